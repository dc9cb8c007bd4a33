"""Binary collisions on the GPU (App. F) against the oracle: the standalone
`collide` call on a tet-sorted population (cells of every size from 1 to
60, odd ones included, and long runs of up to 3001 that take the
workgroup ranking path), in FP64 and mixed precision, and the coupled
cycle with collisions after every re-sort."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_08125_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic as P
    P.load_library()
    return P


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _population(mesh, om, seed=3):
    """Cells of sizes 1..60 and a few long runs (tets chosen at random,
    ascending), velocities
    of a few nm/fs, unit weights, scattered ids."""
    rng = np.random.default_rng(seed)
    T = om.tets()
    sizes = np.concatenate([np.arange(1, 61), [65, 100, 257, 1000, 2049, 3001],
                            rng.integers(1, 6, 3000)])
    sizes = sizes[rng.permutation(sizes.size)]
    cells = np.sort(rng.choice(om.n_tets, sizes.size, replace=False))
    tet = np.repeat(cells, sizes).astype(np.int32)
    n = tet.size
    pos = T["vert"].mean(axis=1)[tet]
    vel = rng.normal(0.0, 1.5, (n, 3))
    ids = rng.permutation(n).astype(np.int64) * 13 + 5
    return tet, pos, vel, ids


def _gpu_state(pic, gm, tet, pos, vel, ids, precision):
    n = tet.size
    gs = pic.State(gm, n + 16, precision=precision)
    dt = gs.x.dtype
    for k, col in enumerate((gs.x, gs.y, gs.z)):
        col[:n] = torch.from_numpy(pos[:, k]).to(dt)
    for k, col in enumerate((gs.vx, gs.vy, gs.vz)):
        col[:n] = torch.from_numpy(vel[:, k]).to(dt)
    gs.w[:n] = 1.0
    gs.tet[:n] = torch.from_numpy(tet)
    gs.id[:n] = torch.from_numpy(ids)
    gs.n_slots[0] = n
    return gs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_collide_matches_oracle(pic, tiny_mesh, precision):
    om = O.OracleMesh(tiny_mesh, 0.01)
    gm = pic.Mesh(tiny_mesh, 0.01)
    tet, pos, vel, ids = _population(tiny_mesh, om)
    mixed = precision == "mixed"
    if mixed:
        vel = vel.astype(np.float32).astype(np.float64)
    gs = _gpu_state(pic, gm, tet, pos, vel, ids,
                    pic.PIC_MIXED if mixed else pic.PIC_FP64)
    ost = O.OracleState(om, tet.size + 16)
    ost.add(pos, vel, tet, ids=ids)
    kw = dict(dt_coll=2.0, w_sp=2e-5, seed=77, step=11)
    gs.collide(**kw)
    ost.collide(**kw)
    torch.cuda.synchronize()
    n = tet.size
    vg = np.stack([t[:n].cpu().numpy().astype(np.float64)
                   for t in (gs.vx, gs.vy, gs.vz)], 1)
    vo = np.stack([ost.vx[:n], ost.vy[:n], ost.vz[:n]], 1)
    assert not np.array_equal(vo, vel)            # collisions happened
    moved = np.any(vo != vel, axis=1)
    # every superparticle in a cell of two or more collided
    cnt = np.bincount(np.searchsorted(np.unique(tet), tet))
    multi = np.repeat(cnt >= 2, cnt)
    assert moved[multi].all() and not moved[~multi].any()
    assert _rel(vg, vo) < (1e-6 if mixed else 1e-12)
    # positions, tets and ids untouched
    assert (gs.tet[:n].cpu().numpy() == tet).all()
    assert (gs.id[:n].cpu().numpy() == ids).all()
    if not mixed:
        # per-cell momentum and energy on the device result
        for c in np.unique(tet)[:200]:
            sel = tet == c
            assert np.abs(vg[sel].sum(0) - vel[sel].sum(0)).max() < 1e-12 * \
                max(1.0, np.abs(vel[sel]).sum())
            e0, e1 = (vel[sel] ** 2).sum(), (vg[sel] ** 2).sum()
            assert abs(e1 - e0) <= 1e-12 * e0


def test_collide_checks_arguments(pic, tiny_mesh):
    gm = pic.Mesh(tiny_mesh, 0.01)
    gs = pic.State(gm, 64)
    with pytest.raises(pic.PicError):
        gs.collide(dt_coll=0.0, w_sp=1.0, seed=1, step=0)
    with pytest.raises(pic.PicError):   # collisions need re-sorting
        gs.init_field(0.4)
        gs.step(dt=0.5, E0=0.4, w_sp=1e-3, phi_w=4.5, step0=0, seed=1,
                collide=1, resort_every=0)


def _run(pic, cfg, n_steps, collide, precision=0):
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, 60_000)
    ost.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = om.emission_rate(ost.E, cfg.phi_w)
    per_run = rate * cfg.dt * cfg.transit_steps
    j_scale = 0.01 / per_run
    w_sp = 0.01 / 3000
    gm = pic.Mesh(tip, cfg.emit_zmin)
    gs = pic.State(gm, 60_000, precision=precision)
    gs.init_field(cfg.E0, tol=cfg.tol)
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, seed=cfg.seed,
              j_scale=j_scale, tol=cfg.tol)
    so, sg = [], []
    for k in range(n_steps):
        so.append(ost.step(step=k, collide_every=5 if collide else 0, **kw))
        sg.append(pic.State.decode_stats(
            gs.step(step0=k, resort_every=5, collide=collide, **kw))[0])
    torch.cuda.synchronize()
    return ost, gs, so, sg


def test_pic_step_with_collisions_matches_oracle(pic):
    """Tiny tip with space charge, collisions after every re-sort (every 5
    steps): counts, ids, tets and charge as in the oracle, positions,
    velocities and potential to 1e-9; the collisions change the result."""
    cfg = W.config_tiny()
    ost, gs, so, sg = _run(pic, cfg, 20, 1)
    for k, (a, b) in enumerate(zip(so, sg)):
        for key in ("n_inj", "n_anode", "n_cathode", "n_after", "q_after",
                    "status"):
            assert a[key] == b[key], (k, key, a[key], b[key])
    P, Q = gs.live(), ost.particles()
    ia, ib = np.argsort(P["id"]), np.argsort(Q["id"])
    assert (P["id"][ia] == Q["id"][ib]).all()
    assert (P["tet"][ia] == Q["tet"][ib]).all()
    for f in (("x", "y", "z"), ("vx", "vy", "vz")):
        g = np.stack([P[c][ia] for c in f], 1)
        o = np.stack([Q[c][ib] for c in f], 1)
        assert _rel(g, o) < 1e-9, f
    assert _rel(gs.phi.cpu().numpy(), ost.phi) < 1e-9
    assert int(gs.charge.sum().item()) == int(ost.c.sum())
    # without collisions the velocities differ
    ost0, gs0, _, _ = _run(pic, cfg, 20, 0)
    R = gs0.live()
    ic = np.argsort(R["id"])
    common = min(ia.size, ic.size)
    assert not np.allclose(P["vx"][ia][:common], R["vx"][ic][:common],
                           rtol=1e-6, atol=0)


def test_collide_edge_cases(pic, tiny_mesh):
    """No superparticles, and only singletons (nothing to pair): the call
    succeeds and no velocity changes; a step with collisions on an empty
    gap does too."""
    om = O.OracleMesh(tiny_mesh, 0.01)
    gm = pic.Mesh(tiny_mesh, 0.01)
    gs = pic.State(gm, 64)
    gs.collide(dt_coll=1.0, w_sp=1.0, seed=1, step=0)
    T = om.tets()
    tet = np.arange(0, 40, 2, dtype=np.int32)          # one per tet
    pos = T["vert"].mean(axis=1)[tet]
    vel = np.random.default_rng(2).normal(size=(tet.size, 3))
    g1 = _gpu_state(pic, gm, tet, pos, vel, np.arange(tet.size) * 3 + 1,
                    pic.PIC_FP64)
    g1.collide(dt_coll=1.0, w_sp=1.0, seed=1, step=0)
    torch.cuda.synchronize()
    assert np.array_equal(g1.vx[:tet.size].cpu().numpy(), vel[:, 0])
    # nearly equal velocities (the variance overflows): finite, as the oracle
    pair = np.array([5, 5], dtype=np.int32)
    vv = np.array([[0.3, -0.2, 1.1], [0.3, -0.2, 1.1 + 1e-120]])
    g3 = _gpu_state(pic, gm, pair, T["vert"].mean(axis=1)[pair], vv,
                    np.array([7, 9]), pic.PIC_FP64)
    g3.collide(dt_coll=1.0, w_sp=1.0, seed=1, step=0)
    o3 = O.OracleState(om, 4)
    o3.add(T["vert"].mean(axis=1)[pair], vv, pair, ids=np.array([7, 9]))
    o3.collide(dt_coll=1.0, w_sp=1.0, seed=1, step=0)
    vg = np.stack([t[:2].cpu().numpy() for t in (g3.vx, g3.vy, g3.vz)], 1)
    assert np.isfinite(vg).all()
    assert np.array_equal(vg, np.stack([o3.vx[:2], o3.vy[:2], o3.vz[:2]], 1))
    g2 = pic.State(gm, 64)
    g2.init_field(0.4)
    st = pic.State.decode_stats(g2.step(dt=0.5, E0=0.4, w_sp=1.0, phi_w=4.5,
                                        step0=4, seed=1, collide=1,
                                        resort_every=5, j_scale=0.0))[0]
    assert st["status"] == 0 and st["n_after"] == 0


def test_pic_step_with_collisions_mixed(pic):
    """The same run in mixed precision (FP32 velocities collided in FP64
    arithmetic): against the FP64 oracle within the mixed-precision bound."""
    from tests.test_gpu_parity import _compare_mixed
    cfg = W.config_tiny()
    ost, gs, so, sg = _run(pic, cfg, 15, 1, precision=pic.PIC_MIXED)
    err = [_rel(gs.phi.cpu().numpy(), ost.phi)]
    _compare_mixed(ost, gs, so, sg, err)
