"""Batched stepping (pic_batch_step): three uneven instances advanced in
shared launches, each checked against the oracle like a single run, and
against the single-instance entry point (integer results bit-exact)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_08125_amd import workloads as W
from tests.test_gpu_parity import _compare_runs, _rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic as P
    P.load_library()
    return P


def _cases():
    base = W.config_tiny()
    return [
        base,
        W.RunConfig("tiny_b", 12, 12, 24, 0.5, 1.5, 6.0, 0.5, 4.5, 0.5, 10,
                     1e-12, 4000, 0.01, 3, 0, 8),
        W.RunConfig("tiny_c", 16, 16, 32, 0.5, 2.5, 7.0, 0.35, 4.5, 0.5, 10,
                    1e-12, 6000, 0.01, 5, 0, 10),
    ]


def _setup(pic, cfg, live_charge, n_live, cap):
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, cap)
    ost.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = om.emission_rate(ost.E, cfg.phi_w)
    per_run = rate * cfg.dt * cfg.transit_steps
    j_scale = live_charge / per_run
    w_sp = per_run * j_scale / n_live
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w,
              seed=cfg.seed, j_scale=j_scale, tol=cfg.tol)
    gm = pic.Mesh(tip, cfg.emit_zmin)
    return tip, om, ost, gm, kw


def test_batch_matches_oracle_and_single(pic):
    cap, steps = 40_000, 12
    cases = [_setup(pic, c, 0.01, 3000, cap) for c in _cases()]
    states, params = [], []
    for tip, om, ost, gm, kw in cases:
        gs = pic.State(gm, cap)
        gs.init_field(kw["E0"], tol=kw["tol"])
        states.append(gs)
        params.append(dict(kw, resort_every=5))
    batch = pic.Batch([c[3] for c in cases], states, params)
    so_all = [[] for _ in cases]
    sg_all = [[] for _ in cases]
    for k in range(steps):
        for i, (tip, om, ost, gm, kw) in enumerate(cases):
            so_all[i].append(ost.step(step=k, **kw))
        rows = pic.Batch.decode(batch.step(k, 1), len(cases))[0]
        for i in range(len(cases)):
            sg_all[i].append(rows[i])
    torch.cuda.synchronize()
    assert any(s["cg_iters"] > 0 for s in sg_all[0][1:])
    for i, (tip, om, ost, gm, kw) in enumerate(cases):
        _compare_runs(ost, states[i], so_all[i], sg_all[i])
    # the single-instance path from the same start gives the same integers
    for i, (tip, om, ost, gm, kw) in enumerate(cases):
        g2 = pic.State(gm, cap)
        g2.init_field(kw["E0"], tol=kw["tol"])
        for k in range(steps):
            g2.step(step0=k, resort_every=5, **kw)
        A, B = g2.live(), states[i].live()
        a, b = np.argsort(A["id"]), np.argsort(B["id"])
        assert (A["id"][a] == B["id"][b]).all()
        assert (A["tet"][a] == B["tet"][b]).all()
        # the solver's reduction order differs with its workgroup count, so
        # positions agree to rounding and node charges to a few units
        dc = (g2.charge - states[i].charge).abs().max().item()
        assert dc <= 4
        assert int(g2.charge.sum()) == int(states[i].charge.sum())
        assert _rel(B["x"][b], A["x"][a]) < 1e-12


def test_batch_autotune_and_mixed(pic):
    """Mixed precision batch with the autotuned schedule stays within the
    mixed-precision bound of the oracle."""
    cap, steps = 40_000, 8
    cases = [_setup(pic, c, 0.01, 3000, cap) for c in _cases()]
    states, params = [], []
    for tip, om, ost, gm, kw in cases:
        gs = pic.State(gm, cap, precision=pic.PIC_MIXED)
        gs.init_field(kw["E0"], tol=kw["tol"])
        states.append(gs)
        params.append(dict(kw))
    batch = pic.Batch([c[3] for c in cases], states, params)
    for k in range(3):   # some particles in flight before tuning
        batch.step(k, 1)
    for i, (tip, om, ost, gm, kw) in enumerate(cases):
        for k in range(3):
            ost.step(step=k, **kw)
    best = batch.autotune(3, push_tiles=(256, 1024), cg_rows=(256, 2048))
    assert len(batch.tuning) == 4 and best[2] > 0
    for k in range(3, steps):
        batch.step(k, 1)
        for i, (tip, om, ost, gm, kw) in enumerate(cases):
            ost.step(step=k, **kw)
    torch.cuda.synchronize()
    for i, (tip, om, ost, gm, kw) in enumerate(cases):
        assert _rel(states[i].phi.cpu().numpy(), ost.phi) < 1e-6
        P, Q = states[i].live(), ost.particles()
        common, ia, ib = np.intersect1d(P["id"], Q["id"], return_indices=True)
        assert common.size >= 0.999 * max(P["id"].size, Q["id"].size)
        pg = np.stack([P["x"][ia], P["y"][ia], P["z"][ia]], 1)
        po = np.stack([Q["x"][ib], Q["y"][ib], Q["z"][ib]], 1)
        assert _rel(pg, po) < 1e-6


def test_batch_with_collisions_matches_oracle(pic):
    """Binary collisions after every re-sort in the batched path: each
    instance as in the oracle with collisions every 5 steps."""
    cap, steps = 40_000, 10
    cases = [_setup(pic, c, 0.01, 3000, cap) for c in _cases()[:2]]
    states, params = [], []
    for tip, om, ost, gm, kw in cases:
        gs = pic.State(gm, cap)
        gs.init_field(kw["E0"], tol=kw["tol"])
        states.append(gs)
        params.append(dict(kw, resort_every=5, collide=1))
    batch = pic.Batch([c[3] for c in cases], states, params)
    so_all = [[] for _ in cases]
    sg_all = [[] for _ in cases]
    for k in range(steps):
        for i, (tip, om, ost, gm, kw) in enumerate(cases):
            so_all[i].append(ost.step(step=k, collide_every=5, **kw))
        rows = pic.Batch.decode(batch.step(k, 1), len(cases))[0]
        for i in range(len(cases)):
            sg_all[i].append(rows[i])
    torch.cuda.synchronize()
    for i, (tip, om, ost, gm, kw) in enumerate(cases):
        _compare_runs(ost, states[i], so_all[i], sg_all[i])


def test_batch_held_counts(pic):
    """Held emission counts per instance in the batched path: every
    instance injects exactly its counts_in and reports them in counts_out."""
    cap = 40_000
    cases = [_setup(pic, c, 0.01, 3000, cap) for c in _cases()[:2]]
    rng = np.random.default_rng(8)
    states, params, held, outs = [], [], [], []
    for tip, om, ost, gm, kw in cases:
        gs = pic.State(gm, cap)
        gs.init_field(kw["E0"], tol=kw["tol"])
        states.append(gs)
        h = rng.integers(0, 3, om.n_emit).astype(np.int32)
        held.append(h)
        o = torch.zeros(om.n_emit, dtype=torch.int32, device="cuda")
        outs.append(o)
        params.append(dict(kw, counts_in=torch.from_numpy(h).cuda(),
                           counts_out=o))
    batch = pic.Batch([c[3] for c in cases], states, params)
    rows = pic.Batch.decode(batch.step(0, 1), len(cases))[0]
    torch.cuda.synchronize()
    for i in range(len(cases)):
        assert rows[i]["n_inj"] == int(held[i].sum())
        assert (outs[i].cpu().numpy() == held[i]).all()


@pytest.mark.parametrize("layout", ["amg_jacobi_amg", "all_amg"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_amg_instances(pic, precision, layout):
    """Instances preconditioned by AMG, next to a Jacobi one or all of them,
    in one batch (AMG instances iterating in the same round share the
    V-cycle launches, each stage one launch over their hierarchies of
    different depths; in mixed precision the V-cycle runs in FP32 inside the
    FP64 CG): every instance against the oracle, with the FP64 bounds
    (counts, ids, tets exact; positions and phi 1e-9) or the mixed-precision
    ones, and fewer iterations for the AMG ones."""
    cap, steps = 40_000, 12
    cases = [_setup(pic, c, 0.01, 3000, cap) for c in _cases()]
    mixed = precision == "mixed"
    A, J = pic.PIC_PRECOND_AMG, pic.PIC_PRECOND_JACOBI
    pre = [A, J, A] if layout == "amg_jacobi_amg" else [A, A, A]
    states, params = [], []
    for (tip, om, ost, gm, kw), pc in zip(cases, pre):
        gs = pic.State(gm, cap, precision=pic.PIC_MIXED if mixed else pic.PIC_FP64,
                       precond=pc)
        gs.init_field(kw["E0"], tol=kw["tol"])
        states.append(gs)
        params.append(dict(kw, resort_every=5))
    batch = pic.Batch([c[3] for c in cases], states, params)
    so_all = [[] for _ in cases]
    sg_all = [[] for _ in cases]
    for k in range(steps):
        for i, (tip, om, ost, gm, kw) in enumerate(cases):
            so_all[i].append(ost.step(step=k, **kw))
        rows = pic.Batch.decode(batch.step(k, 1), len(cases))[0]
        for i in range(len(cases)):
            sg_all[i].append(rows[i])
    torch.cuda.synchronize()
    for i, (tip, om, ost, gm, kw) in enumerate(cases):
        it_g = sum(s["cg_iters"] for s in sg_all[i])
        it_o = sum(s["cg_iters"] for s in so_all[i])
        print(i, "precond", pre[i], "iterations", it_g, "oracle", it_o)
        assert it_o > 0
        if pre[i] == pic.PIC_PRECOND_AMG:
            assert it_g < it_o
        if mixed:
            assert _rel(states[i].phi.cpu().numpy(), ost.phi) < 1e-6
            P, Q = states[i].live(), ost.particles()
            common, ia, ib = np.intersect1d(P["id"], Q["id"], return_indices=True)
            assert common.size >= 0.999 * max(P["id"].size, Q["id"].size)
            pg = np.stack([P["x"][ia], P["y"][ia], P["z"][ia]], 1)
            po = np.stack([Q["x"][ib], Q["y"][ib], Q["z"][ib]], 1)
            assert _rel(pg, po) < 1e-6
        else:
            _compare_runs(ost, states[i], so_all[i], sg_all[i],
                          same_solver=pre[i] == pic.PIC_PRECOND_JACOBI)
