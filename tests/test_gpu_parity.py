"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Integer results (tet ids, where-codes, fixed-point charge, particle counts,
collected charge) must be bit-exact; floating-point results meet the
relative-L2 bound of 1e-9 (potential, positions)."""
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


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


MESHES = {
    "small_tip": lambda: W.kuhn_tip_mesh(3, 3, 4, 0.5, 0.5, 1.0),
    "plates": lambda: W.kuhn_tip_mesh(4, 4, 8, 0.5),
    "tiny_tip": lambda: W.config_tiny().mesh(),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_mesh_counts_and_faces(pic, name):
    tip = MESHES[name]()
    zmin = 0.01 if name != "plates" else -1.0
    om = O.OracleMesh(tip, zmin)
    gm = pic.Mesh(tip, zmin)
    i = gm.info
    print(name, i)
    assert (i["n_nodes"], i["n_tets"], i["n_free"], i["nnz"], i["n_emit"],
            i["n_top"], i["n_metal"]) == (om.n_nodes, om.n_tets, om.n_free,
                                          om.nnz, om.n_emit, om.n_top,
                                          om.n_metal)
    ge = gm.emit_faces()
    oe = om.emit()
    assert (ge["tet"] == oe["tet"]).all()
    assert (ge["nodes"] == oe["nodes"]).all()
    assert (ge["area"] == oe["area"]).all()


def test_poisson_plates_closed_form(pic):
    tip = MESHES["plates"]()
    gm = pic.Mesh(tip, 0.01)
    phi = torch.zeros(tip.n_nodes, dtype=torch.float64, device="cuda")
    E = torch.zeros(4 * tip.n_nodes, dtype=torch.float64, device="cuda")
    st = gm.poisson_solve(None, 0.0, 0.7, phi, E, tol=1e-13)
    s = gm.solve_stats(st)
    assert s["status"] == 0 and s["relres"] <= 1e-13
    assert np.abs(phi.cpu().numpy() - 0.7 * tip.xyz[:, 2]).max() < 1e-11
    e = E.cpu().numpy().reshape(-1, 4)
    assert np.abs(e[:, :3] - np.array([0, 0, -0.7])).max() < 1e-10
    assert (e[:, 3] == 0).all()


@pytest.mark.parametrize("name", ["small_tip", "tiny_tip"])
def test_poisson_matches_oracle(pic, name):
    tip = MESHES[name]()
    om = O.OracleMesh(tip, 0.01)
    gm = pic.Mesh(tip, 0.01)
    rng = np.random.default_rng(3)
    c = rng.integers(-2**44, 2**44, tip.n_nodes).astype(np.int64)
    phi_o, info = om.poisson_solve(c, 1e-3, 0.4, tol=1e-12)
    E_o = om.field(phi_o)
    phi = torch.zeros(tip.n_nodes, dtype=torch.float64, device="cuda")
    E = torch.zeros(4 * tip.n_nodes, dtype=torch.float64, device="cuda")
    st = gm.poisson_solve(_dev(c), 1e-3, 0.4, phi, E, tol=1e-12)
    s = gm.solve_stats(st)
    print(name, s, info)
    assert s["status"] == 0 and s["relres"] <= 1e-12
    assert abs(s["iters"] - info["iters"]) <= 3
    assert _rel(phi.cpu().numpy(), phi_o) < 1e-9
    e = E.cpu().numpy().reshape(-1, 4)[:, :3]
    assert _rel(e, E_o) < 1e-9
    # warm start from the solution: zero iterations, unchanged potential
    phi2 = phi.clone()
    st2 = gm.poisson_solve(_dev(c), 1e-3, 0.4, phi2, None, tol=1e-12)
    assert gm.solve_stats(st2)["iters"] == 0
    assert torch.equal(phi2, phi)


@pytest.mark.parametrize("name", ["small_tip", "tiny_tip"])
def test_poisson_amg_matches_oracle(pic, name):
    """The smoothed-aggregation AMG preconditioner: the same potential and
    field as the oracle's Jacobi-PCG solution to the paper's tolerance, in
    a small fraction of the Jacobi iterations; the hierarchy is reused by a
    second solve and a warm start from the solution needs no iteration."""
    tip = MESHES[name]()
    om = O.OracleMesh(tip, 0.01)
    gm = pic.Mesh(tip, 0.01)
    rng = np.random.default_rng(5)
    c = rng.integers(-2**44, 2**44, tip.n_nodes).astype(np.int64)
    phi_o, info = om.poisson_solve(c, 1e-3, 0.4, tol=1e-12)
    E_o = om.field(phi_o)
    for rep in range(2):
        phi = torch.zeros(tip.n_nodes, dtype=torch.float64, device="cuda")
        E = torch.zeros(4 * tip.n_nodes, dtype=torch.float64, device="cuda")
        st = gm.poisson_solve(_dev(c), 1e-3, 0.4, phi, E, tol=1e-12,
                              precond=pic.PIC_PRECOND_AMG)
        s = gm.solve_stats(st)
        print(name, rep, s, info["iters"])
        assert s["status"] == 0 and s["relres"] <= 1e-12
        assert s["iters"] <= max(info["iters"] // 4, 10)
        assert _rel(phi.cpu().numpy(), phi_o) < 1e-9
        e = E.cpu().numpy().reshape(-1, 4)[:, :3]
        assert _rel(e, E_o) < 1e-9
    st2 = gm.poisson_solve(_dev(c), 1e-3, 0.4, phi, None, tol=1e-12,
                           precond=pic.PIC_PRECOND_AMG)
    assert gm.solve_stats(st2)["iters"] == 0
    # mixed precision: the V-cycle in FP32 inside the FP64 CG; the stopping
    # test stays on the FP64 true residual, so the potential is the FP64 one
    phi3 = torch.zeros(tip.n_nodes, dtype=torch.float64, device="cuda")
    E3 = torch.zeros(4 * tip.n_nodes, dtype=torch.float32, device="cuda")
    st3 = gm.poisson_solve(_dev(c), 1e-3, 0.4, phi3, E3, tol=1e-12,
                           precision=pic.PIC_MIXED, precond=pic.PIC_PRECOND_AMG)
    s3 = gm.solve_stats(st3)
    print(name, "fp32 v-cycle", s3)
    assert s3["status"] == 0 and s3["relres"] <= 1e-12
    assert s3["restarts"] <= 2
    assert s3["iters"] <= max(info["iters"] // 4, 10)
    assert _rel(phi3.cpu().numpy(), phi_o) < 1e-9
    assert _rel(E3.cpu().numpy().reshape(-1, 4)[:, :3], E_o) < 1e-6


def _locate_case(pic, tip, pts, hint=None):
    om = O.OracleMesh(tip, 0.01)
    gm = pic.Mesh(tip, 0.01)
    t_o, w_o = om.locate(pts, hint)
    x, y, z = (_dev(pts[:, k].copy()) for k in range(3))
    h = np.full(len(pts), -1, np.int32) if hint is None else hint
    tet = _dev(h.astype(np.int32))
    where = torch.zeros(len(pts), dtype=torch.uint8, device="cuda")
    gm.locate(x, y, z, tet, where)
    assert (tet.cpu().numpy() == t_o).all()
    assert (where.cpu().numpy() == w_o).all()
    return t_o


@pytest.mark.parametrize("name", ["small_tip", "tiny_tip"])
def test_locate_bit_exact(pic, name):
    tip = MESHES[name]()
    pts = np.concatenate([W.random_points_in_box(tip, 20000, 5),
                          W.lattice_points(tip, 5000, 6)])
    t_o = _locate_case(pic, tip, pts)
    # hints: the answer itself, a random tet, and -1
    rng = np.random.default_rng(1)
    om = O.OracleMesh(tip, 0.01)
    hint = np.where(rng.random(len(pts)) < 0.5, t_o,
                    rng.integers(0, om.n_tets, len(pts))).astype(np.int32)
    _locate_case(pic, tip, pts, hint)


@pytest.mark.parametrize("name", ["small_tip", "tiny_tip"])
def test_locate_on_face_interiors(pic, name):
    """Points exactly on the relative interior of random faces (dyadic
    weights of the face's three vertices, exact in FP64; the case a
    position stored in FP32 meets most often): the oracle's canonical tet
    (the lower index of the two holding the point, or the one tet on a
    boundary or periodic face; both occur), from hints on either side of
    the face and far away."""
    tip = MESHES[name]()
    rng = np.random.default_rng(11)
    n = 6000
    t = rng.integers(0, tip.n_tets, n)
    k = rng.integers(0, 4, n)                   # the face opposite vertex k
    wts = np.array([[0.25, 0.25, 0.5], [0.125, 0.375, 0.5],
                    [0.375, 0.375, 0.25]])[rng.integers(0, 3, n)]
    V = tip.xyz[tip.tet[t]].copy()              # [n, 4, 3]
    V[:, :, 0] += tip.shift[t, :, 0] * tip.Lx
    V[:, :, 1] += tip.shift[t, :, 1] * tip.Ly
    others = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])[k]
    F = np.take_along_axis(V, others[:, :, None], axis=1)   # [n, 3, 3]
    pts = np.einsum("nj,njc->nc", wts, F)
    keep = (pts[:, 0] < tip.Lx) & (pts[:, 1] < tip.Ly) & (pts[:, 2] < tip.z_top)
    pts, t = pts[keep], t[keep]
    t_o = _locate_case(pic, tip, pts, t.astype(np.int32))
    assert (t_o >= 0).mean() > 0.9
    _locate_case(pic, tip, pts, t_o.astype(np.int32))
    far = rng.integers(0, tip.n_tets, len(pts)).astype(np.int32)
    _locate_case(pic, tip, pts, far)


def test_locate_empty(pic):
    tip = MESHES["small_tip"]()
    gm = pic.Mesh(tip, 0.01)
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    gm.locate(e, e, e, torch.zeros(0, dtype=torch.int32, device="cuda"),
              torch.zeros(0, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("name", ["small_tip", "tiny_tip"])
def test_deposit_bit_exact(pic, name):
    tip = MESHES[name]()
    om = O.OracleMesh(tip, 0.01)
    gm = pic.Mesh(tip, 0.01)
    pts = np.concatenate([W.random_points_in_box(tip, 30000, 7),
                          W.lattice_points(tip, 3000, 8)])
    tet, where = om.locate(pts)
    keep = where == 0
    pts, tet = pts[keep], tet[keep]
    w = np.random.default_rng(2).uniform(0.1, 2.0, len(pts))
    c_o = om.deposit(pts, tet, w)
    c = torch.zeros(tip.n_nodes, dtype=torch.int64, device="cuda")
    args = [_dev(pts[:, k].copy()) for k in range(3)]
    gm.deposit(*args, _dev(tet), _dev(w), c)
    assert (c.cpu().numpy() == c_o).all()
    # order independence on the device
    perm = np.random.default_rng(3).permutation(len(pts))
    c2 = torch.zeros_like(c)
    gm.deposit(*[_dev(pts[perm, k].copy()) for k in range(3)],
               _dev(tet[perm]), _dev(w[perm]), c2)
    assert torch.equal(c, c2)


def test_emission_rate_matches_oracle(pic):
    cfg = W.config_tiny()
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, 10)
    ost.init_field(cfg.E0, tol=1e-12)
    r_o, F_o = om.emission_rate(ost.E, cfg.phi_w)
    gm = pic.Mesh(tip, cfg.emit_zmin)
    gs = pic.State(gm, 10)
    gs.init_field(cfg.E0, tol=1e-12)
    rate, F = gm.emission_rate(gs.E, cfg.phi_w)
    assert abs(rate.item() / r_o - 1) < 1e-8
    assert _rel(F.cpu().numpy(), F_o) < 1e-10


def _run_pair(pic, cfg, n_steps, live_charge, n_live, cap, seed=None,
              resort_every=0, precision=0, solve_precision=None,
              phi_err=None, precond=0, field_mode=0):
    """live_charge: electrons in flight wanted (None = physical emission).
    phi_err: a list that receives the relative L2 distance of the device
    potential from the oracle's after every step."""
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, cap)
    ost.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = om.emission_rate(ost.E, cfg.phi_w,
                               ost.phi if field_mode == 1 else None)
    per_run = rate * cfg.dt * cfg.transit_steps
    j_scale = 1.0 if live_charge is None else live_charge / per_run
    w_sp = per_run * j_scale / n_live
    gm = pic.Mesh(tip, cfg.emit_zmin)
    gs = pic.State(gm, cap, precision=precision,
                   solve_precision=solve_precision, precond=precond)
    gs.init_field(cfg.E0, tol=cfg.tol)
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w,
              seed=cfg.seed if seed is None else seed, j_scale=j_scale,
              tol=cfg.tol)
    so_all, sg_all = [], []
    for k in range(n_steps):
        so_all.append(ost.step(step=k, field_mode=field_mode, **kw))
        sg_all.append(pic.State.decode_stats(
            gs.step(step0=k, resort_every=resort_every, field_mode=field_mode,
                    **kw))[0])
        if phi_err is not None:
            phi_err.append(_rel(gs.phi.cpu().numpy(), ost.phi))
    torch.cuda.synchronize()
    return om, ost, gm, gs, so_all, sg_all


def _compare_runs(ost, gs, so_all, sg_all, same_solver=True):
    for k, (so, sg) in enumerate(zip(so_all, sg_all)):
        for key in ("n_inj", "n_anode", "n_cathode", "n_after", "q_before",
                    "q_inj", "q_anode", "q_cathode", "q_after", "status",
                    "n_trunc", "n_clamp"):
            assert so[key] == sg[key], (k, key, so[key], sg[key])
        if same_solver:
            assert abs(so["cg_iters"] - sg["cg_iters"]) <= 3
        else:
            assert sg["cg_iters"] <= so["cg_iters"] + 1
        assert sg["cg_relres"] <= 1e-12 or sg["cg_iters"] == 0
        for key in ("emit_current", "mean_face_E", "max_face_E"):
            assert abs(sg[key] - so[key]) <= 1e-9 * abs(so[key]) + 1e-300
        # fixed-point conservation on the device
        assert sg["q_before"] + sg["q_inj"] - sg["q_anode"] - \
            sg["q_cathode"] == sg["q_after"]
    P, Q = gs.live(), ost.particles()
    assert P["id"].size == Q["id"].size
    a = np.argsort(P["id"])
    b = np.argsort(Q["id"])
    assert (P["id"][a] == Q["id"][b]).all()
    assert (P["tet"][a] == Q["tet"][b]).all()
    assert (P["birth"][a] == Q["birth"][b]).all()
    assert (P["w"][a] == Q["w"][b]).all()
    pos_g = np.stack([P["x"][a], P["y"][a], P["z"][a]], 1)
    pos_o = np.stack([Q["x"][b], Q["y"][b], Q["z"][b]], 1)
    assert _rel(pos_g, pos_o) < 1e-9
    vel_g = np.stack([P["vx"][a], P["vy"][a], P["vz"][a]], 1)
    vel_o = np.stack([Q["vx"][b], Q["vy"][b], Q["vz"][b]], 1)
    assert _rel(vel_g, vel_o) < 1e-9
    assert _rel(gs.phi.cpu().numpy(), ost.phi) < 1e-9
    # total deposited charge is exact (per-node values may differ in the
    # last unit where positions differ by rounding)
    assert int(gs.charge.sum().item()) == int(ost.c.sum())


def test_pic_step_tiny_physical(pic):
    """The tiny-tip workload at its physical emission: 10 steps."""
    cfg = W.config_tiny()
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 10, None, 10_000, 60_000)
    assert sum(s["n_inj"] for s in sg) > 1000
    _compare_runs(ost, gs, so, sg)


def test_pic_step_tiny_space_charge(pic):
    """Emission scaled up so that the deposited charge moves the field
    (coupled parity): 8 steps, some particles reach the anode."""
    cfg = W.config_tiny()
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 36, 0.01, 3000, 60_000,
                                        resort_every=5)
    # the space charge is visible in the potential
    assert all(s["cg_iters"] > 0 for s in sg[1:])
    assert sum(s["n_anode"] for s in sg) > 0
    _compare_runs(ost, gs, so, sg)


def test_pic_step_space_charge_amg(pic):
    """The coupled space-charge run with the AMG-preconditioned solve: every
    count, charge and particle as in the oracle (whose solve is Jacobi-PCG
    to the same tolerance), with fewer iterations per step."""
    cfg = W.config_tiny()
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 12, 0.01, 3000, 60_000,
                                        resort_every=5,
                                        precond=pic.PIC_PRECOND_AMG)
    assert sum(s["cg_iters"] for s in sg) < sum(s["cg_iters"] for s in so)
    _compare_runs(ost, gs, so, sg, same_solver=False)


def test_pic_step_cell_field(pic):
    """The cell field mode (E = -(grad phi)_t in the particle's tet; the
    emitting face's tet for the FN current and the injection velocity) with
    space charge and re-sorting: every count, charge and particle as in the
    oracle's cell mode."""
    cfg = W.config_tiny()
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 24, 0.01, 3000, 60_000,
                                        resort_every=5,
                                        field_mode=pic.PIC_FIELD_CELL)
    assert sum(s["n_inj"] for s in sg) > 1000
    assert all(s["cg_iters"] > 0 for s in sg[1:])
    _compare_runs(ost, gs, so, sg)


def test_pic_step_cell_field_differs_from_nodal(pic):
    """The two field modes give different trajectories (the mode reaches
    the kernels), and the cell-mode FN current is that of the oracle's
    per-tet field of the device potential."""
    cfg = W.config_tiny()
    runs = []
    for mode in (pic.PIC_FIELD_NODAL, pic.PIC_FIELD_CELL):
        om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 4, None, 10_000, 60_000,
                                            field_mode=mode)
        runs.append((gs.live(), sg))
    (P0, s0), (P1, s1) = runs
    assert s0[0]["emit_current"] != s1[0]["emit_current"]
    a, b = np.argsort(P0["id"]), np.argsort(P1["id"])
    n = min(a.size, b.size)
    assert not np.array_equal(P0["z"][a][:n], P1["z"][b][:n])


def test_pic_step_cell_field_mixed(pic):
    """The cell field mode in mixed precision (FP32 particles; the field
    from FP64 potential differences rounded to FP32)."""
    cfg = W.config_tiny()
    err = []
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 12, 0.01, 3000, 60_000,
                                        resort_every=5,
                                        precision=pic.PIC_MIXED,
                                        phi_err=err,
                                        field_mode=pic.PIC_FIELD_CELL)
    _compare_mixed(ost, gs, so, sg, err)


def test_field_mode_checked(pic):
    cfg = W.config_tiny()
    tip = cfg.mesh()
    gm = pic.Mesh(tip, cfg.emit_zmin)
    gs = pic.State(gm, 1000)
    gs.init_field(cfg.E0, tol=cfg.tol)
    with pytest.raises(pic.PicError):
        gs.step(dt=cfg.dt, E0=cfg.E0, w_sp=1e-3, phi_w=cfg.phi_w, step0=0,
                seed=1, field_mode=7)


def test_pic_step_deterministic(pic):
    cfg = W.config_tiny()
    outs = []
    for _ in range(2):
        _, _, gm, gs, _, sg = _run_pair(pic, cfg, 8, 0.01, 3000, 60_000,
                                        resort_every=3)
        P = gs.live()
        outs.append((P, gs.phi.cpu().numpy().copy(), sg))
    (P1, f1, s1), (P2, f2, s2) = outs
    for k in P1:
        assert (P1[k] == P2[k]).all()
    assert (f1 == f2).all()


@pytest.mark.parametrize("live_charge", [None, 0.01])
def test_pic_step_many_per_call(pic, live_charge):
    """Twelve steps in one pic_step call against twelve calls of one step.
    Inside a call, each step's pre-solve kernels are enqueued behind the
    previous solve's first report, gated on its outcome, and the first pass
    of each later solve forms the residual from the previous one ((b -
    b_prev) + r_prev, the same quantity as b - K phi up to rounding).  With
    physical emission no solve iterates and both runs agree bit for bit but
    for the reported residual; with space charge every solve iterates past
    its first round (the gated launches are skipped and enqueued again) and
    the two runs agree to the solver tolerance."""
    cfg = W.config_tiny()
    gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
    runs = []
    for per_call in (1, 12):
        gs = pic.State(gm, 60_000)
        gs.init_field(cfg.E0, tol=cfg.tol)
        rate, _ = gm.emission_rate(gs.E, cfg.phi_w)
        per_run = rate.item() * cfg.dt * cfg.transit_steps
        j_scale = 1.0 if live_charge is None else live_charge / per_run
        kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=per_run * j_scale / 3000,
                  phi_w=cfg.phi_w, seed=cfg.seed, j_scale=j_scale, tol=cfg.tol,
                  resort_every=5)
        recs = []
        for k0 in range(0, 12, per_call):
            recs += pic.State.decode_stats(gs.step(step0=k0, n_steps=per_call, **kw))
        runs.append((gs, recs))
    (ga, ra), (gb, rb) = runs
    exact = live_charge is None
    for a, b in zip(ra, rb):
        for key in ("n_before", "n_inj", "n_anode", "n_cathode", "n_after",
                    "q_before", "q_inj", "q_anode", "q_cathode", "q_after",
                    "status", "n_trunc", "n_fallback", "n_slots"):
            assert a[key] == b[key], key
        assert b["cg_relres"] <= cfg.tol
        if exact:
            assert a["cg_iters"] == b["cg_iters"] == 0
        else:
            assert a["cg_iters"] > 0 and abs(a["cg_iters"] - b["cg_iters"]) <= 3
    n = int(ga.n_slots.item())
    assert n == int(gb.n_slots.item())
    for key in ("tet", "birth", "id", "w"):
        assert torch.equal(getattr(ga, key)[:n], getattr(gb, key)[:n]), key
    for key in ("x", "y", "z", "vx", "vy", "vz"):
        A, B = getattr(ga, key)[:n], getattr(gb, key)[:n]
        if exact:
            assert torch.equal(A, B), key
        else:
            assert ((A - B).norm() / B.norm()).item() <= 1e-9, key
    for key in ("phi", "E"):
        A, B = getattr(ga, key), getattr(gb, key)
        if exact:
            assert torch.equal(A, B), key
        else:
            assert ((A - B).norm() / B.norm()).item() <= 1e-9, key
    dq = (ga.charge - gb.charge).abs().max().item()
    assert dq == 0 if exact else dq <= 16


def test_pic_step_lean_solve_that_iterates(pic):
    """A step solve after one that needed no iteration starts lean: its
    first pass leaves x and u undone and its test starts no product.  Where
    the warm start then misses the tolerance (the charge in flight grows
    until its change per step matters), the host makes up x and u and the
    test's product before the iterations; the next step's particle launch,
    gated on that test, does nothing and is enqueued again.  The
    space-charge scale is scanned for a call with such a step; the run then
    agrees with one step per call (no lean solves) to the solver tolerance,
    counts exactly."""
    cfg = W.config_tiny()
    gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)

    def run(live_charge, per_call):
        gs = pic.State(gm, 60_000)
        gs.init_field(cfg.E0, tol=cfg.tol)
        rate, _ = gm.emission_rate(gs.E, cfg.phi_w)
        per_run = rate.item() * cfg.dt * cfg.transit_steps
        j_scale = live_charge / per_run
        kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=per_run * j_scale / 3000,
                  phi_w=cfg.phi_w, seed=cfg.seed, j_scale=j_scale, tol=cfg.tol)
        recs = []
        for k0 in range(0, 16, per_call):
            recs += pic.State.decode_stats(gs.step(step0=k0, n_steps=per_call, **kw))
        return gs, recs

    found, seen = None, []
    for lc in (1e-14, 1e-13, 1e-12, 1e-11, 1e-10, 1e-9, 1e-8, 1e-7, 1e-6,
               1e-5, 1e-4, 1e-3):
        gb, rb = run(lc, 16)
        its = [r["cg_iters"] for r in rb]
        seen.append((lc, its))
        if any(its[k - 1] == 0 and its[k] > 0 for k in range(1, 15)):
            found = lc
            break
    assert found is not None, f"no solve iterating after one that did not: {seen}"
    ga, ra = run(found, 1)
    for a, b in zip(ra, rb):
        for key in ("n_before", "n_inj", "n_anode", "n_cathode", "n_after",
                    "q_before", "q_inj", "q_anode", "q_cathode", "q_after",
                    "status", "n_trunc", "n_fallback", "n_slots"):
            assert a[key] == b[key], key
        assert b["status"] == 0
        assert b["cg_relres"] <= cfg.tol
    n = int(ga.n_slots.item())
    assert n == int(gb.n_slots.item())
    for key in ("tet", "birth", "id", "w"):
        assert torch.equal(getattr(ga, key)[:n], getattr(gb, key)[:n]), key
    for key in ("x", "y", "z", "vx", "vy", "vz"):
        A, B = getattr(ga, key)[:n], getattr(gb, key)[:n]
        assert ((A - B).norm() / B.norm()).item() <= 1e-9, key
    for key in ("phi", "E"):
        A, B = getattr(ga, key), getattr(gb, key)
        assert ((A - B).norm() / B.norm()).item() <= 1e-9, key
    assert (ga.charge - gb.charge).abs().max().item() <= 16


def test_wrap_and_absorption_explicit(pic):
    """Hand-placed particles crossing x = L, x = 0, y = L, reaching the
    anode and entering the cathode, on both sides."""
    tip = MESHES["plates"]()
    om = O.OracleMesh(tip, -1.0)
    ost = O.OracleState(om, 16)
    ost.init_field(1e-6, tol=1e-12)
    L, Lz = tip.Lx, tip.z_top
    p = np.array([[L - 0.05, 1.0, 2.0], [0.02, 0.5, 1.0], [1.0, L - 0.01, 3.0],
                  [1.0, 1.0, Lz - 0.1], [1.0, 1.0, 0.1], [0.7, 1.3, 2.2]])
    v = np.array([[0.3, 0, 0], [-0.1, 0, 0], [0, 0.1, 0], [0, 0, 0.5],
                  [0, 0, -0.5], [0.01, -0.02, 0.03]])
    w = np.array([1.0, 0.5, 0.25, 1.0, 0.75, 1.5])
    tet, _ = om.locate(p)
    ost.add(p, v, tet, w=w, ids=np.arange(6))
    gm = pic.Mesh(tip, -1.0)
    gs = pic.State(gm, 16)
    gs.init_field(1e-6, tol=1e-12)
    n = len(p)
    for k, t in enumerate((gs.x, gs.y, gs.z)):
        t[:n] = _dev(p[:, k].copy())
    for k, t in enumerate((gs.vx, gs.vy, gs.vz)):
        t[:n] = _dev(v[:, k].copy())
    gs.w[:n] = _dev(w)
    gs.tet[:n] = _dev(tet)
    gs.id[:n] = _dev(np.arange(6, dtype=np.int64))
    gs.n_slots.fill_(n)
    kw = dict(dt=0.5, E0=1e-6, w_sp=1e-30, phi_w=4.5, seed=1, j_scale=0.0,
              tol=1e-12)
    so = ost.step(step=0, **kw)
    sg = pic.State.decode_stats(gs.step(step0=0, **kw))[0]
    assert sg["n_anode"] == 1 and sg["n_cathode"] == 1
    assert sg["q_anode"] == 2**40 and sg["q_cathode"] == int(0.75 * 2**40)
    _compare_runs(ost, gs, [so], [sg])


def test_resort_compacts_and_orders(pic):
    """After a re-sort the slots hold exactly the live particles, ordered by
    tet (ties in the previous slot order), with the particle set unchanged."""
    cfg = W.config_tiny()
    _, ost, gm, gs, so, sg = _run_pair(pic, cfg, 6, None, 10_000, 60_000,
                                       resort_every=6)
    n = int(gs.n_slots.item())
    tet = gs.tet[:n].cpu().numpy()
    assert n == sg[-1]["n_after"] == sg[-1]["n_slots"]
    assert (tet >= 0).all() and (np.diff(tet) >= 0).all()
    # before this first re-sort the slots held the injected particles in
    # injection order, which is id order: a stable sort keeps ties that way
    ids = gs.id[:n].cpu().numpy()
    assert (np.diff(ids)[np.diff(tet) == 0] > 0).all()
    _compare_runs(ost, gs, so, sg)


def test_resort_three_digit_passes(pic):
    """A mesh of more than 2^16 tets (three 8-bit digit passes) and a
    population spanning several sort tiles: a run that re-sorts after its
    last step holds exactly the particles of the same run without re-sort,
    compacted, ordered by tet, ties in slot (= injection = id) order."""
    cfg = W.batch_configs(1)[0]
    tip = cfg.mesh()
    gm = pic.Mesh(tip, cfg.emit_zmin)
    assert gm.n_tets >= 1 << 16
    out = []
    for every in (0, 8):
        gs = pic.State(gm, 200_000)
        gs.init_field(cfg.E0, tol=cfg.tol)
        rate, _ = gm.emission_rate(gs.E, cfg.phi_w)
        w_sp = rate.item() * cfg.dt * cfg.transit_steps / 100_000
        st = pic.State.decode_stats(gs.step(
            step0=0, n_steps=8, dt=cfg.dt, E0=cfg.E0, w_sp=w_sp,
            phi_w=cfg.phi_w, seed=cfg.seed, tol=cfg.tol, resort_every=every))
        out.append((gs, st))
    (ga, sa), (gb, sb) = out
    A, B = ga.live(), gb.live()
    assert B["id"].size == sb[-1]["n_after"] == int(gb.n_slots.item())
    assert B["id"].size > 3 * 4096
    assert (np.diff(B["tet"]) >= 0).all()
    assert (np.diff(B["id"])[np.diff(B["tet"]) == 0] > 0).all()
    a, b = np.argsort(A["id"]), np.argsort(B["id"])
    for key in ("id", "x", "y", "z", "vx", "vy", "vz", "w", "tet", "birth"):
        assert (A[key][a] == B[key][b]).all(), key


@pytest.mark.parametrize("n_inj", [1, 3, 9, 17, 4101])
def test_resort_small_and_ragged_populations(pic, n_inj):
    """Populations smaller than the sort's eight per-XCD parts of the gather,
    not a multiple of eight, and one tile plus a ragged tail: the step that
    injects exactly n_inj particles (held counts) and re-sorts after itself
    leaves the same particles as the same step without re-sort, compacted
    and ordered by tet (ties in injection = id order)."""
    cfg = W.config_tiny()
    gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
    held = np.zeros(gm.n_emit, np.int32)
    np.add.at(held, np.random.default_rng(n_inj).integers(0, gm.n_emit, n_inj), 1)
    out = []
    for every in (0, 1):
        gs = pic.State(gm, 20_000)
        gs.init_field(cfg.E0, tol=cfg.tol)
        st = pic.State.decode_stats(gs.step(
            step0=0, n_steps=1, dt=cfg.dt, E0=cfg.E0, w_sp=1e-6,
            phi_w=cfg.phi_w, seed=cfg.seed, tol=cfg.tol, resort_every=every,
            counts_in=torch.from_numpy(held).cuda()))
        assert st[0]["n_inj"] == n_inj
        out.append((gs, st))
    (ga, sa), (gb, sb) = out
    A, B = ga.live(), gb.live()
    n_live = sb[-1]["n_after"]
    assert B["id"].size == n_live == int(gb.n_slots.item()) == A["id"].size
    assert (gb.tet[:n_live].cpu().numpy() >= 0).all()
    assert (np.diff(B["tet"]) >= 0).all()
    assert (np.diff(B["id"])[np.diff(B["tet"]) == 0] > 0).all()
    a, b = np.argsort(A["id"]), np.argsort(B["id"])
    for key in ("id", "x", "y", "z", "vx", "vy", "vz", "w", "tet", "birth"):
        assert (A[key][a] == B[key][b]).all(), key


# ---------------------------------------------------------------------------
# Mixed precision: FP32 particles, field and CG recursion against the FP64
# oracle.  Bound: relative L2 <= 1e-6 for the potential (every step) and the
# positions; the particle sets may differ by the rare particle whose count,
# absorption or injection decision sits within FP32 rounding of a threshold.

def _compare_mixed(ost, gs, so_all, sg_all, phi_err, bound=1e-6):
    assert max(phi_err) < bound, phi_err
    for k, (so, sg) in enumerate(zip(so_all, sg_all)):
        assert sg["status"] == 0
        assert sg["cg_relres"] <= 1e-9 or sg["cg_iters"] == 0
        assert sg["q_before"] + sg["q_inj"] - sg["q_anode"] - \
            sg["q_cathode"] == sg["q_after"]
        for key in ("n_inj", "n_anode", "n_cathode", "n_after"):
            assert abs(so[key] - sg[key]) <= 2 + 1e-3 * so[key], (k, key)
    P, Q = gs.live(), ost.particles()
    common, ia, ib = np.intersect1d(P["id"], Q["id"], return_indices=True)
    assert common.size >= 0.999 * max(P["id"].size, Q["id"].size)
    pos_g = np.stack([P["x"][ia], P["y"][ia], P["z"][ia]], 1)
    pos_o = np.stack([Q["x"][ib], Q["y"][ib], Q["z"][ib]], 1)
    assert _rel(pos_g, pos_o) < bound
    vel_g = np.stack([P["vx"][ia], P["vy"][ia], P["vz"][ia]], 1)
    vel_o = np.stack([Q["vx"][ib], Q["vy"][ib], Q["vz"][ib]], 1)
    assert _rel(vel_g, vel_o) < bound
    # where the FP32 positions sit in the same tet, the ids agree exactly
    assert (P["tet"][ia] == Q["tet"][ib]).mean() > 0.999


def test_poisson_mixed_refinement(pic):
    """FP32 recursion + FP64 refinement reaches the FP64 tolerance on the
    true residual; phi then matches the oracle like the FP64 solver."""
    cfg = W.config_tiny()
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    rng = np.random.default_rng(7)
    c = rng.integers(-2**44, 2**44, tip.n_nodes).astype(np.int64)
    phi_o, info = om.poisson_solve(c, 1e-3, cfg.E0, tol=1e-12)
    assert info["status"] == 0
    E_o = om.field(phi_o)
    gm = pic.Mesh(tip, cfg.emit_zmin)
    phi = torch.zeros(tip.n_nodes, dtype=torch.float64, device="cuda")
    E = torch.zeros(4 * tip.n_nodes, dtype=torch.float32, device="cuda")
    st = gm.poisson_solve(_dev(c), 1e-3, cfg.E0, phi, E, tol=1e-11,
                          precision=pic.PIC_MIXED, inner_tol=1e-3)
    s = pic.Mesh.solve_stats(st)
    assert s["status"] == 0 and s["relres"] <= 1e-11
    assert s["restarts"] >= 2          # refinement sweeps did happen
    assert _rel(phi.cpu().numpy(), phi_o) < 1e-9
    Eg = E.cpu().numpy().reshape(-1, 4)[:, :3].astype(np.float64)
    assert _rel(Eg, E_o) < 1e-6


def test_pic_step_mixed_tiny(pic):
    """Mixed precision PIC on the tiny tip, physical emission, 10 steps."""
    cfg = W.config_tiny()
    err = []
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 10, None, 10_000, 60_000,
                                        precision=pic.PIC_MIXED,
                                        phi_err=err)
    assert gs.x.dtype == torch.float32 and gs.E.dtype == torch.float32
    _compare_mixed(ost, gs, so, sg, err)


def test_pic_step_mixed_space_charge(pic):
    """Mixed precision with space charge and re-sorting, 36 steps."""
    cfg = W.config_tiny()
    err = []
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 36, 0.01, 3000, 60_000,
                                        resort_every=5,
                                        precision=pic.PIC_MIXED,
                                        phi_err=err)
    assert all(s["cg_iters"] > 0 for s in sg[1:])
    _compare_mixed(ost, gs, so, sg, err)


def test_pic_step_mixed_amg(pic):
    """Mixed precision with the FP32 V-cycle preconditioning the FP64 CG
    (space charge, re-sorting, 24 steps): the mixed-precision bounds
    against the oracle, fewer iterations than the oracle's Jacobi PCG."""
    cfg = W.config_tiny()
    err = []
    om, ost, gm, gs, so, sg = _run_pair(pic, cfg, 24, 0.01, 3000, 60_000,
                                        resort_every=5,
                                        precision=pic.PIC_MIXED,
                                        precond=pic.PIC_PRECOND_AMG,
                                        phi_err=err)
    assert all(s["cg_iters"] > 0 for s in sg[1:])
    assert sum(s["cg_iters"] for s in sg) < sum(s["cg_iters"] for s in so)
    _compare_mixed(ost, gs, so, sg, err)


def test_pic_step_held_counts(pic):
    """Emission counts held from outside (counts_in, as finite differences
    of a window need): counts twice those of the rounding, the same on
    both sides, for 6 steps of the space-charge run; counts_out returns
    them."""
    cfg = W.config_tiny()
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, 60_000)
    ost.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = om.emission_rate(ost.E, cfg.phi_w)
    per_run = rate * cfg.dt * cfg.transit_steps
    j_scale = 0.01 / per_run
    w_sp = per_run * j_scale / 3000
    gm = pic.Mesh(tip, cfg.emit_zmin)
    gs = pic.State(gm, 60_000)
    gs.init_field(cfg.E0, tol=cfg.tol)
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, seed=cfg.seed,
              j_scale=j_scale, tol=cfg.tol)
    rng = np.random.default_rng(4)
    so_all, sg_all = [], []
    out = torch.zeros(om.n_emit, dtype=torch.int32, device="cuda")
    for k in range(6):
        held = rng.integers(0, 3, om.n_emit)
        so_all.append(ost.step(step=k, counts_in=held, **kw))
        sg_all.append(pic.State.decode_stats(gs.step(
            step0=k, counts_in=torch.from_numpy(held.astype(np.int32)).cuda(),
            counts_out=out, **kw))[0])
        assert (out.cpu().numpy() == held).all()
        assert so_all[-1]["n_inj"] == int(held.sum())
    _compare_runs(ost, gs, so_all, sg_all)


def test_mesh_in_caller_workspace(pic):
    """mesh_create_in: the mesh's persistent arrays in a caller workspace
    of mesh_workspace_bytes give the same steps, bit for bit, as a handle
    that allocates them; a workspace one byte short is rejected."""
    import ctypes as C
    cfg = W.config_tiny()
    tip = cfg.mesh()
    ga = pic.Mesh(tip, cfg.emit_zmin)
    gb = pic.Mesh(tip, cfg.emit_zmin, workspace=True)
    assert gb.workspace.numel() >= ga.info["device_bytes"]
    assert gb.info["device_bytes"] == ga.info["device_bytes"]
    out = []
    for gm in (ga, gb):
        gs = pic.State(gm, 30000)
        gs.init_field(cfg.E0, tol=cfg.tol)
        rate, _ = gm.emission_rate(gs.E, cfg.phi_w)
        per_run = rate.item() * cfg.dt * cfg.transit_steps
        st = gs.step(dt=cfg.dt, E0=cfg.E0, w_sp=0.5 / 2000, phi_w=cfg.phi_w,
                     step0=0, seed=cfg.seed, j_scale=0.5 / per_run, tol=cfg.tol,
                     resort_every=4, n_steps=9)
        torch.cuda.synchronize()
        out.append((gs.live(), gs.phi.cpu().numpy(), st.cpu().numpy()))
    (Pa, phia, sa), (Pb, phib, sb) = out
    assert Pa["id"].size > 0
    for k in ("x", "y", "z", "vx", "vy", "vz", "tet", "id"):
        assert np.array_equal(Pa[k], Pb[k]), k
    assert np.array_equal(phia, phib) and np.array_equal(sa, sb)
    L = pic.load_library()
    keep = (np.ascontiguousarray(tip.xyz, np.float64),
            np.ascontiguousarray(tip.tet, np.int32),
            np.ascontiguousarray(tip.shift, np.int8))
    d = pic.MeshDesc(tip.n_nodes, keep[0].ctypes.data, tip.n_tets,
                     keep[1].ctypes.data, keep[2].ctypes.data, tip.Lx, tip.Ly,
                     tip.z_top, cfg.emit_zmin)
    nb = C.c_size_t()
    assert L.mesh_workspace_bytes(C.byref(d), C.byref(nb)) == pic.PIC_OK
    assert nb.value == gb.workspace.numel()
    h = C.c_void_p()
    assert L.mesh_create_in(C.byref(d), C.c_void_p(gb.workspace.data_ptr()),
                            nb.value - 1, None, C.byref(h)) == pic.PIC_E_ARG
    gb.close()
    ga.close()
