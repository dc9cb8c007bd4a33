"""The device adjoint at the production size (3.1M tets) against central
finite differences of the device forward itself, in the coupled regime
(emission scaled so that the charge in flight is 10 % of the emitting
faces' surface charge; ~1e5 superparticles after 60 steps), a window of 10
steps with the emission counts held (as the adjoint holds them): dJ_E/dE0
and, for 8 seeded strongly emitting faces, dJ_E/ds_f and dJ_Q/ds_f.  The
solves run to 1e-11 (an FP64 solve of this size stalls before 1e-13), so
the steps are 1e-5 relative."""
import numpy as np
import pytest

from paper_1906_08125_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def window():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic
    pic.load_library()
    cfg = W.config_production()
    tip = cfg.mesh()
    gm = pic.Mesh(tip, cfg.emit_zmin)
    phi = torch.zeros(gm.n_nodes, dtype=torch.float64, device="cuda")
    E = torch.zeros(4 * gm.n_nodes, dtype=torch.float64, device="cuda")
    gm.poisson_solve(None, 0.0, cfg.E0, phi, E, tol=1e-12)
    rate, faceF = gm.emission_rate(E, cfg.phi_w)
    eps0 = 8.8541878128e-12 / 1.602176634e-19 * 1e-9
    q_target = 0.1 * eps0 * float((faceF.cpu().numpy()
                                   * gm.emit_faces()["area"]).sum())
    per_run = rate.item() * cfg.dt * cfg.transit_steps
    m_j = q_target / per_run
    w_sp = per_run * m_j / 2e5
    gs = pic.State(gm, int(6e5), precond=pic.PIC_PRECOND_AMG)
    gs.init_field(cfg.E0, tol=1e-12)
    gs.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, step0=0,
            seed=cfg.seed, tol=1e-12, resort_every=10, n_steps=60, j_scale=m_j)
    torch.cuda.synchronize()
    win = pic.Window(gm, gs, T=10, step0=60, dt=cfg.dt, w_sp=w_sp,
                     phi_w=cfg.phi_w, seed=cfg.seed, j_scale=m_j, tol=1e-11,
                     max_iter=3000, adjoint_precond=pic.PIC_PRECOND_AMG)
    s = torch.ones(gm.n_emit, dtype=torch.float64, device="cuda")
    JQ, JE = win.forward(cfg.E0, s)
    counts = [c.clone() for c in win.counts]
    gE = win.backward(cfg.E0, s, 0.0, 1.0)
    gQ = win.backward(cfg.E0, s, 1.0, 0.0)
    return pic, cfg, gm, win, s, counts, (float(JQ), float(JE)), gE, gQ, faceF


def test_held_counts_reproduce_the_forward(window):
    pic, cfg, gm, win, s, counts, J, gE, gQ, faceF = window
    jq, je = win.forward(cfg.E0, s, counts=counts)
    assert float(jq) == J[0] and float(je) == J[1]
    assert J[0] > 0        # charge reached the anode within the window


def test_dJE_dE0_matches_central_differences(window):
    pic, cfg, gm, win, s, counts, J, gE, gQ, faceF = window
    d = 1e-5 * cfg.E0
    jp = win.forward(cfg.E0 + d, s, counts=counts)
    jm = win.forward(cfg.E0 - d, s, counts=counts)
    fd = (float(jp[1]) - float(jm[1])) / (2 * d)
    assert abs(fd / float(gE[0]) - 1) < 1e-6
    # the collected charge does not depend on E0 with the counts held
    assert float(jp[0]) == float(jm[0]) == J[0] and float(gQ[0]) == 0.0


def test_face_multipliers_match_central_differences(window):
    pic, cfg, gm, win, s, counts, J, gE, gQ, faceF = window
    rng = np.random.default_rng(5)
    strong = np.argsort(-faceF.cpu().numpy())[:60]
    for f in rng.choice(strong, 8, replace=False):
        sp, sm = s.clone(), s.clone()
        sp[f] += 1e-5
        sm[f] -= 1e-5
        a = win.forward(cfg.E0, sp, counts=counts)
        b = win.forward(cfg.E0, sm, counts=counts)
        fE = (float(a[1]) - float(b[1])) / 2e-5
        fQ = (float(a[0]) - float(b[0])) / 2e-5
        print(f"face {f}: dJE/ds FD {fE:.7e} adjoint {float(gE[1][f]):.7e}; "
              f"dJQ/ds FD {fQ:.7e} adjoint {float(gQ[1][f]):.7e}", flush=True)
        assert abs(fE / float(gE[1][f]) - 1) < 1e-4
        assert abs(fQ / float(gQ[1][f]) - 1) < 1e-5


@pytest.fixture(scope="module")
def config5():
    """The adjoint workload as configured: the production geometry, about
    2e5 superparticles after 100 mixed-precision warm-up steps at the
    physical emission, a window of 20 steps.  The same population (FP32
    positions, widened exactly) runs the window in FP64 and in mixed
    precision (FP32 particles and field, FP64-refined forward solves, FP64
    transposed solves)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic
    pic.load_library()
    cfg = W.config_production()
    tip = cfg.mesh()
    gm = pic.Mesh(tip, cfg.emit_zmin)
    phi = torch.zeros(gm.n_nodes, dtype=torch.float64, device="cuda")
    E = torch.zeros(4 * gm.n_nodes, dtype=torch.float64, device="cuda")
    gm.poisson_solve(None, 0.0, cfg.E0, phi, E, tol=1e-12)
    rate, _ = gm.emission_rate(E, cfg.phi_w)
    w_sp = rate.item() * cfg.dt * cfg.transit_steps / 2e5
    cap, warm = int(6e5), 100
    g32 = pic.State(gm, cap, precision=pic.PIC_MIXED)
    g32.init_field(cfg.E0, tol=cfg.tol)
    g32.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, step0=0,
             seed=cfg.seed, tol=cfg.tol, resort_every=10, n_steps=warm)
    torch.cuda.synchronize()
    g64 = pic.State(gm, cap, precision=pic.PIC_FP64)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        getattr(g64, k).copy_(getattr(g32, k).to(torch.float64))
    for k in ("w", "tet", "birth", "id", "n_slots"):
        getattr(g64, k).copy_(getattr(g32, k))
    live = int((g32.tet >= 0).sum().item())
    kw = dict(T=20, step0=warm, dt=cfg.dt, w_sp=w_sp, phi_w=cfg.phi_w,
              seed=cfg.seed, tol=1e-11, max_iter=5000,
              adjoint_precond=pic.PIC_PRECOND_AMG)
    s = torch.ones(gm.n_emit, dtype=torch.float64, device="cuda")
    out = {}
    for name, st in (("fp64", g64), ("mixed", g32)):
        win = pic.Window(gm, st, **kw)
        J = win.forward(cfg.E0, s)
        counts = [c.clone() for c in win.counts]
        gE = win.backward(cfg.E0, s, 0.0, 1.0)
        gQ = win.backward(cfg.E0, s, 1.0, 0.0)
        out[name] = dict(win=win, J=(float(J[0]), float(J[1])), counts=counts,
                         gE=(float(gE[0]), gE[1].cpu().numpy()),
                         gQ=(float(gQ[0]), gQ[1].cpu().numpy()))
    return pic, cfg, s, live, out


def test_config5_fp64_gradient_against_central_differences(config5):
    pic, cfg, s, live, out = config5
    assert live > 1.5e5
    r = out["fp64"]
    d = 1e-6 * cfg.E0
    jp = r["win"].forward(cfg.E0 + d, s, counts=r["counts"])
    jm = r["win"].forward(cfg.E0 - d, s, counts=r["counts"])
    fd = (float(jp[1]) - float(jm[1])) / (2 * d)
    print("dJE/dE0 FD", fd, "adjoint", r["gE"][0])
    assert abs(fd / r["gE"][0] - 1) < 1e-5
    assert r["J"][0] > 0          # charge reached the anode in the window


def test_config5_mixed_gradient_against_fp64(config5):
    """The smooth terms (dJ_E/dE0, dJ_E/ds) to 1e-5.  dJ_Q/ds_f is, at the
    physical emission, w_sp times the number of collected superparticles
    born at face f (the space-charge coupling is ~1e-20 of it): a count,
    which FP32 rounding may change by an absorption decided on the other
    side of the anode plane; both are checked to be whole counts, differing
    by at most three events."""
    pic, cfg, s, live, out = config5
    a, b = out["fp64"], out["mixed"]
    rel = lambda u, v: float(np.linalg.norm(np.asarray(u) - v) / np.linalg.norm(v))
    e0 = abs(b["gE"][0] / a["gE"][0] - 1)
    es = rel(b["gE"][1], a["gE"][1])
    w_sp = a["win"].kw["w_sp"]
    na, nb = a["gQ"][1] / w_sp, b["gQ"][1] / w_sp
    flips = int(np.abs(np.rint(na) - np.rint(nb)).sum())
    print(f"live {live}; J fp64 {a['J']} mixed {b['J']}; dJE/dE0 rel {e0:.2e}, "
          f"dJE/ds rel {es:.2e}; collected {int(np.rint(na).sum())}, "
          f"counts differing by {flips}")
    assert abs(b["J"][1] / a["J"][1] - 1) <= 1e-6
    assert e0 <= 1e-5 and es <= 1e-5
    assert np.abs(na - np.rint(na)).max() < 1e-6
    assert np.abs(nb - np.rint(nb)).max() < 1e-6
    assert flips <= 3
