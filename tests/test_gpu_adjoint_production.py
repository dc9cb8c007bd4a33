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
