"""Device adjoint (adjoint_step through the C ABI, driven by pic.Window)
against the oracle's adjoint, which its own pins tie to central finite
differences.  Bound: 1e-5 relative (FP64); the objective values to 1e-9."""
import numpy as np
import pytest

from tests.adjoint_cases import tiny_window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic as P
    P.load_library()
    return P


@pytest.fixture(scope="module")
def case():
    cfg, tip, om, win = tiny_window(T=4)
    s = np.ones(om.n_emit)
    JQ, JE, cks, counts = win.forward(cfg.E0, s, keep=True)
    gE = win.adjoint(cfg.E0, s, cks, wQ=0.0, wE=1.0)
    gQ = win.adjoint(cfg.E0, s, cks, wQ=1.0, wE=0.0)
    return cfg, tip, om, win, (JQ, JE, gE, gQ)


def _device_window(pic, cfg, tip, win, precision, adjoint_precond=0):
    gm = pic.Mesh(tip, cfg.emit_zmin)
    gs = pic.State(gm, win.cap, precision=precision)
    I = win.init
    n = len(I["x"])
    rd = gs.x.dtype
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        getattr(gs, k)[:n] = torch.from_numpy(I[k]).to(rd).cuda()
    gs.w[:n] = torch.from_numpy(I["omega"]).cuda()
    gs.tet[:n] = torch.from_numpy(I["tet"].astype(np.int32)).cuda()
    gs.birth[:n] = torch.from_numpy(I["birth"].astype(np.int32)).cuda()
    gs.id[:n] = torch.from_numpy(I["id"].astype(np.int64)).cuda()
    gs.n_slots.fill_(n)
    gw = pic.Window(gm, gs, T=win.T, step0=win.step0, dt=cfg.dt,
                    w_sp=win.w_sp, phi_w=cfg.phi_w, seed=cfg.seed,
                    j_scale=win.j_scale, tol=1e-13,
                    adjoint_precond=adjoint_precond)
    return gm, gs, gw


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "amg"])
def test_adjoint_fp64_matches_oracle(pic, case, precond):
    """precond: that of the transposed solves (Jacobi or AMG)."""
    cfg, tip, om, win, (JQ, JE, gE, gQ) = case
    gm, gs, gw = _device_window(pic, cfg, tip, win, pic.PIC_FP64, precond)
    s = torch.ones(om.n_emit, dtype=torch.float64, device="cuda")
    jq, je = gw.forward(cfg.E0, s)
    print("J", float(jq), JQ, float(je), JE)
    assert abs(float(je) - JE) <= 1e-9 * JE
    assert abs(float(jq) - JQ) <= 1e-9 * JQ
    e0, es = gw.backward(cfg.E0, s, 0.0, 1.0)
    q0, qs = gw.backward(cfg.E0, s, 1.0, 0.0)
    print("dJE/dE0", float(e0), gE[0], "rel ds", _rel(es.cpu(), gE[1]),
          "dJQ/ds rel", _rel(qs.cpu(), gQ[1]))
    assert abs(float(e0) - gE[0]) <= 1e-5 * abs(gE[0])
    assert _rel(es.cpu().numpy(), gE[1]) <= 1e-5
    assert float(q0) == 0.0
    assert _rel(qs.cpu().numpy(), gQ[1]) <= 1e-5


def test_adjoint_autograd(pic, case):
    """torch.autograd through window_objective gives the same gradient."""
    cfg, tip, om, win, (JQ, JE, gE, gQ) = case
    gm, gs, gw = _device_window(pic, cfg, tip, win, pic.PIC_FP64)
    E0 = torch.tensor(cfg.E0, dtype=torch.float64, requires_grad=True)
    s = torch.ones(om.n_emit, dtype=torch.float64, device="cuda",
                   requires_grad=True)
    J = pic.window_objective(E0, s, gw, 1.0, 1.0)
    J.backward()
    assert abs(float(J) - (JQ + JE)) <= 1e-9 * (JQ + JE)
    assert abs(float(E0.grad) - (gE[0] + gQ[0])) <= 1e-5 * abs(gE[0] + gQ[0])
    assert _rel(s.grad.cpu().numpy(), gE[1] + gQ[1]) <= 1e-5


def test_adjoint_mixed_precision(pic, case):
    """FP32 particles and field with FP64-refined solves: the gradient of
    each objective term against the FP64 oracle, to the 1e-5 bound of the
    adjoint gradients."""
    cfg, tip, om, win, (JQ, JE, gE, gQ) = case
    gm, gs, gw = _device_window(pic, cfg, tip, win, pic.PIC_MIXED)
    s = torch.ones(om.n_emit, dtype=torch.float64, device="cuda")
    jq, je = gw.forward(cfg.E0, s)
    e0, es = gw.backward(cfg.E0, s, 0.0, 1.0)
    r0 = abs(float(e0) - gE[0]) / abs(gE[0])
    rs = _rel(es.cpu().numpy(), gE[1])
    print("mixed: J_E rel", abs(float(je) - JE) / JE, "dE0 rel", r0, "ds rel", rs)
    assert abs(float(je) - JE) <= 1e-6 * JE
    assert r0 <= 1e-5 and rs <= 1e-5
    q0, qs = gw.backward(cfg.E0, s, 1.0, 0.0)
    rq = _rel(qs.cpu().numpy(), gQ[1])
    print("mixed: dJQ/ds rel", rq)
    assert float(q0) == 0.0 and rq <= 1e-5
