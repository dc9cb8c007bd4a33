"""Pins of the oracle's adjoint: transpose identity of the field operator,
homogeneity in E0, the direct collection term, and central finite
differences (counts held) of each objective term separately."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.adjoint_cases import central_fd, tiny_window


def test_field_adj_is_transpose(tiny_mesh):
    om = O.OracleMesh(tiny_mesh, 0.01)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(om.n_nodes)
    Eb = rng.standard_normal((om.n_nodes, 3))
    lhs = float(np.sum(Eb * om.field(phi)))
    rhs = float(om.field_adj(Eb) @ phi)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-300) * 10


def test_adjoint_homogeneity_no_particles():
    """Without superparticles E is linear in E0: dJ_E/dE0 = J_E / E0."""
    cfg, tip, om, win = tiny_window(T=3, empty=True)
    s = np.ones(om.n_emit)
    JQ, JE, cks, counts = win.forward(cfg.E0, s, keep=True)
    assert JQ == 0.0 and JE > 0
    g0, gs = win.adjoint(cfg.E0, s, cks, wQ=0.0, wE=1.0)
    assert abs(g0 - JE / cfg.E0) <= 1e-9 * JE / cfg.E0
    assert np.all(gs == 0.0)


@pytest.fixture(scope="module")
def coupled():
    cfg, tip, om, win = tiny_window(T=4)
    s = np.ones(om.n_emit)
    fwd = win.forward(cfg.E0, s, keep=True)
    return cfg, om, win, s, fwd


def test_adjoint_direct_collection_term(coupled):
    """dJ_Q/ds_f = w_sp sum of the base weights of the superparticles born
    at f that the anode collects in the window."""
    cfg, om, win, s, (JQ, JE, cks, counts) = coupled
    assert JQ > 0
    want = np.zeros(om.n_emit)
    for ck in cks:
        det = ck["det"]
        face = det["inj"][:, 3].astype(np.int64)
        birth = np.concatenate([ck["pre"]["birth"], face])
        w = np.concatenate([ck["pre"]["w"], s[face]])
        an = det["fate"] == 1
        np.add.at(want, birth[an], win.w_sp * (w / s[birth])[an])
    g0, gs = win.adjoint(cfg.E0, s, cks, wQ=1.0, wE=0.0)
    assert g0 == 0.0
    assert np.allclose(gs, want, rtol=1e-14, atol=0)


def test_adjoint_fd_E0(coupled):
    cfg, om, win, s, (JQ, JE, cks, counts) = coupled
    fq, fe = central_fd(win, cfg.E0, s, counts, "E0")
    g0, _ = win.adjoint(cfg.E0, s, cks, wQ=0.0, wE=1.0)
    assert abs(g0 - fe) <= 1e-5 * abs(fe)
    assert fq == 0.0  # no collection event moves for a 1e-6 change


def test_adjoint_fd_faces(coupled):
    cfg, om, win, s, (JQ, JE, cks, counts) = coupled
    _, gE = win.adjoint(cfg.E0, s, cks, wQ=0.0, wE=1.0)
    _, gQ = win.adjoint(cfg.E0, s, cks, wQ=1.0, wE=0.0)
    births = np.bincount(win.init["birth"], minlength=om.n_emit)
    for f in np.argsort(births)[-3:]:
        fq, fe = central_fd(win, cfg.E0, s, counts, int(f))
        assert abs(gE[f] - fe) <= 1e-5 * abs(fe) + 1e-12 * abs(JE)
        assert abs(gQ[f] - fq) <= 1e-6 * abs(fq) + 1e-15
