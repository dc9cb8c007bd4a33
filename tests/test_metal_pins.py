"""Pins of the oracle's metal-side solves (Sec. II D, App. C-D) against
what the equations and the mesh fix independently of the oracle's code:

* the continuity equation with a layered conductivity sigma(z) and the
  interface flux of a uniform vertical current J: the exact solution is
  piecewise linear, Phi(z) = int J / sigma, which P1 elements reproduce at
  the nodes (patch test on the tip's staircase geometry); Joule heating is
  then J^2 / sigma;
* the consistent mass and stiffness matrices on a slab: v^T C v and
  v^T K v for a linear v are the closed-form integrals of C_v v^2 and
  kappa |grad v|^2;
* the heat step with no Dirichlet nodes: uniform heating raises every
  nodal temperature by dt P / C_v, and the heat content int C_v T (every
  Kuhn tetrahedron has volume h^3 / 6) grows by dt times the total source
  (int P_J + int P_N, face areas by Heron's formula), for any Theta;
* the steady state of the heat equation with kappa = L sigma T
  (Eq. wied_franz) in a slab heated through its top face: T(z)^2 =
  T_amb^2 + 2 q (z - z_b) / (L sigma), to the discretisation error."""
import numpy as np
import pytest

from oracle import metal as OM
from paper_1906_08125_amd import workloads as W

L_CU = 2.0e-8      # the paper's finite-size Lorentz number, W Ohm K^-2


@pytest.fixture(scope="module")
def tip():
    return W.kuhn_metal_mesh(16, 16, 32, 0.5, 2.0, 8.0, 4)


def _layer(m, h):
    """Cube layer index of each tetrahedron."""
    return np.floor(m.xyz[m.tet][:, :, 2].min(axis=1) / h + 0.5).astype(int)


def _outward_nz(m):
    """z component of the unit outward normal of each interface face (away
    from the fourth vertex of its metal tetrahedron)."""
    P = m.xyz[m.faces]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    n /= np.linalg.norm(n, axis=1)[:, None]
    opp = m.xyz[m.tet[m.face_tet]].sum(axis=1) - P.sum(axis=1)
    s = np.sign(((P[:, 0] - opp) * n).sum(axis=1))
    return n[:, 2] * s


def test_metal_mesh_shape(tip):
    v = W.kuhn_tip_mesh(16, 16, 32, 0.5, 2.0, 8.0)
    assert tip.n_tets == 16 * 16 * 32 * 6 - v.n_tets + 16 * 16 * 4 * 6
    assert tip.dirichlet.sum() == 17 * 17
    assert (tip.xyz[tip.dirichlet == 1, 2] == tip.z_bottom).all()
    g, V = OM.geometry(tip.xyz, tip.tet)
    assert np.allclose(V, 0.5 ** 3 / 6, rtol=1e-14, atol=0)
    nz = _outward_nz(tip)
    assert (np.abs(nz) <= 1 + 1e-12).all()
    assert np.isclose(np.abs(nz), 1.0).sum() > 0


def test_continuity_layered_conductivity(tip):
    h, J = 0.5, 0.37
    k = _layer(tip, h)
    sig_layer = {kk: 1.0 + 0.5 * ((kk + 7) % 3) for kk in range(-4, 32)}
    sigma = np.array([sig_layer[kk] for kk in k])
    flux = J * _outward_nz(tip)
    phi = OM.continuity_solve(tip, sigma, flux)
    # exact: Phi(z) = sum of J h / sigma over the layers below z
    z = tip.xyz[:, 2]
    want = np.zeros_like(z)
    for i, zz in enumerate(z):
        kk = int(round(zz / h))
        want[i] = sum(J * h / sig_layer[q] for q in range(-4, kk))
    assert np.abs(phi - want).max() <= 1e-11 * np.abs(want).max()
    PJ = OM.joule(tip, sigma, phi)
    assert np.allclose(PJ, J * J / sigma, rtol=1e-10, atol=0)


def test_continuity_without_current_is_zero(tip):
    phi = OM.continuity_solve(tip, np.ones(tip.n_tets), np.zeros(tip.n_faces))
    assert np.abs(phi).max() == 0.0


@pytest.fixture(scope="module")
def slab():
    return W.kuhn_metal_mesh(6, 5, 4, 0.5, 0.0, 0.0, 8)


def test_mass_and_stiffness_integrate_exactly(slab):
    Lx, Ly, D = 3.0, 2.5, 4.0
    Cv, kap = 3.45, 0.7
    C = OM.mass(slab.xyz, slab.tet, np.full(slab.n_tets, Cv))
    K = OM.stiffness(slab.xyz, slab.tet, np.full(slab.n_tets, kap))
    x, y, z = slab.xyz.T
    a, b = 1.3, -0.4
    v = a * z + b
    # int_{-D}^{0} (a z + b)^2 dz = ((a 0 + b)^3 - (-a D + b)^3) / (3 a)
    want = Cv * Lx * Ly * (b ** 3 - (b - a * D) ** 3) / (3 * a)
    assert abs(v @ (C @ v) - want) <= 1e-12 * abs(want)
    assert abs(v @ (K @ v) - kap * a * a * Lx * Ly * D) <= \
        1e-12 * kap * a * a * Lx * Ly * D
    w = 0.8 * x - 1.1 * y + 0.3
    want_w = Cv * D * (0.64 * Lx ** 3 * Ly / 3 + 1.21 * Ly ** 3 * Lx / 3
                       + 0.09 * Lx * Ly - 2 * 0.88 * Lx ** 2 * Ly ** 2 / 4
                       + 2 * 0.24 * Lx ** 2 * Ly / 2
                       - 2 * 0.33 * Ly ** 2 * Lx / 2)
    assert abs(w @ (C @ w) - want_w) <= 1e-12 * abs(want_w)


def _no_dirichlet(m):
    return W.MetalMesh(m.xyz, m.tet, m.faces, m.face_tet,
                       np.zeros_like(m.dirichlet), m.z_bottom)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_heat_uniform_heating(tip, theta):
    m = _no_dirichlet(tip)
    T0, p, Cv, dt = 300.0, 2.5e-3, 3.45e-3, 40.0
    T1 = OM.heat_step(m, np.full(m.n_nodes, T0), np.full(m.n_tets, 5.0),
                      np.full(m.n_tets, p), np.zeros(m.n_faces), Cv, L_CU,
                      dt, theta, 300.0)
    assert np.allclose(T1, T0 + dt * p / Cv, rtol=1e-12, atol=0)


def _heron(P):
    a = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
    b = np.linalg.norm(P[:, 2] - P[:, 1], axis=1)
    c = np.linalg.norm(P[:, 0] - P[:, 2], axis=1)
    s = 0.5 * (a + b + c)
    return np.sqrt(s * (s - a) * (s - b) * (s - c))


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.0])
def test_heat_energy_balance(tip, theta):
    m = _no_dirichlet(tip)
    rng = np.random.default_rng(12)
    T0 = 300.0 + 50.0 * rng.random(m.n_nodes)
    PJ = rng.random(m.n_tets) * 1e-3
    PN = (rng.random(m.n_faces) - 0.3) * 1e-3
    Cv, dt = 3.45e-3, 40.0
    T1 = OM.heat_step(m, T0, 1.0 + rng.random(m.n_tets), PJ, PN, Cv, L_CU,
                      dt, theta, 300.0)
    V = 0.5 ** 3 / 6

    def content(T):
        return Cv * V * T[m.tet].mean(axis=1).sum()

    src = (PJ * V).sum() + (PN * _heron(m.xyz[m.faces])).sum()
    assert abs(content(T1) - content(T0) - dt * src) <= 1e-9 * dt * abs(src)
    assert not np.allclose(T1, T1.mean())


def _steady(m, sigma, q, T_amb):
    T = np.full(m.n_nodes, T_amb)
    for _ in range(80):
        Tn = OM.heat_step(m, T, np.full(m.n_tets, sigma),
                          np.zeros(m.n_tets), np.full(m.n_faces, q),
                          3.45e-3, L_CU, 1e12, 1.0, T_amb)
        if np.abs(Tn - T).max() < 1e-11:
            return Tn
        T = Tn
    raise AssertionError("the lagged conductivity did not settle")


def test_heat_steady_state_wiedemann_franz(slab):
    """Implicit Euler with a huge step is the steady solve with kappa lagged
    one step; iterated, it settles on the nonlinear steady state, within a
    discretisation error that falls like h^2."""
    sigma, q, T_amb = 1.0, 1.35e-3, 300.0
    assert np.isclose(_outward_nz(slab), 1.0).all()   # only the top face
    err = []
    for m in (slab, W.kuhn_metal_mesh(12, 10, 4, 0.25, 0.0, 0.0, 16)):
        T = _steady(m, sigma, q, T_amb)
        z = m.xyz[:, 2]
        want = np.sqrt(T_amb ** 2 + 2 * q * (z - m.z_bottom) / (L_CU * sigma))
        assert want.max() > 1.8 * T_amb
        err.append(np.abs(T - want).max() / (want.max() - T_amb))
        assert (T[m.dirichlet == 1] == T_amb).all()
    assert err[0] < 3e-3, err
    assert 3.0 < err[0] / err[1] < 5.0, err
