"""Metal-side solves on the GPU (Sec. II D, App. C-D) against the oracle:
the continuity solve and its Joule heating, and Theta-scheme heat steps
(implicit Euler and Crank-Nicolson) on the tiny tip's metal mesh, with
random conductivities and sources; at the production size, the exact
solutions that hold at any size (layered conductivity: piecewise-linear
Phi; uniform heating without Dirichlet nodes: T + dt P / C_v)."""
import numpy as np
import pytest

from oracle import metal as OM
from paper_1906_08125_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L_CU = 2.0e-8


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic as P
    P.load_library()
    return P


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


@pytest.fixture(scope="module")
def tiny():
    return W.kuhn_metal_mesh(16, 16, 32, 0.5, 2.0, 8.0, 4)


def test_continuity_matches_oracle(pic, tiny):
    rng = np.random.default_rng(3)
    sigma = 0.5 + 1.5 * rng.random(tiny.n_tets)
    flux = rng.normal(0.0, 0.2, tiny.n_faces)
    gm = pic.Metal(tiny)
    phi, pj, st = gm.continuity_solve(_dev(sigma), _dev(flux), tol=1e-13)
    torch.cuda.synchronize()
    want = OM.continuity_solve(tiny, sigma, flux)
    assert st["converged"] and st["iters"] > 10
    assert _rel(phi.cpu().numpy(), want) < 1e-9
    assert _rel(pj.cpu().numpy(), OM.joule(tiny, sigma, want)) < 1e-9
    assert (phi.cpu().numpy()[tiny.dirichlet == 1] == 0.0).all()
    # a second call from the solution as guess converges at once, same answer
    phi2, _, st2 = gm.continuity_solve(_dev(sigma), _dev(flux), phi=phi.clone(),
                                       tol=1e-13)
    assert st2["iters"] <= 2
    assert _rel(phi2.cpu().numpy(), want) < 1e-9


def test_continuity_zero_current(pic, tiny):
    gm = pic.Metal(tiny)
    guess = _dev(np.linspace(0.0, 1.0, tiny.n_nodes))
    phi, pj, st = gm.continuity_solve(_dev(np.ones(tiny.n_tets)),
                                      _dev(np.zeros(tiny.n_faces)), phi=guess)
    assert st["converged"] and st["iters"] == 0
    assert np.abs(phi.cpu().numpy()).max() == 0.0
    assert np.abs(pj.cpu().numpy()).max() == 0.0


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_heat_steps_match_oracle(pic, tiny, theta):
    rng = np.random.default_rng(7)
    sigma = 0.5 + rng.random(tiny.n_tets)
    PJ = rng.random(tiny.n_tets) * 2e-3
    PN = rng.normal(0.0, 1e-3, tiny.n_faces)
    Cv, dt, T_amb = 3.45e-3, 40.0, 300.0
    T_o = T_amb + 80.0 * rng.random(tiny.n_nodes)
    T_g = _dev(T_o)
    gm = pic.Metal(tiny)
    for k in range(3):
        st = gm.heat_step(T_g, _dev(sigma), _dev(PJ), _dev(PN), Cv, L_CU, dt,
                          theta=theta, T_amb=T_amb, tol=1e-13)
        T_o = OM.heat_step(tiny, T_o, sigma, PJ, PN, Cv, L_CU, dt, theta, T_amb)
        torch.cuda.synchronize()
        assert st["converged"], k
        assert _rel(T_g.cpu().numpy(), T_o) < 1e-9, k
    assert (T_g.cpu().numpy()[tiny.dirichlet == 1] == T_amb).all()


def test_heat_without_dirichlet_nodes(pic, tiny):
    m = W.MetalMesh(tiny.xyz, tiny.tet, tiny.faces, tiny.face_tet,
                    np.zeros_like(tiny.dirichlet), tiny.z_bottom)
    rng = np.random.default_rng(9)
    T0 = 300.0 + 20.0 * rng.random(m.n_nodes)
    sigma = 1.0 + rng.random(m.n_tets)
    PN = rng.normal(0.0, 1e-3, m.n_faces)
    gm = pic.Metal(m)
    T = _dev(T0)
    gm.heat_step(T, _dev(sigma), None, _dev(PN), 3.45e-3, L_CU, 40.0,
                 tol=1e-13)
    want = OM.heat_step(m, T0, sigma, np.zeros(m.n_tets), PN, 3.45e-3, L_CU,
                        40.0, 1.0, 300.0)
    assert _rel(T.cpu().numpy(), want) < 1e-9


def test_metal_checks_arguments(pic, tiny):
    gm = pic.Metal(tiny)
    s = _dev(np.ones(tiny.n_tets))
    with pytest.raises(pic.PicError):
        gm.continuity_solve(s, _dev(np.zeros(tiny.n_faces)), tol=0.0)
    with pytest.raises(pic.PicError):
        gm.heat_step(_dev(np.full(tiny.n_nodes, 300.0)), s, None,
                     _dev(np.zeros(tiny.n_faces)), 1.0, L_CU, 1.0, theta=1.5)
    # max_iter reached: PIC_E_NOCONV, the iterate is returned in place
    with pytest.raises(pic.PicError) as e:
        gm.continuity_solve(s, _dev(np.full(tiny.n_faces, 0.1)), max_iter=3)
    assert e.value.status == pic.PIC_E_NOCONV
    bad = W.MetalMesh(tiny.xyz, tiny.tet.copy(), tiny.faces, tiny.face_tet,
                      tiny.dirichlet, tiny.z_bottom)
    bad.tet[5, 3] = bad.tet[5, 2]          # a flat element
    with pytest.raises(pic.PicError):
        pic.Metal(bad)
    bad.tet[5, 3] = tiny.n_nodes           # a node out of range
    with pytest.raises(pic.PicError):
        pic.Metal(bad)


def test_metal_on_reused_memory(pic, tiny):
    """A handle whose device buffers are memory that earlier work left full
    of NaN: the first CG iteration must not read its search directions
    (regression: it multiplied them by beta = 0).  The library itself
    fills the search directions with NaN when a handle is created, so this
    and every other metal solve here would fail deterministically if the
    first iteration read them."""
    junk = torch.full((1 << 27,), float("nan"), dtype=torch.float64,
                      device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    rng = np.random.default_rng(5)
    sigma = 0.5 + rng.random(tiny.n_tets)
    flux = rng.normal(0.0, 0.2, tiny.n_faces)
    gm = pic.Metal(tiny)
    phi, _, st = gm.continuity_solve(_dev(sigma), _dev(flux), tol=1e-13)
    assert st["converged"]
    assert _rel(phi.cpu().numpy(), OM.continuity_solve(tiny, sigma, flux)) < 1e-9
    T = _dev(np.full(tiny.n_nodes, 300.0))
    st = gm.heat_step(T, _dev(sigma), _dev(np.full(tiny.n_tets, 1e-3)),
                      _dev(np.zeros(tiny.n_faces)), 3.45e-3, L_CU, 40.0,
                      tol=1e-13)
    assert st["converged"] and np.isfinite(T.cpu().numpy()).all()


def _outward_nz(m):
    P = m.xyz[m.faces]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    n /= np.linalg.norm(n, axis=1)[:, None]
    opp = m.xyz[m.tet[m.face_tet]].sum(axis=1) - P.sum(axis=1)
    return n[:, 2] * np.sign(((P[:, 0] - opp) * n).sum(axis=1))


def test_production_metal_exact_solutions(pic):
    """The production tip's metal (tip plus a 10 nm substrate): the layered
    conductivity's piecewise-linear potential and uniform heating, both
    exact for P1 elements at any size."""
    m = W.metal_production()
    h, J = 0.5, 0.37
    k = np.floor(m.xyz[m.tet][:, :, 2].min(axis=1) / h + 0.5).astype(int)
    sig_of = lambda kk: 1.0 + 0.5 * ((kk + 7) % 3)
    gm = pic.Metal(m)
    phi, pj, st = gm.continuity_solve(_dev(sig_of(k)), _dev(J * _outward_nz(m)),
                                      tol=1e-13)
    torch.cuda.synchronize()
    assert st["converged"]
    kn = np.round(m.xyz[:, 2] / h).astype(int)
    kmin = int(round(m.z_bottom / h))
    steps = np.array([J * h / sig_of(q) for q in range(kmin, kn.max())])
    want = np.concatenate([[0.0], np.cumsum(steps)])[kn - kmin]
    assert np.abs(phi.cpu().numpy() - want).max() <= 1e-9 * want.max()
    assert np.allclose(pj.cpu().numpy(), J * J / sig_of(k), rtol=1e-8, atol=0)
    free = W.MetalMesh(m.xyz, m.tet, m.faces, m.face_tet,
                       np.zeros_like(m.dirichlet), m.z_bottom)
    gf = pic.Metal(free)
    T = _dev(np.full(m.n_nodes, 300.0))
    st = gf.heat_step(T, _dev(np.ones(m.n_tets)),
                      _dev(np.full(m.n_tets, 2.5e-3)),
                      _dev(np.zeros(m.n_faces)), 3.45e-3, L_CU, 40.0,
                      tol=1e-13)
    assert st["converged"]
    assert np.allclose(T.cpu().numpy(), 300.0 + 40.0 * 2.5e-3 / 3.45e-3,
                       rtol=1e-10, atol=0)
