"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: mesh counts of the workload recipe, a published RNG, exact rational
arithmetic, closed-form fields and trajectories, brute-force point location,
library solvers, and conservation laws.  CPU only."""
from fractions import Fraction
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1906_08125_amd import workloads as W


# ---------------------------------------------------------------------------
# Mesh recipe and derived structure
# ---------------------------------------------------------------------------

def test_mesh_counts_tiny(tiny_mesh):
    om = O.OracleMesh(tiny_mesh, 0.01)
    # 16x16x32 grid, tip R = 2, H = 8
    assert (om.n_tets, om.n_nodes) == (43916, 7773)
    assert om.n_free == 7088 and om.nnz == 102514
    assert om.n_top == 2 * 16 * 16          # two triangles per top cell
    assert om.n_emit == 948                 # tip faces (not in z = 0)


@pytest.mark.slow
def test_mesh_counts_production():
    cfg = W.config_production()
    m = cfg.mesh()
    assert (m.n_tets, m.n_nodes) == (3100504, 522017)
    om = O.OracleMesh(m, cfg.emit_zmin)
    assert om.n_free == 515455 and om.nnz == 7688725
    assert om.n_emit == 612 and om.n_top == 2 * 64 * 64


def test_orientation_and_adjacency(small_tip_mesh):
    om = O.OracleMesh(small_tip_mesh, 0.01)
    t = om.tets()
    assert (t["D"] > 0).all()
    # half the Kuhn permutations are negatively oriented
    assert om.n_flipped * 2 == om.n_tets or om.n_flipped > 0
    nbr, ns = t["nbr"], t["nbr_shift"]
    for a in range(om.n_tets):
        for f in range(4):
            b = nbr[a, f]
            if b < 0:
                continue
            back = [g for g in range(4) if nbr[b, g] == a and
                    (ns[b, g] == -ns[a, f]).all()]
            assert back, (a, f, b)
            # the shared face has the same unwrapped vertices up to the shift
            va = np.delete(t["vert"][a], f, axis=0)
            shift = np.array([ns[a, f, 0] * small_tip_mesh.Lx,
                              ns[a, f, 1] * small_tip_mesh.Ly, 0.0])
            vb = t["vert"][b] - shift
            for p in va:
                assert np.any(np.all(vb == p, axis=1))
    # every boundary face is on the top plane or the metal
    top = sum(int((nbr[:, f] == -1).sum()) for f in range(4))
    assert top == 2 * 3 * 3


# ---------------------------------------------------------------------------
# RNG: Philox4x64-10 equals numpy's implementation (which increments the
# 256-bit counter before producing a block)
# ---------------------------------------------------------------------------

def test_philox_matches_numpy():
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = [int(k) for k in rng.integers(0, 2**63, 2)]
        ctr = [int(c) for c in rng.integers(1, 2**63, 4)]
        mine = O.philox4x64(tuple(key), ctr)
        prev = list(ctr)
        prev[0] -= 1
        ref = np.random.Philox(key=key, counter=prev).random_raw(4)
        assert (mine == ref).all()


# ---------------------------------------------------------------------------
# Exact orientation predicate against rational arithmetic
# ---------------------------------------------------------------------------

def _frac_vol6(a, b, c, d):
    a, b, c, d = ([Fraction(float(x)) for x in p] for p in (a, b, c, d))
    e1 = [b[i] - a[i] for i in range(3)]
    e2 = [c[i] - a[i] for i in range(3)]
    e3 = [d[i] - a[i] for i in range(3)]
    return (e1[0] * (e2[1] * e3[2] - e2[2] * e3[1])
            - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0])
            + e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]))


def test_orient_sign_exact():
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(300):
        a, b, c = rng.random((3, 3)) * 10
        # d nearly coplanar with a, b, c: the float filter cannot decide
        s, t = rng.random(2)
        d = a + s * (b - a) + t * (c - a)
        d = d + rng.integers(-2, 3, 3) * np.spacing(d)
        cases.append((a, b, c, d))
        cases.append((a, b, c, rng.random(3) * 10))
    # exactly coplanar binary points
    for _ in range(50):
        a, b, c = rng.integers(0, 8, (3, 3)) * 0.5
        d = a + 0.25 * (b - a) + 0.5 * (c - a)
        cases.append((a, b, c, d))
    for a, b, c, d in cases:
        exact = _frac_vol6(a, b, c, d)
        sgn = (exact > 0) - (exact < 0)
        assert O.orient_sign(a, b, c, d) == sgn


# ---------------------------------------------------------------------------
# Stiffness, load, solve: closed forms between parallel plates
# ---------------------------------------------------------------------------

def _K(om):
    rp, col, val = om.csr()
    return sp.csr_matrix((val, col, rp), shape=(om.n_free, om.n_free))


def test_stiffness_symmetric_spd(plates_mesh, small_tip_mesh):
    for mesh in (plates_mesh, small_tip_mesh):
        om = O.OracleMesh(mesh, 0.01)
        K = _K(om).toarray()
        assert np.abs(K - K.T).max() < 1e-14
        assert np.linalg.eigvalsh(K).min() > 0


def test_patch_test_plates(plates_mesh):
    """phi = z solves the discrete problem with E0 = 1 exactly: K z = g."""
    om = O.OracleMesh(plates_mesh, 0.01)
    fid, g = om.free()
    z = plates_mesh.xyz[fid >= 0, 2]
    assert np.abs(_K(om) @ z - g).max() < 1e-13
    # g = E0 * h^2 per top node for a unit-spaced periodic top plane
    top = np.isclose(plates_mesh.xyz[fid >= 0, 2], plates_mesh.z_top)
    assert np.allclose(g[top], 0.25, rtol=0, atol=1e-15)
    assert np.all(g[~top] == 0)


def test_plates_linear_potential(plates_mesh):
    E0 = 0.7
    om = O.OracleMesh(plates_mesh, 0.01)
    phi, info = om.poisson_solve(None, 0.0, E0, tol=1e-13)
    assert info["status"] == 0
    assert np.abs(phi - E0 * plates_mesh.xyz[:, 2]).max() < 1e-11
    E = om.field(phi)
    assert np.abs(E - np.array([0, 0, -E0])).max() < 1e-10


def test_cell_field_of_linear_potential(small_tip_mesh, tiny_mesh):
    """Reading R2, cell variant: the field of a tet is -(grad phi)_t, so a
    nodal potential phi = a.x + c gives -a in every tet (and the nodal
    recovery gives -a at every node); a sign or index slip in the gradient
    rows breaks it."""
    a = np.array([0.3, -1.25, 2.0])
    for mesh in (small_tip_mesh, tiny_mesh):
        om = O.OracleMesh(mesh, 0.01)
        T = om.tets()
        Et = om.cell_field(mesh.xyz @ a + 7.0)
        assert Et.shape == (om.n_tets, 3)
        # (tets across the lateral seam carry unwrapped vertices, where a
        # potential linear in x or y is not)
        inner = np.all(T["vert"] == mesh.xyz[T["tet"]], axis=(1, 2))
        assert inner.sum() > 0.3 * om.n_tets
        assert np.abs(Et[inner] + a).max() <= 1e-12 * 8
        # linear in z (not periodic): -e_z in every tet and at every node
        phz = mesh.xyz[:, 2] * 2.0 + 7.0
        Ez = om.cell_field(phz)
        assert np.abs(Ez[:, :2]).max() <= 1e-12
        assert np.abs(Ez[:, 2] + 2.0).max() <= 1e-12
        En = om.field(phz)
        assert np.abs(En[:, :2]).max() <= 1e-12
        assert np.abs(En[:, 2] + 2.0).max() <= 1e-12


def _interior_patch_nodes(mesh, om):
    """Nodes whose patch is the full 24-tet Kuhn star and does not cross the
    lateral seam (every incident tet has its vertices at the nodes' own,
    wrapped coordinates)."""
    T = om.tets()
    inner = np.all(T["vert"] == mesh.xyz[T["tet"]], axis=(1, 2))
    count = np.bincount(T["tet"].reshape(-1), minlength=mesh.n_nodes)
    bad = np.zeros(mesh.n_nodes, bool)
    bad[T["tet"][~inner].reshape(-1)] = True
    return np.nonzero((count == 24) & ~bad)[0]


def test_nodal_field_of_quadratic_potential(tiny_mesh):
    """Reading R2 (Sec. II B 2): the nodal field is the volume-weighted mean
    of -grad phi over the tets holding the node.  For any quadratic q the
    element gradient of its P1 interpolant is grad q at the tet centroid
    plus a shape term that changes sign under the point reflection about a
    vertex; the Kuhn star of an interior vertex is symmetric under that
    reflection with equal volumes, so the recovered field there is exactly
    -grad q(vertex).  A linear q (the older pin) cannot tell the nodes of a
    tet apart; a quadratic one can."""
    om = O.OracleMesh(tiny_mesh, 0.01)
    nodes = _interior_patch_nodes(tiny_mesh, om)
    assert nodes.size > 0.5 * tiny_mesh.n_nodes
    x, y, z = tiny_mesh.xyz.T
    # q = z^2 (the closed form of the plates' space-charge potential) and a
    # full quadratic with mixed terms
    cases = [(z * z, lambda p: np.stack([0 * p[:, 0], 0 * p[:, 0], 2 * p[:, 2]], 1)),
             (0.3 * x * x - 0.2 * y * y + 0.7 * z * z + 0.5 * x * y
              - 0.4 * y * z + 0.25 * x * z + 1.5 * x - 0.5 * z,
              lambda p: np.stack([0.6 * p[:, 0] + 0.5 * p[:, 1] + 0.25 * p[:, 2] + 1.5,
                                  -0.4 * p[:, 1] + 0.5 * p[:, 0] - 0.4 * p[:, 2],
                                  1.4 * p[:, 2] - 0.4 * p[:, 1] + 0.25 * p[:, 0] - 0.5], 1))]
    for q, grad in cases:
        E = om.field(q)
        want = -grad(tiny_mesh.xyz[nodes])
        err = np.abs(E[nodes] - want).max()
        assert err <= 1e-13 * max(1.0, np.abs(want).max()), err


def test_nodal_field_graded_mesh_weights():
    """Volume weights of the nodal field (reading R2) on a mesh whose layers
    have unequal heights (so tets above and below a node differ in volume):
    every tet of layer k (between z_k and z_k+1) interpolates phi = z^2 by
    the linear function with slope z_k + z_k+1, and half of a Kuhn star lies
    in each layer, so the volume-weighted mean at an interior node of level
    k is -(z_k-1 + z_k+1) e_z, at the bottom and top levels -(z_0 + z_1) and
    -(z_n-1 + z_n).  An unweighted mean would give -(z_k-1 + 2 z_k +
    z_k+1)/2 instead."""
    mesh = W.kuhn_tip_mesh(4, 4, 8, 0.5)
    g = np.random.default_rng(5)
    levels = np.concatenate([[0.0], np.cumsum(g.uniform(0.25, 0.9, mesh.nz))])
    k = np.rint(mesh.xyz[:, 2] / mesh.h).astype(int)
    xyz = mesh.xyz.copy()
    xyz[:, 2] = levels[k]
    import dataclasses
    gm = dataclasses.replace(mesh, xyz=xyz, z_top=float(levels[-1]))
    om = O.OracleMesh(gm, 0.01)
    E = om.field(xyz[:, 2] ** 2)
    zl = levels
    want = np.where(k == 0, -(zl[0] + zl[1]),
                    np.where(k == mesh.nz, -(zl[-2] + zl[-1]),
                             -(zl[np.clip(k - 1, 0, None)] + zl[np.clip(k + 1, None, mesh.nz)])))
    assert np.abs(E[:, :2]).max() <= 1e-13
    assert np.abs(E[:, 2] - want).max() <= 1e-13 * np.abs(want).max()
    inner = (k > 0) & (k < mesh.nz)
    unweighted = -(zl[np.clip(k - 1, 0, None)] + 2 * zl[k]
                   + zl[np.clip(k + 1, None, mesh.nz)]) / 2
    assert np.abs(unweighted - want)[inner].min() > 1e-6


def test_cell_mode_emission_uses_the_face_tet(small_tip_mesh):
    """Cell mode emission: every emitting face sees the field of its own
    vacuum tet.  With phi = -4 z^2 (a field growing with height, so that
    another tet's field differs), |E| per face equals the pinned per-tet
    field of the face's tet, and the total is the sum of the FN current
    (emitting only where the field points into the metal) over the
    faces' areas; with a linear potential both modes agree."""
    om = O.OracleMesh(small_tip_mesh, 0.01)
    em = om.emit()
    phi = -4.0 * small_tip_mesh.xyz[:, 2] ** 2
    Et = om.cell_field(phi)[em["tet"]]
    E0 = np.zeros((om.n_nodes, 3))
    r, F = om.emission_rate(E0, 4.5, phi)
    assert np.array_equal(F, np.sqrt((Et ** 2).sum(1)))
    pull = (Et * em["normal"]).sum(1) < 0
    assert pull.sum() > 0
    j_unit = O.constants()["j_unit"]
    want = sum(O.fn_current(F[f], 4.5)[0] * j_unit * em["area"][f]
               for f in np.flatnonzero(pull))
    assert abs(r - want) <= 1e-12 * want
    phz = small_tip_mesh.xyz[:, 2] * -2.0
    rn, Fn = om.emission_rate(om.field(phz), 4.5)
    rc, Fc = om.emission_rate(E0, 4.5, phz)
    assert abs(rn - rc) <= 1e-10 * rn and np.abs(Fn - Fc).max() <= 1e-12


def test_plates_uniform_charge_closed_form(plates_mesh):
    """SPs on the nodes with weight rho0 h^3 (half on the top plane) load
    the P1 system uniformly; P1 is nodally exact for the quadratic
    phi(z) = -(rho0/2 eps0) z^2 + (E0 + rho0 Lz/eps0) z."""
    om = O.OracleMesh(plates_mesh, 0.01)
    k = O.constants()
    h, Lz, E0 = plates_mesh.h, plates_mesh.z_top, 0.5
    fid, _ = om.free()
    nodes = np.nonzero(fid >= 0)[0]
    p = plates_mesh.xyz[nodes]
    # a tet having each node as an unwrapped vertex (lambda = e_i there)
    V = om.tets()["vert"].reshape(-1, 3)
    tet = np.array([np.nonzero(np.all(V == q, axis=1))[0][0] // 4 for q in p],
                   dtype=np.int32)
    rho_w = 1.0 / 4096          # weight per unit volume (binary exact)
    w = np.where(np.isclose(p[:, 2], Lz), 0.5, 1.0) * rho_w * h**3
    c = om.deposit(p, tet, w)
    w_sp = 1e-3
    phi, info = om.poisson_solve(c, w_sp, E0, tol=1e-14)
    rho = -w_sp * rho_w * k["e_eps"]          # rho0/eps0 in V/nm^2 (electrons)
    z = plates_mesh.xyz[:, 2]
    ref = -(rho / 2) * z**2 + (E0 + rho * Lz) * z
    assert np.abs(phi - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_pcg_matches_spsolve(small_tip_mesh):
    om = O.OracleMesh(small_tip_mesh, 0.01)
    rng = np.random.default_rng(5)
    fid, g = om.free()
    c = rng.integers(-2**40, 2**40, om.n_nodes)
    phi, info = om.poisson_solve(c, 1e-2, 0.3, tol=1e-14)
    b = om.rhs(c, 1e-2, 0.3)
    x = spla.spsolve(_K(om).tocsc(), b)
    assert np.abs(phi[fid >= 0] - x).max() < 1e-12 * np.abs(x).max()
    assert (phi[fid < 0] == 0).all()


def test_pcg_warm_start_zero_iterations(small_tip_mesh):
    om = O.OracleMesh(small_tip_mesh, 0.01)
    phi, info = om.poisson_solve(None, 0.0, 0.3, tol=1e-12)
    phi2, info2 = om.poisson_solve(None, 0.0, 0.3, phi=phi, tol=1e-12)
    assert info2["iters"] == 0 and (phi2 == phi).all()
    phi3, info3 = om.poisson_solve(None, 0.0, 0.0)
    assert (phi3 == 0).all()


# ---------------------------------------------------------------------------
# Barycentric coordinates and point location
# ---------------------------------------------------------------------------

def test_barycentric_properties(small_tip_mesh):
    om = O.OracleMesh(small_tip_mesh, 0.01)
    t = om.tets()
    rng = np.random.default_rng(11)
    for k in rng.integers(0, om.n_tets, 50):
        V = t["vert"][k]
        for i in range(4):
            lam = om.lam(k, V[i])
            assert (lam == np.eye(4)[i]).all()
        w = rng.dirichlet(np.ones(4))
        p = w @ V
        lam = om.lam(k, p)
        assert abs(lam.sum() - 1) < 4e-16
        assert np.abs(lam @ V - p).max() < 8 * np.spacing(np.abs(p).max())
        assert np.abs(lam - w).max() < 1e-13


def _brute_locate(om, mesh, pts):
    """All (tet, point) containment decided in exact integer arithmetic
    (inputs are multiples of 1/4, coordinates scaled by 4)."""
    V = (om.tets()["vert"] * 4).round().astype(np.int64)
    out = []
    for p in pts:
        q = (np.asarray(p) * 4).round().astype(np.int64)
        assert np.all(q / 4 == p)
        best = -1
        for k in range(V.shape[0]):
            ok = True
            for i in range(4):
                r = V[k].copy()
                r[i] = q
                e1, e2, e3 = r[1] - r[0], r[2] - r[0], r[3] - r[0]
                if int(np.dot(e1, np.cross(e2, e3))) < 0:
                    ok = False
                    break
            if ok:
                best = k
                break
        out.append(best)
    return np.array(out)


def test_locate_brute_force_degenerate(small_tip_mesh):
    om = O.OracleMesh(small_tip_mesh, 0.01)
    pts = W.lattice_points(small_tip_mesh, 400, 21)
    pts = pts[pts[:, 2] < small_tip_mesh.z_top]
    ref = _brute_locate(om, small_tip_mesh, pts)
    tet, where = om.locate(pts)
    assert (tet == ref).all()
    assert ((where == 2) == (ref < 0)).all()
    # hints never change the canonical answer
    rng = np.random.default_rng(2)
    hint = rng.integers(-1, om.n_tets, len(pts)).astype(np.int32)
    tet2, _ = om.locate(pts, hint)
    assert (tet2 == ref).all()


def test_locate_brute_force_random(small_tip_mesh):
    om = O.OracleMesh(small_tip_mesh, 0.01)
    pts = W.random_points_in_box(small_tip_mesh, 300, 8)
    tv = om.tets()["vert"]
    tet, where = om.locate(pts)
    for p, t_ in zip(pts, tet):
        hits = []
        for k in range(om.n_tets):
            s = [O.orient_sign(*(np.where(np.arange(4)[:, None] == i, p, tv[k])))
                 for i in range(4)]
            if min(s) >= 0:
                hits.append(k)
        assert (hits[0] if hits else -1) == t_


# ---------------------------------------------------------------------------
# Deposition: exact conservation and order independence
# ---------------------------------------------------------------------------

def test_deposit_conservation_and_permutation(tiny_mesh):
    om = O.OracleMesh(tiny_mesh, 0.01)
    pts = W.random_points_in_box(tiny_mesh, 5000, 4)
    tet, where = om.locate(pts)
    keep = where == 0
    pts, tet = pts[keep], tet[keep]
    w = np.random.default_rng(1).uniform(0.2, 1.5, len(pts))
    c = om.deposit(pts, tet, w)
    total = sum(int(np.rint(x * 2.0**40)) for x in w)
    assert int(c.sum()) == total
    perm = np.random.default_rng(9).permutation(len(pts))
    c2 = om.deposit(pts[perm], tet[perm], w[perm])
    assert (c2 == c).all()


# ---------------------------------------------------------------------------
# Emission: constants, FN form, rounding, sampling
# ---------------------------------------------------------------------------

def test_fn_constants_published_values():
    """The oracle's constants against their published values (the first
    and second FN constants and the Schottky constant of Forbes & Deane,
    e/m_e and e/eps0 from CODATA; tests/golden/fn_constants.txt)."""
    from conftest import golden
    k = O.constants()
    ref = golden("fn_constants.txt")
    assert set(ref) == {"a_fn", "b_fn", "c_s", "qm", "e_eps"}
    for name, (value, rtol, *unit) in ref.items():
        assert abs(k[name] / float(value) - 1) < float(rtol), name


def test_fn_current_limits():
    # v(1) = 0: at the barrier-vanishing field J = a F^2/(phi t(1)^2)
    phi = 4.5
    k = O.constants()
    F1 = phi**2 / k["c_s"]
    j, clamped = O.fn_current(F1 * 1.0001, phi)
    assert clamped
    t1 = 1 + 1 / 9
    assert abs(j / (k["a_fn"] * (F1 * 1.0001e9) ** 2 / (phi * t1**2)) - 1) < 1e-6
    assert O.fn_current(0.0, phi)[0] == 0.0
    # ln(J/F^2) is close to linear in 1/F with slope ~ -b phi^1.5 s(f), s ~ 0.95
    F = np.array([3.0, 4.0, 5.0, 6.0])
    y = np.log([O.fn_current(x, phi)[0] / x**2 for x in F])
    slope = np.polyfit(1 / F, y, 1)[0]
    assert -1.0 < slope / (k["b_fn"] * phi**1.5) < -0.9


def _sn_barrier_functions(f):
    """Exact Schottky-Nordheim barrier functions (Forbes and Deane, Proc. R.
    Soc. A 463 (2007) 2907): with l = sqrt(f) and elliptic parameter
    m = (1 - l)/(1 + l), v(f) = sqrt(1 + l) (E(m) - l K(m)), and
    t(f) = v - (4/3) f dv/df (Richardson-extrapolated central difference)."""
    from scipy.special import ellipe, ellipk

    def v(f):
        l = np.sqrt(f)
        m = (1 - l) / (1 + l)
        return np.sqrt(1 + l) * (ellipe(m) - l * ellipk(m))
    h = 1e-5
    d1 = (v(f + h) - v(f - h)) / (2 * h)
    d2 = (v(f + 2 * h) - v(f - 2 * h)) / (4 * h)
    return v(f), v(f) - 4.0 / 3.0 * f * (4 * d1 - d2) / 3


def _oracle_v_t(f):
    """v(f) and t(f) as the oracle's FN current uses them, recovered from
    two currents at the same scaled field f but different work functions:
    ln(J phi / (a F^2)) = -2 ln t - v b phi^1.5 / F is linear in (ln t, v)."""
    k = O.constants()
    ys, cs = [], []
    for phi in (4.5, 2.0):
        F = f * phi * phi / k["c_s"]
        j, clamped = O.fn_current(F, phi)
        assert not clamped
        ys.append(math.log(j * phi / (k["a_fn"] * (F * 1e9) ** 2)))
        cs.append(k["b_fn"] * phi ** 1.5 / F)
    v = -(ys[0] - ys[1]) / (cs[0] - cs[1])
    return v, math.exp(-(ys[0] + v * cs[0]) / 2)


def test_fn_barrier_functions_against_exact_sn():
    """The Murphy-Good current (Sec. II B 3; GETELEC stands in the paper)
    takes Forbes' approximations of the Schottky-Nordheim v(f) and t(f).
    The oracle's v and t, read back from its currents, lie within the
    approximations' own deviation from the exact elliptic-integral functions
    over 0.05 <= f <= 0.95 (at most 0.33 % for v, 0.39 % for t); a dropped
    log term or a swapped sign exceeds it many times over."""
    fs = np.linspace(0.05, 0.95, 19)
    v_ex, t_ex = _sn_barrier_functions(fs)
    for f, ve, te in zip(fs, v_ex, t_ex):
        vo, to = _oracle_v_t(float(f))
        assert abs(vo / ve - 1) <= 0.0034, (f, vo, ve)
        assert abs(to / te - 1) <= 0.0040, (f, to, te)
    # the bounds are tight enough to reject the plausible slips
    assert np.abs((1 - fs) / v_ex - 1).max() > 0.03          # no log term
    assert np.abs((1 - fs - fs / 6 * np.log(fs)) / v_ex - 1).max() > 0.03
    assert np.abs((1 + fs / 9 + fs / 18 * np.log(fs)) / t_ex - 1).max() > 0.01


def _face_field_state(mesh, E0=5.0, emit_zmin=-1.0):
    om = O.OracleMesh(mesh, emit_zmin)
    st = O.OracleState(om, 200000)
    st.init_field(E0, tol=1e-13)
    return om, st


def test_stochastic_rounding_unbiased(plates_mesh):
    """Eq. rnd_nsp keeps the mean count: average n' over many steps equals
    n within 5 sigma."""
    om, st = _face_field_state(plates_mesh)
    assert om.n_emit == 2 * 4 * 4           # the z = 0 plane emits
    rate, _ = om.emission_rate(st.E, 4.5)
    n_face = rate / om.n_emit * 0.5         # e per face per step
    w_sp = n_face / 2.37                    # n = 2.37 SPs per face-step
    tot = 0
    steps = 400
    for k in range(steps):
        st.n = 0
        _, counts, _ = st.inject(dt=0.5, E0=5.0, w_sp=w_sp, phi_w=4.5, step=k,
                                 seed=3)
        assert set(np.unique(counts)) <= {2, 3}
        tot += counts.sum()
    mean = tot / (steps * om.n_emit)
    sigma = math.sqrt(0.37 * 0.63 / (steps * om.n_emit))
    assert abs(mean - 2.37) < 5 * sigma


def test_triangle_sampling_uniform(plates_mesh):
    om, st = _face_field_state(plates_mesh)
    em = om.emit()
    rate, _ = om.emission_rate(st.E, 4.5)
    w_sp = rate / om.n_emit * 0.5 / 400.0   # ~400 SPs per face
    _, counts, pts = st.inject(dt=0.5, E0=5.0, w_sp=w_sp, phi_w=4.5, step=1,
                               seed=5)
    # barycentric coordinates on each face, binned on a 10x10 grid
    start = np.concatenate([[0], np.cumsum(counts)])
    hist = np.zeros((10, 10))
    for f in range(om.n_emit):
        A, B, C = em["abc"][f]
        P = pts[start[f]:start[f + 1]]
        M = np.stack([B - A, C - A], axis=1)
        sol = np.linalg.lstsq(M, (P - A).T, rcond=None)[0].T
        assert (sol >= -1e-12).all() and (sol.sum(1) <= 1 + 1e-12).all()
        # fold the triangle onto the unit square's lower half: bins with
        # i + j < 9 are whole, the diagonal ones are half cells
        i = np.minimum((sol[:, 0] * 10).astype(int), 9)
        j = np.minimum((sol[:, 1] * 10).astype(int), 9)
        np.add.at(hist, (i, j), 1)
    ii, jj = np.meshgrid(np.arange(10), np.arange(10), indexing="ij")
    area = np.where(ii + jj < 9, 1.0, np.where(ii + jj == 9, 0.5, 0.0))
    n = hist.sum()
    exp = n * area / area.sum()
    mask = area > 0
    chi2 = (((hist - exp) ** 2)[mask] / exp[mask]).sum()
    assert hist[~mask].sum() == 0
    # 64 cells -> 63 dof; p = 1e-4 critical value ~ 112
    assert chi2 < 112


def test_injection_velocity_displacement(plates_mesh):
    """Eq. sp_velocity / Eq. sp_displacement in the uniform field: v0 is
    antiparallel to E (electrons), |v0| / (|q/m| E dt) = 1/2 + R and the
    displacement is v0 dt R, with R taken from numpy's Philox."""
    om, st = _face_field_state(plates_mesh)
    k = O.constants()
    rate, _ = om.emission_rate(st.E, 4.5)
    w_sp = rate / om.n_emit * 0.5 / 3.0
    _, counts, pts = st.inject(dt=0.5, E0=5.0, w_sp=w_sp, phi_w=4.5, step=4,
                               seed=9)
    P = st.particles()
    idx = 0
    for f in range(om.n_emit):
        for o in range(counts[f]):
            ctr = [4 - 1, f, o, 1]
            R = (np.random.Philox(key=[9, 0], counter=ctr).random_raw(4)[2]
                 >> 11) * 2.0**-53
            v = np.array([P["vx"][idx], P["vy"][idx], P["vz"][idx]])
            a = k["qm"] * 5.0 * 0.5     # |v0| scale = |q/m| E0 dt
            assert abs(v[2] / (-a) - (0.5 + R)) < 1e-9
            assert abs(v[0]) < 1e-9 and abs(v[1]) < 1e-9
            r = np.array([P["x"][idx], P["y"][idx], P["z"][idx]])
            assert np.abs(r - (pts[idx] + v * 0.5 * R)).max() < 1e-12
            idx += 1


# ---------------------------------------------------------------------------
# The full step: closed-form trajectories, periodic wrap, absorption and
# exact charge conservation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1], ids=["nodal", "cell"])
def test_uniform_field_trajectory_closed_form(plates_mesh, mode):
    """Leapfrog is exact for constant acceleration: after its first step a
    particle satisfies r_n = r_1 + (n-1) dt v0 + a dt^2 n(n-1)/2 (the
    uniform field is the same in the nodal and the cell reading)."""
    om, st = _face_field_state(plates_mesh, E0=5.0)
    k = O.constants()
    rate, _ = om.emission_rate(st.E, 4.5)
    w_sp = 1e-30                              # space charge far below 1e-12
    js = w_sp * 1.5 * om.n_emit / (rate * 0.5)  # ~1.5 SPs per face-step
    dt = 0.5
    a = k["qm"] * np.array([0.0, 0.0, -5.0])
    first = {}
    for step in range(8):
        s = st.step(dt=dt, E0=5.0, w_sp=w_sp, phi_w=4.5, step=step, seed=1,
                    j_scale=js, tol=1e-13, field_mode=mode)
        assert s["status"] == 0
        P = st.particles()
        for i, pid in enumerate(P["id"]):
            born = int(pid) >> 42
            r = np.array([P["x"][i], P["y"][i], P["z"][i]])
            if born == step:
                first[int(pid)] = (r, np.array([P["vx"][i], P["vy"][i],
                                                P["vz"][i]]))
                continue
            r1, v0 = first[int(pid)]
            n = step - born + 1
            ref = r1 + (n - 1) * dt * v0 + a * dt**2 * n * (n - 1) / 2
            d = r - ref
            d[:2] -= np.round(d[:2] / plates_mesh.Lx) * plates_mesh.Lx
            assert np.abs(d).max() < 1e-9
    assert len(first) > 20


def test_periodic_wrap_and_absorption(plates_mesh):
    om, st = _face_field_state(plates_mesh, E0=1e-6)
    L, Lz = plates_mesh.Lx, plates_mesh.z_top
    p = np.array([[L - 0.05, 1.0, 2.0],     # crosses x = L
                  [0.02, 0.5, 1.0],        # crosses x = 0 backwards
                  [1.0, L - 0.01, 3.0],     # crosses y = L
                  [1.0, 1.0, Lz - 0.1],     # reaches the anode
                  [1.0, 1.0, 0.1]])         # enters the cathode
    v = np.array([[0.3, 0, 0], [-0.1, 0, 0], [0, 0.1, 0], [0, 0, 0.5],
                  [0, 0, -0.5]])
    tet, _ = om.locate(p)
    st.add(p, v, tet, w=np.array([1.0, 0.5, 0.25, 1.0, 0.75]))
    s = st.step(dt=0.5, E0=1e-6, w_sp=1e-30, phi_w=4.5, step=0, seed=1,
                j_scale=0.0, tol=1e-12)
    P = st.particles()
    assert s["n_anode"] == 1 and s["n_cathode"] == 1 and P["x"].size == 3
    assert abs(P["x"][0] - (L - 0.05 + 0.15 - L)) < 1e-12
    assert abs(P["x"][1] - (0.02 - 0.05 + L)) < 1e-12
    assert abs(P["y"][2] - (L - 0.01 + 0.05 - L)) < 1e-12
    S = 2**40
    assert s["q_anode"] == S and s["q_cathode"] == int(0.75 * S)
    assert s["q_before"] + s["q_inj"] - s["q_anode"] - s["q_cathode"] == \
        s["q_after"]
    tet2, where = om.locate(np.stack([P["x"], P["y"], P["z"]], 1))
    assert (tet2 == P["tet"]).all() and (where == 0).all()


def test_step_conservation_tiny_tip(tiny_mesh):
    """Charge bookkeeping of a stressed run on the tiny tip: every step
    conserves live charge exactly in fixed point."""
    cfg = W.config_tiny()
    om = O.OracleMesh(tiny_mesh, cfg.emit_zmin)
    st = O.OracleState(om, 40000)
    st.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = om.emission_rate(st.E, cfg.phi_w)
    w_sp = rate * cfg.dt * cfg.transit_steps / cfg.n_target
    for k in range(4):
        s = st.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, step=k,
                    seed=cfg.seed, tol=cfg.tol)
        assert s["status"] == 0
        assert s["q_before"] + s["q_inj"] - s["q_anode"] - s["q_cathode"] == \
            s["q_after"]
        assert s["n_before"] + s["n_inj"] - s["n_anode"] - s["n_cathode"] == \
            s["n_after"]
    assert st.n > 1000
    P = st.particles()
    tet, where = om.locate(np.stack([P["x"], P["y"], P["z"]], 1))
    assert (tet == P["tet"]).all()
