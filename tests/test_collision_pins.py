"""Pins of the oracle's binary collisions (App. F, after Takizuka and Abe)
against what the appendix and mechanics fix: momentum and kinetic energy
of every cell conserved, every superparticle of a cell with two or more
colliding (odd-count rule included), and the scattering statistics of
Eq. variance evaluated from SI constants: the mean squared velocity change
of a pair, 2 <delta^2> |u|^2 in the small-angle limit, with <delta^2>
scaling as n dt / (u^3 V), and half the variance in the three collisions
of an odd cell."""
import math

import numpy as np
import pytest

from oracle import oracle as O

E = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
LANDAU = 13.0


def _var_full(n_e, dt, u, V):
    """<delta^2> of Eq. variance with SI constants, in the oracle's units
    (nm, fs): e^4 / (2 pi eps0^2 m^2) in m^6 s^-4 is 1e-6 nm^6 fs^-4."""
    c = E ** 4 / (2 * math.pi * EPS0 ** 2 * ME ** 2) * 1e54 * 1e-60
    return c * n_e * LANDAU * dt / (u ** 3 * V)


def _state(mesh, cells, vel, w=None):
    om = O.OracleMesh(mesh, 0.01)
    T = om.tets()
    tet = np.repeat(np.asarray(cells, np.int32),
                    [len(v) for v in vel]).astype(np.int32)
    v = np.concatenate(vel)
    cen = T["vert"].mean(axis=1)[tet]
    st = O.OracleState(om, len(tet) + 8)
    st.add(cen, v, tet, w=w, ids=np.arange(len(tet)) * 7 + 3)
    return om, T, st, tet


def test_collisions_conserve_momentum_and_energy(tiny_mesh):
    rng = np.random.default_rng(21)
    sizes = [2, 3, 4, 5, 7, 8, 11, 50, 1]
    cells = [5, 900, 1234, 20000, 31000, 7, 43000, 15000, 333]
    vel = [rng.normal(0.0, 1.0, (n, 3)) for n in sizes]
    om, T, st, tet = _state(tiny_mesh, cells, vel)
    v0 = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1).copy()
    st.collide(dt_coll=2.5, w_sp=40.0, seed=9, step=3)
    v1 = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1)
    for c, n in zip(cells, sizes):
        sel = tet == c
        p0, p1 = v0[sel].sum(0), v1[sel].sum(0)
        e0, e1 = (v0[sel] ** 2).sum(), (v1[sel] ** 2).sum()
        assert np.abs(p1 - p0).max() <= 1e-13 * max(1.0, np.abs(v0[sel]).sum())
        assert abs(e1 - e0) <= 1e-13 * e0
        changed = np.any(v1[sel] != v0[sel], axis=1)
        assert changed.all() if n >= 2 else not changed.any()
    # the same call again with another step draws other pairs and angles
    st2 = O.OracleState(om, st.cap)
    st2.add(v0 * 0 + T["vert"].mean(axis=1)[tet], v0, tet,
            ids=np.arange(len(tet)) * 7 + 3)
    st2.collide(dt_coll=2.5, w_sp=40.0, seed=9, step=4)
    assert not np.array_equal(st2.vx[:st2.n], st.vx[:st.n])


def _msq_change(mesh, groups, dt, w_sp, seed=5):
    """Mean over cells of sum_i |dv_i|^2, and the cells' volumes."""
    om, T, st, tet = _state(mesh, range(len(groups)), groups)
    v0 = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1).copy()
    st.collide(dt_coll=dt, w_sp=w_sp, seed=seed, step=0)
    v1 = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1)
    dv2 = ((v1 - v0) ** 2).sum(1)
    per_cell = np.bincount(tet, weights=dv2, minlength=len(groups))
    V = T["D"][: len(groups)] / 6.0
    return per_cell, V


def _unit(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1)[:, None]


@pytest.mark.parametrize("u", [1.0, 2.0])
def test_pair_scattering_follows_the_variance(tiny_mesh, u):
    """Two-particle cells with relative speed u: E[sum |dv|^2] =
    2 <delta^2> u^2 (small angles), with <delta^2> from Eq. variance."""
    rng = np.random.default_rng(31)
    N = 20000
    d = _unit(rng, N)
    groups = [np.stack([np.zeros(3), u * d[i]]) for i in range(N)]
    dt, w_sp = 1.0, 5e-6
    per_cell, V = _msq_change(tiny_mesh, groups, dt, w_sp)
    var = _var_full(2 * w_sp, dt, u, V)
    assert var.max() < 0.02                  # small-angle regime
    want = 2.0 * var * u * u
    r = per_cell.sum() / want.sum()
    assert abs(r - 1) < 0.03, r


def test_odd_cells_collide_three_times_at_half_variance(tiny_mesh):
    """Three-particle cells with equal relative speeds s (an equilateral
    triangle in velocity space): three collisions at half variance give
    E[sum |dv|^2] = 3 <delta^2>_full s^2 (at full variance it would be
    twice that)."""
    rng = np.random.default_rng(41)
    N = 12000
    s = 1.0
    groups = []
    for i in range(N):
        a, b = _unit(rng, 2)
        b = b - a * (a @ b)
        b /= np.linalg.norm(b)
        r = s / math.sqrt(3.0)
        pts = [r * (math.cos(t) * a + math.sin(t) * b)
               for t in (0.0, 2 * math.pi / 3, 4 * math.pi / 3)]
        groups.append(np.stack(pts))
    dt, w_sp = 1.0, 3e-6
    per_cell, V = _msq_change(tiny_mesh, groups, dt, w_sp)
    var = _var_full(3 * w_sp, dt, s, V)
    assert var.max() < 0.02
    want = 3.0 * var * s * s
    r = per_cell.sum() / want.sum()
    assert abs(r - 1) < 0.04, r


def test_scattering_angles_are_gaussian_in_tan_half_theta(tiny_mesh):
    """delta = tan(theta/2) of the pair's relative velocity is normal with
    the variance of Eq. variance: its second moment matches and 68.3 % of
    the draws fall within one standard deviation."""
    rng = np.random.default_rng(51)
    N = 20000
    u = 1.5
    d = _unit(rng, N)
    groups = [np.stack([np.zeros(3), u * d[i]]) for i in range(N)]
    dt, w_sp = 1.0, 5e-4
    om, T, st, tet = _state(tiny_mesh, range(N), groups)
    st.collide(dt_coll=dt, w_sp=w_sp, seed=17, step=2)
    v = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1).reshape(N, 2, 3)
    rel1 = v[:, 1] - v[:, 0]
    rel0 = u * d
    cos_t = (rel0 * rel1).sum(1) / (u * np.linalg.norm(rel1, axis=1))
    cos_t = np.clip(cos_t, -1.0, 1.0)
    tan_half = np.sqrt((1 - cos_t) / (1 + cos_t))
    var = _var_full(2 * w_sp, dt, u, T["D"][:N] / 6.0)
    z = tan_half / np.sqrt(var)
    assert abs((z ** 2).mean() - 1) < 0.04
    assert abs((z < 1).mean() - 0.6827) < 0.015
    # the relative speed is unchanged
    assert np.abs(np.linalg.norm(rel1, axis=1) - u).max() < 1e-13


def test_extreme_variance_stays_finite(tiny_mesh):
    """Pairs with nearly equal velocities (relative speed 1e-120 nm/fs:
    <delta^2> overflows) still conserve momentum and energy and stay
    finite: Eq. sin_theta in its theta -> pi limit."""
    rng = np.random.default_rng(61)
    N = 200
    base = rng.normal(size=(N, 3))
    d = _unit(rng, N) * 1e-120
    groups = [np.stack([base[i], base[i] + d[i]]) for i in range(N)]
    om, T, st, tet = _state(tiny_mesh, range(N), groups)
    v0 = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1).copy()
    st.collide(dt_coll=1.0, w_sp=1.0, seed=3, step=1)
    v1 = np.stack([st.vx[:st.n], st.vy[:st.n], st.vz[:st.n]], 1)
    assert np.isfinite(v1).all()
    assert np.abs(v1 - v0).max() < 1e-100
