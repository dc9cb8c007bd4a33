"""Planar-diode validation (the paper's PIC check, Sec. III A), CPU side.

The semianalytic model of oracle/diode.py is pinned against the Child-
Langmuir law, the FN current without space charge and a numerical
integration of the 1D Poisson equation; the oracle's PIC cycle on a coarse
diode is then checked against the model and against the momentum balance
of the beam (a law of 1D steady flow that holds whatever the emission)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import diode as D
from oracle import oracle as O
from paper_1906_08125_amd import workloads as W


def test_diode_workload_is_the_papers_geometry():
    """The diode workload's default mesh is the paper's validation geometry
    (Sec. III A; tests/golden/diode_validation.txt): the gap exactly, the
    electrode area to the lattice (32 x 32 cubes of 0.364 nm: 135.7 nm^2)."""
    from conftest import golden
    g = golden("diode_validation.txt")
    cfg = W.config_diode(14.0)
    assert abs(cfg.nz * cfg.h - float(g["gap_nm"][0])) < 1e-12
    area = (cfg.nx * cfg.h) * (cfg.ny * cfg.h)
    assert abs(area / float(g["area_nm2"][0]) - 1) < 0.006
    assert 0.0 < float(g["rms_vs_semianalytic"][0]) < 0.05


def test_gap_reduces_to_child_langmuir():
    """E_c = 0: the closed-form gap of the Child-Langmuir density is d."""
    for Ea in (2.0, 7.5, 14.0, 30.0):
        for d in (5.0, 18.2, 100.0):
            J = D.child_langmuir(Ea, d)
            assert abs(D.gap(0.0, Ea, J) / d - 1) < 1e-12
            # and the anode sits at V = (3/4) E_a d
            assert abs(D.voltage(0.0, Ea, J) / (0.75 * Ea * d) - 1) < 1e-12


def test_weak_emission_is_plain_fn():
    """With negligible current the cathode field is the applied one and the
    density is the FN density there."""
    s = D.steady_state(3.0, 18.2, 4.5)
    assert abs(s["E_c"] / 3.0 - 1) < 1e-6
    assert abs(s["J"] / D.fn_density(3.0, 4.5) - 1) < 1e-5
    assert abs(s["V"] / (3.0 * 18.2) - 1) < 1e-5


@pytest.mark.parametrize("Ea", [8.0, 14.0, 25.0])
def test_steady_state_solves_poisson(Ea):
    """Integrate phi'' = (J / eps0) / v(phi), v = sqrt(2 |q/m| phi), from the
    model's E_c over z in [0, d]: the field reaches E_a and the potential V
    at z = d (an independent check of the closed-form integral)."""
    d = 18.2
    s = D.steady_state(Ea, d, 4.5)
    k = O.constants()
    eps0, qm = 1.0 / k["e_eps"], abs(k["qm"])
    Ec, J = s["E_c"], s["J"]
    assert 0 < Ec < Ea and s["J"] < D.child_langmuir(Ea, d)
    # near z = 0: phi = Ec z + (4/3) c z^(3/2) with E' = c z^(-1/2),
    # c = J / (eps0 sqrt(2 qm Ec))
    c = J / (eps0 * math.sqrt(2 * qm * Ec))
    z0 = 1e-9
    y0 = [Ec * z0 + (4.0 / 3.0) * c * z0 ** 1.5, Ec + 2.0 * c * math.sqrt(z0)]

    def rhs(z, y):
        return [y[1], J / (eps0 * math.sqrt(2 * qm * max(y[0], 1e-300)))]

    sol = solve_ivp(rhs, (z0, d), y0, rtol=1e-11, atol=1e-14, method="DOP853")
    phi_d, E_d = sol.y[0, -1], sol.y[1, -1]
    assert abs(E_d / Ea - 1) < 1e-6
    assert abs(phi_d / s["V"] - 1) < 1e-6


def _run_oracle_diode(E0, n_steps, per_step, dt=0.02):
    cfg = W.config_diode(E0, nx=8, nz=36, h=0.5, dt=dt, n_steps=n_steps)
    mesh = cfg.mesh()
    om = O.OracleMesh(mesh, cfg.emit_zmin)
    ost = O.OracleState(om, 200_000)
    ost.init_field(E0, tol=1e-12)
    A, d = mesh.Lx * mesh.Ly, mesh.z_top
    s = D.steady_state(E0, d, cfg.phi_w)
    w_sp = s["J"] * A * dt / per_step
    top = np.isclose(mesh.xyz[:, 2], d)
    q_a, Q, V = 0, 0.0, 0.0
    n = 0
    for k in range(n_steps):
        st = ost.step(dt=dt, E0=E0, w_sp=w_sp, phi_w=cfg.phi_w, step=k,
                      seed=cfg.seed, tol=cfg.tol)
        assert st["status"] == 0
        if k >= n_steps // 2:
            n += 1
            q_a += st["q_anode"]
            Q += st["q_after"] / 2.0 ** 40 * w_sp
            V += ost.phi[top].mean()
    J = q_a / 2.0 ** 40 * w_sp / (n * dt) / A
    return dict(J=J, Q=Q / n, V=V / n, A=A, d=d, semi=s)


def _balance(E0, r):
    """E_a^2 - E_c^2 against (4 J / eps0) sqrt(m V / (2 e)), with E_c from
    Gauss's law over the charge in flight."""
    k = O.constants()
    eps0, qm = 1.0 / k["e_eps"], abs(k["qm"])
    Ec = E0 - r["Q"] / (eps0 * r["A"])
    lhs = E0 ** 2 - Ec ** 2
    rhs = 4.0 * r["J"] / eps0 * math.sqrt(r["V"] / (2.0 * qm))
    return Ec, rhs / lhs


def test_oracle_diode_fn_regime():
    """Weak space charge (E_a = 5 V/nm): the anode current is the FN
    current of the applied field and the gap voltage is E_a d."""
    r = _run_oracle_diode(5.0, 800, 20)
    assert abs(r["J"] / r["semi"]["J"] - 1) < 0.03
    assert abs(r["V"] / r["semi"]["V"] - 1) < 1e-3
    Ec, ratio = _balance(5.0, r)
    assert abs(ratio - 1) < 0.02


def test_oracle_diode_space_charge_regime():
    """Strong space charge (E_a = 14 V/nm): the current falls to a few
    tenths of the FN current of the applied field, stays below the
    Child-Langmuir bound, follows the semianalytic model within the
    discretization error of the surface field (first-order in the cathode
    layer), and the beam's momentum balance holds."""
    r = _run_oracle_diode(14.0, 1200, 40)
    J_fn = D.fn_density(14.0, 4.5)
    assert r["J"] < 0.3 * J_fn
    assert r["J"] < D.child_langmuir(14.0, r["d"])
    assert abs(r["J"] / r["semi"]["J"] - 1) < 0.12
    assert abs(r["V"] / r["semi"]["V"] - 1) < 0.03
    Ec, ratio = _balance(14.0, r)
    assert Ec < 0.8 * 14.0
    assert abs(ratio - 1) < 0.03
