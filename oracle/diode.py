"""Semianalytic planar vacuum diode: the reference curve of the paper's PIC
validation (Sec. III A).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.

The paper checks its PIC cycle on two parallel plane electrodes (area 135
nm^2, gap 18.2 nm): the steady current follows from a stationary-point
iteration between the Fowler-Nordheim current density J(E_c) at the
cathode field E_c and the analytic solution of the 1D Poisson equation
with space charge, and tends to the Child-Langmuir law at high voltage.

Here the anode carries the applied field E_a (the Neumann condition of the
top plane, Eq. poisson_bc) instead of a fixed voltage.  In 1D, for a cold
steady beam leaving the cathode from rest (energy e phi = m v^2 / 2,
charge density rho = J / v), phi'' = (J / eps0) sqrt(m / (2 e phi)), whose
first integral is

    phi'(z)^2 = E_c^2 + kappa sqrt(phi(z)),   kappa = (4 J / eps0) sqrt(m / (2 e)),

so that E_a^2 = E_c^2 + kappa sqrt(V) (the momentum balance of the beam)
and the gap is the closed-form integral

    d = int_0^V dphi / phi'
      = (2 / kappa^2) [ (2/3) (E_a^3 - E_c^3) - 2 E_c^2 (E_a - E_c) ]
      = (4 / (3 kappa^2)) (E_a - E_c)^2 (E_a + 2 E_c)

(with s = phi'^2 as the variable of integration; the factored form has no
cancellation when E_c is close to E_a).

Given E_a and d, E_c in (0, E_a] solves d(E_c, J_FN(E_c)) = d (bisection:
the gap shrinks as E_c grows, since the current grows).  E_c -> 0 gives the
Child-Langmuir law with V = (3/4) E_a d; J -> 0 gives E_c = E_a.

Units: nm, fs, V, elementary charges (J in e fs^-1 nm^-2).
"""
from __future__ import annotations

import math

from oracle import oracle as O


def _consts():
    k = O.constants()
    return 1.0 / k["e_eps"], abs(k["qm"]), k["j_unit"]


def fn_density(F: float, phi_w: float) -> float:
    """FN current density (e fs^-1 nm^-2) at the surface field F (V/nm)."""
    _, _, ju = _consts()
    return O.fn_current(F, phi_w)[0] * ju


def kappa(J: float) -> float:
    """(4 J / eps0) sqrt(m / (2 e)) in V^(3/2) nm^-2."""
    eps0, qm, _ = _consts()
    return 4.0 * J / eps0 * math.sqrt(1.0 / (2.0 * qm))


def gap(E_c: float, E_a: float, J: float) -> float:
    """Gap (nm) over which a beam of density J raises the field from E_c at
    the cathode to E_a at the anode."""
    k = kappa(J)
    return 4.0 / (3.0 * k ** 2) * (E_a - E_c) ** 2 * (E_a + 2.0 * E_c)


def voltage(E_c: float, E_a: float, J: float) -> float:
    """Anode potential V from E_a^2 = E_c^2 + kappa sqrt(V)."""
    return ((E_a - E_c) * (E_a + E_c) / kappa(J)) ** 2


def child_langmuir(E_a: float, d: float) -> float:
    """Space-charge-limited density at anode field E_a (E_c = 0):
    J = (4 eps0 / 9) sqrt(2 e / m) (3 E_a / 4)^(3/2) / sqrt(d)."""
    eps0, qm, _ = _consts()
    return (4.0 * eps0 / 9.0) * math.sqrt(2.0 * qm) * (0.75 * E_a) ** 1.5 \
        / math.sqrt(d)


def steady_state(E_a: float, d: float, phi_w: float) -> dict:
    """Self-consistent cathode field, current density and anode potential
    of the FN-emitting planar diode at anode field E_a."""
    lo, hi = 0.0, E_a
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if gap(mid, E_a, fn_density(mid, phi_w)) > d:
            lo = mid
        else:
            hi = mid
    E_c = 0.5 * (lo + hi)
    J = fn_density(E_c, phi_w)
    return dict(E_c=E_c, J=J, V=voltage(E_c, E_a, J))
