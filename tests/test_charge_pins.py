"""Pins of the oracle's surface charge (Sec. II C: Eq. face_charge,
Eq. atom_charge, Eq. charge_weight) against what the physics and the
definition fix: between parallel plates every face carries eps0 E0 A_f
(uniform field, exact) and the cathode carries -eps0 E0 Lx Ly (Gauss's
law); the distribution to atoms conserves the total charge; one atom takes
all of it; an atom sitting on a face takes that face's charge when every
other atom is many r_c away; the cell-field mode agrees with the nodal one
where the field is uniform."""
import math

import numpy as np

from oracle import oracle as O
from paper_1906_08125_amd import workloads as W


def _eps0():
    return 1.0 / O.constants()["e_eps"]


def _plates():
    m = W.kuhn_tip_mesh(6, 6, 8, 0.5)
    om = O.OracleMesh(m, -1.0)
    st = O.OracleState(om, 4)
    st.init_field(0.7, tol=1e-13)
    return m, om, st


def test_plates_face_charge_is_gauss():
    m, om, st = _plates()
    em = om.emit()
    assert om.n_emit == 2 * 6 * 6
    Q, _ = om.surface_charge(st.E, np.zeros((0, 3)))
    assert np.allclose(Q, -_eps0() * 0.7 * em["area"], rtol=1e-11, atol=0)
    assert abs(Q.sum() / (-_eps0() * 0.7 * m.Lx * m.Ly) - 1) < 1e-11
    Qc, _ = om.surface_charge(st.E, np.zeros((0, 3)), phi=st.phi)
    assert np.allclose(Qc, Q, rtol=1e-11, atol=0)


def test_distribution_conserves_charge(tiny_mesh):
    om = O.OracleMesh(tiny_mesh, -1.0)
    st = O.OracleState(om, 4)
    st.init_field(0.4, tol=1e-12)
    atoms = W.surface_atoms(tiny_mesh, density=4.0, seed=3)
    Q, q = om.surface_charge(st.E, atoms, r_c=0.1)
    assert len(q) == len(atoms) > 100
    assert abs(q.sum() / Q.sum() - 1) < 1e-12
    assert (Q <= 0).all()           # the cathode is charged negatively
    # a wider r_c spreads the same total
    _, q2 = om.surface_charge(st.E, atoms, r_c=0.5)
    assert abs(q2.sum() / Q.sum() - 1) < 1e-12
    assert q2.std() < q.std()


def test_single_atom_takes_everything():
    m, om, st = _plates()
    Q, q = om.surface_charge(st.E, np.array([[1.3, 2.1, 0.0]]))
    assert abs(q[0] / Q.sum() - 1) < 1e-13


def test_atoms_on_faces_take_their_faces_charge():
    """One atom on every face centroid and r_c = 0.01 nm (the nearest other
    centroid is 20 r_c or more away): every atom takes its face's charge,
    up to exp(-20)."""
    m, om, st = _plates()
    em = om.emit()
    c = em["abc"].mean(axis=1)
    Q, q = om.surface_charge(st.E, c, r_c=0.01)
    d = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2)
    np.fill_diagonal(d, np.inf)
    assert d.min() >= 0.2
    assert np.abs(q / Q - 1).max() < 1e-7
