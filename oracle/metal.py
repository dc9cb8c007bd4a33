"""Metal-side solves of Sec. II D: the current continuity equation (Eq.
cont with Eq. cont_bc, weak form of App. C), Joule heating (Eq. joule) and
one step of the heat equation (Eq. heat with Eq. heat_bc, weak form and
Theta-scheme of App. D), in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's
CPU-baseline leg, never by the product path.  It shares no code with the
HIP library; both sides read the same mesh arrays of
``paper_1906_08125_amd.workloads.MetalMesh``.

Every matrix is assembled from its definition, element by element, over
linear tetrahedra (P1): with shape-function gradients g_a (constant on a
tetrahedron of volume V),

    stiffness  int c grad N_a . grad N_b  = c V g_a . g_b
    mass       int c N_a N_b             = c V (1 + delta_ab) / 20
    volume load int N_a p                = p V / 4
    face load  int_face N_a q            = q A / 3     (triangle of area A)

with c, p constant per tetrahedron and q constant per face.  The linear
systems are solved directly (scipy's sparse LU): the oracle's result is the
exact discrete solution, which the device's iterative solver approaches to
its tolerance.

Readings (the paper leaves these open):
* the conductivity sigma is an input per tetrahedron (sigma(T) and its
  finite-size correction come from sources outside the paper);
* the flux through an interface face is an input J_n = J_e . n per face
  (n the outward normal of the metal; GETELEC is outside the paper), and so
  is the Nottingham flux P_N;
* kappa = L T sigma (Eq. wied_franz) per tetrahedron with T the mean of its
  four nodal temperatures at the start of the step: the conductivities are
  lagged, kappa^{n+1} ~ kappa^n, as App. D states;
* the volumetric heat capacity C_v is a constant and the sources P_J, P_N
  are held over the step, so f^{n+1} = f^n in Eq. heat_theta2;
* Dirichlet values (Phi = 0, T = T_amb on the bottom plane) are imposed by
  elimination.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def geometry(xyz, tet):
    """Shape-function gradients [n_tets, 4, 3] and volumes [n_tets] of P1
    tetrahedra: N_a(x) = c_a + g_a . x solves N_a(x_b) = delta_ab, i.e. the
    coefficients are the columns of the inverse of [1 x y z] over the four
    vertices."""
    X = xyz[tet]
    A = np.concatenate([np.ones(X.shape[:2] + (1,)), X], axis=2)
    inv = np.linalg.inv(A)
    grads = np.transpose(inv[:, 1:4, :], (0, 2, 1))
    vol = np.abs(np.linalg.det(A)) / 6.0
    return grads, vol


def stiffness(xyz, tet, coef):
    """sum over tetrahedra of coef_t int grad N_a . grad N_b (sparse)."""
    g, V = geometry(xyz, tet)
    loc = np.einsum("tai,tbi->tab", g, g) * (coef * V)[:, None, None]
    return _scatter(tet, loc, xyz.shape[0])


def mass(xyz, tet, coef):
    """sum over tetrahedra of coef_t int N_a N_b (consistent mass)."""
    _, V = geometry(xyz, tet)
    ref = (np.ones((4, 4)) + np.eye(4)) / 20.0
    loc = ref[None] * (coef * V)[:, None, None]
    return _scatter(tet, loc, xyz.shape[0])


def _scatter(tet, loc, n):
    rows = np.repeat(tet, 4, axis=1).reshape(-1)
    cols = np.tile(tet, (1, 4)).reshape(-1)
    return sp.coo_matrix((loc.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()


def volume_load(xyz, tet, p):
    """int N_a p over the tetrahedra, p constant per tetrahedron."""
    _, V = geometry(xyz, tet)
    f = np.zeros(xyz.shape[0])
    np.add.at(f, tet.reshape(-1), np.repeat(p * V / 4.0, 4))
    return f


def face_load(xyz, faces, q):
    """int_face N_a q over triangles, q constant per triangle."""
    P = xyz[faces]
    A = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]),
                             axis=1)
    f = np.zeros(xyz.shape[0])
    np.add.at(f, faces.reshape(-1), np.repeat(q * A / 3.0, 3))
    return f


def _solve_dirichlet(A, b, fixed, value):
    """A x = b with x = value on the fixed nodes (elimination)."""
    n = b.size
    x = np.zeros(n)
    x[fixed] = value
    free = ~fixed
    rhs = b[free] - A[free][:, fixed] @ x[fixed]
    x[free] = spla.spsolve(A[free][:, free].tocsc(), rhs)
    return x


def continuity_solve(mesh, sigma, flux):
    """Eq. cont_mat: K(sigma) Phi = f, f_a = int_Gamma3 N_a J_n, Phi = 0 on
    the Dirichlet nodes (Gamma5); the lateral faces carry no flux (Gamma4,
    the natural condition)."""
    K = stiffness(mesh.xyz, mesh.tet, np.asarray(sigma, np.float64))
    f = face_load(mesh.xyz, mesh.faces, np.asarray(flux, np.float64))
    return _solve_dirichlet(K, f, mesh.dirichlet.astype(bool), 0.0)


def joule(mesh, sigma, phi):
    """Eq. joule per tetrahedron: sigma |grad Phi|^2 with the P1 gradient."""
    g, _ = geometry(mesh.xyz, mesh.tet)
    grad = np.einsum("tai,ta->ti", g, phi[mesh.tet])
    return sigma * (grad * grad).sum(axis=1)


def heat_step(mesh, T, sigma, P_J, P_N, Cv, L, dt, theta, T_amb):
    """One step of Eq. heat_theta2:
    (C/dt + theta K) T^{n+1} = (C/dt - (1 - theta) K) T^n + f,
    C = int C_v N_a N_b, K = int kappa grad N_a . grad N_b with
    kappa = L T sigma (lagged), f = int N_a P_J + int_Gamma3 N_a P_N,
    T = T_amb on the Dirichlet nodes."""
    T = np.asarray(T, np.float64)
    kappa = L * np.asarray(sigma, np.float64) * T[mesh.tet].mean(axis=1)
    K = stiffness(mesh.xyz, mesh.tet, kappa)
    C = mass(mesh.xyz, mesh.tet, np.full(mesh.n_tets, float(Cv)))
    f = volume_load(mesh.xyz, mesh.tet, np.asarray(P_J, np.float64)) + \
        face_load(mesh.xyz, mesh.faces, np.asarray(P_N, np.float64))
    A = C / dt + theta * K
    b = (C / dt - (1.0 - theta) * K) @ T + f
    return _solve_dirichlet(A.tocsr(), b, mesh.dirichlet.astype(bool), T_amb)
