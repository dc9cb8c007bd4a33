"""Adjoint of a window of PIC steps, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the reference the
device adjoint is checked against, itself checked against central finite
differences of the oracle's forward window.

The paper has no adjoint; what is differentiated is this reading of it:

* Objective J = J_Q + J_E over a window of T steps.  J_Q = w_sp * sum of w
  over the superparticles the anode collects (the collected charge in e).
  J_E = mean over the emitting faces f and over the post-solve fields
  E_1 .. E_T of |e_f|, with e_f = ((E_a + E_b) + E_c) / 3 the field at the
  face centroid (the quantity Eq. nsp's current density is evaluated at).
* Parameters: the applied field E0 (Eq. poisson_bc) and a multiplier s_f
  of the weight of every superparticle born at face f, w = s_f omega
  (omega the base weight), including those in flight at the window start.
* Held fixed: the emission counts (Eq. rnd_nsp is not differentiable), the
  injection draws, which superparticles are absorbed, and the containing
  tets; the fixed-point rounding of the deposition is taken as exact, so
  the charge is c = sum lambda w (scaled by 2^40).

One step k maps (r, v, w; E_k) to (r', v'; E_{k+1}): the gather
E_p = sum_i lambda_i(r) E_k[i] (tet fixed, lambda affine in r), the kick
v' = v + 2Q E_p (Q = q/m dt / 2, Eq. leapfrog1 and leapfrog3), the drift
r' = r + dt v' (Eq. leapfrog2); injected superparticles start at
x_f + dt (1 + R) v0 with v0 = (q/m) dt (0.5 + R) sum (l0, R1, R2) E_k
(Eq. sp_velocity, Eq. sp_displacement); then c = sum lambda(r') w,
K phi = (-e/eps0) w_sp c + E0 g (App. B) and E_{k+1} = R phi.  The reverse
of a step, with adjoints rb, vb of (r', v') and Eb of E_{k+1}:

  phib = R^T Eb,  K mu = phib (K symmetric),  dJ/dE0 += g . mu,
  cb = (-e/eps0) w_sp mu,
  rb += w sum_j (cb[n_j] - cb[n_0]) m_j           (deposition, j = 1..3)
  sb[f] += omega sum_i cb[n_i] lambda_i(r')        (deposition)
  sb[f] += omega w_sp                               (anode collection)
  vt = vb + dt rb,  a = 2Q vt,
  rb_prev = rb + sum_j m_j ((E_k[n_j] - E_k[n_0]) . a),  vb_prev = vt,
  Eb_k[n_i] += lambda_i(r) a                        (gather)
  injected: v0b = vb + dt (1 + R) rb,  Eb_k[face nodes] += (l0, R1, R2)
            (q/m) dt (0.5 + R) v0b.
The window starts with phi_0 solved from the in-flight charge and E0, whose
reverse ends the sweep.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import oracle as O


def lam_of(geo, tet, p):
    """Barycentric coordinates of points p [n,3] in tets [n] (the oracle's
    fixed arithmetic: d = p - v0, l_k = (m_k.x d.x + m_k.y d.y) + m_k.z d.z,
    l_0 = ((1 - l_1) - l_2) - l_3)."""
    v0 = geo["vert"][tet, 0, :]
    m = geo["m"][tet]
    d = p - v0
    l = (m[:, :, 0] * d[:, None, 0] + m[:, :, 1] * d[:, None, 1]) + \
        m[:, :, 2] * d[:, None, 2]
    l0 = ((1.0 - l[:, 0]) - l[:, 1]) - l[:, 2]
    return np.concatenate([l0[:, None], l], axis=1)


class Window:
    """A window of T oracle steps from a given in-flight population."""

    def __init__(self, om, init, *, dt, w_sp, phi_w, seed, j_scale, step0,
                 T, cap, tol=1e-13):
        self.om = om
        self.init = {k: np.asarray(v).copy() for k, v in init.items()}
        self.dt, self.w_sp, self.phi_w = dt, w_sp, phi_w
        self.seed, self.j_scale, self.step0 = seed, j_scale, step0
        self.T, self.cap, self.tol = T, cap, tol
        self.geo = om.tets()
        self.fid, self.g = om.free()
        rp, col, val = om.csr()
        nf = om.n_free
        self.K = sp.csr_matrix((val, col, rp), shape=(nf, nf)).tocsc()
        self.free_nodes = np.flatnonzero(self.fid >= 0)
        order = self.fid[self.free_nodes]
        self.free_nodes = self.free_nodes[np.argsort(order)]
        self.faces = om.emit()["nodes"]
        k = O.constants()
        self.qm = k["qm"]
        self.e_eps = k["e_eps"]

    # ---- forward ----------------------------------------------------------
    def face_mean_abs(self, E):
        e = ((E[self.faces[:, 0]] + E[self.faces[:, 1]]) + E[self.faces[:, 2]]) / 3.0
        return float(np.mean(np.sqrt(np.sum(e * e, axis=1)))) if len(e) else 0.0

    def forward(self, E0, s, counts=None, keep=False):
        """Returns (J_Q, J_E, checkpoints or None, counts per step)."""
        om, I = self.om, self.init
        s = np.asarray(s, np.float64)
        st = O.OracleState(om, self.cap)
        p = np.stack([I["x"], I["y"], I["z"]], 1)
        v = np.stack([I["vx"], I["vy"], I["vz"]], 1)
        w = I["omega"] * s[I["birth"]]
        st.add(p, v, I["tet"], w=w, birth=I["birth"], ids=I["id"])
        c0 = om.deposit(p, I["tet"], w)
        st.phi, info = om.poisson_solve(c0, self.w_sp, E0, tol=self.tol)
        st.E = om.field(st.phi)
        JQ = JE = 0.0
        cks, used = [], []
        for k in range(self.T):
            pre = st.particles()
            Ek = st.E.copy()
            det = {}
            st.step(dt=self.dt, E0=E0, w_sp=self.w_sp, phi_w=self.phi_w,
                    step=self.step0 + k, seed=self.seed, j_scale=self.j_scale,
                    tol=self.tol, s_face=s,
                    counts_in=None if counts is None else counts[k],
                    detail=det)
            face = det["inj"][:, 3].astype(np.int64)
            w_all = np.concatenate([pre["w"], s[face]])
            JQ += self.w_sp * float(np.sum(w_all[det["fate"] == 1]))
            JE += self.face_mean_abs(st.E) / self.T
            used.append(det["counts"])
            if keep:
                cks.append(dict(pre=pre, Ek=Ek, det=det, post=st.particles(),
                                Ek1=st.E.copy()))
        return JQ, JE, (cks if keep else None), used

    # ---- reverse ----------------------------------------------------------
    def _solve_adj(self, Eb):
        phib = self.om.field_adj(Eb)[self.free_nodes]
        mu = spla.spsolve(self.K, phib)
        cb = np.zeros(self.om.n_nodes)
        cb[self.free_nodes] = (-self.e_eps * self.w_sp) * mu
        return float(self.g @ mu), cb

    def _dJE_dE(self, E):
        F = len(self.faces)
        out = np.zeros_like(E)
        if F == 0:
            return out
        e = ((E[self.faces[:, 0]] + E[self.faces[:, 1]]) + E[self.faces[:, 2]]) / 3.0
        n = np.sqrt(np.sum(e * e, axis=1))
        gdir = np.where(n[:, None] > 0, e / np.where(n > 0, n, 1.0)[:, None], 0.0)
        for q in range(3):
            np.add.at(out, self.faces[:, q], gdir / (3.0 * F * self.T))
        return out

    def adjoint(self, E0, s, cks, wQ=1.0, wE=1.0):
        """Gradient of wQ J_Q + wE J_E: (dJ/dE0, dJ/ds [n_emit])."""
        s = np.asarray(s, np.float64)
        geo, dt = self.geo, self.dt
        two_q = self.qm * dt  # 2Q
        E0b = 0.0
        sb = np.zeros(len(s))
        Eb_next = np.zeros((self.om.n_nodes, 3))
        rb_post = vb_post = None
        for k in range(self.T - 1, -1, -1):
            ck = cks[k]
            pre, det, post = ck["pre"], ck["det"], ck["post"]
            Ek = ck["Ek"]
            n0 = det["n_before"]
            fate = det["fate"]
            inj = det["inj"]
            face = inj[:, 3].astype(np.int64)
            birth_all = np.concatenate([pre["birth"], face])
            w_all = np.concatenate([pre["w"], s[face]])
            om_all = w_all / s[birth_all]
            # objective on E_{k+1}, then the solve
            Et = Eb_next + wE * self._dJE_dE(ck["Ek1"])
            g_mu, cb = self._solve_adj(Et)
            E0b += g_mu
            # anode collection
            an = np.flatnonzero(fate == 1)
            np.add.at(sb, birth_all[an], wQ * self.w_sp * om_all[an])
            # deposition at the post-step positions
            kept = np.flatnonzero(fate == 0)
            npost = len(kept)
            rp = np.stack([post["x"], post["y"], post["z"]], 1)
            tp = post["tet"]
            lamp = lam_of(geo, tp, rp)
            cbn = cb[geo["tet"][tp]]
            np.add.at(sb, birth_all[kept], om_all[kept] * np.sum(cbn * lamp, 1))
            mp = geo["m"][tp]
            rb = np.zeros((npost, 3)) if rb_post is None else rb_post.copy()
            vb = np.zeros((npost, 3)) if vb_post is None else vb_post.copy()
            rb += w_all[kept][:, None] * np.einsum(
                "nj,njc->nc", cbn[:, 1:] - cbn[:, [0]], mp)
            Eb_k = np.zeros_like(Eb_next)
            # pre-step superparticles that survive: kick and drift reversed
            sel = kept < n0
            i = kept[sel]
            vt = vb[sel] + dt * rb[sel]
            a = two_q * vt
            r0 = np.stack([pre["x"], pre["y"], pre["z"]], 1)[i]
            t0 = pre["tet"][i]
            lam0 = lam_of(geo, t0, r0)
            nd0 = geo["tet"][t0]
            En = Ek[nd0]                       # [n, 4, 3]
            proj = np.einsum("njc,nc->nj", En[:, 1:, :] - En[:, [0], :], a)
            rb_prev = np.zeros((n0, 3))
            vb_prev = np.zeros((n0, 3))
            rb_prev[i] = rb[sel] + np.einsum("nj,njc->nc", proj, geo["m"][t0])
            vb_prev[i] = vt
            for q in range(4):
                np.add.at(Eb_k, nd0[:, q], lam0[:, [q]] * a)
            # superparticles injected in this step
            si = np.flatnonzero(~sel)
            if len(si):
                qi = kept[si] - n0
                R1, R2, Rf = inj[qi, 0], inj[qi, 1], inj[qi, 2]
                f = face[qi]
                v0b = vb[si] + (dt * (1.0 + Rf))[:, None] * rb[si]
                aa = ((self.qm * dt) * (0.5 + Rf))[:, None] * v0b
                l0 = (1.0 - R1) - R2
                for q, wq in enumerate((l0, R1, R2)):
                    np.add.at(Eb_k, self.faces[f, q], wq[:, None] * aa)
            Eb_next = Eb_k
            rb_post, vb_post = rb_prev, vb_prev
        # the window's initial field: phi_0 from the in-flight charge and E0
        g_mu, cb = self._solve_adj(Eb_next)
        E0b += g_mu
        I = self.init
        p = np.stack([I["x"], I["y"], I["z"]], 1)
        lam = lam_of(geo, I["tet"], p)
        np.add.at(sb, I["birth"], I["omega"] * np.sum(cb[geo["tet"][I["tet"]]] * lam, 1))
        return E0b, sb
