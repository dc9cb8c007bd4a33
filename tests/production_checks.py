"""Checks of a device PIC state against the oracle that work at any size
(shared by the production-size and batched-size parity tests): the oracle
computes them one superparticle or one pass at a time.

* fields_and_charge: the oracle's deposition of every live device
  superparticle (bit-exact) and its total; the true residual of the device
  potential under the oracle's K and right-hand side; the oracle's nodal
  field of the device potential.
* replay_sample: one step of sampled superparticles replayed by the
  oracle's arithmetic from the device state before it (gather, kick,
  drift, wrap, absorption), against the device state after it, and the
  oracle's canonical location of every sampled survivor (bit-exact)."""
import numpy as np

from oracle import oracle as O


def host(gs):
    n = int(gs.n_slots.item())
    g = lambda t: t[:n].cpu().numpy().astype(np.float64)
    i = lambda t: t[:n].cpu().numpy()
    return dict(n=n, x=g(gs.x), y=g(gs.y), z=g(gs.z), vx=g(gs.vx), vy=g(gs.vy),
                vz=g(gs.vz), w=g(gs.w), tet=i(gs.tet), id=i(gs.id),
                phi=gs.phi.cpu().numpy(),
                E=gs.E.cpu().numpy().astype(np.float64).reshape(-1, 4)[:, :3],
                charge=gs.charge.cpu().numpy())


def fields_and_charge(om, cfg, kw, S, ftol):
    live = S["tet"] >= 0
    p = np.stack([S["x"], S["y"], S["z"]], 1)[live]
    c = om.deposit(p, S["tet"][live], S["w"][live])
    assert np.array_equal(c, S["charge"])
    q = np.rint(S["w"][live] * 2.0**40).astype(np.int64)
    assert int(S["charge"].sum()) == int(q.sum())
    fid, _ = om.free()
    free = np.flatnonzero(fid >= 0)
    free = free[np.argsort(fid[free])]
    b = om.rhs(S["charge"], kw["w_sp"], cfg.E0)
    r = b - om.spmv(S["phi"][free])
    assert np.linalg.norm(r) <= 1.5 * cfg.tol * np.linalg.norm(b)
    E = om.field(S["phi"])
    assert np.linalg.norm(E - S["E"]) <= ftol * np.linalg.norm(E)



def replay_sample(om, tip, dt, A, B, ftol, cell=False, n_pick=3000, seed=11,
                  max_mismatch=None):
    """A, B: host() snapshots before and after one device step."""
    cfg_dt = dt
    Et = om.cell_field(A["phi"]) if cell else None
    live = np.flatnonzero(A["tet"] >= 0)
    rng = np.random.default_rng(seed)
    pick = rng.choice(live, size=min(n_pick, live.size), replace=False)
    where_b = {int(i): k for k, i in enumerate(B["id"]) if B["tet"][k] >= 0}
    k_ = O.constants()
    Q = (k_["qm"] * cfg_dt) * 0.5
    Lx, Ly, ztop = tip.Lx, tip.Ly, tip.z_top
    nodes = om.tets()["tet"]
    survivors = []
    # FP32 storage can put a particle on the other side of a decision
    # boundary (anode plane, lateral wrap, metal surface) than the FP64
    # replay when it lies within rounding of it: counted, none allowed
    # in FP64, a few in mixed precision
    mism = 0
    for i in pick:
        p = np.array([A["x"][i], A["y"][i], A["z"][i]])
        v = np.array([A["vx"][i], A["vy"][i], A["vz"][i]])
        t = int(A["tet"][i])
        if cell:
            E = Et[t]
        else:
            lam = om.lam(t, p)
            e = A["E"][nodes[t]]
            E = ((lam[0] * e[0] + lam[1] * e[1]) + lam[2] * e[2]) + lam[3] * e[3]
        qE = Q * E
        v = (v + qE) + qE
        p = p + cfg_dt * v
        if p[0] >= Lx:
            p[0] -= Lx
        elif p[0] < 0.0:
            p[0] += Lx
        if p[1] >= Ly:
            p[1] -= Ly
        elif p[1] < 0.0:
            p[1] += Ly
        k = where_b.get(int(A["id"][i]))
        if p[2] >= ztop:  # anode-absorbed on the device too
            mism += k is not None
            continue
        if k is None:  # absorbed by the cathode: outside every vacuum tet
            tt, wh = om.locate(p[None, :])
            mism += not (tt[0] < 0 and wh[0] == 2)
            continue
        q = np.array([B["x"][k], B["y"][k], B["z"][k]])
        if np.abs(q - p).max() > ftol * max(1.0, np.abs(p).max()):
            mism += 1  # (wrapped on the other side)
            continue
        assert np.abs(np.array([B["vx"][k], B["vy"][k], B["vz"][k]]) - v).max() \
            <= ftol * max(1.0, np.abs(v).max())
        survivors.append(k)
    limit = (0 if ftol < 1e-9 else 3) if max_mismatch is None else max_mismatch
    assert mism <= limit, mism
    assert len(survivors) > 0.9 * len(pick)
    ks = np.array(survivors)
    pts = np.stack([B["x"][ks], B["y"][ks], B["z"][ks]], 1)
    tt, wh = om.locate(pts)
    assert np.array_equal(tt, B["tet"][ks])
    return len(pick), len(survivors)
