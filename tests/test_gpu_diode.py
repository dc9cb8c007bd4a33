"""Planar-diode validation on the GPU (the paper's PIC check, Sec. III A):
a flat FN emitter of 135.7 nm^2 under an 18.2 nm gap, the whole cathode
plane emitting.

* parity: the coupled cycle with emission from the plane against the
  oracle, step by step (counts, ids, tets and charge bit-exact; positions
  and potential to 1e-9);
* the current-field curve at the paper's geometry against the semianalytic
  model (FN current at the self-consistent cathode field of the 1D space-
  charge solution), the Child-Langmuir bound, and the momentum balance of
  the beam E_a^2 - E_c^2 = (4 J / eps0) sqrt(m V / (2 e)) with E_c from
  Gauss's law over the charge in flight."""
import math

import numpy as np
import pytest

from oracle import diode as D
from oracle import oracle as O
from paper_1906_08125_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def test_diode_parity_with_oracle(pic):
    """Coarse diode (8 x 8 x 36 cubes of 0.5 nm) at E_a = 14 V/nm from an
    empty gap: 60 coupled steps, the space charge building up."""
    E0, dt = 14.0, 0.02
    cfg = W.config_diode(E0, nx=8, nz=36, h=0.5, dt=dt)
    mesh = cfg.mesh()
    om = O.OracleMesh(mesh, cfg.emit_zmin)
    assert om.n_emit == 2 * 8 * 8
    A = mesh.Lx * mesh.Ly
    w_sp = D.steady_state(E0, mesh.z_top, cfg.phi_w)["J"] * A * dt / 40
    ost = O.OracleState(om, 100_000)
    ost.init_field(E0, tol=1e-12)
    gm = pic.Mesh(mesh, cfg.emit_zmin)
    assert gm.n_emit == om.n_emit
    gs = pic.State(gm, 100_000)
    gs.init_field(E0, tol=1e-12)
    kw = dict(dt=dt, E0=E0, w_sp=w_sp, phi_w=cfg.phi_w, seed=cfg.seed,
              tol=1e-12)
    for k in range(60):
        so = ost.step(step=k, **kw)
        sg = pic.State.decode_stats(gs.step(step0=k, resort_every=20,
                                            **kw))[0]
        for key in ("n_inj", "n_anode", "n_cathode", "n_after", "q_inj",
                    "q_anode", "q_cathode", "q_after", "status", "n_clamp"):
            assert so[key] == sg[key], (k, key, so[key], sg[key])
        for key in ("emit_current", "mean_face_E"):
            assert abs(sg[key] - so[key]) <= 1e-9 * abs(so[key])
    assert sg["n_after"] > 1000
    P, Q = gs.live(), ost.particles()
    a, b = np.argsort(P["id"]), np.argsort(Q["id"])
    assert (P["id"][a] == Q["id"][b]).all()
    assert (P["tet"][a] == Q["tet"][b]).all()
    pg = np.stack([P["x"][a], P["y"][a], P["z"][a]], 1)
    po = np.stack([Q["x"][b], Q["y"][b], Q["z"][b]], 1)
    assert _rel(pg, po) < 1e-9
    assert _rel(gs.phi.cpu().numpy(), ost.phi) < 1e-9
    assert int(gs.charge.sum().item()) == int(ost.c.sum())


def _run_diode(pic, E0, n_steps=1600, per_step=200, chunk=50, cfg=None):
    if cfg is None:
        cfg = W.config_diode(E0, n_steps=n_steps)
    mesh = cfg.mesh()
    A, d = mesh.Lx * mesh.Ly, mesh.z_top
    semi = D.steady_state(E0, d, cfg.phi_w)
    w_sp = semi["J"] * A * cfg.dt / per_step
    gm = pic.Mesh(mesh, cfg.emit_zmin)
    gs = pic.State(gm, 400_000)
    gs.init_field(E0, tol=cfg.tol)
    top = torch.from_numpy(np.isclose(mesh.xyz[:, 2], d)).cuda()
    kw = dict(dt=cfg.dt, E0=E0, w_sp=w_sp, phi_w=cfg.phi_w, seed=cfg.seed,
              tol=cfg.tol, resort_every=cfg.resort_every)
    q_a, Q, V, emit, n, nV = 0, 0.0, 0.0, 0.0, 0, 0
    for k0 in range(0, n_steps, chunk):
        rows = pic.State.decode_stats(gs.step(step0=k0, n_steps=chunk, **kw))
        for r in rows:
            assert r["status"] == 0
        if k0 >= n_steps // 2:
            for r in rows:
                q_a += r["q_anode"]
                Q += r["q_after"] / 2.0 ** 40 * w_sp
                emit += r["emit_current"]
                n += 1
            V += gs.phi[top].mean().item()
            nV += 1
    J = q_a / 2.0 ** 40 * w_sp / (n * cfg.dt) / A
    k = O.constants()
    eps0, qm = 1.0 / k["e_eps"], abs(k["qm"])
    Q /= n
    V /= nV
    Ec = E0 - Q / (eps0 * A)
    balance = 4.0 * J / eps0 * math.sqrt(V / (2.0 * qm)) / (E0 ** 2 - Ec ** 2)
    return dict(E0=E0, J=J, J_semi=semi["J"], J_fn=D.fn_density(E0, cfg.phi_w),
                J_cl=D.child_langmuir(E0, d), V=V, V_semi=semi["V"], Ec=Ec,
                Ec_semi=semi["E_c"], balance=balance, emit=emit / n / A,
                live=int(gs.n_slots.item()))


def test_diode_current_field_curve(pic):
    """Anode fields 5 .. 40 V/nm at A = 135.7 nm^2, d = 18.2 nm, 0.02 fs
    steps, 1600 steps each (the second half averaged): from emission-limited
    (J close to the FN current of the anode field) into the space-charge-
    limited regime (J above 0.8 of the Child-Langmuir current)."""
    out = []
    for E0 in (5.0, 8.0, 10.0, 12.0, 14.0, 16.0, 20.0, 25.0, 30.0, 40.0):
        r = _run_diode(pic, E0)
        out.append(r)
        print("diode E_a %5.1f  J %.4e  J/J_semi %.4f  J/J_FN(E_a) %.4f  "
              "J/J_CL %.4f  V %.2f (semi %.2f)  E_c %.3f (semi %.3f)  "
              "balance %.4f  emit/J %.4f  live %d" % (
                  E0, r["J"], r["J"] / r["J_semi"], r["J"] / r["J_fn"],
                  r["J"] / r["J_cl"], r["V"], r["V_semi"], r["Ec"],
                  r["Ec_semi"], r["balance"], r["emit"] / r["J"], r["live"]),
              flush=True)
    rel = np.array([r["J"] / r["J_semi"] - 1 for r in out])
    print("diode RMS relative deviation from the semianalytic curve: %.4f"
          % math.sqrt((rel ** 2).mean()), flush=True)
    for r in out:
        assert abs(r["balance"] - 1) < 0.03
        assert abs(r["V"] / r["V_semi"] - 1) < 0.03
        assert r["J"] < r["J_cl"]
        assert abs(r["emit"] / r["J"] - 1) < 0.03   # steady: emitted = collected
    assert abs(out[0]["J"] / out[0]["J_semi"] - 1) < 0.03
    assert np.abs(rel).max() < 0.12
    assert out[-1]["J"] < 0.3 * out[-1]["J_fn"]       # space charge limits
    assert out[-1]["J"] > 0.8 * out[-1]["J_cl"]       # close to Child-Langmuir
    assert all(b["J"] > a["J"] for a, b in zip(out, out[1:]))
    assert all(b["J"] / b["J_cl"] > a["J"] / a["J_cl"] for a, b in zip(out, out[1:]))


def test_diode_surface_field_convergence(pic):
    """The gap to the semianalytic current at E_a = 14 V/nm comes from the
    recovered cathode field (the gradient averaged over the first cell
    layer, where phi grows like z + z^(3/2)): it shrinks like sqrt(h) as
    the mesh is refined (h = 0.5, 0.25, 0.125 nm at a fixed 18.2 nm gap
    within half a cell), while the momentum balance holds throughout."""
    dev = []
    for nx, nz, h in ((8, 36, 0.5), (16, 73, 0.25), (32, 146, 0.125)):
        cfg = W.config_diode(14.0, nx=nx, nz=nz, h=h)
        r = _run_diode(pic, 14.0, cfg=cfg)
        dev.append(r["J"] / r["J_semi"] - 1)
        print("diode h %.3f  J/J_semi - 1 = %.4f  balance %.4f"
              % (h, dev[-1], r["balance"]), flush=True)
        assert abs(r["balance"] - 1) < 0.01
    assert dev[0] > dev[1] > dev[2] > 0
    for a, b in zip(dev, dev[1:]):
        assert 1.2 < a / b < 1.7     # sqrt(2) per halving
