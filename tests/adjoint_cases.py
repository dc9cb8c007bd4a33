"""Adjoint windows on the tiny tip, shared by the oracle and device tests.

The in-flight population comes from an oracle warm-up run whose emission is
scaled so that the space charge moves the field (coupled case); the window
then starts after the first superparticles have reached the anode."""
import numpy as np

from oracle import oracle as O
from oracle.adjoint import Window
from paper_1906_08125_amd import workloads as W


def tiny_window(T=4, live_charge=0.5, n_live=2000, warm=22, cap=40_000,
                tol=1e-13, empty=False):
    cfg = W.config_tiny()
    tip = cfg.mesh()
    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, cap)
    ost.init_field(cfg.E0, tol=tol)
    rate, _ = om.emission_rate(ost.E, cfg.phi_w)
    per_run = rate * cfg.dt * cfg.transit_steps
    j_scale = 0.0 if empty else live_charge / per_run
    w_sp = per_run * (live_charge / per_run) / n_live
    if not empty:
        for k in range(warm):
            ost.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, step=k,
                     seed=cfg.seed, j_scale=j_scale, tol=tol)
    P = ost.particles()
    init = dict(x=P["x"], y=P["y"], z=P["z"], vx=P["vx"], vy=P["vy"],
                vz=P["vz"], tet=P["tet"], birth=P["birth"], id=P["id"],
                omega=P["w"])
    win = Window(om, init, dt=cfg.dt, w_sp=w_sp, phi_w=cfg.phi_w,
                 seed=cfg.seed, j_scale=j_scale, step0=warm, T=T, cap=cap,
                 tol=tol)
    return cfg, tip, om, win


def central_fd(win, E0, s, counts, param, delta=1e-6):
    """Central differences of (J_Q, J_E) with the counts held; param is
    'E0' or a face index."""
    s = np.asarray(s, np.float64)
    if param == "E0":
        h = delta * E0
        p = win.forward(E0 + h, s, counts)
        m = win.forward(E0 - h, s, counts)
    else:
        h = delta * s[param]
        sp, sm = s.copy(), s.copy()
        sp[param] += h
        sm[param] -= h
        p = win.forward(E0, sp, counts)
        m = win.forward(E0, sm, counts)
    return (p[0] - m[0]) / (2 * h), (p[1] - m[1]) / (2 * h)
