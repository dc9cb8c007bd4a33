"""Benchmark of the electron PIC cycle on one MI355X.

Workload: the production-shaped tip (box 32 x 32 x 64 nm, 64 x 64 x 128
Kuhn grid, 3,100,504 tets, tip R = 3 nm, H = 30 nm, E0 = 0.5 V/nm, apex
faces emitting, w_sp set for ~1e6 live superparticles, dt = 0.5 fs,
PCG tolerance 1e-10).  An untimed fill runs from the empty gap until at
least 95 % of the ~1e6 target population is live (the steady state,
whatever W says), then W untimed warm-up steps, then K steps are timed
between device synchronizations.

Prints one JSON line.  Roofline byte model of the push: 112 B per live
superparticle and step in FP64 (read x, y, z, vx, vy, vz, w and the tet
id; write the six reals and the tet id), 64 B in mixed precision.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("PIC steps/s & pushes/s at 3M tets/1M e-; mixed vs FP64 speedup; "
          "adjoint/fwd")
HBM_PEAK_GBS = 8000.0
# the timed steps bracket the push with HIP events in every this many steps
PUSH_TIMING_EVERY = 5

# HBM traffic from rocprofv3 FETCH_SIZE and WRITE_SIZE counter runs, scaled
# by what the counters read for a plain 1 GiB device copy (fetch 1.9999,
# write 1.0000).  A figure is reported only while the sources it was taken
# on are unchanged and the run's load matches the one profiled.
# The dominant kernel (FP64 push) per launch at the production workload
# (profiles/pic_step_fp64_production_tip.md):
PUSH_TRAFFIC = dict(bytes=220.4e6, read=155.9e6, written=64.6e6, live=992_300,
                    sources=("paper_1906_08125_amd/csrc/particles.hip",
                             "paper_1906_08125_amd/csrc/common.h"),
                    sha256=("5770ae084b9f9585a4b0d54bd5d8e7f9e881e1d3cf0fe7c783617cdb6aa6d220",
                            "df664d921b2048d0e38d5de9ccce0edb99bc52cb2a034c6b94b3b69f07cb3843"))

# One step of the 32-instance batch (every dispatch between consecutive
# batched particle launches, averaged over the timed steps;
# profiles/pic_batch_step_32_instances.md):
BATCH_TRAFFIC = dict(bytes=3345.7e6, read=2717.9e6, written=627.8e6,
                     live=3_371_102,
                     sources=("paper_1906_08125_amd/csrc/particles.hip",
                              "paper_1906_08125_amd/csrc/solver.hip",
                              "paper_1906_08125_amd/csrc/amg.hip",
                              "paper_1906_08125_amd/csrc/api.hip",
                              "paper_1906_08125_amd/csrc/common.h"),
                     sha256=("5770ae084b9f9585a4b0d54bd5d8e7f9e881e1d3cf0fe7c783617cdb6aa6d220",
                             "48dc7dedd15d958bcf9d263391b89c760b31dc43d7838b22276f98ba3273aebf",
                             "b7134060afc401da45819d5e18d224beee6fb57e6660ef3331fb9b6bb80d9af9",
                             "e86b16e48b77a312e297ff1664407f4a6d70ef7381df77a5ce39d568443292e9",
                             "df664d921b2048d0e38d5de9ccce0edb99bc52cb2a034c6b94b3b69f07cb3843"))


def measured_traffic(rec, live):
    """The counters' bytes of record `rec`, when they were taken on the
    sources as they are now and at the population the figure it goes with
    is measured at (within 5 %); else None."""
    import hashlib
    for path, digest in zip(rec["sources"], rec["sha256"]):
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    if abs(live / rec["live"] - 1) > 0.05:
        return None
    return rec["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solve_bytes(info, rows, first_full=True):
    """Algorithmic HBM bytes of the solves of a run of consecutive steps of
    one pic_step call (rows: their stats).  The first solve of a call starts
    with the fused residual + field pass over phi (rows: node map, own phi,
    charge, Neumann load, x, r, u, D^-1, E; entries: node column, K, R (3));
    every later one with the incremental residual pass r = (b - b_prev) +
    r_prev, which needs no product with K because phi and the field have
    not changed since the previous solve ended: node map, charge, Neumann
    load, b_prev and r read and written, x written, phi, D^-1, u written
    (84 B per free row).  Where the step before needed no iteration and a
    step follows (the lean pass), it leaves x and u to a launch made only
    if the test asks for iterations (node map, phi, r, D^-1 read, x and u
    written: 44 B per free row) and clears the charges it reads (60 B per
    free row, 12 B per Dirichlet node).  Per CG iteration: the update (7
    vector reads, 5 writes) and the K u product (column + value per entry,
    u and w per row); a solve that iterated ends with phi = x (20 B per
    free row) and a fused re-check pass."""
    n, nnz = info["n_free"], info["nnz"]
    N, nf = info["n_nodes"], info["nnz_field"]
    fused = 100 * n + 36 * nnz + 28 * (nf - nnz) + 40 * (N - n)
    inc = 84 * n
    lean = 60 * n + 12 * (N - n)
    prep = 44 * n
    it = 96 * n + 12 * nnz + 16 * n
    total = 0
    for k, r in enumerate(rows):
        if k == 0 and first_full:
            total += fused
        elif k > 0 and k + 1 < len(rows) and rows[k - 1]["cg_iters"] == 0:
            total += lean + (prep if r["cg_iters"] > 0 else 0)
        else:
            total += inc
        if r["cg_iters"] > 0:
            total += r["cg_iters"] * it + 20 * n + fused
    return total


def push_bytes(n_live, real_bytes=8):
    """Particle stream of the push kernel: read x,y,z,vx,vy,vz (6 reals),
    tet (4), w (8); write x,y,z,vx,vy,vz (6 reals), tet (4)."""
    return (12 * real_bytes + 16) * n_live


def run_leg(gm, cfg, w_sp, precision, args, fill_steps=None):
    """Warm-up then K timed steps of one run at the given precision."""
    import torch

    from paper_1906_08125_amd import pic

    gs = pic.State(gm, int(args.capacity), precision=precision,
                   inner_tol=args.inner_tol)
    gs.init_field(cfg.E0, tol=cfg.tol)   # captures this precision's graphs
    gs.phi.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st0 = gs.init_field(cfg.E0, tol=cfg.tol)
    torch.cuda.synchronize()
    cold = dict(pic.Mesh.solve_stats(st0), ms=round(1e3 * (time.perf_counter() - t0), 3))
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w,
              seed=cfg.seed, tol=cfg.tol, resort_every=args.resort)
    step, fill = fill_to_steady_state(gm, gs, kw, cfg.n_target, args,
                                      fill_steps)
    log(f"fill ({precision}): {fill['steps']} steps to "
        f"{fill['live']} live superparticles")
    if args.warmup:
        wstats = gs.step(step0=step, n_steps=args.warmup, **kw)
        torch.cuda.synchronize()
        log(f"after warmup ({precision}): "
            f"{pic.State.decode_stats(wstats)[-1]}")
        step += args.warmup
    stats = torch.zeros(args.steps * pic.STEP_STATS_BYTES // 8,
                        dtype=torch.int64, device="cuda")
    # timed region: K steps, bracketed by synchronizations; HIP events
    # bracket the push kernel (the dominant one) only, and only in every
    # fifth step: every event is a packet of its own in the stream, and the
    # GPU idles some 5 us at each (two per timed push)
    gm.profile(True, classes=("push",), every=PUSH_TIMING_EVERY)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    gs.step(step0=step, n_steps=args.steps, stats=stats, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    kt_timed = gm.profile_read()
    gm.profile(False)
    rows = pic.State.decode_stats(stats)
    step += args.steps
    # state after the timed steps (the two precisions compared there)
    snap = dict(phi=gs.phi.cpu().numpy().copy(), live=gs.live(),
                mean_face_E=rows[-1]["mean_face_E"])
    # per-class breakdown: a further, untimed stretch of steps with every
    # kernel class bracketed
    kt = {}
    if args.breakdown_steps > 0:
        gm.profile(True)
        bstats = gs.step(step0=step, n_steps=args.breakdown_steps, **kw)
        torch.cuda.synchronize()
        kt = gm.profile_read()
        gm.profile(False)
        rows_b = pic.State.decode_stats(bstats)
    else:
        rows_b = []
    # binary collisions (App. F) after every re-sort: a further untimed
    # stretch with the collision launches bracketed
    kt_coll = {}
    if args.collide_steps > 0 and precision == pic.PIC_FP64:
        # one untimed stretch first: the first launch of a kernel also loads
        # its code object
        gs.step(step0=step, n_steps=args.resort, collide=1, **kw)
        step += args.resort
        torch.cuda.synchronize()
        gm.profile(True, classes=("collide",))
        cstats = gs.step(step0=step, n_steps=args.collide_steps, collide=1,
                         **kw)
        torch.cuda.synchronize()
        kt_coll = gm.profile_read()
        gm.profile(False)
        rows_b = rows_b + pic.State.decode_stats(cstats)
        step += args.collide_steps
    for r in rows + rows_b:
        if r["status"] != 0:
            raise RuntimeError(f"step status {r['status']}: {r}")
    return dict(elapsed=elapsed, kt=kt, kt_timed=kt_timed, rows=rows,
                rows_b=rows_b, state=gs, cold=cold, kt_coll=kt_coll, snap=snap,
                fill=fill)


def fill_to_steady_state(gm, gs, kw, n_target, args, steps=None):
    """Untimed steps from the empty gap until at least args.fill_frac of the
    target population is live, one step per call with the push kernel timed
    by HIP events: the pairs (superparticles pushed, push time) of the fill
    separate the push's fixed cost per launch from its cost per particle
    (least-squares line).  steps: run exactly this many instead (the
    mixed-precision leg repeats the FP64 leg's fill, so that both are
    compared after the same steps).  Returns the next step index and the
    fill record."""
    import numpy as np
    import torch

    from paper_1906_08125_amd import pic

    pts = []
    step, live = 0, 0
    while (live < args.fill_frac * n_target if steps is None
           else step < steps):
        if step >= args.max_fill:
            raise RuntimeError(f"fill: {live} live after {step} steps, "
                               f"target {args.fill_frac} x {n_target}")
        gm.profile(True, classes=("push",))
        st = pic.State.decode_stats(gs.step(step0=step, n_steps=1, **kw))[0]
        kt = gm.profile_read()
        gm.profile(False)
        if st["status"] != 0:
            raise RuntimeError(f"fill step status {st['status']}: {st}")
        pts.append((st["n_before"] + st["n_inj"], 1e3 * kt["push"]["ms"]))
        live = st["n_after"]
        step += 1
    torch.cuda.synchronize()
    n = np.array([p[0] for p in pts], float)
    us = np.array([p[1] for p in pts])
    # the first steps also load code objects and page the mesh in
    use = slice(3, None) if len(pts) > 8 else slice(0, None)
    b, a = np.polyfit(n[use], us[use], 1)
    return step, dict(steps=step, live=int(live),
                      push_fixed_us=round(float(a), 2),
                      push_us_per_million=round(float(b) * 1e6, 2),
                      samples=[(int(x), round(float(y), 2))
                               for x, y in zip(n[::5], us[::5])])


def precision_drift(a, b):
    """Mixed against FP64 after the same steps: rel-L2 of phi, relative
    error of the mean apex-face field, and over the superparticles present
    in both (matched by id) rel-L2 and max abs of the positions."""
    import numpy as np
    phi = float(np.linalg.norm(b["phi"] - a["phi"]) / np.linalg.norm(a["phi"]))
    Pa, Pb = a["live"], b["live"]
    common, ia, ib = np.intersect1d(Pa["id"], Pb["id"], return_indices=True)
    pa = np.stack([Pa[c][ia] for c in ("x", "y", "z")], 1)
    pb = np.stack([Pb[c][ib] for c in ("x", "y", "z")], 1)
    d = pb - pa
    return dict(phi_rel_l2=phi,
                mean_apex_field_rel=abs(b["mean_face_E"] / a["mean_face_E"] - 1),
                positions_rel_l2=float(np.linalg.norm(d) / np.linalg.norm(pa)),
                positions_max_abs_nm=float(np.abs(d).max()),
                matched=int(common.size), fp64_live=int(Pa["id"].size),
                mixed_live=int(Pb["id"].size))


def run_gpu(args):
    import torch

    from paper_1906_08125_amd import pic, workloads as W

    cfg = W.config_production()
    tip = cfg.mesh()
    t0 = time.time()
    gm = pic.Mesh(tip, cfg.emit_zmin)
    log(f"mesh_create {time.time() - t0:.1f}s {gm.info}")
    # cold Laplace solve: CG throughput on the production matrix (the
    # first solve also captures the iteration graphs; the second is timed)
    phi = torch.zeros(gm.n_nodes, dtype=torch.float64, device="cuda")
    E = torch.zeros(4 * gm.n_nodes, dtype=torch.float64, device="cuda")
    gm.poisson_solve(None, 0.0, cfg.E0, phi, E, tol=cfg.tol)
    phi.zero_()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st = gm.poisson_solve(None, 0.0, cfg.E0, phi, E, tol=cfg.tol)
    e1.record()
    torch.cuda.synchronize()
    cold = gm.solve_stats(st)
    cold_ms = e0.elapsed_time(e1)
    log(f"cold solve {cold} {cold_ms:.2f} ms")
    # the same cold solve preconditioned by AMG: the first call builds the
    # hierarchy (host setup, timed apart), the second is timed
    phi.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gm.poisson_solve(None, 0.0, cfg.E0, phi, E, tol=cfg.tol,
                     precond=pic.PIC_PRECOND_AMG)
    torch.cuda.synchronize()
    amg_setup_ms = 1e3 * (time.perf_counter() - t0)
    phi.zero_()
    torch.cuda.synchronize()
    e0.record()
    st = gm.poisson_solve(None, 0.0, cfg.E0, phi, E, tol=cfg.tol,
                          precond=pic.PIC_PRECOND_AMG)
    e1.record()
    torch.cuda.synchronize()
    cold_amg = gm.solve_stats(st)
    cold_amg_ms = e0.elapsed_time(e1)
    log(f"cold solve (AMG) {cold_amg} {cold_amg_ms:.2f} ms, "
        f"first call with setup {amg_setup_ms:.1f} ms")
    rate, faceF = gm.emission_rate(E, cfg.phi_w)
    rate = rate.item()
    w_sp = rate * cfg.dt * cfg.transit_steps / cfg.n_target
    log(f"emission {rate:.3e} e/fs -> w_sp {w_sp:.3e}")
    del phi, E

    leg = run_leg(gm, cfg, w_sp, pic.PIC_FP64, args)
    elapsed, kt, rows = leg["elapsed"], leg["kt"], leg["rows"]
    kt_timed, rows_b = leg["kt_timed"], leg["rows_b"]
    snap64 = leg["snap"]
    fill64 = leg["fill"]
    collisions = None
    if "collide" in leg["kt_coll"]:
        c = leg["kt_coll"]["collide"]
        us = 1e3 * c["ms"] / c["launches"]
        collisions = dict(calls=c["launches"], us_per_call=round(us, 2),
                          every_steps=args.resort,
                          us_per_step_amortised=round(us / args.resort, 2))
    del leg
    pushes = sum(r["n_before"] + r["n_inj"] for r in rows)
    live_mean = sum(r["n_before"] for r in rows) / len(rows)
    ms_step = 1e3 * elapsed / args.steps
    # per-kernel times of the breakdown stretch; the push also from the
    # timed region (the roofline figure)
    kernels = {}
    for name, v in kt.items():
        kernels[name] = dict(ms_total=round(v["ms"], 4), launches=v["launches"],
                             us_per_launch=round(1e3 * v["ms"] / v["launches"], 2))
    push_us = kt_timed["push"]["ms"] * 1e3 / kt_timed["push"]["launches"]
    pb = push_bytes(live_mean)
    kernels["push_timed"] = dict(
        ms_total=round(kt_timed["push"]["ms"], 4),
        launches=kt_timed["push"]["launches"], us_per_launch=round(push_us, 2),
        algo_bytes=pb, GBps=round(pb / push_us / 1e3, 1))
    dom, dom_bytes, dom_us = "push", pb, push_us
    if "solve" in kt and rows_b:
        solve_us = kt["solve"]["ms"] * 1e3 / kt["solve"]["launches"]
        nb = args.breakdown_steps
        live_b = sum(r["n_before"] for r in rows_b[:nb]) / nb
        sb = solve_bytes(gm.info, rows_b[:nb]) / nb
        kernels["solve"]["algo_bytes"] = sb
        kernels["solve"]["GBps"] = round(sb / solve_us / 1e3, 1)
        pbb = push_bytes(live_b)
        kernels["push"]["algo_bytes"] = pbb
        kernels["push"]["GBps"] = round(pbb / (kt["push"]["ms"] * 1e3 / kt["push"]["launches"]) / 1e3, 1)
        if kt["solve"]["ms"] > kt["push"]["ms"]:
            dom, dom_bytes, dom_us = "solve", sb, solve_us
    achieved = dom_bytes / dom_us / 1e3  # GB/s
    for name, v in kernels.items():
        if v.get("GBps", 0.0) > HBM_PEAK_GBS:
            # only a working set held in the 256 MB Infinity Cache could
            # do this; the byte model of that kernel is to be checked
            log(f"warning: {name} at {v['GBps']} GB/s of algorithmic bytes "
                f"exceeds the HBM peak")
            v["above_hbm_peak"] = True

    mixed = None
    if not args.no_mixed:
        torch.cuda.empty_cache()
        ml = run_leg(gm, cfg, w_sp, pic.PIC_MIXED, args,
                     fill_steps=fill64["steps"])
        mr = ml["rows"]
        m_live = sum(r["n_before"] for r in mr) / len(mr)
        mk = ml["kt"]
        mt = ml["kt_timed"]["push"]
        m_push_us = mt["ms"] * 1e3 / mt["launches"]
        mixed = dict(
            value=round(args.steps / ml["elapsed"], 3), unit="steps/s",
            ms_per_step=round(1e3 * ml["elapsed"] / args.steps, 4),
            speedup_vs_fp64=round(elapsed / ml["elapsed"], 4),
            pushes_per_s=round(sum(r["n_before"] + r["n_inj"] for r in mr)
                               / ml["elapsed"], 1),
            live_particles_mean=round(m_live),
            cg_iters_per_step=sum(r["cg_iters"] for r in mr) / len(mr),
            inner_tol=args.inner_tol,
            cold_solve=ml["cold"],
            fill=ml["fill"],
            kernels={n: dict(ms_total=round(v["ms"], 4),
                             launches=v["launches"],
                             us_per_launch=round(1e3 * v["ms"] / v["launches"], 2))
                     for n, v in mk.items()},
            push_GBps=round(push_bytes(m_live, 4) / m_push_us / 1e3, 1),
            drift_vs_fp64=precision_drift(snap64, ml["snap"]))
        del ml
    batch = None
    if args.batch_instances > 0:
        torch.cuda.empty_cache()
        batch = run_batch_leg(args)
    stress = None
    if args.stress_steps > 0:
        torch.cuda.empty_cache()
        stress = [run_stress_leg(gm, cfg, rate, faceF, args, pc, pr)
                  for pc, pr in ((pic.PIC_PRECOND_JACOBI, pic.PIC_FP64),
                                 (pic.PIC_PRECOND_JACOBI, pic.PIC_MIXED),
                                 (pic.PIC_PRECOND_AMG, pic.PIC_FP64),
                                 (pic.PIC_PRECOND_AMG, pic.PIC_MIXED))]
        log(f"stress leg {stress}")
    charge = None
    if args.charge_calls > 0:
        torch.cuda.empty_cache()
        charge = run_charge_leg(tip, args)
    metal = None
    if args.metal_calls > 0:
        torch.cuda.empty_cache()
        metal = run_metal_leg(args)
    adjoint = None
    if not args.no_adjoint:
        torch.cuda.empty_cache()
        adjoint = run_adjoint_leg(gm, cfg, rate, args)
    out = dict(
        metric=METRIC, value=round(args.steps / elapsed, 3), unit="steps/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms_step, 4), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=cfg.name, tets=gm.n_tets, nodes=gm.n_nodes,
                    free_nodes=gm.n_free, nnz=gm.info["nnz"],
                    live_particles_mean=round(live_mean), precision="fp64",
                    w_sp=w_sp, dt_fs=cfg.dt, tol=cfg.tol,
                    resort_every=args.resort),
        pushes_per_s=round(pushes / elapsed, 1),
        cg_iters_per_step=sum(r["cg_iters"] for r in rows) / len(rows),
        fill=fill64,
        cold_solve=dict(iters=cold["iters"], ms=round(cold_ms, 3),
                        iters_per_s=round(cold["iters"] / cold_ms * 1e3, 1),
                        relres=cold["relres"], precond="jacobi"),
        cold_solve_amg=dict(iters=cold_amg["iters"], ms=round(cold_amg_ms, 3),
                            relres=cold_amg["relres"],
                            first_call_with_setup_ms=round(amg_setup_ms, 1),
                            speedup_vs_jacobi=round(cold_ms / cold_amg_ms, 2)),
        kernels=kernels,
        mixed=mixed,
        adjoint=adjoint,
        batch=batch,
        collisions=collisions,
        surface_charge=charge,
        metal=metal,
        stress=stress,
        roofline=dict(kernel=dom, bound="hbm", achieved=round(achieved, 1),
                      peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4),
                      traffic=(measured_traffic(PUSH_TRAFFIC, live_mean) if dom == "push"
                               else None),
                      live_particles=round(live_mean),
                      limiter=("dependent gathers (tet record, nodal field, "
                               "walk) at the occupancy the registers allow"
                               if dom == "push" else "HBM")),
    )
    gm.close()
    return out, dict(cfg=cfg, tip=tip, w_sp=w_sp)


def run_stress_leg(gm, cfg, rate, faceF, args, precond, precision=0):
    """The coupled ("stress") variant of the production workload: the FN
    current scaled by M_J so that the charge in flight is 10 % of the
    surface charge eps0 sum_f |E_f| A_f of the emitting faces (space charge
    visible in phi, a CG solve every step); the same 1e6 superparticles."""
    import torch

    from paper_1906_08125_amd import pic

    eps0 = 8.8541878128e-12 / 1.602176634e-19 * 1e-9   # e V^-1 nm^-1
    area = gm.emit_faces()["area"]
    q_target = 0.1 * eps0 * float((faceF.cpu().numpy() * area).sum())
    per_run = rate * cfg.dt * cfg.transit_steps          # electrons in flight
    m_j = q_target / per_run
    w_sp = per_run * m_j / cfg.n_target
    gs = pic.State(gm, int(args.capacity), precond=precond,
                   precision=precision, inner_tol=args.inner_tol)
    gs.init_field(cfg.E0, tol=cfg.tol)
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, seed=cfg.seed,
              tol=cfg.tol, resort_every=args.resort, j_scale=m_j)
    gs.step(step0=0, n_steps=args.stress_warmup, **kw)
    torch.cuda.synchronize()
    stats = torch.zeros(args.stress_steps * pic.STEP_STATS_BYTES // 8,
                        dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    gs.step(step0=args.stress_warmup, n_steps=args.stress_steps, stats=stats,
            **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rows = pic.State.decode_stats(stats)
    for r in rows:
        if r["status"] != 0:
            raise RuntimeError(f"stress step status {r['status']}: {r}")
    live_q = rows[-1]["q_after"] / 2.0 ** 40 * w_sp
    out = dict(precond="amg" if precond == pic.PIC_PRECOND_AMG else "jacobi",
               precision="mixed" if precision == pic.PIC_MIXED else "fp64",
               M_J=m_j, w_sp=w_sp, value=round(args.stress_steps / el, 2),
               unit="steps/s", ms_per_step=round(1e3 * el / args.stress_steps, 4),
               cg_iters_per_step=sum(r["cg_iters"] for r in rows) / len(rows),
               live_particles=rows[-1]["n_after"], live_charge_e=live_q,
               target_charge_e=q_target,
               mean_face_E=rows[-1]["mean_face_E"])
    del gs
    return out


def run_charge_leg(tip, args):
    """Surface charge of every metal face of the production tip (a second
    mesh handle with all metal faces listed) distributed to seeded surface
    atoms: time per call with events on the stream."""
    import torch

    from paper_1906_08125_amd import pic, workloads as W

    t0 = time.time()
    gmc = pic.Mesh(tip, -1.0)
    gs = pic.State(gmc, 16)
    gs.init_field(0.5, tol=1e-10)
    atoms = torch.from_numpy(W.surface_atoms(tip, density=4.0)).cuda()
    log(f"surface-charge mesh {time.time() - t0:.1f}s: {gmc.n_emit} faces, "
        f"{atoms.shape[0]} atoms")
    gmc.surface_charge(atoms, E=gs.E)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.charge_calls):
        Q, q = gmc.surface_charge(atoms, E=gs.E)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.charge_calls
    out = dict(faces=gmc.n_emit, atoms=int(atoms.shape[0]),
               us_per_call=round(1e3 * ms, 1),
               face_atom_pairs_per_s=round(3 * gmc.n_emit * atoms.shape[0]
                                           / (ms * 1e-3), 1),
               total_charge_e=round(float(Q.sum().item()), 6),
               conservation=float(q.sum().item() / Q.sum().item()))
    del gs
    gmc.close()
    return out


def run_metal_leg(args):
    """Metal-side solves (Sec. II D) on the metal under the production tip:
    the continuity solve with Joule heating from a synthetic apex-centred
    emission current, then implicit-Euler heat steps with those sources.
    Times per call are host wall times (each call waits for its solve)."""
    import torch

    import numpy as np

    from paper_1906_08125_amd import pic, workloads as W

    t0 = time.time()
    m = W.metal_production()
    gm = pic.Metal(m)
    torch.cuda.synchronize()
    setup = time.time() - t0
    flux, PN = (torch.from_numpy(a).cuda() for a in W.metal_sources(m))
    sigma = torch.ones(m.n_tets, dtype=torch.float64, device="cuda")
    gm.continuity_solve(sigma, flux, tol=1e-12)          # code-object load
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.metal_calls):
        phi, pj, st = gm.continuity_solve(sigma, flux, tol=1e-12)
    torch.cuda.synchronize()
    cont_s = (time.perf_counter() - t1) / args.metal_calls
    T = torch.full((m.n_nodes,), 300.0, dtype=torch.float64, device="cuda")
    t2 = time.perf_counter()
    iters = []
    for _ in range(args.metal_calls):
        sh = gm.heat_step(T, sigma, pj, PN, Cv=3.45e-3, L=2.0e-8, dt=40.0,
                          theta=1.0, T_amb=300.0, tol=1e-12)
        iters.append(sh["iters"])
    torch.cuda.synchronize()
    heat_s = (time.perf_counter() - t2) / args.metal_calls
    # algorithmic bytes of one CG iteration: the CSR product (8-byte values
    # and 4-byte columns per entry, the row pointers, z, r and w once) and
    # the step's vector updates (7 vectors read, 5 written)
    e = np.sort(m.tet[:, [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]]
                .reshape(-1, 2), axis=1)
    nnz = 2 * int(np.unique(e[:, 0].astype(np.int64) * m.n_nodes + e[:, 1]).size) \
        + m.n_nodes
    it_bytes = 12 * nnz + (4 + 32 + 96) * m.n_nodes
    out = dict(nodes=m.n_nodes, tets=m.n_tets, interface_faces=m.n_faces,
               nnz=nnz, cg_bytes_per_iter=it_bytes,
               cg_GBps_wall=round(it_bytes * st["iters"] / cont_s / 1e9, 1),
               setup_s=round(setup, 2),
               continuity_ms=round(1e3 * cont_s, 3),
               continuity_iters=int(st["iters"]),
               heat_step_ms=round(1e3 * heat_s, 3),
               heat_iters=iters,
               us_per_cg_iter=round(1e6 * cont_s / max(st["iters"], 1), 2),
               T_max=round(float(T.max().item()), 4))
    log(f"metal leg {out}")
    gm.close()
    return out


def run_adjoint_leg(gm, cfg, rate, args):
    """Adjoint window on the production mesh: mixed precision (FP32
    particles and field, FP64-refined forward solves, FP64 transposed
    solves preconditioned as --adjoint-precond says), about 2e5 live
    superparticles after 100 warm-up steps, a window of 20 steps with
    per-step checkpoints; the backward recomputes every step from its
    checkpoint.  Reports forward and backward wall time on the device (the
    second of two passes: the first also builds the AMG hierarchy)."""
    import torch

    from paper_1906_08125_amd import pic

    n_target = 2e5
    w_sp = rate * cfg.dt * cfg.transit_steps / n_target
    gs = pic.State(gm, int(6e5), precision=pic.PIC_MIXED,
                   inner_tol=args.inner_tol)
    gs.init_field(cfg.E0, tol=cfg.tol)
    warm = 100
    gs.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, step0=0,
            seed=cfg.seed, tol=cfg.tol, resort_every=10, n_steps=warm)
    torch.cuda.synchronize()
    live = int((gs.tet[: int(gs.n_slots.item())] >= 0).sum().item())
    T = args.adjoint_steps
    precond = pic.PIC_PRECOND_AMG if args.adjoint_precond == "amg" \
        else pic.PIC_PRECOND_JACOBI
    win = pic.Window(gm, gs, T=T, step0=warm, dt=cfg.dt, w_sp=w_sp,
                     phi_w=cfg.phi_w, seed=cfg.seed, tol=cfg.tol,
                     adjoint_precond=precond)
    s = torch.ones(gm.n_emit, dtype=torch.float64, device="cuda")
    times = []
    for rep in range(2):  # the first pass warms the allocator
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        JQ, JE = win.forward(cfg.E0, s)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dE0, ds = win.backward(cfg.E0, s)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = times[-1]
    recs = [pic.Mesh.solve_stats(win.adjoint_solve_stats[6 * j: 6 * j + 6])
            for j in range(T + 1)]
    return dict(window_steps=T, live_particles=live, precision="mixed",
                adjoint_solves="fp64", adjoint_precond=args.adjoint_precond,
                adjoint_cg_iters=[r["iters"] for r in recs],
                fwd_ms=round(1e3 * fwd, 3), bwd_ms=round(1e3 * bwd, 3),
                adjoint_over_fwd=round(bwd / fwd, 4),
                J_E=float(JE), J_Q=float(JQ), dJ_dE0=float(dE0),
                dJ_ds_norm=float(ds.norm()),
                note="backward includes the recompute of every step")


def run_batch_leg(args):
    """Uneven tip instances (grid n x n x 2n, n in 32..64, tip and field
    drawn per instance, 1e4..1e6 superparticles each) advanced together by
    pic_batch_step in mixed precision with the autotuned schedule, against
    the plain FP64 form: the same instances stepped one after another by
    pic_step.  Both from the empty gap: W warm-up steps, then K timed."""
    import torch

    from paper_1906_08125_amd import pic, workloads as W

    cfgs = W.batch_configs(args.batch_instances, seed=4)
    t0 = time.time()
    meshes, kws = [], []
    for c in cfgs:
        gm = pic.Mesh(c.mesh(), c.emit_zmin)
        phi = torch.zeros(gm.n_nodes, dtype=torch.float64, device="cuda")
        E = torch.zeros(4 * gm.n_nodes, dtype=torch.float64, device="cuda")
        gm.poisson_solve(None, 0.0, c.E0, phi, E, tol=c.tol)
        rate, _ = gm.emission_rate(E, c.phi_w)
        w_sp = rate.item() * c.dt * c.transit_steps / c.n_target
        meshes.append(gm)
        kws.append(dict(dt=c.dt, E0=c.E0, w_sp=w_sp, phi_w=c.phi_w, seed=c.seed,
                        instance=len(kws), tol=c.tol, resort_every=10))
        del phi, E
    log(f"batch: {len(cfgs)} instances, "
        f"{sum(m.n_tets for m in meshes) / 1e6:.1f}M tets, "
        f"setup {time.time() - t0:.1f}s")
    warm, K = args.batch_warmup, args.batch_steps

    def states(precision, precond=pic.PIC_PRECOND_JACOBI):
        out = []
        for c, m, kw in zip(cfgs, meshes, kws):
            st = pic.State(m, int(2.5 * c.n_target) + 50_000, precision=precision,
                           precond=precond)
            st.init_field(c.E0, tol=c.tol)
            out.append(st)
        return out

    # batched, mixed precision (the FP32 V-cycle preconditioning the FP64 CG
    # of every instance), autotuned
    sts = states(pic.PIC_MIXED, pic.PIC_PRECOND_AMG)
    batch = pic.Batch(meshes, sts, kws)
    batch.step(0, warm)
    best = batch.autotune(warm)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    stats = batch.step(warm, K)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - w0
    rows = pic.Batch.decode(stats, len(cfgs))
    for r in rows:
        for x in r:
            if x["status"] != 0:
                raise RuntimeError(f"batch step status {x['status']}")
    pushes = sum(x["n_before"] + x["n_inj"] for r in rows for x in r)
    # algorithmic bytes of the timed batch steps: the particle streams (64 B
    # per superparticle in mixed precision) and, per instance, the solver
    # passes that ran (the fused residual + field pass of the call's first
    # step, the incremental residual pass after it, a re-check pass after
    # iterations); the V-cycle iterations themselves (a few per step over
    # all instances) are not counted, so the figure is a lower bound
    algo = 0.0
    for i, m in enumerate(meshes):
        ri = [r[i] for r in rows]
        algo += sum(push_bytes(x["n_before"] + x["n_inj"], 4) for x in ri)
        inf = m.info
        n, nnz, N, nf = inf["n_free"], inf["nnz"], inf["n_nodes"], inf["nnz_field"]
        fused = 100 * n + 36 * nnz + 28 * (nf - nnz) + 40 * (N - n)
        algo += fused + 84 * n * (len(ri) - 1)
        algo += sum(20 * n + fused for x in ri if x["cg_iters"] > 0)
    batch_gbps = algo / t_batch / 1e9
    csr_bytes = sum(12 * m.info["nnz"] + 36 * (m.info["nnz_field"]) for m in meshes)
    live_b = sum(x["n_after"] for x in rows[-1])
    batch.close()
    del sts
    torch.cuda.empty_cache()
    # plain FP64, one instance after another: with the default (Jacobi)
    # preconditioner, and with the FP64 AMG one
    def sequential(precond):
        sts = states(pic.PIC_FP64, precond)
        t = 0.0
        for st, kw in zip(sts, kws):
            st.step(step0=0, n_steps=warm, **kw)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            st.step(step0=warm, n_steps=K, **kw)
            torch.cuda.synchronize()
            t += time.perf_counter() - w0
        del sts
        torch.cuda.empty_cache()
        return t
    t_seq = sequential(pic.PIC_PRECOND_JACOBI)
    t_seq_amg = sequential(pic.PIC_PRECOND_AMG)
    for m in meshes:
        m.close()
    n = len(cfgs)
    return dict(instances=n, tets=int(sum(m.n_tets for m in meshes)),
                live_particles=int(live_b),
                warmup=warm, steps=K, precision="mixed",
                instance_steps_per_s=round(n * K / t_batch, 1),
                pushes_per_s=round(pushes / t_batch, 1),
                ms_per_batch_step=round(1e3 * t_batch / K, 4),
                fp64_sequential_ms_per_step=round(1e3 * t_seq / K, 4),
                speedup_vs_fp64_sequential=round(t_seq / t_batch, 4),
                fp64_amg_sequential_ms_per_step=round(1e3 * t_seq_amg / K, 4),
                speedup_vs_fp64_amg_sequential=round(t_seq_amg / t_batch, 4),
                precond="amg (FP32 V-cycle in the FP64 CG)",
                roofline=dict(bound="hbm", achieved=round(batch_gbps, 1),
                              peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(batch_gbps / HBM_PEAK_GBS, 4),
                              algo_bytes_per_step=round(algo / K),
                              traffic=measured_traffic(BATCH_TRAFFIC, live_b),
                              note="particle streams and solver passes over "
                                   "the wall time of the batch steps; V-cycle "
                                   "iterations not counted (the traffic "
                                   "figure counts them)"),
                operators_bytes=csr_bytes,
                mall_resident=bool(csr_bytes < 256e6),
                schedule=dict(push_tile=best[0], cg_rows=best[1]),
                autotune=[dict(push_tile=a, cg_rows=b, ms=round(c, 4))
                          for a, b, c in batch.tuning])


def cpu_baseline(cfg, tip, n_particles, n_steps):
    """The FP64 oracle on the host: the same mesh, a seeded synthetic
    population of superparticles in the gap above the apex, n_steps steps.
    The PIC steps run in the oracle's -fopenmp timing build on every thread
    OpenMP gives it (its parallel loops -- kick, drift and location,
    deposition, SpMV -- give the plain build's results bit for bit); the
    collision pass, the surface charge and the metal solves are serial."""
    import numpy as np

    from oracle import oracle as O
    O.use_openmp()

    om = O.OracleMesh(tip, cfg.emit_zmin)
    ost = O.OracleState(om, n_particles + 50 * 20000)
    ost.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = om.emission_rate(ost.E, cfg.phi_w)
    w_sp = rate * cfg.dt * cfg.transit_steps / cfg.n_target
    g = np.random.Generator(np.random.Philox(key=[cfg.seed, 77]))
    cx, cy = tip.Lx / 2, tip.Ly / 2
    r = 6.0 * np.sqrt(g.random(n_particles))
    a = 2 * np.pi * g.random(n_particles)
    p = np.stack([cx + r * np.cos(a), cy + r * np.sin(a),
                  cfg.tip_H + (tip.z_top - cfg.tip_H - 0.5) * g.random(n_particles)], 1)
    v = np.zeros_like(p)
    v[:, 2] = 0.2 + 1.5 * g.random(n_particles)
    v[:, :2] = 0.05 * (g.random((n_particles, 2)) - 0.5)
    tet, where = om.locate(p)
    keep = where == 0
    ost.add(p[keep], v[keep], tet[keep])
    n0 = ost.n
    t0 = time.perf_counter()
    for k in range(n_steps):
        ost.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w, step=k,
                 seed=cfg.seed, tol=cfg.tol)
    dt = time.perf_counter() - t0
    # the oracle's binary collisions on the same population (App. F)
    t1 = time.perf_counter()
    ost.collide(dt_coll=10 * cfg.dt, w_sp=w_sp, seed=cfg.seed, step=n_steps)
    coll_s = time.perf_counter() - t1
    # and its surface charge of every metal face to the seeded atoms
    from paper_1906_08125_amd import workloads as W
    omc = O.OracleMesh(tip, -1.0)
    sc = O.OracleState(omc, 4)
    sc.init_field(cfg.E0, tol=cfg.tol)
    atoms = W.surface_atoms(tip, density=4.0)
    t2 = time.perf_counter()
    omc.surface_charge(sc.E, atoms)
    charge_s = time.perf_counter() - t2
    # and its metal-side solves on a bounded sample: the same tip's metal
    # with a 2 nm substrate (the production metal has a 10 nm one)
    from oracle import metal as OM
    mm = W.kuhn_metal_mesh(tip.nx, tip.ny, tip.nz, tip.h, tip.tip_R,
                           tip.tip_H, 4)
    flux, PN = W.metal_sources(mm)
    sig = np.ones(mm.n_tets)
    t3 = time.perf_counter()
    mphi = OM.continuity_solve(mm, sig, flux)
    cont_s = time.perf_counter() - t3
    t4 = time.perf_counter()
    OM.heat_step(mm, np.full(mm.n_nodes, 300.0), sig, OM.joule(mm, sig, mphi),
                 PN, 3.45e-3, 2.0e-8, 40.0, 1.0, 300.0)
    heat_s = time.perf_counter() - t4
    return dict(value=round(n_steps / dt, 5), unit="steps/s", cores=O.threads(),
                kind="oracle",
                sample=(f"{n_steps} steps of the FP64 oracle ({O.threads()} "
                        "OpenMP threads) on "
                        f"the same 3.1M-tet mesh with {n0} seeded synthetic "
                        "superparticles in the gap above the apex; then, "
                        "serially, one "
                        "collision pass over them and one surface charge of "
                        f"the {omc.n_emit} metal faces to {len(atoms)} atoms; "
                        "one continuity solve and one heat step (sparse LU, "
                        f"scipy) on the tip's metal with a 2 nm substrate "
                        f"({mm.n_nodes} nodes)"),
                pushes_per_s=round(n0 * n_steps / dt, 1),
                collide_s_per_call=round(coll_s, 4),
                surface_charge_s_per_call=round(charge_s, 4),
                metal_sample_nodes=mm.n_nodes,
                continuity_s_per_solve=round(cont_s, 4),
                heat_s_per_step=round(heat_s, 4))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed steps after the fill, before the timed ones")
    ap.add_argument("--fill-frac", type=float, default=0.95,
                    help="the untimed fill runs until this fraction of the "
                         "target population is live")
    ap.add_argument("--max-fill", type=int, default=400)
    ap.add_argument("--capacity", type=float, default=2.5e6)
    ap.add_argument("--resort", type=int, default=10)
    ap.add_argument("--breakdown-steps", type=int, default=20,
                    help="untimed steps after the timed ones with every "
                         "kernel class bracketed by events (0: none)")
    ap.add_argument("--cpu-particles", type=int, default=1_000_000)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision leg")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint window leg")
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--adjoint-precond", choices=("amg", "jacobi"),
                    default="amg",
                    help="preconditioner of the adjoint's transposed solves")
    ap.add_argument("--batch-instances", type=int, default=32,
                    help="instances of the batched leg (0: skip it)")
    ap.add_argument("--batch-warmup", type=int, default=30)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--stress-steps", type=int, default=20,
                    help="timed steps of the coupled variant (current scaled "
                         "so that space charge shows; 0: skip)")
    ap.add_argument("--stress-warmup", type=int, default=60)
    ap.add_argument("--metal-calls", type=int, default=3,
                    help="continuity solves and heat steps timed on the "
                         "production tip's metal (0: skip)")
    ap.add_argument("--charge-calls", type=int, default=5,
                    help="timed surface-charge calls over every metal face "
                         "of the production tip (0: skip)")
    ap.add_argument("--collide-steps", type=int, default=20,
                    help="untimed steps with binary collisions after every "
                         "re-sort, to time the collision launches (0: none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (the "
                         "reference kernel for HBM byte counters)")
    ap.add_argument("--inner-tol", type=float, default=1e-4,
                    help="FP32 inner CG target of the mixed leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: a multi-GPU layout of this "
              "PIC cycle (z-slab domains, particle migration, halo exchange "
              "in the solve) is designed, not implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    out, ctx = run_gpu(args)
    if not args.no_cpu_baseline:
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(ctx["cfg"], ctx["tip"],
                                           args.cpu_particles, args.cpu_steps)
        log(f"cpu baseline {time.time() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
