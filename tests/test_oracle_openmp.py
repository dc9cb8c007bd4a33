"""The oracle's -fopenmp timing build (the benchmark's CPU baseline) gives
the plain build's results bit for bit: 20 PIC steps of the tiny tip from
the empty gap (injection, push, location, absorption, deposition, solve,
field), with 4 threads, each build in a process of its own."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_RUN = r"""
import hashlib, json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_1906_08125_amd import workloads as W
if sys.argv[2] == "omp":
    O.use_openmp()
cfg = W.config_tiny()
om = O.OracleMesh(cfg.mesh(), cfg.emit_zmin)
st = O.OracleState(om, 200_000)
st.init_field(cfg.E0, tol=cfg.tol)
rate, _ = om.emission_rate(st.E, cfg.phi_w)
w_sp = rate * cfg.dt * cfg.transit_steps / cfg.n_target
rows = []
for k in range(20):
    rows.append(st.step(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w,
                        step=k, seed=cfg.seed, tol=cfg.tol))
P = st.particles()
h = hashlib.sha256()
for key in sorted(P):
    h.update(np.ascontiguousarray(P[key]).tobytes())
h.update(np.ascontiguousarray(st.phi).tobytes())
h.update(np.ascontiguousarray(st.E).tobytes())
print(json.dumps(dict(threads=O.threads(), digest=h.hexdigest(),
                      n=int(P["x"].shape[0]),
                      stats=[{k: float(v) for k, v in r.items()} for r in rows])))
"""


def _run(kind):
    env = dict(os.environ, OMP_NUM_THREADS="4")
    out = subprocess.run([sys.executable, "-c", _RUN, ROOT, kind], env=env,
                         capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_openmp_build_matches_plain_build():
    plain, omp = _run("plain"), _run("omp")
    assert plain["threads"] == 1 and omp["threads"] == 4
    assert plain["n"] > 1000          # particles were injected and pushed
    assert omp["stats"] == plain["stats"]
    assert omp["digest"] == plain["digest"]
