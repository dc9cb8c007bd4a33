"""Process exit with library handles still open.

A program that leaves a vacuum mesh, a batch and a metal mesh open (no
close(), objects alive until the interpreter exits) must end cleanly: the
binding's exit hook destroys them while the HIP runtime is still up, and
finalizers make no HIP calls while the interpreter finalizes."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
import sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_1906_08125_amd import pic, workloads as W
cfg = W.config_tiny()
gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
gs = pic.State(gm, 20000)
gs.init_field(cfg.E0, tol=cfg.tol)
kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=1e-3, phi_w=cfg.phi_w, seed=1, tol=cfg.tol,
          j_scale=1e30)
gs.step(step0=0, n_steps=2, **kw)
b = pic.Batch([gm], [gs], [dict(kw)])
b.step(2, 1)
mm = pic.Metal(W.kuhn_metal_mesh(8, 8, 16, 0.5, 2.0, 5.0, 2))
torch.cuda.synchronize()
keep = (gm, gs, b, mm)          # alive until the interpreter exits
closed = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
closed.close()                  # closed early: its finalizer runs at exit
print("left open", flush=True)
"""


def test_exit_with_open_handles():
    r = subprocess.run([sys.executable, "-c", PROGRAM, ROOT],
                       capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.returncode
    assert "left open" in r.stdout
    assert "Exception ignored" not in r.stderr
