"""The C ABI library loads on the host and exports every entry point the
public header declares; host-side argument checks reject bad input before
any device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "femocs_pic.h")


def declared_functions():
    src = open(HEADER).read()
    return re.findall(r"PIC_API\s+[\w\s\*]+?\b(\w+)\s*\(", src)


def test_header_declares_the_boundary():
    names = set(declared_functions())
    for n in ("mesh_create", "pic_step", "poisson_solve", "deposit", "locate",
              "adjoint_step", "mesh_destroy", "pic_last_error"):
        assert n in names, n


def test_library_exports_header_symbols():
    from paper_1906_08125_amd import pic
    if not os.path.exists(pic.LIB_PATH):
        pytest.skip("library not built")
    lib = C.CDLL(pic.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_host_argument_checks():
    from paper_1906_08125_amd import pic
    if not os.path.exists(pic.LIB_PATH):
        pytest.skip("library not built")
    L = pic.load_library()
    h = C.c_void_p()
    assert L.mesh_create(None, None, C.byref(h)) == pic.PIC_E_ARG
    d = pic.MeshDesc(0, None, 0, None, None, 1.0, 1.0, 1.0, 0.0)
    assert L.mesh_create(C.byref(d), None, C.byref(h)) == pic.PIC_E_ARG
    assert b"empty" in L.pic_last_error()
    assert L.locate(None, 1, None, None, None, None, None, None) == pic.PIC_E_ARG
    assert L.deposit(None, 1, None, None, None, None, None, None, None) == \
        pic.PIC_E_ARG
    assert L.pic_step(None, None, None, None, 1, None, None) == pic.PIC_E_ARG
    assert L.adjoint_step(None, None, None, None, None, None, None, None,
                          None) == pic.PIC_E_ARG


def test_collide_rejects_null():
    from paper_1906_08125_amd import pic
    if not os.path.exists(pic.LIB_PATH):
        pytest.skip("library not built")
    L = pic.load_library()
    assert L.collide(None, None, None, None) == pic.PIC_E_ARG
    assert L.surface_charge(None, None, None, None, None, None) == pic.PIC_E_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes records have the header's sizes and offsets
    (compiled with the host C compiler)."""
    import subprocess
    from paper_1906_08125_amd import pic
    checks = {
        "pic_step_params": (pic.StepParams, ["resort_every", "field_mode",
                                             "collide", "counts_in",
                                             "counts_out", "solve"]),
        "pic_collide_params": (pic.CollideParams, ["dt_coll", "w_sp", "seed",
                                                   "step", "instance"]),
        "pic_solve_params": (pic.SolveParams, ["tol", "precond"]),
        "pic_kernel_times": (pic.KernelTimes, ["ms", "launches"]),
        "pic_charge_params": (pic.ChargeParams, ["n_atoms", "atoms", "r_c",
                                                 "field_mode", "precision"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>',
             f'#include "{HEADER}"', 'int main(void) {']
    for cname, (_, fields) in checks.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", str(src), "-o", str(exe)], capture_output=True,
                       text=True)
    if r.returncode != 0:
        pytest.skip("no host C compiler: " + r.stderr[:200])
    out = dict(l.split() for l in subprocess.run(
        [str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for cname, (cls, fields) in checks.items():
        assert int(out[cname]) == C.sizeof(cls), cname
        for f in fields:
            assert int(out[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    """No CPU fallback: a missing library is an error, not a slower path."""
    from paper_1906_08125_amd import pic
    monkeypatch.setattr(pic, "_lib", None)
    with pytest.raises(ImportError):
        pic.load_library(str(tmp_path / "absent.so"))


def test_metal_rejects_null():
    from paper_1906_08125_amd import pic
    if not os.path.exists(pic.LIB_PATH):
        pytest.skip("library not built")
    L = pic.load_library()
    h = C.c_void_p()
    assert L.metal_create(None, None, C.byref(h)) == pic.PIC_E_ARG
    d = pic.MetalDesc(0, None, 0, None, 0, None, None)
    assert L.metal_create(C.byref(d), None, C.byref(h)) == pic.PIC_E_ARG
    assert b"empty" in L.pic_last_error()
    # out-of-range node ids are caught on the host, before any device work
    xyz = (C.c_double * 12)(0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1)
    tets = (C.c_int32 * 4)(0, 1, 2, 4)
    dr = (C.c_uint8 * 4)(1, 0, 0, 0)
    d = pic.MetalDesc(4, C.cast(xyz, C.c_void_p), 1, C.cast(tets, C.c_void_p),
                      0, None, C.cast(dr, C.c_void_p))
    assert L.metal_create(C.byref(d), None, C.byref(h)) == pic.PIC_E_ARG
    assert b"range" in L.pic_last_error()
    st = pic.MetalStats()
    assert L.continuity_solve(None, None, None, 1e-10, 10, None, None,
                              C.byref(st), None) == pic.PIC_E_ARG
    hp = pic.HeatParams(1.0, 2e-8, 1.0, 1.0, 300.0, 1e-10, 10)
    assert L.heat_step(None, C.byref(hp), None, None, None, None, None,
                       None) == pic.PIC_E_ARG


def test_binding_rejects_bad_arrays_before_the_library():
    """The binding checks dtype, length, contiguity and device of every
    array it passes to the metal solves and the single calls before
    anything is enqueued (a float32 temperature or a short conductivity
    would otherwise be read and written out of bounds by the kernels).
    Runs on the host: every case fails before the library is called."""
    import torch
    from paper_1906_08125_amd import pic

    m = pic.Metal.__new__(pic.Metal)
    m.n_nodes, m.n_tets, m.n_faces, m._h = 10, 20, 4, None
    f64 = lambda n: torch.zeros(n, dtype=torch.float64)
    with pytest.raises(TypeError, match="T: dtype float32"):
        m.heat_step(torch.full((10,), 300.0), f64(20), None, f64(4),
                    1.0, 1.0, 1.0)
    with pytest.raises(ValueError, match="sigma: 19 elements"):
        m.heat_step(f64(10), f64(19), None, f64(4), 1.0, 1.0, 1.0)
    with pytest.raises(ValueError, match="P_N: 3 elements"):
        m.heat_step(f64(10), f64(20), f64(20), f64(3), 1.0, 1.0, 1.0)
    with pytest.raises(ValueError, match="not contiguous"):
        m.heat_step(f64(20)[::2], f64(20), None, f64(4), 1.0, 1.0, 1.0)
    with pytest.raises(TypeError, match="HIP device"):
        m.heat_step(f64(10), f64(20), None, f64(4), 1.0, 1.0, 1.0)
    with pytest.raises(TypeError, match="flux: dtype int64"):
        m.continuity_solve(f64(20), torch.zeros(4, dtype=torch.int64))
    with pytest.raises(ValueError, match="phi: 9 elements"):
        m.continuity_solve(f64(20), f64(4), phi=f64(9))
    g = pic.Mesh.__new__(pic.Mesh)
    g.n_nodes, g._h = 7, None
    with pytest.raises(TypeError, match="E .*dtype float32"):
        g.emission_rate(torch.zeros(28, dtype=torch.float32), 4.5)
    with pytest.raises(ValueError, match="phi: 6 elements"):
        g.poisson_solve(None, 0.0, 0.5, f64(6))
    with pytest.raises(TypeError, match="tet: dtype int64"):
        g.deposit(f64(3), f64(3), f64(3), torch.zeros(3, dtype=torch.int64),
                  f64(3), torch.zeros(7, dtype=torch.int64))
    with pytest.raises(TypeError, match="where_out: dtype int32"):
        g.locate(f64(3), f64(3), f64(3), torch.zeros(3, dtype=torch.int32),
                 torch.zeros(3, dtype=torch.int32))
