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
