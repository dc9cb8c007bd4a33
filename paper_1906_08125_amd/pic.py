"""Python binding of libfemocs_pic.so: argument marshalling only.

Torch supplies device memory and the stream; every step of the PIC cycle
runs in the library's HIP kernels.  The binding raises when the library is
missing or a GPU is not available -- there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfemocs_pic.so")

PIC_OK, PIC_E_ARG, PIC_E_DEVICE, PIC_E_MESH = 0, -1, -2, -3
PIC_E_NOCONV, PIC_E_CAPACITY, PIC_E_NUMERIC = -4, -5, -6
PIC_FP64, PIC_MIXED = 0, 1
PIC_PRECOND_JACOBI, PIC_PRECOND_AMG = 0, 1
PIC_FIELD_NODAL, PIC_FIELD_CELL = 0, 1
CHARGE_SCALE = float(2 ** 40)


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.c_void_p),
                ("n_tets", C.c_int64), ("tet", C.c_void_p),
                ("shift", C.c_void_p), ("Lx", C.c_double), ("Ly", C.c_double),
                ("z_top", C.c_double), ("emit_zmin", C.c_double)]


class MeshInfo(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_nodes", "n_tets", "n_free", "nnz", "nnz_field", "n_emit", "n_top",
        "n_metal", "device_bytes")]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double),
                ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("precond", C.c_int32), ("pad", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("status", C.c_int64),
                ("restarts", C.c_int64), ("pad", C.c_int64),
                ("relres", C.c_double), ("bnorm", C.c_double)]


class Particles(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("precision", C.c_int32),
                ("pad", C.c_int32)] + [(n, C.c_void_p) for n in (
                    "x", "y", "z", "vx", "vy", "vz", "w", "tet", "birth", "id",
                    "n_slots")]


class Fields(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("E", C.c_void_p), ("charge", C.c_void_p)]


class StepParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("E0", C.c_double), ("w_sp", C.c_double),
                ("phi_w", C.c_double), ("j_scale", C.c_double),
                ("seed", C.c_uint64), ("step0", C.c_int64),
                ("instance", C.c_int64), ("s_face", C.c_void_p),
                ("resort_every", C.c_int32), ("field_mode", C.c_int32),
                ("collide", C.c_int32), ("pad", C.c_int32),
                ("counts_in", C.c_void_p), ("counts_out", C.c_void_p),
                ("solve", SolveParams)]


class ChargeParams(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("atoms", C.c_void_p),
                ("r_c", C.c_double), ("field_mode", C.c_int32),
                ("precision", C.c_int32)]


class MetalDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.c_void_p),
                ("n_tets", C.c_int64), ("tets", C.c_void_p),
                ("n_faces", C.c_int64), ("faces", C.c_void_p),
                ("dirichlet", C.c_void_p)]


class MetalStats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres", C.c_double),
                ("converged", C.c_int32), ("pad", C.c_int32)]


class HeatParams(C.Structure):
    _fields_ = [("Cv", C.c_double), ("L", C.c_double), ("dt", C.c_double),
                ("theta", C.c_double), ("T_amb", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_int64)]


class CollideParams(C.Structure):
    _fields_ = [("dt_coll", C.c_double), ("w_sp", C.c_double),
                ("seed", C.c_uint64), ("step", C.c_int64),
                ("instance", C.c_int64)]


STEP_STATS_FIELDS = (
    "n_before", "n_inj", "n_anode", "n_cathode", "n_after", "q_before",
    "q_inj", "q_anode", "q_cathode", "q_after", "cg_iters", "n_clamp",
    "status", "n_trunc", "walk_steps", "walk_max", "n_fallback", "n_slots")
STEP_STATS_FLOATS = ("cg_relres", "emit_current", "mean_face_E", "max_face_E")
STEP_STATS_BYTES = 8 * (len(STEP_STATS_FIELDS) + len(STEP_STATS_FLOATS))

class AdjointArgs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("rb", "vb", "Eb", "mu", "dJ_dE0",
                                          "dJ_ds", "bref")] + [
        ("wQ", C.c_double), ("wE", C.c_double), ("T", C.c_int32),
        ("mode", C.c_int32)]


PIC_ADJ_STEP, PIC_ADJ_INITIAL = 0, 1
PIC_MAX_BATCH = 64


class BatchSchedule(C.Structure):
    _fields_ = [("push_blocks", C.c_int32 * PIC_MAX_BATCH),
                ("inject_blocks", C.c_int32 * PIC_MAX_BATCH),
                ("cg_blocks", C.c_int32 * PIC_MAX_BATCH),
                ("clear_blocks", C.c_int32 * PIC_MAX_BATCH),
                ("fallback_blocks", C.c_int32), ("pad", C.c_int32)]

_lib = None

# Handles still open when the interpreter exits are closed by an atexit
# hook (registered when the library loads, so it runs before torch's own
# exit hooks and long before the HIP runtime's teardown at process exit):
# batches first, then metal meshes, then vacuum meshes.  Finalizers do not
# call into HIP while the interpreter is finalizing.
_open_handles = weakref.WeakSet()


def _close_all():
    objs = list(_open_handles)
    order = {"Batch": 0, "Metal": 1, "Mesh": 2}
    for o in sorted(objs, key=lambda o: order.get(type(o).__name__, 3)):
        try:
            o.close()
        except Exception:
            pass


LOCATE_NOALLOC_MAX = (1 << 20) - 64

EXPORTS = ("mesh_create", "mesh_workspace_bytes", "mesh_create_in",
           "mesh_destroy", "mesh_query", "mesh_emit_faces",
           "locate", "locate_noalloc", "deposit", "poisson_solve", "pic_step", "emission_rate",
           "adjoint_step", "pic_batch_create", "pic_batch_destroy",
           "pic_batch_step", "pic_profile", "pic_profile_every", "pic_profile_read",
           "pic_last_error", "collide", "surface_charge", "window_objective",
           "apply_face_weights", "metal_create",
           "metal_destroy", "continuity_solve", "heat_step")
KERNEL_CLASSES = ("push", "emit", "inject", "fallback", "solve", "sort",
                  "clear", "adjoint", "collide")


class KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 9), ("launches", C.c_int64 * 9)]


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m "
            "paper_1906_08125_amd.build` (hipcc, gfx950)")
    L = C.CDLL(path)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.mesh_create.argtypes = [C.POINTER(MeshDesc), vp, C.POINTER(vp)]
    L.mesh_workspace_bytes.argtypes = [C.POINTER(MeshDesc), C.POINTER(C.c_size_t)]
    L.mesh_create_in.argtypes = [C.POINTER(MeshDesc), vp, C.c_size_t, vp,
                                 C.POINTER(vp)]
    L.mesh_destroy.argtypes = [vp]
    L.mesh_query.argtypes = [vp, C.POINTER(MeshInfo)]
    L.mesh_emit_faces.argtypes = [vp, vp, vp, vp]
    L.locate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.locate_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.deposit.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.poisson_solve.argtypes = [vp, vp, dbl, dbl, vp, vp,
                                C.POINTER(SolveParams), vp, vp]
    L.pic_step.argtypes = [vp, C.POINTER(Particles), C.POINTER(Fields),
                           C.POINTER(StepParams), i32, vp, vp]
    L.emission_rate.argtypes = [vp, vp, dbl, vp, vp, vp]
    L.pic_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp), vp]
    L.pic_batch_destroy.argtypes = [vp]
    L.pic_batch_step.argtypes = [vp, C.POINTER(Particles), C.POINTER(Fields),
                                 C.POINTER(StepParams),
                                 C.POINTER(BatchSchedule), i32, vp, vp]
    L.adjoint_step.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles),
                               C.POINTER(Fields), C.POINTER(Fields),
                               C.POINTER(StepParams), C.POINTER(AdjointArgs),
                               vp, vp]
    L.pic_profile.argtypes = [vp, i32]
    L.pic_profile_every.argtypes = [vp, i32]
    L.window_objective.argtypes = [vp, vp, i32, vp, dbl, i32, dbl, dbl, vp, vp]
    L.apply_face_weights.argtypes = [vp, C.POINTER(Particles), vp, vp, vp]
    L.collide.argtypes = [vp, C.POINTER(Particles), C.POINTER(CollideParams), vp]
    L.surface_charge.argtypes = [vp, C.POINTER(Fields), C.POINTER(ChargeParams),
                                 vp, vp, vp]
    L.pic_profile_read.argtypes = [vp, C.POINTER(KernelTimes)]
    L.metal_create.argtypes = [C.POINTER(MetalDesc), vp, C.POINTER(vp)]
    L.metal_destroy.argtypes = [vp]
    L.continuity_solve.argtypes = [vp, vp, vp, dbl, i64, vp, vp,
                                   C.POINTER(MetalStats), vp]
    L.heat_step.argtypes = [vp, C.POINTER(HeatParams), vp, vp, vp, vp,
                            C.POINTER(MetalStats), vp]
    L.pic_last_error.restype = C.c_char_p
    for n in EXPORTS:
        if n != "pic_last_error":
            getattr(L, n).restype = C.c_int32
    _lib = L
    atexit.register(_close_all)
    return L


def _check(status):
    if status != PIC_OK:
        raise PicError(status, load_library().pic_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required (no CPU fallback)")
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_arrays(*specs):
    """Checks, before anything reaches the library, that each (tensor,
    dtype names, n, name) spec is a contiguous tensor of one of the dtypes
    ("float64", "int32", ...) holding exactly n elements (the kernels index
    it up to n), and then that every one of them is on the HIP device."""
    for t, dtypes, n, name in specs:
        if isinstance(dtypes, str):
            dtypes = (dtypes,)
        dt = str(getattr(t, "dtype", "")).replace("torch.", "")
        if dt not in dtypes:
            raise TypeError(f"{name}: dtype {dt or type(t).__name__}, "
                            f"expected {' or '.join(dtypes)}")
        if t.numel() != n:
            raise ValueError(f"{name}: {t.numel()} elements, expected {n}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: not contiguous")
    for t, _, _, name in specs:
        if t.device.type != "cuda":
            raise TypeError(f"{name}: on {t.device}, expected a HIP device "
                            "tensor")


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """Device mesh handle (mesh_create; with workspace=True, mesh_create_in
    into a torch-allocated workspace of mesh_workspace_bytes)."""

    def __init__(self, tip_mesh, emit_zmin: float, workspace: bool = False):
        torch = _torch()
        L = load_library()
        self._keep = (np.ascontiguousarray(tip_mesh.xyz, np.float64),
                      np.ascontiguousarray(tip_mesh.tet, np.int32),
                      np.ascontiguousarray(tip_mesh.shift, np.int8))
        d = MeshDesc(tip_mesh.n_nodes, self._keep[0].ctypes.data,
                     tip_mesh.n_tets, self._keep[1].ctypes.data,
                     self._keep[2].ctypes.data, tip_mesh.Lx, tip_mesh.Ly,
                     tip_mesh.z_top, emit_zmin)
        h = C.c_void_p()
        self.workspace = None
        if workspace:
            nb = C.c_size_t()
            _check(L.mesh_workspace_bytes(C.byref(d), C.byref(nb)))
            self.workspace = torch.empty(nb.value, dtype=torch.uint8,
                                         device="cuda")
            _check(L.mesh_create_in(C.byref(d), _ptr(self.workspace),
                                    nb.value, _stream(torch), C.byref(h)))
        else:
            _check(L.mesh_create(C.byref(d), _stream(torch), C.byref(h)))
        self._h = h
        _open_handles.add(self)
        info = MeshInfo()
        _check(L.mesh_query(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in info._fields_}
        self.n_nodes = info.n_nodes
        self.n_tets = info.n_tets
        self.n_free = info.n_free
        self.n_emit = info.n_emit
        self.tip = tip_mesh
        del self._keep

    @property
    def handle(self):
        return self._h

    def close(self):
        """Frees the device mesh (mesh_destroy); later calls do nothing."""
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _open_handles.discard(self)
            load_library().mesh_destroy(h)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (module globals may already be None while the interpreter
        # finalizes: the check is bound at definition time)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True, classes=None, every: int = 1):
        """Time the kernels of the named classes (KERNEL_CLASSES; all when
        None) with HIP events on the stream; enable=False stops.  Each
        event costs GPU time, so time only what is read: every > 1 times
        only the steps of pic_step whose index is a multiple of it."""
        mask = 0
        if enable:
            mask = 0x1FF if classes is None else sum(
                1 << KERNEL_CLASSES.index(c) for c in classes)
        L = load_library()
        _check(L.pic_profile_every(self._h, int(every) if enable else 1))
        _check(L.pic_profile(self._h, mask))

    def surface_charge(self, atoms, r_c=0.1, E=None, phi=None):
        """Face charges of the emitting faces and charges of the atoms
        (device [n, 3] f64): from the nodal field E (f64 or f32), or the
        cell field of phi when phi is given.  Returns (face_Q, atom_q)."""
        torch = _torch()
        atoms = atoms.contiguous()
        n = int(atoms.shape[0]) if atoms.numel() else 0
        dev = atoms.device
        fq = torch.zeros(max(self.n_emit, 1), dtype=torch.float64, device=dev)
        aq = torch.zeros(max(n, 1), dtype=torch.float64, device=dev)
        cell = phi is not None
        prec = PIC_FP64
        if not cell and E is not None and E.dtype == torch.float32:
            prec = PIC_MIXED
        f = Fields(phi.data_ptr() if cell else None,
                   None if cell or E is None else E.data_ptr(), None)
        prm = ChargeParams(n, atoms.data_ptr() if n else None, float(r_c),
                           PIC_FIELD_CELL if cell else PIC_FIELD_NODAL, prec)
        _check(load_library().surface_charge(self._h, C.byref(f), C.byref(prm),
                                             fq.data_ptr(), aq.data_ptr(),
                                             _stream(torch)))
        return fq[: self.n_emit], aq[:n]

    def profile_read(self) -> dict:
        kt = KernelTimes()
        _check(load_library().pic_profile_read(self._h, C.byref(kt)))
        return {n: dict(ms=kt.ms[i], launches=kt.launches[i])
                for i, n in enumerate(KERNEL_CLASSES) if kt.launches[i]}

    def emit_faces(self):
        F = self.n_emit
        tet = np.zeros(F, np.int32)
        nodes = np.zeros((F, 3), np.int32)
        area = np.zeros(F)
        _check(load_library().mesh_emit_faces(self._h, tet.ctypes.data,
                                              nodes.ctypes.data,
                                              area.ctypes.data))
        return dict(tet=tet, nodes=nodes, area=area)

    # ---- single calls ---------------------------------------------------
    def locate(self, x, y, z, tet_inout, where_out):
        n = x.numel()
        _dev_arrays((x, "float64", n, "x"), (y, "float64", n, "y"),
                    (z, "float64", n, "z"), (tet_inout, "int32", n, "tet_inout"),
                    (where_out, "uint8", n, "where_out"))
        torch = _torch()
        _check(load_library().locate(self._h, x.numel(), _ptr(x), _ptr(y),
                                     _ptr(z), _ptr(tet_inout), _ptr(where_out),
                                     _stream(torch)))

    def locate_noalloc(self, x, y, z, tet_inout, where_out):
        """locate with the library's fixed scratch (no device allocation;
        at most LOCATE_NOALLOC_MAX points per call)."""
        n = x.numel()
        _dev_arrays((x, "float64", n, "x"), (y, "float64", n, "y"),
                    (z, "float64", n, "z"), (tet_inout, "int32", n, "tet_inout"),
                    (where_out, "uint8", n, "where_out"))
        torch = _torch()
        _check(load_library().locate_noalloc(self._h, n, _ptr(x), _ptr(y),
                                             _ptr(z), _ptr(tet_inout),
                                             _ptr(where_out), _stream(torch)))

    def deposit(self, x, y, z, tet, w, charge):
        n = x.numel()
        _dev_arrays((x, "float64", n, "x"), (y, "float64", n, "y"),
                    (z, "float64", n, "z"), (w, "float64", n, "w"),
                    (tet, "int32", n, "tet"),
                    (charge, "int64", self.n_nodes, "charge"))
        torch = _torch()
        _check(load_library().deposit(self._h, x.numel(), _ptr(x), _ptr(y),
                                      _ptr(z), _ptr(tet), _ptr(w),
                                      _ptr(charge), _stream(torch)))

    def poisson_solve(self, charge, w_sp, E0, phi, E=None, tol=1e-12,
                      max_iter=20000, precision=PIC_FP64, inner_tol=1e-4,
                      precond=PIC_PRECOND_JACOBI):
        specs = [(phi, "float64", self.n_nodes, "phi")]
        if charge is not None:
            specs.append((charge, "int64", self.n_nodes, "charge"))
        if E is not None:
            specs.append((E, "float64" if precision == PIC_FP64 else "float32",
                          4 * self.n_nodes, "E"))
        _dev_arrays(*specs)
        torch = _torch()
        st = torch.zeros(6, dtype=torch.float64, device=phi.device)
        prm = SolveParams(tol, inner_tol, max_iter, precision, precond)
        _check(load_library().poisson_solve(
            self._h, _ptr(charge), float(w_sp), float(E0), _ptr(phi), _ptr(E),
            C.byref(prm), _ptr(st), _stream(torch)))
        return st

    @staticmethod
    def solve_stats(st) -> dict:
        raw = st.cpu().numpy()
        ints = raw[:4].view(np.int64)
        return dict(iters=int(ints[0]), status=int(ints[1]),
                    restarts=int(ints[2]), relres=float(raw[4]),
                    bnorm=float(raw[5]))

    def emission_rate(self, E, phi_w):
        """FN rate (e/fs) and |E| per emitting face for the FP64 nodal field
        E [4 n_nodes]."""
        _dev_arrays((E, "float64", 4 * self.n_nodes, "E (FP64 nodal field)"))
        torch = _torch()
        rate = torch.zeros(1, dtype=torch.float64, device=E.device)
        faceF = torch.zeros(max(self.n_emit, 1), dtype=torch.float64,
                            device=E.device)
        _check(load_library().emission_rate(self._h, _ptr(E), float(phi_w),
                                            _ptr(rate), _ptr(faceF),
                                            _stream(torch)))
        return rate, faceF[: self.n_emit]


class State:
    """Device particle SoA + fields for one run."""

    def __init__(self, mesh: Mesh, capacity: int, precision: int = PIC_FP64,
                 device="cuda", solve_precision: int | None = None,
                 inner_tol: float = 1e-4, precond: int = PIC_PRECOND_JACOBI):
        """precision: PIC_FP64, or PIC_MIXED for FP32 particles and field;
        solve_precision (default: precision) picks the Poisson solver;
        precond its preconditioner (PIC_PRECOND_AMG with mixed solves: the
        V-cycle in FP32 inside the FP64 CG)."""
        torch = _torch()
        self.mesh = mesh
        self.capacity = int(capacity)
        self.precision = precision
        self.solve_precision = (precision if solve_precision is None
                                else solve_precision)
        self.inner_tol = inner_tol
        self.precond = precond
        rd = torch.float64 if precision == PIC_FP64 else torch.float32
        n = self.capacity
        mk = lambda dt: torch.zeros(n, dtype=dt, device=device)
        self.x, self.y, self.z = mk(rd), mk(rd), mk(rd)
        self.vx, self.vy, self.vz = mk(rd), mk(rd), mk(rd)
        self.w = mk(torch.float64)
        self.tet = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.birth = mk(torch.int32)
        self.id = mk(torch.int64)
        self.n_slots = torch.zeros(1, dtype=torch.int32, device=device)
        nn = mesh.n_nodes
        self.phi = torch.zeros(nn, dtype=torch.float64, device=device)
        self.E = torch.zeros(4 * nn, dtype=rd, device=device)
        self.charge = torch.zeros(nn, dtype=torch.int64, device=device)
        self._p = Particles(n, precision, 0, *[
            t.data_ptr() for t in (self.x, self.y, self.z, self.vx, self.vy,
                                   self.vz, self.w, self.tet, self.birth,
                                   self.id, self.n_slots)])
        self._f = Fields(self.phi.data_ptr(), self.E.data_ptr(),
                         self.charge.data_ptr())

    def init_field(self, E0, tol=1e-12, max_iter=20000):
        """phi and E of the empty gap (the field type follows precision)."""
        st = self.mesh.poisson_solve(
            None, 0.0, E0, self.phi, self.E, tol, max_iter,
            precision=self.precision, inner_tol=self.inner_tol,
            precond=self.precond)
        return st

    def step(self, *, dt, E0, w_sp, phi_w, step0, seed, n_steps=1, instance=0,
             j_scale=1.0, tol=1e-12, max_iter=20000, s_face=None,
             resort_every=0, field_mode=PIC_FIELD_NODAL, collide=0,
             counts_in=None, counts_out=None, stats=None):
        """counts_in / counts_out: device int32 [n_emit] frozen emission
        counts / the counts used (see pic_step_params)."""
        torch = _torch()
        if stats is None:
            stats = torch.zeros(n_steps * STEP_STATS_BYTES // 8,
                                dtype=torch.int64, device=self.phi.device)
        prm = StepParams(dt, E0, w_sp, phi_w, j_scale, seed, step0, instance,
                         None if s_face is None else s_face.data_ptr(),
                         resort_every, field_mode, int(collide), 0,
                         None if counts_in is None else counts_in.data_ptr(),
                         None if counts_out is None else counts_out.data_ptr(),
                         SolveParams(tol, self.inner_tol, max_iter,
                                     self.solve_precision, self.precond))
        _check(load_library().pic_step(self.mesh.handle, C.byref(self._p),
                                       C.byref(self._f), C.byref(prm),
                                       int(n_steps), _ptr(stats),
                                       _stream(torch)))
        return stats

    def collide(self, *, dt_coll, w_sp, seed, step, instance=0):
        """Binary collisions of the superparticles of each tet (slots grouped
        by tet, as a re-sort leaves them); velocities change in place."""
        torch = _torch()
        prm = CollideParams(dt_coll, w_sp, seed, step, instance)
        _check(load_library().collide(self.mesh.handle, C.byref(self._p),
                                      C.byref(prm), _stream(torch)))

    @staticmethod
    def decode_stats(stats) -> list[dict]:
        raw = stats.cpu().numpy().view(np.int64).reshape(-1, STEP_STATS_BYTES // 8)
        out = []
        ni = len(STEP_STATS_FIELDS)
        for row in raw:
            d = {k: int(v) for k, v in zip(STEP_STATS_FIELDS, row[:ni])}
            fl = row[ni:].view(np.float64)
            d.update({k: float(v) for k, v in zip(STEP_STATS_FLOATS, fl)})
            out.append(d)
        return out

    def live(self) -> dict:
        """Host copy of the live particles (tet >= 0)."""
        n = int(self.n_slots.item())
        tet = self.tet[:n].cpu().numpy()
        keep = tet >= 0
        g = lambda t: t[:n].cpu().numpy()[keep]
        return dict(x=g(self.x).astype(np.float64), y=g(self.y).astype(np.float64),
                    z=g(self.z).astype(np.float64), vx=g(self.vx).astype(np.float64),
                    vy=g(self.vy).astype(np.float64), vz=g(self.vz).astype(np.float64),
                    w=g(self.w), tet=tet[keep], birth=g(self.birth), id=g(self.id))


# ---------------------------------------------------------------------------
# Adjoint window: T steps with per-step checkpoints (forward) and the
# reverse sweep that recomputes each step from its checkpoint and calls
# adjoint_step (backward).
# ---------------------------------------------------------------------------
_PARTICLE_ARRAYS = ("x", "y", "z", "vx", "vy", "vz", "w", "tet", "birth", "id",
                    "n_slots")


class _Checkpoint:
    """Device copies of a state's particles, phi and E."""

    def __init__(self, st: "State"):
        for k in _PARTICLE_ARRAYS + ("phi", "E"):
            setattr(self, k, getattr(st, k).clone())
        self.capacity = st.capacity
        self.precision = st.precision
        self.p = Particles(st.capacity, st.precision, 0, *[
            getattr(self, k).data_ptr() for k in _PARTICLE_ARRAYS])
        self.f = Fields(self.phi.data_ptr(), self.E.data_ptr(), 0)

    def restore(self, st: "State"):
        for k in _PARTICLE_ARRAYS + ("phi", "E"):
            getattr(st, k).copy_(getattr(self, k))


class Window:
    """T steps from the population currently in `state`.  The parameters
    are E0 and s (per emitting face: the weight of every superparticle born
    there is s_f times its base weight, the in-flight ones included); the
    objective is J = wQ J_Q + wE J_E (collected charge in e; mean |E| over
    the emitting-face centroids and the fields E_1..E_T)."""

    def __init__(self, mesh: Mesh, state: "State", T: int, step0: int, *,
                 dt, w_sp, phi_w, seed, j_scale=1.0, instance=0, tol=1e-10,
                 max_iter=20000, adjoint_solve_precision=PIC_FP64,
                 adjoint_precond=PIC_PRECOND_JACOBI):
        """adjoint_solve_precision: the transposed solves (FP64 by default:
        on a cold right-hand side the FP32 recursion with FP64 refinement
        needs more iterations than it saves per iteration)."""
        torch = _torch()
        self.adj_precision = adjoint_solve_precision
        self.adj_precond = adjoint_precond
        self.mesh, self.state, self.T, self.step0 = mesh, state, int(T), int(step0)
        self.kw = dict(dt=dt, w_sp=w_sp, phi_w=phi_w, seed=seed,
                       j_scale=j_scale, instance=instance, tol=tol,
                       max_iter=max_iter)
        self.base = _Checkpoint(state)        # population with base weights
        self.scratch = State(mesh, state.capacity, state.precision,
                             solve_precision=state.solve_precision,
                             inner_tol=state.inner_tol)
        self.cks = []
        self.charge = torch.zeros(mesh.n_nodes, dtype=torch.int64,
                                  device=state.phi.device)

    def _params(self, E0, s, step0):
        k = self.kw
        return StepParams(k["dt"], E0, k["w_sp"], k["phi_w"], k["j_scale"],
                          k["seed"], step0, k["instance"], s.data_ptr(), 0, 0, 0, 0,
                          None, None,
                          SolveParams(k["tol"], self.state.inner_tol,
                                      k["max_iter"], self.adj_precision,
                                      self.adj_precond))

    def _initial_field(self, st: "State", E0):
        """phi_0 and E_0 from the in-flight charge (weights already set)."""
        torch = _torch()
        n = int(st.n_slots.item())
        self.charge.zero_()
        if n:
            f64 = lambda t: t[:n].to(torch.float64)
            self.mesh.deposit(f64(st.x), f64(st.y), f64(st.z), st.tet[:n],
                              st.w[:n], self.charge)
        self.mesh.poisson_solve(self.charge, self.kw["w_sp"], E0, st.phi,
                                st.E, tol=self.kw["tol"],
                                max_iter=self.kw["max_iter"],
                                precision=st.precision,
                                inner_tol=st.inner_tol)

    def forward(self, E0: float, s, counts=None, wQ=1.0, wE=1.0):
        """Runs the window from the base population; returns (J_Q, J_E) as
        device scalars (and keeps J = wQ J_Q + wE J_E in self.J[2]) and the
        checkpoints.  counts: None, or the per-step emission counts to hold
        (a list of T device int32 [n_emit], e.g. the `counts` of an earlier
        forward) -- finite differences of J hold them, as the adjoint does.
        The counts used are kept in `counts` (and replayed by backward)."""
        torch = _torch()
        st, k = self.state, self.kw
        L = load_library()
        strm = _stream(torch)
        _dev_arrays((s, "float64", max(self.mesh.n_emit, 1), "s"))
        self.base.restore(st)
        _check(L.apply_face_weights(self.mesh.handle, C.byref(st._p),
                                    _ptr(self.base.w), _ptr(s), strm))
        self._initial_field(st, E0)
        self.cks = []
        used = [torch.zeros(max(self.mesh.n_emit, 1), dtype=torch.int32,
                            device=st.phi.device) for _ in range(self.T)]
        J = torch.zeros(3, dtype=torch.float64, device=st.phi.device)
        for j in range(self.T):
            self.cks.append(_Checkpoint(st))
            stats = st.step(dt=k["dt"], E0=E0, w_sp=k["w_sp"], phi_w=k["phi_w"],
                            step0=self.step0 + j, seed=k["seed"],
                            instance=k["instance"], j_scale=k["j_scale"],
                            tol=k["tol"], max_iter=k["max_iter"], s_face=s,
                            resort_every=0,
                            counts_in=None if counts is None else counts[j],
                            counts_out=used[j])
            _check(L.window_objective(self.mesh.handle, _ptr(st.E),
                                      int(st.precision), _ptr(stats),
                                      float(k["w_sp"]), self.T, float(wQ),
                                      float(wE), _ptr(J), strm))
        self.counts = used
        self.J = J
        return J[0], J[1]

    def backward(self, E0: float, s, wQ=1.0, wE=1.0):
        """dJ/dE0 (device scalar) and dJ/ds (device [n_emit]) of the last
        forward, recomputing each step from its checkpoint."""
        torch = _torch()
        st, sc, k = self.state, self.scratch, self.kw
        dev = st.phi.device
        cap, N = st.capacity, self.mesh.n_nodes
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=dev)
        rb, vb, Eb, mu = z(3 * cap), z(3 * cap), z(4 * N), z(N)
        dE0, ds, bref = z(1), z(max(self.mesh.n_emit, 1)), z(1)
        adj = AdjointArgs(rb.data_ptr(), vb.data_ptr(), Eb.data_ptr(),
                          mu.data_ptr(), dE0.data_ptr(), ds.data_ptr(),
                          bref.data_ptr(), float(wQ), float(wE), self.T,
                          PIC_ADJ_STEP)
        L = load_library()
        sst = torch.zeros(6 * (self.T + 1), dtype=torch.float64, device=dev)
        for j in range(self.T - 1, -1, -1):
            ck = self.cks[j]
            ck.restore(sc)
            sc.step(dt=k["dt"], E0=E0, w_sp=k["w_sp"], phi_w=k["phi_w"],
                    step0=self.step0 + j, seed=k["seed"], instance=k["instance"],
                    j_scale=k["j_scale"], tol=k["tol"], max_iter=k["max_iter"],
                    s_face=s, resort_every=0, counts_in=self.counts[j])
            prm = self._params(E0, s, self.step0 + j)
            _check(L.adjoint_step(self.mesh.handle, C.byref(ck.p),
                                  C.byref(sc._p), C.byref(ck.f),
                                  C.byref(sc._f), C.byref(prm), C.byref(adj),
                                  C.c_void_p(sst[6 * j:].data_ptr()),
                                  _stream(torch)))
        # the first field's adjoint solves another system: start from zero
        mu.zero_()
        adj.mode = PIC_ADJ_INITIAL
        ck = self.cks[0]
        prm = self._params(E0, s, self.step0)
        _check(L.adjoint_step(self.mesh.handle, C.byref(ck.p), None,
                              C.byref(ck.f), None, C.byref(prm), C.byref(adj),
                              C.c_void_p(sst[6 * self.T:].data_ptr()),
                              _stream(torch)))
        self.adjoint_solve_stats = sst   # [T + 1] pic_solve_stats records
        return dE0[0], ds[: self.mesh.n_emit]


def _window_function():
    torch = _torch()

    class PICWindowFn(torch.autograd.Function):
        """J(E0, s) = wQ J_Q + wE J_E of a Window, with the hand-written
        adjoint as its backward."""

        @staticmethod
        def forward(ctx, E0, s, window, wQ, wE):
            e0 = float(E0)
            s64 = s.detach().to(torch.float64).contiguous()
            window.forward(e0, s64, wQ=wQ, wE=wE)
            ctx.window, ctx.e0, ctx.w = window, e0, (wQ, wE)
            ctx.save_for_backward(s64)
            return window.J[2].clone().to(E0.dtype)

        @staticmethod
        def backward(ctx, g):
            (s64,) = ctx.saved_tensors
            dE0, ds = ctx.window.backward(ctx.e0, s64, *ctx.w)
            return (g * dE0).to(g.dtype), (g * ds).to(s64.dtype), None, None, None

    return PICWindowFn


def window_objective(E0, s, window: Window, wQ=1.0, wE=1.0):
    """Differentiable J(E0, s) (torch.autograd) over `window`."""
    return _window_function().apply(E0, s, window, wQ, wE)



# ---------------------------------------------------------------------------
# Batched stepping of independent instances, with a schedule autotuner.
# ---------------------------------------------------------------------------
class Batch:
    """Instances (Mesh, State, per-instance step keywords) advanced together
    by pic_batch_step.  The schedule gives each instance a number of
    workgroups per kernel from its size: live particles per push workgroup
    (push_tile) and free rows per solver workgroup (cg_rows);
    `autotune` picks these two from measured step times."""

    def __init__(self, meshes, states, params):
        torch = _torch()
        L = load_library()
        self.meshes, self.states, self.params = list(meshes), list(states), list(params)
        n = len(self.meshes)
        arr = (C.c_void_p * n)(*[m.handle for m in self.meshes])
        lim = (C.c_int32 * (4 * n))()
        h = C.c_void_p()
        _check(L.pic_batch_create(arr, n, C.byref(h), lim))
        self._h = h
        _open_handles.add(self)
        self.limits = np.array(list(lim), dtype=np.int64).reshape(n, 4)
        self.push_tile, self.cg_rows = 4096, 1024
        self.inject_blocks, self.clear_blocks, self.fallback_blocks = 16, 16, 8
        self.tuning = []
        self.last_iters = [0] * n

    def close(self):
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _open_handles.discard(self)
            load_library().pic_batch_destroy(h)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (module globals may already be None while the interpreter
        # finalizes: the check is bound at definition time)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def schedule(self, push_tile=None, cg_rows=None) -> BatchSchedule:
        pt = push_tile or self.push_tile
        cr = cg_rows or self.cg_rows
        sc = BatchSchedule()
        r8 = lambda x: max(8, (int(x) + 7) // 8 * 8)
        for i, (m, st) in enumerate(zip(self.meshes, self.states)):
            live = int(st.n_slots.item())
            lim = self.limits[i]
            sc.push_blocks[i] = min(r8(-(-live // pt)), int(lim[0]) // 8 * 8)
            sc.inject_blocks[i] = min(r8(self.inject_blocks), int(lim[1]) // 8 * 8)
            # an instance whose solve iterated gets the full solver grid,
            # the others (one residual pass per step) a grid by cg_rows
            full = int(lim[2]) // 8 * 8
            sc.cg_blocks[i] = full if self.last_iters[i] > 0 else min(
                r8(-(-m.n_free // cr)), full)
            sc.clear_blocks[i] = r8(self.clear_blocks)
        sc.fallback_blocks = min(self.fallback_blocks, int(self.limits[:, 3].min()) // 8 * 8)
        return sc

    def step(self, step0, n_steps=1, sched=None, stats=None):
        torch = _torch()
        n = len(self.meshes)
        if stats is None:
            stats = torch.zeros(n_steps * n * STEP_STATS_BYTES // 8,
                                dtype=torch.int64, device="cuda")
        P = (Particles * n)(*[st._p for st in self.states])
        F = (Fields * n)(*[st._f for st in self.states])
        prms = []
        for st, kw in zip(self.states, self.params):
            sf = kw.get("s_face")
            prms.append(StepParams(
                kw["dt"], kw["E0"], kw["w_sp"], kw["phi_w"], kw.get("j_scale", 1.0),
                kw["seed"], step0, kw.get("instance", 0),
                None if sf is None else sf.data_ptr(), kw.get("resort_every", 0),
                kw.get("field_mode", PIC_FIELD_NODAL), int(kw.get("collide", 0)), 0,
                None if kw.get("counts_in") is None else kw["counts_in"].data_ptr(),
                None if kw.get("counts_out") is None else kw["counts_out"].data_ptr(),
                SolveParams(kw.get("tol", 1e-10), st.inner_tol,
                            kw.get("max_iter", 20000), st.solve_precision,
                            kw.get("precond", st.precond))))
        S = (StepParams * n)(*prms)
        sc = sched if sched is not None else self.schedule()
        _check(load_library().pic_batch_step(self._h, P, F, S, C.byref(sc),
                                             int(n_steps), _ptr(stats),
                                             _stream(torch)))
        last = stats.view(n_steps, n, -1)[-1, :, STEP_STATS_FIELDS.index("cg_iters")]
        self.last_iters = [int(v) for v in last.cpu()]
        return stats

    @staticmethod
    def decode(stats, n):
        rows = State.decode_stats(stats)
        return [rows[k * n:(k + 1) * n] for k in range(len(rows) // n)]

    def autotune(self, step0, push_tiles=(1024, 2048, 4096, 8192),
                 cg_rows=(512, 1024, 2048, 4096), steps=2):
        """Times `steps` batched steps from a snapshot for every (push_tile,
        cg_rows) pair, restores the snapshot and keeps the fastest pair."""
        torch = _torch()
        snaps = [_Checkpoint(st) for st in self.states]
        best = None
        self.tuning = []
        for pt in push_tiles:
            for cr in cg_rows:
                for snap, st in zip(snaps, self.states):
                    snap.restore(st)
                sc = self.schedule(pt, cr)
                self.step(step0, 1, sc)          # warm the schedule
                for snap, st in zip(snaps, self.states):
                    snap.restore(st)
                torch.cuda.synchronize()
                import time as _t
                w0 = _t.perf_counter()
                self.step(step0, steps, sc)
                torch.cuda.synchronize()
                ms = 1e3 * (_t.perf_counter() - w0) / steps
                self.tuning.append((pt, cr, ms))
                if best is None or ms < best[2]:
                    best = (pt, cr, ms)
        for snap, st in zip(snaps, self.states):
            snap.restore(st)
        self.push_tile, self.cg_rows = best[0], best[1]
        return best


class Metal:
    """Device metal mesh (metal_create) for the solves of Sec. II D: the
    continuity equation with Joule heating and the Theta-scheme heat step.
    `mesh` is a workloads.MetalMesh (host arrays)."""

    def __init__(self, mesh):
        torch = _torch()
        L = load_library()
        self.n_nodes, self.n_tets = mesh.n_nodes, mesh.n_tets
        self.n_faces = mesh.n_faces
        self._keep = [np.ascontiguousarray(mesh.xyz, np.float64),
                      np.ascontiguousarray(mesh.tet, np.int32),
                      np.ascontiguousarray(mesh.faces, np.int32).reshape(-1, 3),
                      np.ascontiguousarray(mesh.dirichlet, np.uint8)]
        xyz, tet, fac, dr = self._keep
        d = MetalDesc(self.n_nodes, xyz.ctypes.data, self.n_tets,
                      tet.ctypes.data, self.n_faces,
                      fac.ctypes.data if self.n_faces else None, dr.ctypes.data)
        h = C.c_void_p()
        _check(L.metal_create(C.byref(d), _stream(torch), C.byref(h)))
        self._h = h
        _open_handles.add(self)

    def close(self):
        """Frees the device metal mesh (metal_destroy)."""
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _open_handles.discard(self)
            load_library().metal_destroy(h)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (module globals may already be None while the interpreter
        # finalizes: the check is bound at definition time)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def continuity_solve(self, sigma, flux, phi=None, tol=1e-12,
                         max_iter=100_000, joule=True):
        """Phi of Eq. cont_mat (device f64 tensors sigma [n_tets], flux
        [n_faces]); returns (Phi, P_J or None, stats dict)."""
        specs = [(sigma, "float64", self.n_tets, "sigma")]
        if self.n_faces:
            specs.append((flux, "float64", self.n_faces, "flux"))
        if phi is not None:
            specs.append((phi, "float64", self.n_nodes, "phi"))
        _dev_arrays(*specs)
        torch = _torch()
        if phi is None:
            phi = torch.zeros(self.n_nodes, dtype=torch.float64,
                              device=sigma.device)
        pj = torch.empty(self.n_tets, dtype=torch.float64,
                         device=sigma.device) if joule else None
        st = MetalStats()
        _check(load_library().continuity_solve(
            self._h, sigma.data_ptr(), _ptr(flux) if self.n_faces else None,
            float(tol), int(max_iter), phi.data_ptr(),
            pj.data_ptr() if joule else None, C.byref(st), _stream(torch)))
        return phi, pj, dict(iters=st.iters, relres=st.relres,
                             converged=bool(st.converged))

    def heat_step(self, T, sigma, P_J, P_N, Cv, L, dt, theta=1.0,
                  T_amb=300.0, tol=1e-12, max_iter=100_000):
        """One step of Eq. heat_theta2 in place on T (device f64 [n_nodes]);
        returns the solver stats."""
        specs = [(T, "float64", self.n_nodes, "T"),
                 (sigma, "float64", self.n_tets, "sigma")]
        if P_J is not None:
            specs.append((P_J, "float64", self.n_tets, "P_J"))
        if self.n_faces:
            specs.append((P_N, "float64", self.n_faces, "P_N"))
        _dev_arrays(*specs)
        torch = _torch()
        prm = HeatParams(float(Cv), float(L), float(dt), float(theta),
                         float(T_amb), float(tol), int(max_iter))
        st = MetalStats()
        _check(load_library().heat_step(
            self._h, C.byref(prm), sigma.data_ptr(),
            None if P_J is None else P_J.data_ptr(),
            _ptr(P_N) if self.n_faces else None, T.data_ptr(), C.byref(st),
            _stream(torch)))
        return dict(iters=st.iters, relres=st.relres,
                    converged=bool(st.converged))
