"""ctypes binding of the FP64 CPU oracle (femocs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  The oracle shares
no code with the HIP library; both sides only share the seeded input arrays
of ``paper_1906_08125_amd.workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "femocs_oracle.c")
_LIB = os.path.join(_HERE, "libfemocs_oracle.so")
_LIB_OMP = os.path.join(_HERE, "libfemocs_oracle_omp.so")
_openmp = False

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build(openmp: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math);
    openmp: the timing build of the CPU baseline (-fopenmp; its parallel
    loops give the plain build's results bit for bit)."""
    out = _LIB_OMP if openmp else _LIB
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas"]
    cmd += ["-fopenmp"] if openmp else []
    cmd += ["-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def use_openmp() -> None:
    """Load the -fopenmp timing build instead of the plain one (before the
    first use of the oracle in this process)."""
    global _openmp
    if _lib is not None and not _openmp:
        raise RuntimeError("the plain oracle build is already loaded")
    _openmp = True


def threads() -> int:
    """Threads of the loaded build's parallel loops (1: plain build)."""
    return int(lib().om_threads())


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = _LIB_OMP if _openmp else _LIB
    if (not os.path.exists(path)
            or os.path.getmtime(path) < os.path.getmtime(_SRC)
            or os.path.getmtime(path) < os.path.getmtime(
                os.path.join(_HERE, "femocs_oracle.h"))):
        build(_openmp)
    L = C.CDLL(path)
    L.om_threads.restype = C.c_int
    L.om_threads.argtypes = []
    L.om_create.restype = C.c_void_p
    L.om_create.argtypes = [C.c_int64, _dp, C.c_int64, _i32p, _i8p,
                            C.c_double, C.c_double, C.c_double, C.c_double,
                            C.c_char_p, C.c_int]
    L.om_destroy.argtypes = [C.c_void_p]
    L.om_info.restype = C.c_int64
    L.om_info.argtypes = [C.c_void_p, C.c_int]
    L.om_get_tets.argtypes = [C.c_void_p, _i32p, _dp, _dp, _dp, _i32p, _i8p]
    L.om_get_csr.argtypes = [C.c_void_p, _i64p, _i32p, _dp]
    L.om_get_free.argtypes = [C.c_void_p, _i32p, _dp]
    L.om_get_emit.argtypes = [C.c_void_p, _i32p, _i32p, _dp, _dp, _dp, _i32p]
    L.om_orient_sign.restype = C.c_int
    L.om_orient_sign.argtypes = [_dp, _dp, _dp, _dp]
    L.om_lambda.argtypes = [C.c_void_p, C.c_int32, _dp, _dp]
    L.om_locate.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, _dp, C.c_void_p,
                            _i32p, _u8p]
    L.om_deposit.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, _dp, _i32p, _dp,
                             _i64p]
    L.om_poisson_solve.restype = C.c_int
    L.om_poisson_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_double,
                                   C.c_double, _dp, C.c_double, C.c_int,
                                   C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.om_rhs.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, _dp]
    L.om_spmv.argtypes = [C.c_void_p, _dp, _dp]
    L.om_field.argtypes = [C.c_void_p, _dp, _dp]
    L.om_cell_field.argtypes = [C.c_void_p, _dp, _dp]
    L.om_field_adj.argtypes = [C.c_void_p, _dp, _dp]
    L.om_fn_current.restype = C.c_double
    L.om_fn_current.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int)]
    L.om_constants.argtypes = [_dp]
    L.om_philox4x64.argtypes = [C.c_uint64, C.c_uint64, _u64p, _u64p]
    L.om_pic_step.restype = C.c_int
    L.om_pic_step.argtypes = [C.c_void_p, C.c_void_p, _dp, _dp, _i64p,
                              C.c_void_p, C.c_void_p]
    L.om_surface_charge.restype = None
    L.om_surface_charge.argtypes = [C.c_void_p, _dp, C.c_void_p, C.c_int,
                                    C.c_int64, C.c_void_p, C.c_double, _dp,
                                    _dp]
    L.om_collide.restype = None
    L.om_collide.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.om_inject.restype = C.c_int
    L.om_inject.argtypes = [C.c_void_p, C.c_void_p, _dp, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p]
    L.om_emission_rate.restype = C.c_double
    L.om_emission_rate.argtypes = [C.c_void_p, _dp, C.c_double, C.c_void_p]
    L.om_emission_rate_mode.restype = C.c_double
    L.om_emission_rate_mode.argtypes = [C.c_void_p, _dp, C.c_void_p, C.c_double,
                                        C.c_void_p]
    _lib = L
    return L


class _Particles(C.Structure):
    _fields_ = [("cap", C.c_int64), ("n", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("w", C.c_void_p), ("tet", C.c_void_p), ("birth", C.c_void_p),
                ("id", C.c_void_p)]


class _StepParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("E0", C.c_double), ("w_sp", C.c_double),
                ("phi_w", C.c_double), ("j_scale", C.c_double),
                ("tol", C.c_double), ("seed", C.c_uint64), ("step", C.c_int64),
                ("instance", C.c_int64), ("max_iter", C.c_int32),
                ("field_mode", C.c_int32), ("s_face", C.c_void_p),
                ("counts_in", C.c_void_p), ("counts_out", C.c_void_p),
                ("fate_out", C.c_void_p), ("inj_out", C.c_void_p),
                ("phi", C.c_void_p), ("collide_every", C.c_int32),
                ("pad_c", C.c_int32)]


class _CollideParams(C.Structure):
    _fields_ = [("dt_coll", C.c_double), ("w_sp", C.c_double),
                ("seed", C.c_uint64), ("step", C.c_int64),
                ("instance", C.c_int64)]


class _StepStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_before", "n_inj", "n_anode", "n_cathode", "n_after", "q_before",
        "q_inj", "q_anode", "q_cathode", "q_after", "cg_iters", "n_clamp",
        "status", "n_trunc")] + [(n, C.c_double) for n in (
            "cg_relres", "emit_current", "mean_face_E", "max_face_E")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def constants() -> dict:
    out = np.zeros(8)
    lib().om_constants(out)
    return dict(qm=out[0], e_eps=out[1], a_fn=out[2], b_fn=out[3], c_s=out[4],
                j_unit=out[5], fx_scale=out[6])


def fn_current(F: float, phi_w: float) -> tuple[float, bool]:
    cl = C.c_int(0)
    j = lib().om_fn_current(float(F), float(phi_w), C.byref(cl))
    return j, bool(cl.value)


def philox4x64(key: tuple[int, int], ctr) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().om_philox4x64(C.c_uint64(key[0]), C.c_uint64(key[1]),
                        np.ascontiguousarray(ctr, dtype=np.uint64), out)
    return out


def orient_sign(a, b, c, d) -> int:
    f = lambda v: np.ascontiguousarray(v, dtype=np.float64)
    return int(lib().om_orient_sign(f(a), f(b), f(c), f(d)))


class OracleMesh:
    """FP64 oracle mesh built from the generator's arrays."""

    def __init__(self, mesh, emit_zmin: float = 0.01):
        L = lib()
        err = C.create_string_buffer(256)
        self.mesh = mesh
        self._h = L.om_create(mesh.n_nodes, np.ascontiguousarray(mesh.xyz.reshape(-1)),
                              mesh.n_tets, np.ascontiguousarray(mesh.tet.reshape(-1)),
                              np.ascontiguousarray(mesh.shift.reshape(-1)),
                              mesh.Lx, mesh.Ly, mesh.z_top, emit_zmin, err, 256)
        if not self._h:
            raise ValueError(err.value.decode())
        self.n_nodes = L.om_info(self._h, 0)
        self.n_tets = L.om_info(self._h, 1)
        self.n_free = L.om_info(self._h, 2)
        self.nnz = L.om_info(self._h, 3)
        self.n_emit = L.om_info(self._h, 4)
        self.n_top = L.om_info(self._h, 5)
        self.n_metal = L.om_info(self._h, 6)
        self.n_flipped = L.om_info(self._h, 7)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().om_destroy(self._h)
            self._h = None

    # ---- derived arrays -------------------------------------------------
    def tets(self):
        T = self.n_tets
        tet = np.zeros((T, 4), np.int32)
        vert = np.zeros((T, 4, 3))
        mm = np.zeros((T, 3, 3))
        D = np.zeros(T)
        nbr = np.zeros((T, 4), np.int32)
        ns = np.zeros((T, 4, 2), np.int8)
        lib().om_get_tets(self._h, tet.reshape(-1), vert.reshape(-1),
                          mm.reshape(-1), D, nbr.reshape(-1), ns.reshape(-1))
        return dict(tet=tet, vert=vert, m=mm, D=D, nbr=nbr, nbr_shift=ns)

    def csr(self):
        rp = np.zeros(self.n_free + 1, np.int64)
        col = np.zeros(self.nnz, np.int32)
        val = np.zeros(self.nnz)
        lib().om_get_csr(self._h, rp, col, val)
        return rp, col, val

    def free(self):
        fid = np.zeros(self.n_nodes, np.int32)
        g = np.zeros(max(self.n_free, 1))
        lib().om_get_free(self._h, fid, g)
        return fid, g[: self.n_free]

    def emit(self):
        F = self.n_emit
        t = np.zeros(F, np.int32)
        loc = np.zeros(F, np.int32)
        area = np.zeros(F)
        nrm = np.zeros((F, 3))
        abc = np.zeros((F, 3, 3))
        nodes = np.zeros((F, 3), np.int32)
        if F:
            lib().om_get_emit(self._h, t, loc, area, nrm.reshape(-1),
                              abc.reshape(-1), nodes.reshape(-1))
        return dict(tet=t, local=loc, area=area, normal=nrm, abc=abc,
                    nodes=nodes)

    # ---- operations -----------------------------------------------------
    def lam(self, t: int, p) -> np.ndarray:
        out = np.zeros(4)
        lib().om_lambda(self._h, int(t), np.ascontiguousarray(p, np.float64),
                        out)
        return out

    def locate(self, p, hint=None):
        p = np.ascontiguousarray(p, np.float64)
        n = p.shape[0]
        x = np.ascontiguousarray(p[:, 0])
        y = np.ascontiguousarray(p[:, 1])
        z = np.ascontiguousarray(p[:, 2])
        tet = np.zeros(n, np.int32)
        where = np.zeros(n, np.uint8)
        hp = None
        if hint is not None:
            hint = np.ascontiguousarray(hint, np.int32)
            hp = hint.ctypes.data
        lib().om_locate(self._h, n, x, y, z, hp, tet, where)
        return tet, where

    def deposit(self, p, tet, w, c=None):
        p = np.ascontiguousarray(p, np.float64)
        if c is None:
            c = np.zeros(self.n_nodes, np.int64)
        lib().om_deposit(self._h, p.shape[0], np.ascontiguousarray(p[:, 0]),
                         np.ascontiguousarray(p[:, 1]),
                         np.ascontiguousarray(p[:, 2]),
                         np.ascontiguousarray(tet, np.int32),
                         np.ascontiguousarray(w, np.float64), c)
        return c

    def rhs(self, c, w_sp, E0):
        b = np.zeros(max(self.n_free, 1))
        cp = None if c is None else np.ascontiguousarray(c, np.int64)
        lib().om_rhs(self._h, None if cp is None else cp.ctypes.data,
                     float(w_sp), float(E0), b)
        return b[: self.n_free]

    def spmv(self, x):
        y = np.zeros(self.n_free)
        lib().om_spmv(self._h, np.ascontiguousarray(x, np.float64), y)
        return y

    def poisson_solve(self, c, w_sp, E0, phi=None, tol=1e-12,
                      max_iter=20000):
        if phi is None:
            phi = np.zeros(self.n_nodes)
        phi = np.ascontiguousarray(phi, np.float64).copy()
        it = C.c_int(0)
        rr = C.c_double(0)
        cp = None if c is None else np.ascontiguousarray(c, np.int64)
        s = lib().om_poisson_solve(self._h, None if cp is None else cp.ctypes.data,
                                   float(w_sp), float(E0), phi, float(tol),
                                   int(max_iter), C.byref(it), C.byref(rr))
        return phi, dict(status=s, iters=it.value, relres=rr.value)

    def field_adj(self, Ebar):
        """Transpose of field(): d<Ebar, field(phi)>/d phi over all nodes."""
        out = np.zeros(self.n_nodes)
        lib().om_field_adj(self._h, np.ascontiguousarray(
            np.asarray(Ebar, np.float64).reshape(-1)), out)
        return out

    def cell_field(self, phi):
        """Field of every tet in the cell reading (R2): -(grad phi)_t."""
        E = np.zeros((self.n_tets, 3))
        lib().om_cell_field(self._h, np.ascontiguousarray(phi, np.float64),
                            E.reshape(-1))
        return E

    def field(self, phi):
        E = np.zeros((self.n_nodes, 3))
        lib().om_field(self._h, np.ascontiguousarray(phi, np.float64),
                       E.reshape(-1))
        return E

    def surface_charge(self, E, atoms, r_c=0.1, phi=None):
        """Face charges of the emitting faces and the atoms' charges (nodal
        field E, or the cell field of phi when given)."""
        E = np.ascontiguousarray(E.reshape(-1), dtype=np.float64)
        atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 3)
        Q = np.zeros(max(self.n_emit, 1))
        q = np.zeros(max(len(atoms), 1))
        ph = None
        if phi is not None:
            ph = np.ascontiguousarray(phi, dtype=np.float64)
        lib().om_surface_charge(self._h, E, None if ph is None else ph.ctypes.data,
                                0 if ph is None else 1, len(atoms),
                                atoms.ctypes.data, float(r_c), Q, q)
        return Q[: self.n_emit], q[: len(atoms)]

    def emission_rate(self, E, phi_w, phi=None):
        """Total emission current and per-face |E|: at the nodal field E, or
        (phi given) in the cell field mode, each face at its tet's field."""
        F = np.zeros(max(self.n_emit, 1))
        E = np.ascontiguousarray(E.reshape(-1), dtype=np.float64)
        if phi is None:
            r = lib().om_emission_rate(self._h, E, float(phi_w), F.ctypes.data)
        else:
            phi = np.ascontiguousarray(phi, dtype=np.float64)
            r = lib().om_emission_rate_mode(self._h, E, phi.ctypes.data,
                                            float(phi_w), F.ctypes.data)
        return r, F[: self.n_emit]


class OracleState:
    """Superparticles (SoA, FP64) plus the field state of one run."""

    def __init__(self, om: OracleMesh, cap: int):
        self.om = om
        self.cap = int(cap)
        self.x = np.zeros(cap)
        self.y = np.zeros(cap)
        self.z = np.zeros(cap)
        self.vx = np.zeros(cap)
        self.vy = np.zeros(cap)
        self.vz = np.zeros(cap)
        self.w = np.zeros(cap)
        self.tet = np.zeros(cap, np.int32)
        self.birth = np.zeros(cap, np.int32)
        self.id = np.zeros(cap, np.int64)
        self.n = 0
        self.phi = np.zeros(om.n_nodes)
        self.E = np.zeros((om.n_nodes, 3))
        self.c = np.zeros(om.n_nodes, np.int64)

    def _struct(self):
        s = _Particles()
        s.cap = self.cap
        s.n = self.n
        for k in ("x", "y", "z", "vx", "vy", "vz", "w", "tet", "birth", "id"):
            setattr(s, k, getattr(self, k).ctypes.data)
        return s

    def init_field(self, E0, tol=1e-12, max_iter=20000):
        self.phi, info = self.om.poisson_solve(None, 0.0, E0, self.phi, tol,
                                               max_iter)
        self.E = self.om.field(self.phi)
        return info

    def step(self, *, dt, E0, w_sp, phi_w, step, seed, instance=0,
             j_scale=1.0, tol=1e-12, max_iter=20000, s_face=None,
             counts_in=None, detail=None, field_mode=0,
             collide_every=0) -> dict:
        """One PIC step.  counts_in: frozen emission counts per face.
        detail: a dict that receives the counts used, the fate of every
        particle of the step (pre-step particles, then the injected ones:
        0 kept, 1 anode, 2 cathode) and the injection draws
        (R1, R2, R, face) of the injected ones."""
        ps = self._struct()
        pr = _StepParams()
        pr.dt, pr.E0, pr.w_sp, pr.phi_w = dt, E0, w_sp, phi_w
        pr.j_scale, pr.tol = j_scale, tol
        pr.seed, pr.step, pr.instance = seed, step, instance
        pr.max_iter = max_iter
        pr.field_mode = field_mode
        pr.collide_every = collide_every
        sf = ci = None
        if s_face is not None:
            sf = np.ascontiguousarray(s_face, np.float64)
            pr.s_face = sf.ctypes.data
        if counts_in is not None:
            ci = np.ascontiguousarray(counts_in, np.int64)
            pr.counts_in = ci.ctypes.data
        if detail is not None:
            co = np.zeros(max(self.om.n_emit, 1), np.int64)
            fate = np.zeros(self.cap, np.int8)
            inj = np.zeros((self.cap, 4))
            pr.counts_out = co.ctypes.data
            pr.fate_out = fate.ctypes.data
            pr.inj_out = inj.ctypes.data
        n0 = self.n
        st = _StepStats()
        E = np.ascontiguousarray(self.E.reshape(-1))
        lib().om_pic_step(self.om._h, C.byref(ps), self.phi, E, self.c,
                          C.byref(pr), C.byref(st))
        self.E = E.reshape(-1, 3)
        self.n = ps.n
        out = st.as_dict()
        if detail is not None:
            n_all = n0 + out["n_inj"]
            detail["counts"] = co[: self.om.n_emit].copy()
            detail["fate"] = fate[:n_all].copy()
            detail["inj"] = inj[: out["n_inj"]].copy()
            detail["n_before"] = n0
        return out

    def collide(self, *, dt_coll, w_sp, seed, step, instance=0):
        """Binary collisions of the current superparticles (velocities
        change in place)."""
        ps = self._struct()
        cp = _CollideParams(dt_coll, w_sp, seed, step, instance)
        lib().om_collide(self.om._h, C.byref(ps), C.byref(cp))

    def inject(self, *, dt, E0, w_sp, phi_w, step, seed, instance=0,
               j_scale=1.0, s_face=None, field_mode=0):
        """Injection alone (appends to the state); returns the stats, the
        per-face rounded counts and the sampled face points of the new
        particles."""
        ps = self._struct()
        pr = _StepParams()
        pr.dt, pr.E0, pr.w_sp, pr.phi_w = dt, E0, w_sp, phi_w
        pr.j_scale, pr.seed, pr.step, pr.instance = j_scale, seed, step, instance
        pr.field_mode = field_mode
        pr.phi = self.phi.ctypes.data
        sf = None
        if s_face is not None:
            sf = np.ascontiguousarray(s_face, np.float64)
            pr.s_face = sf.ctypes.data
        st = _StepStats()
        pts = np.zeros((self.cap, 3))
        counts = np.zeros(max(self.om.n_emit, 1), np.int64)
        n_old = self.n
        E = np.ascontiguousarray(self.E.reshape(-1))
        lib().om_inject(self.om._h, C.byref(ps), E, C.byref(pr), C.byref(st),
                        pts.ctypes.data, counts.ctypes.data)
        self.n = ps.n
        return st.as_dict(), counts[: self.om.n_emit], pts[n_old:self.n]

    def add(self, p, v, tet, w=None, birth=None, ids=None):
        """Append particles given explicitly (tests)."""
        k = len(p)
        s = slice(self.n, self.n + k)
        self.x[s], self.y[s], self.z[s] = p[:, 0], p[:, 1], p[:, 2]
        self.vx[s], self.vy[s], self.vz[s] = v[:, 0], v[:, 1], v[:, 2]
        self.tet[s] = tet
        self.w[s] = 1.0 if w is None else w
        self.birth[s] = 0 if birth is None else birth
        self.id[s] = np.arange(k) if ids is None else ids
        self.n += k

    def particles(self) -> dict:
        n = self.n
        return dict(x=self.x[:n].copy(), y=self.y[:n].copy(),
                    z=self.z[:n].copy(), vx=self.vx[:n].copy(),
                    vy=self.vy[:n].copy(), vz=self.vz[:n].copy(),
                    w=self.w[:n].copy(), tet=self.tet[:n].copy(),
                    birth=self.birth[:n].copy(), id=self.id[:n].copy())
