"""Seeded synthetic workloads: the tip-over-cathode tetrahedral mesh and the
run parameters of the benchmark configurations.

This module produces *inputs only*: node coordinates, tetrahedron
connectivity with periodic vertex shifts, and plain parameter records.  It
holds none of the method's arithmetic (no orientation, adjacency, assembly,
field, emission or particle update); both the HIP library and the CPU oracle
derive everything else from these arrays on their own.

Mesh recipe (stands in for the FEMOCS mesh of the paper's Sec. II, which is
built around MD atoms and is out of scope here):

* a structured nx x ny x nz grid of cubes of edge h over the box
  [0, nx h] x [0, ny h] x [0, nz h], periodic in x and y (the lateral
  periodicity of Sec. II B 1);
* every cube (i, j, k) is Kuhn-split into 6 tetrahedra, one per axis
  permutation pi in lexicographic order (012, 021, 102, 120, 201, 210):
  [c, c + e_pi0, c + e_pi0 + e_pi1, c + (1,1,1)];
* the metal tip is a hemisphere-capped cylinder of radius R and total height
  H standing on z = 0 with its axis at (Lx/2, Ly/2); every tetrahedron with a
  vertex strictly inside the tip solid is removed, orphan nodes are dropped
  and the survivors are renumbered in their original order.

Node ids before compaction are ((i mod nx) ny + (j mod ny)) (nz + 1) + k, so
nodes on x = Lx / y = Ly are the same nodes as on x = 0 / y = 0; each
tetrahedron vertex carries a shift (sx, sy) in {0, 1}^2 such that its
unwrapped position is xyz[node] + (sx Lx, sy Ly, 0).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Axis permutations of the Kuhn split, lexicographic order.
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclasses.dataclass
class TipMesh:
    """Arrays describing one vacuum mesh (host, numpy)."""
    xyz: np.ndarray      # float64 [n_nodes, 3], wrapped into [0, Lx) x [0, Ly)
    tet: np.ndarray      # int32 [n_tets, 4]
    shift: np.ndarray    # int8 [n_tets, 4, 2]
    Lx: float
    Ly: float
    z_top: float
    h: float
    nx: int
    ny: int
    nz: int
    tip_R: float
    tip_H: float

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tet.shape[0])


def _inside_tip(x, y, z, cx, cy, R, H):
    """Strict interior of the capped cylinder (squared distances, exact for
    binary-exact grid coordinates)."""
    r2 = (x - cx) ** 2 + (y - cy) ** 2
    zc = H - R
    cyl = (z > 0) & (z <= zc) & (r2 < R * R)
    cap = (z > zc) & (r2 + (z - zc) ** 2 < R * R)
    return cyl | cap


def kuhn_tip_mesh(nx: int, ny: int, nz: int, h: float = 0.5,
                  tip_R: float = 0.0, tip_H: float = 0.0) -> TipMesh:
    """Structured Kuhn mesh of the periodic box with the tip removed.

    tip_R <= 0 gives the plain parallel-plate box (no tip)."""
    Lx, Ly, Lz = nx * h, ny * h, nz * h
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    ii = ii.reshape(-1)
    jj = jj.reshape(-1)
    kk = kk.reshape(-1)
    ncube = ii.size
    # local corner offsets of the 4 vertices for each permutation
    offs = np.zeros((6, 4, 3), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        e0 = np.eye(3, dtype=np.int64)[perm[0]]
        e1 = np.eye(3, dtype=np.int64)[perm[1]]
        offs[p, 1] = e0
        offs[p, 2] = e0 + e1
        offs[p, 3] = (1, 1, 1)
    # unwrapped integer vertex coordinates [ncube, 6, 4, 3]
    base = np.stack([ii, jj, kk], axis=1)[:, None, None, :]
    vint = base + offs[None, :, :, :]
    vint = vint.reshape(ncube * 6, 4, 3)
    vi, vj, vk = vint[..., 0], vint[..., 1], vint[..., 2]
    node = ((vi % nx) * ny + (vj % ny)) * (nz + 1) + vk
    sx = (vi >= nx).astype(np.int8)
    sy = (vj >= ny).astype(np.int8)
    keep = np.ones(ncube * 6, dtype=bool)
    if tip_R > 0.0:
        cx, cy = 0.5 * Lx, 0.5 * Ly
        inside = _inside_tip(vi * h, vj * h, vk * h, cx, cy, tip_R, tip_H)
        keep = ~inside.any(axis=1)
    node = node[keep]
    sx = sx[keep]
    sy = sy[keep]
    n_all = nx * ny * (nz + 1)
    used = np.zeros(n_all, dtype=bool)
    used[node.reshape(-1)] = True
    newid = np.full(n_all, -1, dtype=np.int64)
    newid[used] = np.arange(int(used.sum()))
    tet = newid[node].astype(np.int32)
    old = np.nonzero(used)[0]
    k = old % (nz + 1)
    j = (old // (nz + 1)) % ny
    i = old // ((nz + 1) * ny)
    xyz = np.stack([i * h, j * h, k * h], axis=1).astype(np.float64)
    shift = np.stack([sx, sy], axis=2).astype(np.int8)
    return TipMesh(xyz=np.ascontiguousarray(xyz), tet=np.ascontiguousarray(tet),
                   shift=np.ascontiguousarray(shift), Lx=float(Lx), Ly=float(Ly),
                   z_top=float(Lz), h=float(h), nx=nx, ny=ny, nz=nz,
                   tip_R=float(tip_R), tip_H=float(tip_H))


@dataclasses.dataclass
class MetalMesh:
    """Arrays describing the metal domain (host, numpy): the tip solid and a
    substrate slab under the cathode plane, not periodic (its lateral faces
    carry no flux)."""
    xyz: np.ndarray        # float64 [n_nodes, 3]
    tet: np.ndarray        # int32 [n_tets, 4]
    faces: np.ndarray      # int32 [n_faces, 3] metal-vacuum interface triangles
    face_tet: np.ndarray   # int32 [n_faces] the metal tetrahedron of each face
    dirichlet: np.ndarray  # uint8 [n_nodes] 1 on the substrate's bottom plane
    z_bottom: float

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tet.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.faces.shape[0])


def kuhn_metal_mesh(nx: int, ny: int, nz: int, h: float, tip_R: float,
                    tip_H: float, depth: int) -> MetalMesh:
    """The metal counterpart of kuhn_tip_mesh(nx, ny, nz, h, tip_R, tip_H):
    the tetrahedra that mesh removes (those with a vertex strictly inside the
    tip) plus `depth` layers of Kuhn-split cubes below z = 0.  Nodes are
    numbered by integer grid position (i, j, k), i in [0, nx], j in [0, ny],
    k in [-depth, nz], compacted in that order.  The interface faces are the
    faces that belong to exactly one metal tetrahedron and lie neither on
    the bottom plane z = -depth h nor on a lateral plane of the box; the
    Dirichlet nodes are those of the bottom plane."""
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny),
                             np.arange(-depth, nz), indexing="ij")
    base = np.stack([ii.reshape(-1), jj.reshape(-1), kk.reshape(-1)], 1)
    offs = np.zeros((6, 4, 3), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        e0 = np.eye(3, dtype=np.int64)[perm[0]]
        e1 = np.eye(3, dtype=np.int64)[perm[1]]
        offs[p, 1] = e0
        offs[p, 2] = e0 + e1
        offs[p, 3] = (1, 1, 1)
    vint = (base[:, None, None, :] + offs[None]).reshape(-1, 4, 3)
    vi, vj, vk = vint[..., 0], vint[..., 1], vint[..., 2]
    metal = np.repeat(base[:, 2] < 0, 6)       # substrate cubes
    if tip_R > 0.0:
        cx, cy = 0.5 * nx * h, 0.5 * ny * h
        inside = _inside_tip(vi * h, vj * h, vk * h, cx, cy, tip_R, tip_H)
        metal = metal | inside.any(axis=1)
    vint = vint[metal]
    nk = nz + depth + 1
    gid = (vint[..., 0] * (ny + 1) + vint[..., 1]) * nk + (vint[..., 2] + depth)
    n_all = (nx + 1) * (ny + 1) * nk
    used = np.zeros(n_all, dtype=bool)
    used[gid.reshape(-1)] = True
    newid = np.full(n_all, -1, dtype=np.int64)
    newid[used] = np.arange(int(used.sum()))
    tet = newid[gid].astype(np.int32)
    old = np.nonzero(used)[0]
    k = old % nk - depth
    j = (old // nk) % (ny + 1)
    i = old // (nk * (ny + 1))
    xyz = np.stack([i * h, j * h, k * h], axis=1).astype(np.float64)
    # boundary faces: sorted node triples met once
    tri = np.concatenate([tet[:, [1, 2, 3]], tet[:, [0, 2, 3]],
                          tet[:, [0, 1, 3]], tet[:, [0, 1, 2]]])
    owner = np.tile(np.arange(tet.shape[0], dtype=np.int32), 4)
    key = np.sort(tri, axis=1)
    _, first, cnt = np.unique(key, axis=0, return_index=True,
                              return_counts=True)
    once = first[cnt == 1]
    once.sort()
    f = tri[once]
    fi, fj, fk = (np.stack([i, j, k], 1)[f][..., a] for a in range(3))
    on_plane = ((fk == -depth).all(1) | (fi == 0).all(1) | (fi == nx).all(1)
                | (fj == 0).all(1) | (fj == ny).all(1))
    keep = ~on_plane
    dirichlet = (k == -depth).astype(np.uint8)
    return MetalMesh(xyz=np.ascontiguousarray(xyz),
                     tet=np.ascontiguousarray(tet),
                     faces=np.ascontiguousarray(f[keep].astype(np.int32)),
                     face_tet=np.ascontiguousarray(owner[once][keep]),
                     dirichlet=np.ascontiguousarray(dirichlet),
                     z_bottom=float(-depth * h))


# --------------------------------------------------------------------------
# Run configurations.  The five workloads: a tiny tip, a production-shaped
# tip (about 3.1M tetrahedra), its mixed-precision form, a batch of 32 uneven
# tips, and an adjoint window over the production mesh.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class RunConfig:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    tip_R: float
    tip_H: float
    E0: float              # applied field, V/nm
    phi_w: float           # work function, eV
    dt: float              # fs
    n_steps: int
    tol: float
    n_target: int          # live superparticles wanted in steady state
    emit_zmin: float       # emitting metal faces: centroid z >= emit_zmin
    seed: int
    resort_every: int
    transit_steps: int     # T of the superparticle-weight rule

    def mesh(self) -> TipMesh:
        return kuhn_tip_mesh(self.nx, self.ny, self.nz, self.h,
                             self.tip_R, self.tip_H)


def transit_steps(Lz: float, H: float, E0: float, dt: float) -> int:
    """Steps an electron needs to cross the gap above the apex in the
    uniform applied field: ceil(sqrt(2 (Lz - H) / (|q/m| E0)) / dt), with
    |q/m| = 0.17588 nm fs^-2 per V/nm (this only sizes the weight)."""
    qm = 0.1758820
    return int(math.ceil(math.sqrt(2.0 * (Lz - H) / (qm * E0)) / dt))


def config_tiny() -> RunConfig:
    """Box 8x8x16 nm, 16x16x32 grid, tip R = 2, H = 8, E0 = 0.4 V/nm,
    tip faces emit, 10 steps at 0.5 fs, tol 1e-12, ~1e4 live."""
    return RunConfig("tiny_tip_16x16x32", 16, 16, 32, 0.5, 2.0, 8.0, 0.4, 4.5,
                     0.5, 10, 1e-12, 10_000, 0.01, 1, 10, 10)


def config_production() -> RunConfig:
    """Box 32x32x64 nm, 64x64x128 grid (3,100,504 tets), tip R = 3, H = 30,
    E0 = 0.5 V/nm, apex faces emit, 100 steps, tol 1e-10, ~1e6 live,
    re-sort every 10 steps."""
    # Mean flight time from the apex to the top plane: the uniform-field
    # estimate transit_steps(64, 30, 0.5, 0.5) = 56 steps ignores the field
    # enhancement at the tip; on this mesh the steady state carries 673k
    # particles at T = 56 (17.85k injected and absorbed per step), i.e. a
    # 37.7-step mean transit, so T = 38 gives the ~1e6 live superparticles
    # the workload is defined by.
    T = 38
    return RunConfig("production_tip_64x64x128", 64, 64, 128, 0.5, 3.0, 30.0,
                     0.5, 4.5, 0.5, 100, 1e-10, 1_000_000, 27.0, 2, 10, T)


def config_diode(E0: float, nx: int = 32, nz: int = 50, h: float = 0.364,
                 dt: float = 0.02, n_steps: int = 1600) -> RunConfig:
    """Planar vacuum diode (the paper's PIC check, Sec. III A: a flat
    field emitter of area about 135 nm^2 facing the anode across an 18.2 nm
    gap): the plain box without a tip, the whole cathode plane z = 0
    emitting (emit_zmin = 0), lateral periodicity making the diode
    one-dimensional.  Default: 32 x 32 x 50 cubes of 0.364 nm, so A =
    135.7 nm^2 and d = 18.2 nm.  E0 is the anode field (the Neumann
    condition of the top plane); n_target is not used (the weight is set
    from the expected current by the caller)."""
    T = transit_steps(nz * h, 0.0, E0, dt)
    return RunConfig(f"planar_diode_{nx}x{nx}x{nz}", nx, nx, nz, h, 0.0, 0.0,
                     E0, 4.5, dt, n_steps, 1e-10, 0, 0.0, 5, 20, T)


def metal_production() -> MetalMesh:
    """The metal under the production tip (64 x 64 x 128 cubes of 0.5 nm,
    R = 3, H = 30): the tip solid and a 10 nm substrate (20 layers)."""
    return kuhn_metal_mesh(64, 64, 128, 0.5, 3.0, 30.0, 20)


def metal_sources(m: MetalMesh, J0: float = 0.02, decay: float = 2.0):
    """Synthetic interface fluxes for the metal solves: a current density
    J0 exp((z_f - z_max) / decay) through every interface face (z_f its
    centroid height), concentrated at the apex the way field emission is,
    as J_n = -J (electrons leave, so the current enters the metal), and a
    Nottingham flux of a tenth of it with the opposite sign."""
    zc = m.xyz[m.faces][:, :, 2].mean(axis=1)
    J = J0 * np.exp((zc - zc.max()) / decay)
    return np.ascontiguousarray(-J), np.ascontiguousarray(0.1 * J)


def philox_uniform_stream(seed: int, n: int) -> np.ndarray:
    """Plain seeded uniforms for *input* generation (instance draws, test
    points).  Not used by the method itself."""
    return np.random.Generator(np.random.Philox(seed)).random(n)


def batch_configs(n_inst: int = 32, seed: int = 4) -> list[RunConfig]:
    """Uneven tip instances: grid n x n x 2n with n in U{32..64} at h = 0.5,
    R in U[1.5, 4], H in U[10, 30] (redrawn while H > 0.75 Lz),
    E0 in U[0.3, 0.7], N_target log-uniform in [1e4, 1e6]."""
    out = []
    for i in range(n_inst):
        g = np.random.Generator(np.random.Philox(key=[seed, i]))
        n = int(g.integers(32, 65))
        R = float(g.uniform(1.5, 4.0))
        Lz = 2 * n * 0.5
        H = float(g.uniform(10.0, 30.0))
        while H > 0.75 * Lz:
            H = float(g.uniform(10.0, 30.0))
        E0 = float(g.uniform(0.3, 0.7))
        nt = int(round(10 ** g.uniform(4.0, 6.0)))
        # snap H and R to the grid resolution so node tests stay exact
        H = round(H * 2) / 2
        R = round(R * 4) / 4
        T = transit_steps(Lz, H, E0, 0.5)
        out.append(RunConfig(f"batch_{i}", n, n, 2 * n, 0.5, R, H, E0, 4.5,
                             0.5, 50, 1e-10, nt, H - R, seed, 10, T))
    return out


def random_points_in_box(mesh: TipMesh, n: int, seed: int) -> np.ndarray:
    """Uniform points over the (unwrapped) box; some fall in the metal."""
    g = np.random.Generator(np.random.Philox(seed))
    p = g.random((n, 3))
    p[:, 0] *= mesh.Lx
    p[:, 1] *= mesh.Ly
    p[:, 2] *= mesh.z_top
    return p


def surface_atoms(mesh: TipMesh, density: float = 4.0,
                  seed: int = 6) -> np.ndarray:
    """Synthetic surface atoms (stand-ins for the MD atoms of the paper's
    surface-charge step): seeded uniform points on the analytic metal
    surface -- the cathode plane z = 0 outside the tip's footprint, the tip
    cylinder and its hemispherical cap -- at `density` atoms per nm^2."""
    g = np.random.Generator(np.random.Philox(seed))
    Lx, Ly, R, H = mesh.Lx, mesh.Ly, mesh.tip_R, mesh.tip_H
    cx, cy = 0.5 * Lx, 0.5 * Ly
    n_plane = int(round(density * (Lx * Ly - (np.pi * R * R if R > 0 else 0.0))))
    pts = []
    while sum(len(p) for p in pts) < n_plane:
        p = g.random((n_plane, 3)) * np.array([Lx, Ly, 0.0])
        if R > 0:
            p = p[(p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2 >= R * R]
        pts.append(p)
    out = [np.concatenate(pts)[:n_plane]]
    if R > 0:
        zc = H - R
        n_cyl = int(round(density * 2 * np.pi * R * zc))
        a = g.random(n_cyl) * 2 * np.pi
        z = g.random(n_cyl) * zc
        out.append(np.stack([cx + R * np.cos(a), cy + R * np.sin(a), z], 1))
        n_cap = int(round(density * 2 * np.pi * R * R))
        u = g.random(n_cap)            # uniform on the upper hemisphere
        a = g.random(n_cap) * 2 * np.pi
        r = np.sqrt(1.0 - u * u)
        out.append(np.stack([cx + R * r * np.cos(a), cy + R * r * np.sin(a),
                             zc + R * u], 1))
    return np.ascontiguousarray(np.concatenate(out))


def lattice_points(mesh: TipMesh, n: int, seed: int) -> np.ndarray:
    """Points on vertices, edge midpoints and face centroids of the grid
    (all binary-exact): degenerate cases for point location."""
    g = np.random.Generator(np.random.Philox(seed))
    q = g.integers(0, 4, size=(n, 3)) * 0.25  # quarter-cell offsets
    c = np.stack([g.integers(0, mesh.nx, n), g.integers(0, mesh.ny, n),
                  g.integers(0, mesh.nz, n)], axis=1) * mesh.h
    p = c + q * mesh.h * 2.0
    p[:, 0] = np.minimum(p[:, 0], mesh.Lx)
    p[:, 1] = np.minimum(p[:, 1], mesh.Ly)
    p[:, 2] = np.minimum(p[:, 2], mesh.z_top)
    return p
