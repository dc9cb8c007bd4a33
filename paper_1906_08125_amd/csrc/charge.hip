// Face charge (Eq. face_charge) of the emitting faces -- every metal face
// when the mesh was made with emit_zmin below the cathode -- and its
// distribution to surface atoms (Eq. atom_charge, Eq. charge_weight):
//   Q_f = eps0 (E_f . n_f) A_f, with E_f the mean of the nodal field at the
//       face's vertices (or, in the cell mode, the field of the face's
//       tet) and n_f the normal into the vacuum;
//   q_j = sum_f Q_f w_fj,  w_fj = exp(-d_fj / r_c) / sum_j' exp(-d_fj' / r_c),
//       normalised over the atoms (so that the charge is conserved), d_fj
//       the distance from the face centroid to the atom, minimum image in
//       x and y, evaluated as exp(-(d_fj - d_f,min) / r_c) over the same sum.
// All pairs (a box too small for the cutoff sphere):
// k_face_charge: one workgroup per face (Q_f, d_f,min, the sum);
// k_atom_charge: one thread per (atom, range of faces), the faces in LDS
// tiles, summed in face order; k_atom_reduce adds the ranges in order (no
// atomics: the result does not depend on scheduling).
// Cutoff (every pair beyond d_f,min + kCutRc r_c left out, see ChargeArgs):
// atoms and face centroids binned into cells (k_cut_bin, the k_cut_scan_*
// passes, k_cut_fill, k_cut_rank: the members of a cell in ascending order,
// so the sums below do not depend on scheduling, with their coordinates
// copied in that order); k_face_charge_cut: one wave per face over the
// atom cells near it; k_atom_charge_cut: one wave per atom over the face
// cells near it.  Sums run over the cells in a fixed order and inside a
// cell in index order.
#include "charge.h"

#include <algorithm>
#include <cmath>

namespace fp {

namespace {

constexpr int kThreads = 256;
constexpr int kFaceTile = 512;

__device__ inline double3 face_centroid(const DevMesh& m, int64_t f) {
  const double* p = m.e_abc + 9 * f;
  return make_double3(((p[0] + p[3]) + p[6]) / 3.0, ((p[1] + p[4]) + p[7]) / 3.0,
                      ((p[2] + p[5]) + p[8]) / 3.0);
}

__device__ inline double dist_mi(const DevMesh& m, double3 c, const double* a) {
  double dx = c.x - a[0], dy = c.y - a[1];
  const double dz = c.z - a[2];
  if (dx > 0.5 * m.Lx) dx -= m.Lx;
  else if (dx < -0.5 * m.Lx) dx += m.Lx;
  if (dy > 0.5 * m.Ly) dy -= m.Ly;
  else if (dy < -0.5 * m.Ly) dy += m.Ly;
  return sqrt((dx * dx + dy * dy) + dz * dz);
}

__device__ inline double ld_comp(const void* E, int f32, int64_t i) {
  return f32 ? (double)((const float*)E)[i] : ((const double*)E)[i];
}

__global__ void __launch_bounds__(kThreads) k_face_charge(ChargeArgs a) {
  __shared__ double s_red[kThreads / 64];
  const DevMesh& m = a.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t f = blockIdx.x; f < m.n_emit; f += gridDim.x) {
    double ex, ey, ez;
    if (a.cell) {
      const TetGeom g = m.tg[m.e_tet[f]];
      const double p0 = a.phi[g.node[0]], p1 = a.phi[g.node[1]],
                   p2 = a.phi[g.node[2]], p3 = a.phi[g.node[3]];
      double e[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double g0 = -((g.m[k] + g.m[3 + k]) + g.m[6 + k]);
        e[k] = -(((p0 * g0 + p1 * g.m[k]) + p2 * g.m[3 + k]) + p3 * g.m[6 + k]);
      }
      ex = e[0];
      ey = e[1];
      ez = e[2];
    } else {
      const int32_t* nd = m.e_nodes + 3 * f;
      double e[3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        e[k] = ((ld_comp(a.E, a.f32, 4 * (int64_t)nd[0] + k) +
                 ld_comp(a.E, a.f32, 4 * (int64_t)nd[1] + k)) +
                ld_comp(a.E, a.f32, 4 * (int64_t)nd[2] + k)) / 3.0;
      ex = e[0];
      ey = e[1];
      ez = e[2];
    }
    const double* nr = m.e_nrm + 3 * f;
    const double Q = (((ex * nr[0] + ey * nr[1]) + ez * nr[2]) / a.e_eps) * m.e_area[f];
    if (a.n_atoms == 0) {
      if (threadIdx.x == 0) a.face_Q[f] = Q;
      continue;
    }
    const double3 c = face_centroid(m, f);
    // nearest atom (min is exact in any order)
    double dmin = 1.0 / 0.0;
    for (int64_t j = threadIdx.x; j < a.n_atoms; j += blockDim.x) {
      const double d = dist_mi(m, c, a.atoms + 3 * j);
      dmin = d < dmin ? d : dmin;
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double o = __shfl_xor(dmin, off, 64);
      dmin = o < dmin ? o : dmin;
    }
    if (lane == 0) s_red[wv] = dmin;
    __syncthreads();
    dmin = s_red[0];
    for (int k = 1; k < kThreads / 64; ++k) dmin = s_red[k] < dmin ? s_red[k] : dmin;
    __syncthreads();
    // normalisation (fixed-order tree)
    double S = 0.0;
    for (int64_t j = threadIdx.x; j < a.n_atoms; j += blockDim.x)
      S += exp(-(dist_mi(m, c, a.atoms + 3 * j) - dmin) / a.r_c);
    for (int off = 32; off >= 1; off >>= 1) S += __shfl_xor(S, off, 64);
    if (lane == 0) s_red[wv] = S;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < kThreads / 64; ++k) t += s_red[k];
      a.face_Q[f] = Q;
      a.f_min[f] = dmin;
      a.f_sum[f] = t;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kThreads) k_atom_charge(ChargeArgs a) {
  __shared__ double s_c[3][kFaceTile];
  __shared__ double s_min[kFaceTile], s_Q[kFaceTile], s_S[kFaceTile];
  const DevMesh& m = a.m;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // this workgroup's range of faces
  const int64_t per = (m.n_emit + gridDim.y - 1) / gridDim.y;
  const int64_t f_lo = per * blockIdx.y;
  const int64_t f_hi = f_lo + per < m.n_emit ? f_lo + per : m.n_emit;
  const bool mine = j < a.n_atoms;
  double at[3] = {0.0, 0.0, 0.0};
  if (mine) {
    at[0] = a.atoms[3 * j];
    at[1] = a.atoms[3 * j + 1];
    at[2] = a.atoms[3 * j + 2];
  }
  double q = 0.0;
  for (int64_t f0 = f_lo; f0 < f_hi; f0 += kFaceTile) {
    const int tn = (int)(f_hi - f0 < kFaceTile ? f_hi - f0 : kFaceTile);
    __syncthreads();
    for (int k = threadIdx.x; k < tn; k += blockDim.x) {
      const double3 c = face_centroid(m, f0 + k);
      s_c[0][k] = c.x;
      s_c[1][k] = c.y;
      s_c[2][k] = c.z;
      s_min[k] = a.f_min[f0 + k];
      s_Q[k] = a.face_Q[f0 + k];
      s_S[k] = a.f_sum[f0 + k];
    }
    __syncthreads();
    if (mine) {
      for (int k = 0; k < tn; ++k) {
        const double3 c = make_double3(s_c[0][k], s_c[1][k], s_c[2][k]);
        const double x = dist_mi(m, c, at) - s_min[k];
        q += (s_Q[k] * exp(-x / a.r_c)) / s_S[k];
      }
    }
  }
  if (mine) a.part[blockIdx.y * a.n_atoms + j] = q;
}

__global__ void __launch_bounds__(kThreads) k_atom_reduce(ChargeArgs a) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= a.n_atoms) return;
  double q = 0.0;
  for (int k = 0; k < a.n_split; ++k) q += a.part[k * a.n_atoms + j];
  a.atom_q[j] = q;
}


// ---------------------------------------------------------------------------
// Cutoff path.
// ---------------------------------------------------------------------------
struct Cell3 {
  int x, y, z;
};

__device__ inline Cell3 cell_of(const ChargeArgs& a, double x, double y, double z) {
  const DevMesh& m = a.m;
  double wx = x - m.Lx * floor(x / m.Lx);
  double wy = y - m.Ly * floor(y / m.Ly);
  int ix = (int)(wx / a.cx), iy = (int)(wy / a.cy);
  int iz = (int)floor((z - a.z0) / a.cz);
  ix = ix < 0 ? 0 : (ix >= a.nx ? a.nx - 1 : ix);
  iy = iy < 0 ? 0 : (iy >= a.ny ? a.ny - 1 : iy);
  iz = iz < 0 ? 0 : (iz >= a.nz ? a.nz - 1 : iz);
  return Cell3{ix, iy, iz};
}

__device__ inline int cell_id(const ChargeArgs& a, int x, int y, int z) {
  return (z * a.ny + y) * a.nx + x;
}

__device__ inline double wave_min_d(double v) {
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}
__device__ inline double wave_sum_d(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Counts cleared (both grids) and the far-face counter.
__global__ void __launch_bounds__(kThreads) k_cut_clear(ChargeArgs a) {
  const int64_t n_cells = (int64_t)a.nx * a.ny * a.nz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n_cells;
       i += (int64_t)gridDim.x * blockDim.x) {
    a.a_cnt[i] = 0;
    a.f_cnt[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_far = 0;
}

// Items 0 .. n_atoms - 1 are the atoms, then the faces (their centroids):
// cell, and a slot inside the cell in arrival order.
__global__ void __launch_bounds__(kThreads) k_cut_bin(ChargeArgs a) {
  const int64_t n = a.n_atoms + a.m.n_emit;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < a.n_atoms) {
      const double* p = a.atoms + 3 * i;
      const Cell3 c = cell_of(a, p[0], p[1], p[2]);
      const int id = cell_id(a, c.x, c.y, c.z);
      a.a_cell[i] = id;
      a.a_rank[i] = atomicAdd(a.a_cnt + id, 1);
    } else {
      const int64_t f = i - a.n_atoms;
      const double3 cc = face_centroid(a.m, f);
      const Cell3 c = cell_of(a, cc.x, cc.y, cc.z);
      const int id = cell_id(a, c.x, c.y, c.z);
      a.f_cell[f] = id;
      a.f_rank[f] = atomicAdd(a.f_cnt + id, 1);
    }
  }
}

// Exclusive scan of the counts in place, cnt[c] becoming the first slot of
// cell c and cnt[n_cells] the total, in tiles of 1024 cells (blockIdx.y 0:
// atoms, 1: faces): k_cut_scan_tiles scans each tile and keeps its total,
// k_cut_scan_top scans the totals, k_cut_scan_add adds them back.
__device__ inline int32_t block_excl_scan(int32_t v, int32_t* part, int32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) part[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      const int32_t t = part[w];
      part[w] = run;
      run += t;
    }
    part[16] = run;
  }
  __syncthreads();
  total = part[16];
  const int32_t r = part[wv] + x - v;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(1024) k_cut_scan_tiles(ChargeArgs a) {
  __shared__ int32_t part[17];
  int32_t* cnt = blockIdx.y == 0 ? a.a_cnt : a.f_cnt;
  int32_t* tsum = cnt + a.n_cells_pad;
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  const int64_t i = blockIdx.x * 1024ll + threadIdx.x;
  const int32_t v = i < n ? cnt[i] : 0;
  int32_t total;
  const int32_t e = block_excl_scan(v, part, total);
  if (i < n) cnt[i] = e;
  if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_cut_scan_top(ChargeArgs a) {
  __shared__ int32_t part[17];
  int32_t* cnt = blockIdx.x == 0 ? a.a_cnt : a.f_cnt;
  int32_t* tsum = cnt + a.n_cells_pad;
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  const int tiles = (int)((n + 1023) / 1024);
  const int32_t v = (int)threadIdx.x < tiles ? tsum[threadIdx.x] : 0;
  int32_t total;
  const int32_t e = block_excl_scan(v, part, total);
  if ((int)threadIdx.x < tiles) tsum[threadIdx.x] = e;
  if (threadIdx.x == 0) cnt[n] = total;
}

__global__ void __launch_bounds__(1024) k_cut_scan_add(ChargeArgs a) {
  int32_t* cnt = blockIdx.y == 0 ? a.a_cnt : a.f_cnt;
  const int32_t* tsum = cnt + a.n_cells_pad;
  const int64_t n = (int64_t)a.nx * a.ny * a.nz;
  const int64_t i = blockIdx.x * 1024ll + threadIdx.x;
  if (i < n) cnt[i] += tsum[blockIdx.x];
}

// Every item at its arrival slot of its cell (tmp), then at its place in
// index order inside the cell: idx[pos] = item, with the item's
// coordinates copied to pos (atoms) or its centroid written there (faces).
__global__ void __launch_bounds__(kThreads) k_cut_fill(ChargeArgs a) {
  const int64_t n = a.n_atoms + a.m.n_emit;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < a.n_atoms)
      a.a_tmp[a.a_cnt[a.a_cell[i]] + a.a_rank[i]] = (int32_t)i;
    else {
      const int64_t f = i - a.n_atoms;
      a.f_tmp[a.f_cnt[a.f_cell[f]] + a.f_rank[f]] = (int32_t)f;
    }
  }
}

// Q_f = eps0 (E_f . n_f) A_f (Eq. face_charge), E_f the mean nodal field
// of the face's vertices or the cell field of its tet.
__device__ inline double face_q(const ChargeArgs& a, int64_t f) {
  const DevMesh& m = a.m;
  double e[3];
  if (a.cell) {
    const TetGeom g = m.tg[m.e_tet[f]];
    const double p0 = a.phi[g.node[0]], p1 = a.phi[g.node[1]],
                 p2 = a.phi[g.node[2]], p3 = a.phi[g.node[3]];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double g0 = -((g.m[k] + g.m[3 + k]) + g.m[6 + k]);
      e[k] = -(((p0 * g0 + p1 * g.m[k]) + p2 * g.m[3 + k]) + p3 * g.m[6 + k]);
    }
  } else {
    const int32_t* nd = m.e_nodes + 3 * f;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      e[k] = ((ld_comp(a.E, a.f32, 4 * (int64_t)nd[0] + k) +
               ld_comp(a.E, a.f32, 4 * (int64_t)nd[1] + k)) +
              ld_comp(a.E, a.f32, 4 * (int64_t)nd[2] + k)) / 3.0;
  }
  const double* nr = m.e_nrm + 3 * f;
  return (((e[0] * nr[0] + e[1] * nr[1]) + e[2] * nr[2]) / a.e_eps) * m.e_area[f];
}

// (faces: Q_f too, by face and by position)
__global__ void __launch_bounds__(kThreads) k_cut_rank(ChargeArgs a) {
  const int64_t n = a.n_atoms + a.m.n_emit;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const bool at = i < a.n_atoms;
    const int32_t k = (int32_t)(at ? i : i - a.n_atoms);
    const int32_t* cnt = at ? a.a_cnt : a.f_cnt;
    const int32_t* tmp = at ? a.a_tmp : a.f_tmp;
    const int32_t cell = at ? a.a_cell[k] : a.f_cell[k];
    const int32_t lo = cnt[cell], hi = cnt[cell + 1];
    int32_t pos = lo;
    for (int32_t q = lo; q < hi; ++q) pos += tmp[q] < k ? 1 : 0;
    if (at) {
      a.a_idx[pos] = k;
      const double* p = a.atoms + 3 * (int64_t)k;
      a.a_xyz[3 * (int64_t)pos] = p[0];
      a.a_xyz[3 * (int64_t)pos + 1] = p[1];
      a.a_xyz[3 * (int64_t)pos + 2] = p[2];
    } else {
      a.f_idx[pos] = k;
      const double Q = face_q(a, k);
      a.face_Q[k] = Q;
      a.f_Q_s[pos] = Q;
      const double3 cc = face_centroid(a.m, k);
      a.f_cen[3 * (int64_t)pos] = cc.x;
      a.f_cen[3 * (int64_t)pos + 1] = cc.y;
      a.f_cen[3 * (int64_t)pos + 2] = cc.z;
    }
  }
}

// The members of the cells within K cells of c (K <= kCutKMax), by their
// positions in cell order: the cells of a row along x are consecutive, so
// the block is at most 2 (2K + 1)^2 runs of positions (a row split in two
// where it wraps in x), rows whose lower-bound distance exceeds sqrt(R2)
// left out and each row's x extent cut to what sqrt(R2) can reach (both
// valid for any point of cell c).  Run s = 4 lane + u; the runs' starts
// and prefix sums go to this wave's LDS table.  Every member position p
// (runs in order) is passed to f(p, valid): consecutive lanes take
// consecutive members (coalesced loads), four per lane and trip; lanes
// past the end get p = 0 with valid false (f loads unconditionally and
// only drops the contribution, so the four loads go out together).  Each
// lane sees its own members; the caller reduces over the wave.  Every wave
// of the workgroup calls this alike (it holds workgroup barriers).
constexpr int kCutKMax = 5;
constexpr int kSegMax = 4 * 64;

template <typename F>
__device__ inline void wave_block_members(const ChargeArgs& a, const int32_t* cnt,
                                          Cell3 c, int K, double R2, int32_t* s_lo,
                                          int32_t* s_pre, F&& f) {
  const int lane = threadIdx.x & 63;
  const int w = 2 * K + 1;
  int32_t lo[4], len[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = 2 * lane + (u >> 1), side = u & 1;
    lo[u] = 0;
    len[u] = 0;
    if (r >= w * w) continue;
    const int dy = r % w - K, dz = r / w - K;
    const int z = c.z + dz;
    if (z < 0 || z >= a.nz) continue;
    const int ady = dy < 0 ? -dy : dy, adz = dz < 0 ? -dz : dz;
    const double by = ady > 1 ? (ady - 1) * a.cy : 0.0;
    const double bz = adz > 1 ? (adz - 1) * a.cz : 0.0;
    const double b2 = by * by + bz * bz;
    if (b2 > R2) continue;
    // a point within rx along x of one in cell i lies in a cell within
    // ceil(rx / cx) of i
    const int need = (int)ceil(sqrt(R2 - b2) / a.cx);
    const int kx = need < K ? need : K;
    int y = c.y + dy;
    y = y < 0 ? y + a.ny : (y >= a.ny ? y - a.ny : y);
    const int x0 = c.x - kx, x1 = c.x + kx;
    int xa = 0, xb = -1;
    if (x0 < 0) {
      xa = side == 0 ? x0 + a.nx : 0;
      xb = side == 0 ? a.nx - 1 : x1;
    } else if (x1 >= a.nx) {
      xa = side == 0 ? x0 : 0;
      xb = side == 0 ? a.nx - 1 : x1 - a.nx;
    } else if (side == 0) {
      xa = x0;
      xb = x1;
    }
    if (xb < xa) continue;
    const int base = (z * a.ny + y) * a.nx;
    lo[u] = cnt[base + xa];
    len[u] = cnt[base + xb + 1] - lo[u];
  }
  // exclusive prefix of the run lengths in run order
  const int32_t mine = (len[0] + len[1]) + (len[2] + len[3]);
  int32_t incl = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const int32_t T = __shfl(incl, 63, 64);
  int32_t run = incl - mine;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    s_lo[4 * lane + u] = lo[u];
    s_pre[4 * lane + u] = run;
    run += len[u];
  }
  if (lane == 63) s_pre[kSegMax] = T;
  __syncthreads();
  for (int32_t c0 = lane; c0 < T; c0 += 256) {
    int32_t p[4];
    bool v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t cc = c0 + 64 * u;
      v[u] = cc < T;
      // the last run whose prefix is <= cc (runs of length 0 share a
      // prefix with the next one; the search lands on the last of them)
      int sg = 0;
      for (int step = kSegMax / 2; step >= 1; step >>= 1)
        if (s_pre[sg + step] <= cc) sg += step;
      p[u] = v[u] ? s_lo[sg] + (cc - s_pre[sg]) : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) f(p[u], v[u]);
  }
  __syncthreads();
}

// Squared minimum-image distance in the order dist_mi sums it (its root is
// dist_mi's value).
__device__ inline double dist2_mi(const DevMesh& m, double cx, double cy, double cz,
                                  double x, double y, double z) {
  double dx = cx - x, dy = cy - y;
  const double dz = cz - z;
  if (dx > 0.5 * m.Lx) dx -= m.Lx;
  else if (dx < -0.5 * m.Lx) dx += m.Lx;
  if (dy > 0.5 * m.Ly) dy -= m.Ly;
  else if (dy < -0.5 * m.Ly) dy += m.Ly;
  return (dx * dx + dy * dy) + dz * dz;
}

// The kept-pair test is the same in both passes: t = d - d_f,min <= cut with
// d = dist_mi(face centroid, atom).  Squared distances screen out the pairs
// beyond it (with a relative margin of 1e-12, so the screen never drops a
// kept pair); the root and the weight are taken for the rest only.
constexpr double kScreen = 1.0 + 1e-12;

// One wave per face, the faces taken in cell order (Q_f from k_cut_rank):
// the nearest atom among the 27 cells around the centroid (exact when
// within c_min, else a scan of every atom: a far face), then the sum of the
// kept weights over the cells within reach of d_min + cut (or every atom).
__global__ void __launch_bounds__(kThreads) k_face_charge_cut(ChargeArgs a) {
  __shared__ int32_t s_lo[kThreads / 64][kSegMax];
  __shared__ int32_t s_pre[kThreads / 64][kSegMax + 1];
  const DevMesh& m = a.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // a wave past the last face still takes part in the workgroup barriers
  const int64_t p0 = blockIdx.x * (int64_t)(blockDim.x >> 6) + wv;
  const bool live = p0 < m.n_emit;
  const int64_t pf = live ? p0 : m.n_emit - 1;
  const double cx = a.f_cen[3 * pf], cy = a.f_cen[3 * pf + 1], cz = a.f_cen[3 * pf + 2];
  const Cell3 cc = cell_of(a, cx, cy, cz);
  const double* ax = a.a_xyz;
  double m2 = 1.0 / 0.0;
  wave_block_members(a, a.a_cnt, cc, 1, 1.0 / 0.0, s_lo[wv], s_pre[wv],
                     [&](int32_t p, bool v) {
                       const double d2 = dist2_mi(m, cx, cy, cz, ax[3 * (int64_t)p],
                                                  ax[3 * (int64_t)p + 1],
                                                  ax[3 * (int64_t)p + 2]);
                       m2 = v && d2 < m2 ? d2 : m2;
                     });
  m2 = wave_min_d(m2);
  double dmin = sqrt(m2);
  const bool far = !(dmin <= a.c_min);
  if (far) {
    const double3 c = make_double3(cx, cy, cz);
    for (int64_t j = lane; j < a.n_atoms; j += 64) {
      const double d = dist_mi(m, c, a.atoms + 3 * j);
      dmin = d < dmin ? d : dmin;
    }
    dmin = wave_min_d(dmin);
  }
  const double cut = kCutRc * a.r_c;
  const double bnd = (dmin + cut) * kScreen;
  const double b2 = bnd * bnd;
  double S = 0.0;
  // (every wave takes the walk's barriers; a far face's walk is empty)
  wave_block_members(a, a.a_cnt, cc, far ? 0 : a.K, far ? -1.0 : b2, s_lo[wv], s_pre[wv],
                     [&](int32_t p, bool v) {
                       const double d2 = dist2_mi(m, cx, cy, cz, ax[3 * (int64_t)p],
                                                  ax[3 * (int64_t)p + 1],
                                                  ax[3 * (int64_t)p + 2]);
                       if (v && d2 <= b2) {
                         const double t = sqrt(d2) - dmin;
                         if (t <= cut) S += exp(-t / a.r_c);
                       }
                     });
  if (far) {
    const double3 c = make_double3(cx, cy, cz);
    for (int64_t j = lane; j < a.n_atoms; j += 64) {
      const double t = dist_mi(m, c, a.atoms + 3 * j) - dmin;
      if (t <= cut) S += exp(-t / a.r_c);
    }
  }
  S = wave_sum_d(S);
  if (lane == 0 && live) {
    const int32_t f = a.f_idx[pf];
    a.f_min[f] = dmin;
    a.f_sum[f] = S;
    a.f_min_s[pf] = dmin;
    a.f_sum_s[pf] = S;
    if (far) atomicAdd(a.n_far, 1);
  }
}

// One wave per atom, the atoms taken in cell order: the kept weights of the
// faces within reach of c_min + cut, or, when a face was far, of every face
// (lanes striding over the faces).
__global__ void __launch_bounds__(kThreads) k_atom_charge_cut(ChargeArgs a) {
  __shared__ int32_t s_lo[kThreads / 64][kSegMax];
  __shared__ int32_t s_pre[kThreads / 64][kSegMax + 1];
  const bool any_far = *a.n_far != 0;
  const DevMesh& m = a.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t p0 = blockIdx.x * (int64_t)(blockDim.x >> 6) + wv;
  const bool live = p0 < a.n_atoms;
  const int64_t pa = live ? p0 : a.n_atoms - 1;
  const double at[3] = {a.a_xyz[3 * pa], a.a_xyz[3 * pa + 1], a.a_xyz[3 * pa + 2]};
  const Cell3 cc = cell_of(a, at[0], at[1], at[2]);
  const double cut = kCutRc * a.r_c;
  const double R = a.c_min + cut;
  double q = 0.0;
  wave_block_members(a, a.f_cnt, cc, any_far ? 0 : a.K, any_far ? -1.0 : R * R,
                     s_lo[wv], s_pre[wv], [&](int32_t p, bool v) {
                       const int64_t g = p;
                       const double fm = a.f_min_s[g];
                       const double d2 = dist2_mi(m, a.f_cen[3 * g], a.f_cen[3 * g + 1],
                                                  a.f_cen[3 * g + 2], at[0], at[1], at[2]);
                       const double bd = (fm + cut) * kScreen;
                       if (v && d2 <= bd * bd) {
                         const double t = sqrt(d2) - fm;
                         if (t <= cut) q += (a.f_Q_s[g] * exp(-t / a.r_c)) / a.f_sum_s[g];
                       }
                     });
  if (any_far) {
    for (int64_t g = lane; g < m.n_emit; g += 64) {
      const double3 fc = make_double3(a.f_cen[3 * g], a.f_cen[3 * g + 1], a.f_cen[3 * g + 2]);
      const double t = dist_mi(m, fc, at) - a.f_min_s[g];
      if (t <= cut) q += (a.f_Q_s[g] * exp(-t / a.r_c)) / a.f_sum_s[g];
    }
  }
  q = wave_sum_d(q);
  if (lane == 0 && live) a.atom_q[a.a_idx[pa]] = q;
}

}  // namespace

int charge_splits(int64_t n_emit, int64_t n_atoms, int n_cu) {
  const int64_t blocks = (n_atoms + kThreads - 1) / kThreads;
  int64_t k = ((int64_t)n_cu * 4 + blocks - 1) / (blocks > 0 ? blocks : 1);
  const int64_t tiles = (n_emit + kFaceTile - 1) / kFaceTile;
  if (k > tiles * 4) k = tiles * 4;  // at least a quarter tile per range
  if (k > 1024) k = 1024;
  return (int)(k < 1 ? 1 : k);
}

bool charge_cut_plan(const DevMesh& m, double r_c, ChargeArgs& a) {
  a.cut = 0;
  const double z0 = m.b0[2], z1 = m.b1[2];
  if (!(m.Lx > 0.0 && m.Ly > 0.0 && z1 > z0)) return false;
  double c = 10.0 * r_c;
  int64_t nx, ny, nz;
  for (;;) {
    nx = std::max<int64_t>(1, (int64_t)(m.Lx / c));
    ny = std::max<int64_t>(1, (int64_t)(m.Ly / c));
    nz = std::max<int64_t>(1, (int64_t)((z1 - z0) / c));
    if (nx * ny * nz <= (1 << 20) - 1024) break;
    c *= 1.25;
  }
  const double cx = m.Lx / (double)nx, cy = m.Ly / (double)ny, cz = (z1 - z0) / (double)nz;
  const double c_min = std::min(cx, std::min(cy, cz));
  const double k = std::ceil(kCutRc * r_c / c_min);
  if (!(k <= 16.0)) return false;
  const int K = 1 + (int)k;
  if (K > kCutKMax || nx < 2 * K + 1 || ny < 2 * K + 1) return false;
  a.nx = (int)nx;
  a.ny = (int)ny;
  a.nz = (int)nz;
  a.K = K;
  a.cx = cx;
  a.cy = cy;
  a.cz = cz;
  a.z0 = z0;
  a.c_min = c_min;
  a.n_cells_pad = nx * ny * nz + 1;
  a.cut = 1;
  return true;
}

size_t charge_cut_ints(const ChargeArgs& a, int64_t n_atoms, int64_t n_emit) {
  // per grid: counts and starts (n_cells + 1), then the tile totals
  const int64_t n_cells = (int64_t)a.nx * a.ny * a.nz;
  const int64_t tiles = (n_cells + 1023) / 1024;
  return (size_t)(2 * (n_cells + 1 + tiles) + 4 * n_atoms + 4 * n_emit + 1);
}

hipError_t surface_charge_launch(const ChargeArgs& a, int n_cu, hipStream_t s) {
  if (a.m.n_emit == 0) {
    // no faces: every atom's charge is the empty sum
    if (a.n_atoms > 0) {
      ChargeArgs z = a;
      z.n_split = 0;
      z.cut = 0;
      const int ga = (int)((a.n_atoms + kThreads - 1) / kThreads);
      hipLaunchKernelGGL(k_atom_reduce, dim3(ga), dim3(kThreads), 0, s, z);
    }
    return hipGetLastError();
  }
  auto grid_for = [](int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 4096));
  };
  if (a.cut && a.n_atoms > 0) {
    const int64_t n_cells = (int64_t)a.nx * a.ny * a.nz;
    const int64_t items = a.n_atoms + a.m.n_emit;
    hipLaunchKernelGGL(k_cut_clear, dim3(grid_for(n_cells + 1)), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_cut_bin, dim3(grid_for(items)), dim3(kThreads), 0, s, a);
    const int tiles = (int)((n_cells + 1023) / 1024);
    hipLaunchKernelGGL(k_cut_scan_tiles, dim3(tiles, 2), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_cut_scan_top, dim3(2), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_cut_scan_add, dim3(tiles, 2), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_cut_fill, dim3(grid_for(items)), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_cut_rank, dim3(grid_for(items)), dim3(kThreads), 0, s, a);
    const int per = kThreads / 64;
    hipLaunchKernelGGL(k_face_charge_cut, dim3((int)((a.m.n_emit + per - 1) / per)),
                       dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_atom_charge_cut, dim3((int)((a.n_atoms + per - 1) / per)),
                       dim3(kThreads), 0, s, a);
    return hipGetLastError();
  }
  ChargeArgs b = a;
  b.cut = 0;
  const int gf = (int)(b.m.n_emit < (int64_t)n_cu * 16 ? b.m.n_emit : (int64_t)n_cu * 16);
  hipLaunchKernelGGL(k_face_charge, dim3(gf), dim3(kThreads), 0, s, b);
  if (b.n_atoms > 0) {
    const int ga = (int)((b.n_atoms + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_atom_charge, dim3(ga, b.n_split), dim3(kThreads), 0, s, b);
    hipLaunchKernelGGL(k_atom_reduce, dim3(ga), dim3(kThreads), 0, s, b);
  }
  return hipGetLastError();
}

}  // namespace fp
