// Internal definitions shared by the HIP sources of the PIC library.
// Everything here is compiled for gfx950 with -ffp-contract=off: the
// barycentric and deposition arithmetic is specified operation by operation
// and must not be re-associated or fused.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/femocs_pic.h"

namespace fp {

// ---------------------------------------------------------------------------
// Physical constants (CODATA 2018 base values; derived values computed).
// ---------------------------------------------------------------------------
struct Phys {
  double qm;     // q/m of an electron, nm fs^-2 per V/nm
  double e_eps;  // e/eps0, V nm per elementary charge
  double a_fn;   // A eV V^-2
  double b_fn;   // eV^-3/2 V nm^-1
  double c_s;    // eV^2 V^-1 nm
  double j_unit; // A/m^2 -> e nm^-2 fs^-1
};
Phys phys_constants();  // host

constexpr int kSell = 64;                     // rows per sliced-ELL slice
constexpr double kFx = 1099511627776.0;       // 2^40
constexpr double kFxInv = 1.0 / 1099511627776.0;

// ---------------------------------------------------------------------------
// Device mesh records (one 128-byte line each).
// ---------------------------------------------------------------------------
struct alignas(128) TetWalk {   // vertices (unwrapped) + adjacency
  double v[12];
  int32_t nbr[4];   // neighbour tet, -1 top, -2 metal
  int8_t nsh[8];    // (dx, dy) frame shift when crossing face i
  int32_t pad[2];
};
static_assert(sizeof(TetWalk) == 128, "TetWalk is one line");

// Barycentric map, vertex ids and neighbours: the one record the particle
// loop reads per tet visited.  nbr[k] is the tet across the face opposite
// vertex k in bits 0-27 (kNoNbr when the face is on the boundary), and the
// frame offset (sx + 1, sy + 1) of that tet in bits 28-29 and 30-31.
constexpr uint32_t kNoNbr = 0x0FFFFFFFu;
constexpr int kFineSeed = 4;  // seed sub-cells per bucket edge
constexpr int64_t kMaxTets = kNoNbr;
struct alignas(128) TetGeom {
  double v0[3];
  double m[9];      // rows m1, m2, m3
  int32_t node[4];
  uint32_t nbr[4];
};
static_assert(sizeof(TetGeom) == 128, "TetGeom is one line");

// FP32 copy of the map and vertex ids, for the mixed-precision field
// gather only (the walk and the deposition use TetGeom).
struct alignas(64) TetGeom32 {
  float v0[3];
  float m[9];
  int32_t node[4];
};
static_assert(sizeof(TetGeom32) == 64, "TetGeom32 is half a line");

struct DevMesh {
  int64_t n_nodes, n_tets, n_free, nnz, nnz_field, n_emit;
  double Lx, Ly, z_top;
  const TetWalk* tw;
  const TetGeom* tg;
  const TetGeom32* tg32;
  // Jacobi inverse diagonal of the stiffness on free nodes
  const double* invdiag;
  const float* invdiag32;
  const double* g_unit;      // Neumann load per unit E0 [n_free]
  const int32_t* free2node;  // [n_free]
  const int32_t* node2free;  // [n_nodes], -1 for Dirichlet
  // Stiffness K (rows and columns free nodes) in sliced ELLPACK, kSell rows
  // per slice.  The nodal field operator R (rows all nodes, columns free
  // nodes, three components) has, on a free row, exactly the columns of
  // that row of K: its free rows share K's layout (k_sptr, slot order) with
  // columns given as node ids (k_ncol), so one pass over phi yields both
  // K phi and R phi.  Its Dirichlet rows (dir_nodes order) form a second,
  // small sliced ELLPACK.
  int64_t k_nslices, k_np, d_nslices, d_np;
  const int32_t* k_sptr;   // [k_nslices + 1] slice offsets
  const int32_t* k_scol;   // free-index columns
  const int32_t* k_ncol;   // the same columns as node ids
  const double* k_sval;
  const float* k_sval32;
  const double* r_sval;    // [3][k_np] R on the free rows
  const float* r_sval32;   // [3][k_np]
  const int32_t* d_sptr;   // [d_nslices + 1]
  const int32_t* d_ncol;   // node-id columns
  const double* d_sval;    // [3][d_np] R on the Dirichlet rows
  const float* d_sval32;   // [3][d_np]
  const double4* f_rowsum; // [n_nodes] FP64 row sums of R (w unused)
  // R^T (rows free nodes j, entries R_ij): the part over free i in K's
  // layout (slot of (j, i) holds R_ij), the part over Dirichlet i in a
  // sliced ELLPACK of its own over the free rows
  const double* rt_sval;   // [3][k_np]
  int64_t t_nslices, t_np;
  const int32_t* t_sptr;
  const int32_t* t_ncol;   // Dirichlet node ids
  const double* t_sval;    // [3][t_np]
  // emitting faces
  const int32_t* e_tet;
  const int32_t* e_nodes;    // [3*n_emit]
  const double* e_abc;       // [9*n_emit]
  const double* e_area;
  const double* e_nrm;       // [3*n_emit], into the vacuum
  // nodes of the emitting faces and, per node, its faces in ascending order
  int64_t en_n;
  const int32_t* en_node;    // [en_n]
  const int32_t* en_ptr;     // [en_n + 1]
  const int32_t* en_face;    // [en_ptr[en_n]]
  // bucket grid
  int32_t nb[3];
  double b0[3], b1[3], binv[3];
  const int32_t* bstart;     // [nbx*nby*nbz + 1]
  const int32_t* bitem;
  const int32_t* bseed;      // [nbx*nby*nbz] walk seed per bucket or -1
  // walk seeds on a grid kFineSeed times finer: the tet holding each
  // sub-cell centre (or the coarse seed where the centre is in the metal)
  int32_t fnb[3];
  double finv[3];
  int32_t* fseed;            // [fnb_x*fnb_y*fnb_z]
  double jump_len2;          // displacements beyond this start at the seed
  double lam_c;              // bound factor of the barycentric inside test
};

// Virtual workgroup: index and count within the grid of one instance.  A
// single-instance launch uses (blockIdx.x, gridDim.x); a batched launch
// maps its blocks onto the instances with a schedule table.
struct VB {
  int id, n;
};

// Schedule of a batched launch: segment j (instance inst[j]) owns blocks
// [off[j], off[j+1]).  Offsets and counts are multiples of 8 so that a
// block's XCD (block index mod 8) is its virtual index mod 8.
constexpr int kMaxBatch = 64;
struct BatchMap {
  int32_t n_seg;
  int32_t off[kMaxBatch + 1];
  int8_t inst[kMaxBatch];
};

__device__ inline VB batch_block(const BatchMap& b, int& inst) {
  const int g = (int)blockIdx.x;
  int j = 0;
  while (j + 1 < b.n_seg && b.off[j + 1] <= g) ++j;
  inst = b.inst[j];
  VB v;
  v.id = g - b.off[j];
  v.n = b.off[j + 1] - b.off[j];
  return v;
}

// ---------------------------------------------------------------------------
// Error-free transformations and orientation predicates.
// ---------------------------------------------------------------------------
__host__ __device__ inline void ef_sum(double a, double b, double& s,
                                       double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__host__ __device__ inline void ef_prod(double a, double b, double& p,
                                        double& e) {
  p = a * b;
  e = fma(a, b, -p);
}

// Floating-point vol6(a,b,c,d) = det[b-a; c-a; d-a] and the static error
// bound (7 + 56 u) u * permanent of Shewchuk's orient3d filter: when
// |det| > bound the sign of det is the sign of the exact determinant.
__host__ __device__ inline double vol6_filtered(const double* a,
                                                const double* b,
                                                const double* c,
                                                const double* d,
                                                double& bound) {
  const double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
  const double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
  const double wx = d[0] - a[0], wy = d[1] - a[1], wz = d[2] - a[2];
  const double m1 = vy * wz, m2 = vz * wy;
  const double m3 = vz * wx, m4 = vx * wz;
  const double m5 = vx * wy, m6 = vy * wx;
  const double det = ux * (m1 - m2) + uy * (m3 - m4) + uz * (m5 - m6);
  const double perm = (fabs(m1) + fabs(m2)) * fabs(ux) +
                      (fabs(m3) + fabs(m4)) * fabs(uy) +
                      (fabs(m5) + fabs(m6)) * fabs(uz);
  const double u = 1.1102230246251565e-16;  // 2^-53
  bound = (7.0 + 56.0 * u) * u * perm;
  return det;
}

// Exact sign of det[b-a; c-a; d-a]: the three difference vectors are split
// into exact two-term sums (x = hi + lo), the determinant is expanded
// multilinearly into 6 x 8 triple products, each turned into four doubles
// that sum to it exactly, and all of them are accumulated into one
// nonoverlapping expansion (Shewchuk 1997, Grow-Expansion with zero
// elimination).  The sign of the largest component is the answer.  When
// every difference is exact (all low parts zero, the usual case for a point
// near the tet) only the 6 products of high parts are nonzero, and the
// expansion stays short.
// The case without low parts: the determinant is exactly the sum of 24
// doubles (six triple products, each split exactly into four).  Its sign by
// distillation (iterated VecSum, Ogita, Rump and Oishi 2005): a cascade of
// error-free sums keeps the exact total while concentrating it in the last
// element S; once S exceeds the sum R of the others' magnitudes (with a
// margin for the rounding of R), the sign of S is that of the total.
// Every index is fixed at compile time, so the terms stay in registers.
// Returns 2 when 64 passes do not decide (the caller falls back to the
// general expansion).
__host__ __device__ inline int vol6_sign_exact_short(const double (*U)[2],
                                                     const double (*V)[2],
                                                     const double (*W)[2]) {
  const int P[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1},
                       {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
  double t[24];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const double sg = s < 3 ? 1.0 : -1.0;
    double p, e, p1, e1, p2, e2;
    ef_prod(U[P[s][0]][0], V[P[s][1]][0], p, e);
    ef_prod(p, W[P[s][2]][0], p1, e1);
    ef_prod(e, W[P[s][2]][0], p2, e2);
    t[4 * s] = sg * p1;
    t[4 * s + 1] = sg * e1;
    t[4 * s + 2] = sg * p2;
    t[4 * s + 3] = sg * e2;
  }
  const double margin = 1.0 + 64.0 * 1.1102230246251565e-16;
  for (int pass = 0; pass < 64; ++pass) {
#pragma unroll
    for (int i = 0; i < 23; ++i) {
      double sum, err;
      ef_sum(t[i], t[i + 1], sum, err);
      t[i] = err;
      t[i + 1] = sum;
    }
    double R = 0.0;
#pragma unroll
    for (int i = 0; i < 23; ++i) R += fabs(t[i]);
    const double S = t[23];
    if (R == 0.0) return S > 0.0 ? 1 : (S < 0.0 ? -1 : 0);
    if (fabs(S) > R * margin) return S > 0.0 ? 1 : -1;
  }
  return 2;
}

__host__ __device__ inline int vol6_sign_exact(const double* a,
                                               const double* b,
                                               const double* c,
                                               const double* d) {
  double U[3][2], V[3][2], W[3][2];
  bool tails = false;
  for (int k = 0; k < 3; ++k) {
    ef_sum(b[k], -a[k], U[k][0], U[k][1]);
    ef_sum(c[k], -a[k], V[k][0], V[k][1]);
    ef_sum(d[k], -a[k], W[k][0], W[k][1]);
    tails = tails || U[k][1] != 0.0 || V[k][1] != 0.0 || W[k][1] != 0.0;
  }
  if (!tails) {
    const int sg = vol6_sign_exact_short(U, V, W);
    if (sg != 2) return sg;
  }
  // permutations of (x, y, z) for rows (U, V, W) and their signs
  const int P[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1},
                       {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
  double ex[200];
  int len = 0;
  const int nh = tails ? 8 : 1;
  for (int s = 0; s < 6; ++s) {
    const double sg = s < 3 ? 1.0 : -1.0;
    for (int h = 0; h < nh; ++h) {
      const double f0 = U[P[s][0]][h & 1];
      const double f1 = V[P[s][1]][(h >> 1) & 1];
      const double f2 = W[P[s][2]][(h >> 2) & 1];
      double p, e, p1, e1, p2, e2;
      ef_prod(f0, f1, p, e);
      ef_prod(p, f2, p1, e1);
      ef_prod(e, f2, p2, e2);
      const double t[4] = {p1, e1, p2, e2};
      for (int q = 0; q < 4; ++q) {
        double acc = sg * t[q];
        if (acc == 0.0) continue;
        // in-place grow: output index never passes the input index
        int out = 0;
        for (int i = 0; i < len; ++i) {
          double sum, err;
          ef_sum(acc, ex[i], sum, err);
          acc = sum;
          if (err != 0.0) ex[out++] = err;
        }
        if (acc != 0.0 || out == 0) ex[out++] = acc;
        len = out;
      }
    }
  }
  for (int i = len - 1; i >= 0; --i) {
    if (ex[i] > 0.0) return 1;
    if (ex[i] < 0.0) return -1;
  }
  return 0;
}

__host__ __device__ inline int vol6_sign(const double* a, const double* b,
                                         const double* c, const double* d) {
  double bound;
  const double det = vol6_filtered(a, b, c, d, bound);
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return vol6_sign_exact(a, b, c, d);
}

// ---------------------------------------------------------------------------
// Philox4x64-10 counter-based generator (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
__host__ __device__ inline void philox4x64_10(uint64_t k0, uint64_t k1,
                                              uint64_t c0, uint64_t c1,
                                              uint64_t c2, uint64_t c3,
                                              uint64_t out[4]) {
  for (int r = 0; r < 10; ++r) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint64_t h0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
    const uint64_t h1 = __umul64hi(0xCA5A826395121157ull, c2);
#else
    const uint64_t h0 = (uint64_t)(((unsigned __int128)0xD2E7470EE14C6C93ull * c0) >> 64);
    const uint64_t h1 = (uint64_t)(((unsigned __int128)0xCA5A826395121157ull * c2) >> 64);
#endif
    const uint64_t l0 = 0xD2E7470EE14C6C93ull * c0;
    const uint64_t l1 = 0xCA5A826395121157ull * c2;
    const uint64_t n0 = h1 ^ c1 ^ k0;
    const uint64_t n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__host__ __device__ inline double unit_double(uint64_t w) {
  return (double)(w >> 11) * 1.1102230246251565e-16;
}

// ---------------------------------------------------------------------------
// Barycentric coordinates in a tet (the fixed arithmetic shared with the
// deposition rule): d = p - v0, l_k = (m_k.x d.x + m_k.y d.y) + m_k.z d.z,
// l_0 = ((1 - l_1) - l_2) - l_3.
// ---------------------------------------------------------------------------
__host__ __device__ inline void barycentric(const TetGeom& g, double px,
                                            double py, double pz,
                                            double lam[4]) {
  const double dx = px - g.v0[0], dy = py - g.v0[1], dz = pz - g.v0[2];
  const double l1 = (g.m[0] * dx + g.m[1] * dy) + g.m[2] * dz;
  const double l2 = (g.m[3] * dx + g.m[4] * dy) + g.m[5] * dz;
  const double l3 = (g.m[6] * dx + g.m[7] * dy) + g.m[8] * dz;
  lam[0] = ((1.0 - l1) - l2) - l3;
  lam[1] = l1;
  lam[2] = l2;
  lam[3] = l3;
}

__host__ __device__ inline int64_t fx_round(double x) {
  return (int64_t)rint(x);
}

// Fixed-point split of one particle's charge over its four vertices.
__host__ __device__ inline void charge_split(const double lam[4], double w,
                                             int64_t q[4]) {
  q[1] = fx_round((lam[1] * w) * kFx);
  q[2] = fx_round((lam[2] * w) * kFx);
  q[3] = fx_round((lam[3] * w) * kFx);
  q[0] = fx_round(w * kFx) - ((q[1] + q[2]) + q[3]);
}

// Bucket index along one axis: a monotone map, shared by registration and
// query, so a tet registered from its closed bounding box is found by every
// point it holds.
__host__ __device__ inline int bucket_axis(double x, double x0, double inv,
                                           int n) {
  const double f = floor((x - x0) * inv);
  if (f < 0.0) return 0;
  if (f > (double)(n - 1)) return n - 1;
  return (int)f;
}

// Sum of the per-workgroup counter rows of one step into its stats record
// (rows: [12][n_rows], field-major; counter k = 11 is a maximum, the
// others are sums -- integers, so the order does not matter): one
// workgroup per counter, any block size up to 1024.
constexpr int kStepCounters = 12;
__device__ inline void step_counter_sum(const int64_t* rows, int n_rows,
                                        pic_step_stats* st, int k) {
  __shared__ long long part[16];
  const bool is_max = k == kStepCounters - 1;
  long long s = 0;
  for (int r = threadIdx.x; r < n_rows; r += blockDim.x) {
    const long long v = rows[(int64_t)k * n_rows + r];
    s = is_max ? (v > s ? v : s) : s + v;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const long long o = __shfl_xor(s, off, 64);
    s = is_max ? (o > s ? o : s) : s + o;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w)
      t = is_max ? (part[w] > t ? part[w] : t) : t + part[w];
    int64_t* dst[kStepCounters] = {&st->n_before, &st->q_before, &st->n_anode,
                                   &st->q_anode,  &st->n_after,  &st->q_after,
                                   &st->n_cathode, &st->q_cathode, &st->n_inj,
                                   &st->q_inj,    &st->walk_steps, &st->walk_max};
    *dst[k] = t;
  }
}

// Internal per-handle device scratch layout (counters and scalars).
struct StepScratch {
  // counters used by the particle kernels of one step
  int32_t n_fallback;
  int32_t inj_base;
  int32_t inj_total;
  int32_t inj_fit;
  int32_t n_live;
  int32_t emitted;  // set once the emission counts of the step are published
  int32_t pad[2];
};

}  // namespace fp
