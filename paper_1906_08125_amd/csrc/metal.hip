// Metal-side solves (Sec. II D, weak forms of App. C and App. D): P1
// assembly of the continuity and heat systems in CSR form on the device,
// Joule heating, and a Jacobi-preconditioned CG in FP64.
//
// The metal mesh is small next to the vacuum mesh and its systems change
// every call (sigma, kappa(T), dt), so the design favours a deterministic
// one-pass assembly over reuse: one thread per matrix row walks the
// elements incident to its node (ascending element id) and accumulates the
// row in place, the right-hand side included, so no atomics and no
// run-to-run rounding differences.  Every reduction of the CG is two-level
// (workgroup tree, then every workgroup sums the partials in the same fixed
// order), so every workgroup sees the same scalars.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "metal.h"

namespace fp {
namespace {

constexpr int kMB = 256;       // threads per workgroup
constexpr int kMaxG = 1024;    // workgroups of the row-loop kernels
constexpr int kMaxS = 65536;   // workgroups of the product (a row per thread)
constexpr int kChunk = 24;     // CG iterations before the first host check
constexpr int kChunkBig = 96;  // and between the later ones

struct MetalCtrl {
  double gam[2];     // r.z of the last two iterations (by parity)
  double alpha[2];   // step lengths of the last two iterations (by parity)
  double bb;         // ||b||^2 over the free rows
  double rr;         // ||r||^2 of the last iterate tested
  double tol2;
  // iterations completed: written by k_cg_step and read by k_cg_spmv,
  // whose workgroup 0 copies it to it_cur for the next k_cg_step, so that
  // no kernel reads a counter that its own launch writes
  int64_t iters;
  int64_t it_cur;
  int32_t done;
  int32_t pad;
};

// Element record: shape-function gradients g_a (a = 0..3) and the volume.
struct alignas(128) MetalTet {
  double g[12];
  double vol;
  double pad[3];
};

__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kMB / 64; ++k) s += sh[k];
  return s;   // valid in thread 0
}

__global__ void k_geom(const double* __restrict__ xyz,
                       const int32_t* __restrict__ tet, int64_t nt,
                       MetalTet* __restrict__ out, int32_t* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (t >= nt) return;
  double p[4][3];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) p[a][c] = xyz[3 * (int64_t)tet[4 * t + a] + c];
  double e[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) e[a][c] = p[a + 1][c] - p[0][c];
  // rows of the inverse of the edge matrix: g_a = (e_b x e_c) / det
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double c1[3], c2[3], c3[3];
  cross(e[1], e[2], c1);
  cross(e[2], e[0], c2);
  cross(e[0], e[1], c3);
  const double det = e[0][0] * c1[0] + e[0][1] * c1[1] + e[0][2] * c1[2];
  MetalTet r;
  if (!(det != 0.0) || !std::isfinite(det)) {
    atomicAdd(bad, 1);
    for (int k = 0; k < 12; ++k) r.g[k] = 0.0;
    r.vol = 0.0;
  } else {
    for (int c = 0; c < 3; ++c) {
      r.g[3 + c] = c1[c] / det;
      r.g[6 + c] = c2[c] / det;
      r.g[9 + c] = c3[c] / det;
      r.g[c] = -(r.g[3 + c] + r.g[6 + c] + r.g[9 + c]);
    }
    r.vol = fabs(det) / 6.0;
  }
  r.pad[0] = r.pad[1] = r.pad[2] = 0.0;
  out[t] = r;
}

struct AsmArgs {
  int64_t n;
  const int32_t* row_ptr;
  const int32_t* inc_ptr;
  const int32_t* inc_pos;   // [4] CSR positions per incidence
  const int32_t* fin_ptr;
  const int32_t* fin_face;
  const int32_t* tet;
  const int32_t* face;
  const double* xyz;
  const MetalTet* geo;
  const uint8_t* dir;
  const double* sigma;
  const double* flux;       // face flux (J_n or P_N)
  const double* PJ;         // volume source or null
  const double* T;          // heat: T^n; continuity: null
  double L, Cv, dt, theta;
  const int32_t* elem_inc;  // [4 n_tets] incidence of each element's nodes
  double* stage;            // [5 incidences] element contributions
  double* A;
  double* b;
  double* dinv;
  int64_t nt;
};

__device__ double face_area(const double* xyz, const int32_t* f) {
  double p[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) p[a][c] = xyz[3 * (int64_t)f[a] + c];
  const double u0 = p[1][0] - p[0][0], u1 = p[1][1] - p[0][1], u2 = p[1][2] - p[0][2];
  const double v0 = p[2][0] - p[0][0], v1 = p[2][1] - p[0][1], v2 = p[2][2] - p[0][2];
  const double w0 = u1 * v2 - u2 * v1, w1 = u2 * v0 - u0 * v2, w2 = u0 * v1 - u1 * v0;
  return 0.5 * sqrt(w0 * w0 + w1 * w1 + w2 * w2);
}

// One element per thread: its contributions to the rows of its four nodes
// (continuity: K(sigma); heat: C/dt + theta K(kappa), and the right-hand
// side (C/dt - (1 - theta) K) T^n + int N_a P_J), staged per incidence
// (four matrix entries and one right-hand-side value).
__global__ void k_element(AsmArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (t >= a.nt) return;
  const MetalTet G = a.geo[t];
  int32_t nd[4];
  for (int c = 0; c < 4; ++c) nd[c] = a.tet[4 * t + c];
  const bool heat = a.T != nullptr;
  double Tn[4] = {0.0, 0.0, 0.0, 0.0};
  double kw, mw = 0.0, pj = 0.0;
  if (heat) {
    for (int c = 0; c < 4; ++c) Tn[c] = a.T[nd[c]];
    const double Tbar = (Tn[0] + Tn[1] + Tn[2] + Tn[3]) / 4.0;
    kw = a.L * a.sigma[t] * Tbar * G.vol;
    mw = a.Cv * G.vol / 20.0 / a.dt;
    if (a.PJ) pj = a.PJ[t] * G.vol / 4.0;
  } else {
    kw = a.sigma[t] * G.vol;
  }
  for (int l = 0; l < 4; ++l) {
    const double* gl = &G.g[3 * l];
    double* out = a.stage + 5 * (int64_t)a.elem_inc[4 * t + l];
    double b = pj;
    for (int c = 0; c < 4; ++c) {
      const double* gc = &G.g[3 * c];
      const double kab = kw * (gl[0] * gc[0] + gl[1] * gc[1] + gl[2] * gc[2]);
      if (heat) {
        const double mab = c == l ? 2.0 * mw : mw;
        out[c] = mab + a.theta * kab;
        b += (mab - (1.0 - a.theta) * kab) * Tn[c];
      } else {
        out[c] = kab;
      }
    }
    out[4] = b;
  }
}

// One row per thread: the staged contributions of its node's elements,
// added in ascending element order, and the face loads.  A row of up to
// kRowLds entries (15 for an interior node of a Kuhn mesh) is accumulated
// in the thread's LDS slot and written once; longer rows in place.
constexpr int kRowLds = 16;

__global__ void __launch_bounds__(kMB) k_assemble(AsmArgs a, double dir_value) {
  __shared__ double acc[kMB][kRowLds + 1];
  const int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (i >= a.n) return;
  const int32_t r0 = a.row_ptr[i], r1 = a.row_ptr[i + 1];
  double b = 0.0;
  if (r1 - r0 <= kRowLds) {
    double* row = acc[threadIdx.x];
    for (int k = 0; k < r1 - r0; ++k) row[k] = 0.0;
    for (int32_t q = a.inc_ptr[i]; q < a.inc_ptr[i + 1]; ++q) {
      const double* st = a.stage + 5 * (int64_t)q;
      const int32_t* ps = a.inc_pos + 4 * (int64_t)q;
      for (int c = 0; c < 4; ++c) row[ps[c] - r0] += st[c];
      b += st[4];
    }
    for (int k = 0; k < r1 - r0; ++k) a.A[r0 + k] = row[k];
  } else {
    for (int32_t k = r0; k < r1; ++k) a.A[k] = 0.0;
    for (int32_t q = a.inc_ptr[i]; q < a.inc_ptr[i + 1]; ++q) {
      const double* st = a.stage + 5 * (int64_t)q;
      for (int c = 0; c < 4; ++c) a.A[a.inc_pos[4 * (int64_t)q + c]] += st[c];
      b += st[4];
    }
  }
  for (int32_t q = a.fin_ptr[i]; q < a.fin_ptr[i + 1]; ++q) {
    const int32_t f = a.fin_face[q];
    b += a.flux[f] * face_area(a.xyz, &a.face[3 * (int64_t)f]) / 3.0;
  }
  a.b[i] = a.dir[i] ? dir_value : b;
}

// Second pass over the rows: Dirichlet rows become identity rows, the
// Dirichlet columns of free rows move to the right-hand side, and the
// inverse diagonal of the Jacobi preconditioner.
__global__ void k_eliminate(int64_t n, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col,
                            const uint8_t* __restrict__ dir, double dir_value,
                            double* __restrict__ A, double* __restrict__ b,
                            double* __restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (i >= n) return;
  const int32_t r0 = row_ptr[i], r1 = row_ptr[i + 1];
  if (dir[i]) {
    for (int32_t k = r0; k < r1; ++k) A[k] = col[k] == i ? 1.0 : 0.0;
    dinv[i] = 1.0;
    return;
  }
  double bi = b[i], d = 0.0;
  for (int32_t k = r0; k < r1; ++k) {
    const int32_t j = col[k];
    if (dir[j]) {
      bi -= A[k] * dir_value;
      A[k] = 0.0;
    } else if (j == i) {
      d = A[k];
    }
  }
  b[i] = bi;
  dinv[i] = 1.0 / d;
}

struct CgArgsM {
  int64_t n;
  const int32_t* row_ptr;
  const int32_t* col;
  const double* A;
  // the same matrix in sliced ELLPACK for the product: slices of 64 rows,
  // column-major inside a slice (entry k of row 64 s + l at
  // sptr[s] + 64 k + l), rows padded with zero entries
  const int32_t* sptr;
  const int32_t* scol;
  const double* sval;
  const double* b;
  const double* dinv;
  const uint8_t* dir;
  double dir_value;
  double tol2;       // read by k_cg_init only (the others read ctrl->tol2)
  double *x, *r, *z, *p, *s, *w;
  double* part;      // [3][kMaxS]
  int Gs;            // workgroups of the product
  MetalCtrl* ctrl;
  int G;
};


// Sums nv arrays of nparts partials (stride kMaxS) in index order in one
// workgroup: every reduction of the solver has the same fixed order.
__device__ double sum_fixed(const double* part, int nparts, double* sh, double* bc) {
  double v = 0.0;
#pragma unroll 8
  for (int k = threadIdx.x; k < nparts; k += kMB) v += part[k];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) *bc = s;
  __syncthreads();
  const double r = *bc;
  __syncthreads();
  return r;
}

// The three sums of nparts partials each (arrays at stride kMaxS), in the
// same fixed order as sum_fixed, in one pass: every workgroup gets the
// same values.
__device__ void sum3_fixed(const double* part, int nparts, double out[3]) {
  __shared__ double sh[3][kMB / 64];
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nparts; k += kMB) {
    v[0] += part[k];
    v[1] += part[kMaxS + k];
    v[2] += part[2 * kMaxS + k];
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int j = 0; j < 3; ++j) v[j] += __shfl_down(v[j], o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
    for (int j = 0; j < 3; ++j) sh[j][w] = v[j];
  __syncthreads();
  for (int j = 0; j < 3; ++j) {
    double t = 0.0;
    for (int k = 0; k < kMB / 64; ++k) t += sh[j][k];
    out[j] = t;
  }
  __syncthreads();
}

__global__ void k_cg_dir(CgArgsM a) {
  for (int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x; i < a.n;
       i += (int64_t)a.G * kMB)
    if (a.dir[i]) a.x[i] = a.dir_value;
}

// r = b - A x, z = D^-1 r on free rows (zero on Dirichlet rows), partials
// of b.b; resets the control word
__global__ void k_cg_init(CgArgsM a) {
  __shared__ double sh[kMB / 64];
  double bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x; i < a.n;
       i += (int64_t)a.G * kMB) {
    double ri = 0.0;
    if (!a.dir[i]) {
      const double bi = a.b[i];
      double ax = 0.0;
      for (int32_t k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k)
        ax += a.A[k] * a.x[a.col[k]];
      ri = bi - ax;
      bb += bi * bi;
    }
    a.r[i] = ri;
    a.z[i] = ri * a.dinv[i];
  }
  const double s = block_sum(bb, sh);
  if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

// One workgroup: ||b||^2 from the partials of k_cg_init, and the control
// word reset for a new solve.
__global__ void k_cg_start(CgArgsM a) {
  __shared__ double sh[kMB / 64];
  __shared__ double bc;
  const double bb = sum_fixed(a.part, a.G, sh, &bc);
  if (threadIdx.x == 0) {
    a.ctrl->bb = bb;
    a.ctrl->tol2 = a.tol2;
    a.ctrl->iters = 0;
    a.ctrl->it_cur = 0;
    a.ctrl->done = 0;
  }
}

// The control word's done flag as one value for the whole workgroup (block
// 0 of k_cg_step may set it while other workgroups start).
__device__ bool block_done(const MetalCtrl* c) {
  __shared__ int d;
  if (threadIdx.x == 0) d = __atomic_load_n(&c->done, __ATOMIC_RELAXED);
  __syncthreads();
  const bool r = d != 0;
  __syncthreads();
  return r;
}

// w = A z (one row per lane, 64-row slices of the sliced-ELLPACK copy, so
// that every load of a wave is contiguous; entries summed in row order,
// the padding adding zeros) and the partials of r.z, w.z and r.r; the
// iteration counter for k_cg_step
__global__ void k_cg_spmv(CgArgsM a) {
  if (block_done(a.ctrl)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->it_cur = a.ctrl->iters;
  __shared__ double sh[kMB / 64];
  double gz = 0.0, wz = 0.0, rr = 0.0;
  const int lane = threadIdx.x & 63;
  const int64_t ns = (a.n + 63) / 64;
  for (int64_t sl = (int64_t)blockIdx.x * (kMB / 64) + (threadIdx.x >> 6); sl < ns;
       sl += (int64_t)gridDim.x * (kMB / 64)) {
    const int32_t p0 = a.sptr[sl], p1 = a.sptr[sl + 1];
    double v = 0.0;
    int32_t q = p0 + lane;
    for (; q + 3 * 64 < p1; q += 4 * 64) {
      int32_t c[4];
      double av[4], zv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c[u] = a.scol[q + 64 * u];
        av[u] = a.sval[q + 64 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) zv[u] = a.z[c[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) v += av[u] * zv[u];
    }
    for (; q < p1; q += 64) v += a.sval[q] * a.z[a.scol[q]];
    const int64_t i = sl * 64 + lane;
    if (i < a.n) {
      const double ri = a.r[i], zi = a.z[i];
      a.w[i] = v;
      gz += ri * zi;
      wz += v * zi;
      rr += ri * ri;
    }
  }
  const double s0 = block_sum(gz, sh);
  const double s1 = block_sum(wz, sh);
  const double s2 = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = s0;
    a.part[kMaxS + blockIdx.x] = s1;
    a.part[2 * kMaxS + blockIdx.x] = s2;
  }
}

// The assembled (and eliminated) values into the sliced-ELLPACK copy.
__global__ void k_to_sell(int64_t nnz, const int32_t* __restrict__ c2s,
                          const double* __restrict__ A, double* __restrict__ sval) {
  for (int64_t k = (int64_t)blockIdx.x * kMB + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * kMB)
    sval[c2s[k]] = A[k];
}

// One iteration of the single-reduction (Chronopoulos-Gear) form of
// Jacobi-preconditioned CG: from gamma = r.z, delta = (A z).z,
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
//   (beta = 0, alpha = gamma / delta at the first iteration),
//   p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s, z = D^-1 r.
// The residual of the incoming iterate is tested first.  Every workgroup
// sums the product's partials itself, in the same fixed order (no
// reduction launch between the product and the step).
__global__ void k_cg_step(CgArgsM a) {
  if (block_done(a.ctrl)) return;
  const int64_t it = a.ctrl->it_cur;
  double red[3];
  sum3_fixed(a.part, a.Gs, red);
  const double gam = red[0], del = red[1], rr = red[2];
  const double bb = a.ctrl->bb;
  if (bb == 0.0 || rr <= a.ctrl->tol2 * bb) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.ctrl->rr = rr;
      a.ctrl->iters = it;
      a.ctrl->done = 1;
    }
    return;
  }
  double alpha, beta;
  if (it == 0) {
    beta = 0.0;
    alpha = gam / del;
  } else {
    beta = gam / a.ctrl->gam[it & 1];
    alpha = gam / (del - beta * gam / a.ctrl->alpha[it & 1]);
  }
  for (int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x; i < a.n;
       i += (int64_t)a.G * kMB) {
    // p and s hold nothing yet at the first iteration (not even zeros)
    const double pi = it == 0 ? a.z[i] : a.z[i] + beta * a.p[i];
    const double si = it == 0 ? a.w[i] : a.w[i] + beta * a.s[i];
    a.p[i] = pi;
    a.s[i] = si;
    a.x[i] += alpha * pi;
    const double ri = a.r[i] - alpha * si;
    a.r[i] = ri;
    a.z[i] = ri * a.dinv[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctrl->gam[(it + 1) & 1] = gam;
    a.ctrl->alpha[(it + 1) & 1] = alpha;
    a.ctrl->rr = rr;
    a.ctrl->iters = it + 1;
  }
}

// A zero right-hand side has the zero solution on the free rows.
__global__ void k_cg_zero(CgArgsM a) {
  for (int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x; i < a.n;
       i += (int64_t)a.G * kMB)
    if (!a.dir[i]) a.x[i] = 0.0;
}

__global__ void k_joule(int64_t nt, const int32_t* __restrict__ tet,
                        const MetalTet* __restrict__ geo,
                        const double* __restrict__ sigma,
                        const double* __restrict__ phi, double* __restrict__ pj) {
  const int64_t t = (int64_t)blockIdx.x * kMB + threadIdx.x;
  if (t >= nt) return;
  const MetalTet& G = geo[t];
  double g[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 4; ++a) {
    const double v = phi[tet[4 * t + a]];
    for (int c = 0; c < 3; ++c) g[c] += v * G.g[3 * a + c];
  }
  pj[t] = sigma[t] * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kMB - 1) / kMB); }

}  // namespace

struct MetalImpl {
  int64_t n = 0, nt = 0, nf = 0, nnz = 0, ninc = 0, nfin = 0;
  double *xyz = nullptr, *A = nullptr, *b = nullptr, *dinv = nullptr;
  double *r = nullptr, *z = nullptr, *p = nullptr, *sv = nullptr, *w = nullptr;
  double* part = nullptr;
  int32_t *tet = nullptr, *face = nullptr, *row_ptr = nullptr, *col = nullptr;
  int32_t *sptr = nullptr, *scol = nullptr, *c2s = nullptr;  // sliced ELLPACK
  double* sval = nullptr;
  int64_t nsell = 0;
  int32_t *inc_ptr = nullptr, *inc_pos = nullptr;
  int32_t *fin_ptr = nullptr, *fin_face = nullptr;
  int32_t* elem_inc = nullptr;
  double* stage = nullptr;
  uint8_t* dir = nullptr;
  double* x = nullptr;           // the iterate (the caller's vector is copied)
  MetalTet* geo = nullptr;
  MetalCtrl* ctrl = nullptr;
  MetalCtrl* hctrl = nullptr;   // pinned host mirror
  int G = 1;
  // kChunk and kChunkBig CG iterations captured once per handle (their
  // kernels read every per-solve value from the control word)
  hipGraph_t graph = nullptr, graph_big = nullptr;
  hipGraphExec_t chunk = nullptr, chunk_big = nullptr;
};

}  // namespace fp

struct pic_metal {
  fp::MetalImpl m;
  std::vector<void*> allocs;
  int device = 0;
};

namespace fp {

namespace {
template <typename T>
hipError_t dalloc(pic_metal* h, T** p, size_t n) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) h->allocs.push_back((void*)*p);
  return e;
}

}  // namespace

pic_status metal_build(const pic_metal_desc* d, hipStream_t s, pic_metal** out,
                       std::string* err) {
  const int64_t n = d->n_nodes, nt = d->n_tets, nf = d->n_faces;
  if (n < 4 || nt < 1 || nf < 0 || !d->xyz || !d->tets || !d->dirichlet ||
      (nf > 0 && !d->faces)) {
    *err = "metal_create: empty mesh or null array";
    return PIC_E_ARG;
  }
  if (n >= (1LL << 31) || nt >= (1LL << 31) / 4 || nf >= (1LL << 31) / 3) {
    *err = "metal_create: mesh too large";
    return PIC_E_ARG;
  }
  for (int64_t k = 0; k < 4 * nt; ++k)
    if (d->tets[k] < 0 || d->tets[k] >= n) {
      *err = "metal_create: element node out of range";
      return PIC_E_ARG;
    }
  for (int64_t k = 0; k < 3 * nf; ++k)
    if (d->faces[k] < 0 || d->faces[k] >= n) {
      *err = "metal_create: face node out of range";
      return PIC_E_ARG;
    }
  for (int64_t k = 0; k < 3 * n; ++k)
    if (!std::isfinite(d->xyz[k])) {
      *err = "metal_create: non-finite coordinate";
      return PIC_E_ARG;
    }
  // node -> element incidences (ascending element id)
  std::vector<int32_t> inc_ptr(n + 1, 0), inc_tet(4 * nt);
  std::vector<int8_t> inc_loc(4 * nt);
  std::vector<int32_t> elem_inc(4 * nt);
  for (int64_t k = 0; k < 4 * nt; ++k) ++inc_ptr[d->tets[k] + 1];
  for (int64_t i = 0; i < n; ++i) inc_ptr[i + 1] += inc_ptr[i];
  {
    std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t t = 0; t < nt; ++t)
      for (int a = 0; a < 4; ++a) {
        const int32_t v = d->tets[4 * t + a];
        elem_inc[4 * t + a] = fill[v];
        inc_tet[fill[v]] = (int32_t)t;
        inc_loc[fill[v]++] = (int8_t)a;
      }
  }
  // CSR pattern: the nodes of the incident elements, sorted
  std::vector<int32_t> row_ptr(n + 1, 0), col;
  col.reserve(16 * n);
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < n; ++i) {
    nb.clear();
    for (int32_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q)
      for (int a = 0; a < 4; ++a) nb.push_back(d->tets[4 * (int64_t)inc_tet[q] + a]);
    if (nb.empty()) nb.push_back((int32_t)i);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    col.insert(col.end(), nb.begin(), nb.end());
    if (col.size() >= (size_t)1 << 31) {
      *err = "metal_create: too many matrix entries";
      return PIC_E_ARG;
    }
    row_ptr[i + 1] = (int32_t)col.size();
  }
  std::vector<int32_t> inc_pos(16 * (size_t)nt);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q)
      for (int a = 0; a < 4; ++a) {
        const int32_t v = d->tets[4 * (int64_t)inc_tet[q] + a];
        const int32_t* lo = col.data() + row_ptr[i];
        const int32_t* hi = col.data() + row_ptr[i + 1];
        inc_pos[4 * (size_t)q + a] = (int32_t)(std::lower_bound(lo, hi, v) - col.data());
      }
  // the sliced-ELLPACK copy of the pattern (64-row slices, column-major,
  // rows padded with their own column and a zero value)
  const int64_t n_sl = (n + 63) / 64;
  std::vector<int32_t> sptr(n_sl + 1, 0);
  for (int64_t sl = 0; sl < n_sl; ++sl) {
    int32_t wmax = 0;
    for (int64_t r = 64 * sl; r < std::min<int64_t>(n, 64 * sl + 64); ++r)
      wmax = std::max(wmax, row_ptr[r + 1] - row_ptr[r]);
    if ((int64_t)sptr[sl] + 64 * (int64_t)wmax >= ((int64_t)1 << 31)) {
      *err = "metal_create: too many matrix entries";
      return PIC_E_ARG;
    }
    sptr[sl + 1] = sptr[sl] + 64 * wmax;
  }
  std::vector<int32_t> scol(std::max<int32_t>(sptr[n_sl], 1), 0), c2s(col.size());
  for (int64_t r = 0; r < 64 * n_sl; ++r) {
    const int64_t sl = r / 64, l = r % 64;
    const int32_t w = (sptr[sl + 1] - sptr[sl]) / 64;
    const int32_t len = r < n ? row_ptr[r + 1] - row_ptr[r] : 0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t q = sptr[sl] + 64 * k + (int32_t)l;
      if (k < len) {
        scol[q] = col[row_ptr[r] + k];
        c2s[row_ptr[r] + k] = q;
      } else {
        scol[q] = r < n ? (int32_t)r : 0;
      }
    }
  }
  // node -> interface faces
  std::vector<int32_t> fin_ptr(n + 1, 0), fin_face(3 * nf);
  for (int64_t k = 0; k < 3 * nf; ++k) ++fin_ptr[d->faces[k] + 1];
  for (int64_t i = 0; i < n; ++i) fin_ptr[i + 1] += fin_ptr[i];
  {
    std::vector<int32_t> fill(fin_ptr.begin(), fin_ptr.end() - 1);
    for (int64_t f = 0; f < nf; ++f)
      for (int a = 0; a < 3; ++a) fin_face[fill[d->faces[3 * f + a]]++] = (int32_t)f;
  }

  pic_metal* h = new pic_metal();
  (void)hipGetDevice(&h->device);
  MetalImpl& M = h->m;
  M.n = n; M.nt = nt; M.nf = nf; M.nnz = (int64_t)col.size(); M.ninc = 4 * nt;
  M.nfin = 3 * nf;
  hipError_t e = hipSuccess;
  auto up = [&](auto** dst, const auto* src, size_t count) {
    if (e != hipSuccess) return;
    e = dalloc(h, dst, count);
    if (e == hipSuccess && count)
      e = hipMemcpyAsync(*dst, src, count * sizeof(**dst), hipMemcpyHostToDevice, s);
  };
  up(&M.xyz, d->xyz, 3 * n);
  up(&M.tet, d->tets, 4 * nt);
  up(&M.face, d->faces, 3 * nf);
  up(&M.dir, d->dirichlet, n);
  up(&M.row_ptr, row_ptr.data(), n + 1);
  up(&M.col, col.data(), col.size());
  up(&M.sptr, sptr.data(), sptr.size());
  up(&M.scol, scol.data(), scol.size());
  up(&M.c2s, c2s.data(), c2s.size());
  M.nsell = (int64_t)scol.size();
  if (e == hipSuccess) e = dalloc(h, &M.sval, (size_t)M.nsell);
  // the padding entries stay zero (only real entries are written per call)
  if (e == hipSuccess) e = hipMemsetAsync(M.sval, 0, sizeof(double) * (size_t)M.nsell, s);
  up(&M.inc_ptr, inc_ptr.data(), n + 1);
  up(&M.inc_pos, inc_pos.data(), inc_pos.size());
  up(&M.elem_inc, elem_inc.data(), elem_inc.size());
  if (e == hipSuccess) e = dalloc(h, &M.stage, 5 * (size_t)M.ninc);
  up(&M.fin_ptr, fin_ptr.data(), n + 1);
  up(&M.fin_face, fin_face.data(), fin_face.size());
  if (e == hipSuccess) e = dalloc(h, &M.geo, nt);
  if (e == hipSuccess) e = dalloc(h, &M.A, col.size());
  for (double** v : {&M.b, &M.dinv, &M.r, &M.z, &M.p, &M.sv, &M.w, &M.x})
    if (e == hipSuccess) e = dalloc(h, v, n);
  // the search directions start as NaN (all bits set): the first CG
  // iteration must set them outright, and a read before that write would
  // spoil every solve, not only those on reused memory
  if (e == hipSuccess) e = hipMemsetAsync(M.p, 0xFF, sizeof(double) * (size_t)n, s);
  if (e == hipSuccess) e = hipMemsetAsync(M.sv, 0xFF, sizeof(double) * (size_t)n, s);
  if (e == hipSuccess) e = dalloc(h, &M.part, 3 * kMaxS);
  if (e == hipSuccess) e = dalloc(h, &M.ctrl, 1);
  if (e == hipSuccess) e = hipMemsetAsync(M.ctrl, 0, sizeof(MetalCtrl), s);
  int32_t* bad = nullptr;
  if (e == hipSuccess) e = dalloc(h, &bad, 1);
  if (e == hipSuccess) e = hipHostMalloc((void**)&M.hctrl, sizeof(MetalCtrl), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
  if (e == hipSuccess)
    hipLaunchKernelGGL(k_geom, dim3(blocks_for(nt)), dim3(kMB), 0, s, M.xyz, M.tet,
                       nt, M.geo, bad);
  if (e == hipSuccess) e = hipGetLastError();
  int32_t nbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  M.G = (int)std::min<int64_t>(kMaxG, std::max<int64_t>(1, (n + kMB - 1) / kMB));
  if (e != hipSuccess) {
    *err = std::string("metal_create: ") + hipGetErrorString(e);
    metal_free(h);
    return PIC_E_DEVICE;
  }
  if (nbad) {
    *err = "metal_create: element of zero volume";
    metal_free(h);
    return PIC_E_ARG;
  }
  *out = h;
  return PIC_OK;
}

int64_t metal_n_faces(const pic_metal* h) { return h->m.nf; }

void metal_free(pic_metal* h) {
  if (!h) return;
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->m.hctrl) (void)hipHostFree(h->m.hctrl);
  if (h->m.chunk) (void)hipGraphExecDestroy(h->m.chunk);
  if (h->m.graph) (void)hipGraphDestroy(h->m.graph);
  if (h->m.chunk_big) (void)hipGraphExecDestroy(h->m.chunk_big);
  if (h->m.graph_big) (void)hipGraphDestroy(h->m.graph_big);
  delete h;
}

namespace {

CgArgsM cg_args(MetalImpl& M, double dir_value, double tol) {
  CgArgsM a{};
  a.n = M.n; a.row_ptr = M.row_ptr; a.col = M.col; a.A = M.A; a.b = M.b;
  a.sptr = M.sptr; a.scol = M.scol; a.sval = M.sval;
  a.dinv = M.dinv; a.dir = M.dir; a.dir_value = dir_value; a.tol2 = tol * tol;
  a.x = M.x; a.r = M.r; a.z = M.z; a.p = M.p; a.s = M.sv; a.w = M.w; a.part = M.part;
  a.ctrl = M.ctrl; a.G = M.G;
  a.Gs = (int)std::min<int64_t>(kMaxS, (M.n + kMB - 1) / kMB);  // 4 slices each
  return a;
}

// One iteration: the step (which first tests the incoming iterate) and the
// product for the next one.
void launch_iter(const CgArgsM& a, hipStream_t s) {
  const dim3 g(a.G), b(kMB);
  hipLaunchKernelGGL(k_cg_step, g, b, 0, s, a);
  hipLaunchKernelGGL(k_cg_spmv, dim3(a.Gs), b, 0, s, a);
}

// Capture count iterations into a graph on a private stream (capture is
// not possible on the legacy default stream the caller may use).
hipError_t capture_iters(MetalImpl& M, int count, hipGraph_t* graph, hipGraphExec_t* exec) {
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  const CgArgsM a = cg_args(M, 0.0, 1.0);
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int k = 0; k < count; ++k) launch_iter(a, cs);
    hipError_t e2 = hipStreamEndCapture(cs, graph);
    e = hipGetLastError();
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  return e;
}

hipError_t build_chunk(MetalImpl& M) {
  hipError_t e = capture_iters(M, kChunk, &M.graph, &M.chunk);
  if (e == hipSuccess) e = capture_iters(M, kChunkBig, &M.graph_big, &M.chunk_big);
  return e;
}

pic_status run_cg(pic_metal* h, double* x, double dir_value, double tol,
                  int64_t max_iter, pic_metal_stats* st, hipStream_t s,
                  std::string* err, const char* who) {
  MetalImpl& M = h->m;
  hipError_t e = hipSuccess;
  if (!M.chunk_big) e = build_chunk(M);
  const CgArgsM a = cg_args(M, dir_value, tol);
  const dim3 g(M.G), b(kMB);
  if (e == hipSuccess)
    e = hipMemcpyAsync(M.x, x, sizeof(double) * M.n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_cg_dir, g, b, 0, s, a);
    hipLaunchKernelGGL(k_cg_init, g, b, 0, s, a);
    hipLaunchKernelGGL(k_cg_start, dim3(1), b, 0, s, a);
    hipLaunchKernelGGL(k_cg_spmv, dim3(a.Gs), b, 0, s, a);
    e = hipGetLastError();
  }
  // a first chunk of kChunk iterations (short solves, such as a heat step,
  // end in it), then chunks of kChunkBig between host checks; iterations
  // past convergence return at once
  int64_t it = 0;
  bool done = false;
  while (e == hipSuccess) {
    e = hipMemcpyAsync(M.hctrl, M.ctrl, sizeof(MetalCtrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    done = M.hctrl->done != 0;
    if (done || it >= max_iter) break;
    if (it > 0 && max_iter - it >= kChunkBig) {
      e = hipGraphLaunch(M.chunk_big, s);
      it += kChunkBig;
    } else if (max_iter - it >= kChunk) {
      e = hipGraphLaunch(M.chunk, s);
      it += kChunk;
    } else {
      for (; it < max_iter; ++it) launch_iter(a, s);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess && done && M.hctrl->bb == 0.0) {
    hipLaunchKernelGGL(k_cg_zero, g, b, 0, s, a);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(x, M.x, sizeof(double) * M.n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    *err = std::string(who) + ": " + hipGetErrorString(e);
    return PIC_E_DEVICE;
  }
  const MetalCtrl c = *M.hctrl;
  if (st) {
    st->iters = c.iters;
    st->relres = c.bb > 0.0 ? std::sqrt(c.rr / c.bb) : 0.0;
    st->converged = done ? 1 : 0;
    st->pad = 0;
  }
  if (!done) {
    *err = std::string(who) + ": no convergence within max_iter";
    return PIC_E_NOCONV;
  }
  return PIC_OK;
}

AsmArgs asm_args(const MetalImpl& M) {
  AsmArgs a{};
  a.n = M.n; a.row_ptr = M.row_ptr; a.inc_ptr = M.inc_ptr;
  a.inc_pos = M.inc_pos; a.fin_ptr = M.fin_ptr;
  a.fin_face = M.fin_face; a.tet = M.tet; a.face = M.face; a.xyz = M.xyz;
  a.geo = M.geo; a.dir = M.dir; a.A = M.A; a.b = M.b; a.dinv = M.dinv;
  a.elem_inc = M.elem_inc; a.stage = M.stage; a.nt = M.nt;
  return a;
}

}  // namespace

pic_status metal_continuity(pic_metal* h, const double* sigma, const double* flux,
                            double tol, int64_t max_iter, double* phi, double* pj,
                            pic_metal_stats* st, hipStream_t s, std::string* err) {
  MetalImpl& M = h->m;
  AsmArgs a = asm_args(M);
  a.sigma = sigma;
  a.flux = flux;
  const unsigned g = blocks_for(M.n);
  hipLaunchKernelGGL(k_element, dim3(blocks_for(M.nt)), dim3(kMB), 0, s, a);
  hipLaunchKernelGGL(k_assemble, dim3(g), dim3(kMB), 0, s, a, 0.0);
  hipLaunchKernelGGL(k_eliminate, dim3(g), dim3(kMB), 0, s, M.n, M.row_ptr, M.col,
                     M.dir, 0.0, M.A, M.b, M.dinv);
  hipLaunchKernelGGL(k_to_sell, dim3(blocks_for(M.nnz)), dim3(kMB), 0, s, M.nnz, M.c2s,
                     M.A, M.sval);
  pic_status rc = run_cg(h, phi, 0.0, tol, max_iter, st, s, err, "continuity_solve");
  if (rc != PIC_OK && rc != PIC_E_NOCONV) return rc;
  if (pj) {
    hipLaunchKernelGGL(k_joule, dim3(blocks_for(M.nt)), dim3(kMB), 0, s, M.nt, M.tet,
                       M.geo, sigma, phi, pj);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      *err = std::string("continuity_solve: ") + hipGetErrorString(e);
      return PIC_E_DEVICE;
    }
  }
  return rc;
}

pic_status metal_heat(pic_metal* h, const pic_heat_params* p, const double* sigma,
                      const double* pj, const double* pn, double* T,
                      pic_metal_stats* st, hipStream_t s, std::string* err) {
  MetalImpl& M = h->m;
  AsmArgs a = asm_args(M);
  a.sigma = sigma;
  a.flux = pn;
  a.PJ = pj;
  a.T = T;
  a.L = p->L; a.Cv = p->Cv; a.dt = p->dt; a.theta = p->theta;
  const unsigned g = blocks_for(M.n);
  hipLaunchKernelGGL(k_element, dim3(blocks_for(M.nt)), dim3(kMB), 0, s, a);
  hipLaunchKernelGGL(k_assemble, dim3(g), dim3(kMB), 0, s, a, p->T_amb);
  hipLaunchKernelGGL(k_eliminate, dim3(g), dim3(kMB), 0, s, M.n, M.row_ptr, M.col,
                     M.dir, p->T_amb, M.A, M.b, M.dinv);
  hipLaunchKernelGGL(k_to_sell, dim3(blocks_for(M.nnz)), dim3(kMB), 0, s, M.nnz, M.c2s,
                     M.A, M.sval);
  return run_cg(h, T, p->T_amb, p->tol, p->max_iter, st, s, err, "heat_step");
}

}  // namespace fp
