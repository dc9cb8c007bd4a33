// Poisson solve on the free nodes (Eq. poisson with Eq. poisson_bc in the
// Galerkin form of App. B): Jacobi-preconditioned CG in the single-
// reduction (Chronopoulos-Gear) ordering, warm started, with the stopping
// test re-checked on the true residual, and the nodal field E = R phi.
//
// The solve is a chain of ordinary kernel launches (a launch costs ~3 us on
// MI355X, a device-wide barrier inside a persistent kernel 12-19 us):
//   resfield: one pass over phi: b on the fly, r = b - K phi, u = D^-1 r,
//             x = phi on free nodes, E = R phi on every node, phi = 0 on
//             Dirichlet nodes; (b,b), (r,r)
//   start   : convergence test on that true residual; stats; when not
//             converged, w = K u, (r,u), (w,u)
//   upd(i)  : scalars of iteration i; p, s, x, r, u updates; (r,r), (r,u)
//   spmv(i) : w = K u; (w,u)
//   scatter : phi = x on free nodes, before the re-check (a resfield pass)
// K and R share the sparsity of the free rows, so the field of phi comes out
// of the same pass that tests phi: when the warm start already meets the
// tolerance (no iteration), the step's solve is two launches, and whenever
// the solver stops, E belongs to the final phi.
// Each kernel writes one partial sum per workgroup; the next kernel reduces
// all partials in a fixed order in every workgroup (deterministic, same
// values everywhere), so no cross-workgroup synchronization is needed
// inside a kernel.  A control word in device memory carries the state
// (ITER, RECHECK, DONE, NOCONV); kernels whose state does not apply return
// at once, which lets the host launch iterations in batches.  The last
// kernel before each host wait also writes the state, with a sequence
// number, into host-mapped memory that the host polls.
//
// Storage is sliced ELLPACK (64 rows per slice, column-major in the slice):
// one row per lane, so every load of a wave is contiguous.  Slices are split
// into contiguous blocks per workgroup, grouped so that each of the 8 XCDs
// (workgroup g runs on XCD g mod 8) sweeps one contiguous eighth of the
// matrix, which keeps neighbour gathers in one L2.
#include "amg.h"

#include <algorithm>
#include <cstring>
#include <type_traits>
#include "common.h"
#include "solver.h"

namespace fp {

namespace {

struct Range {
  int64_t lo, hi;
};

__device__ inline Range my_range(int64_t n, VB vb) {
  const int G = vb.n;
  const int g = vb.id;
  int chunk = g;
  if ((G & 7) == 0) chunk = (g & 7) * (G >> 3) + (g >> 3);
  const int64_t per = (n + G - 1) / G;
  Range r;
  r.lo = (int64_t)chunk * per;
  if (r.lo > n) r.lo = n;
  r.hi = r.lo + per < n ? r.lo + per : n;
  return r;
}

// Deterministic block sum; result valid in every thread.
template <int NQ>
__device__ inline void block_sum(double (&v)[NQ]) {
  __shared__ double lds[NQ][16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) lds[q][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[q][w];
    v[q] = s;
  }
  __syncthreads();
}

// Totals of partial sums written by the previous kernel: part[q*stride + j].
template <int NQ>
__device__ inline void totals(const double* part, int P, int stride,
                              double (&t)[NQ]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int j = threadIdx.x; j < P; j += blockDim.x) s += part[q * stride + j];
    t[q] = s;
  }
  block_sum<NQ>(t);
}

template <int NQ>
__device__ inline void write_partials(double* part, int stride,
                                      double (&v)[NQ], VB vb) {
  block_sum<NQ>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[q * stride + vb.id] = v[q];
  }
}

// y_r = sum_j val[j] x[col[j]] over the rows of this workgroup's slices;
// emit(r, y_r) for every row r < nrows.
template <typename T, typename F>
__device__ inline void spmv_sell(const int32_t* __restrict__ sptr,
                                 const int32_t* __restrict__ scol,
                                 const T* __restrict__ sval,
                                 const T* __restrict__ x, int64_t nslices,
                                 int64_t nrows, VB vb, F&& emit) {
  const Range sl = my_range(nslices, vb);
  const int lane = threadIdx.x & (kSell - 1);
  const int sub = threadIdx.x / kSell;
  const int nsub = blockDim.x / kSell;
  for (int64_t s = sl.lo + sub; s < sl.hi; s += nsub) {
    const int64_t r = s * kSell + lane;
    const int32_t p0 = sptr[s], p1 = sptr[s + 1];
    T acc = T(0);
    int32_t p = p0 + lane;
    // four entries per trip (slice widths are uniform across the wave):
    // their loads are in flight together, the sum keeps the entry order
    for (; p + 3 * kSell < p1; p += 4 * kSell) {
      int32_t c[4];
      T v[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c[u] = scol[p + u * kSell];
        v[u] = sval[p + u * kSell];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = x[c[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += v[u] * xv[u];
    }
    for (; p < p1; p += kSell) acc += sval[p] * x[scol[p]];
    if (r < nrows) emit(r, acc);
  }
}

}  // namespace

// Partial-sum slots (each [G] doubles): 0 bb, 1 rr(resid), 2-3 start (ru, wu),
// 4-5 upd even (rr, ru), 6-7 upd odd, 8 spmv even (wu), 9 spmv odd.
__device__ inline double* slot(const CgArgs& a, int k) {
  return a.part + (size_t)k * a.G;
}

__device__ inline void ctrl_reset(CgCtrl* c) {
  CgCtrl z;
  z.state = CG_ITER;
  z.zero_rhs = 0;
  z.iters = 0;
  z.iters_final = 0;
  z.restarts = 0;
  z.bb = 0.0;
  z.relres = 0.0;
  z.rstart = 0.0;
  z.alpha[0] = z.alpha[1] = 0.0;
  z.gamma[0] = z.gamma[1] = 0.0;
  z.it_a = z.it_b = 0;
  z.rc_gate = z.pad = 0;
  *c = z;
}

// Copy of the control state to host-mapped memory; the sequence number is
// stored last with system-scope release so the host sees a complete record.
__device__ inline void report(const CgCtrl* c, CgReport* r, int64_t seq,
                              int32_t state) {
  r->state = state;
  r->iters = state == CG_RECHECK ? c->iters_final : c->iters;
  __hip_atomic_store(&r->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The pass over phi (see the file comment).  reset != 0 starts a new solve
// (control word cleared by workgroup 0; no other workgroup reads it here).
// Mixed precision: the FP64 residual is rounded once into the FP32
// recursion vectors.  FP32 field (e32): E = R phi in the difference form
//   E_i = sum_j R_ij (phi_j - phi_i) + S_i phi_i,   S_i = sum_j R_ij (FP64),
// with R in FP32: the differences are of the size of E h, so rounding R
// costs a relative error of about 2^-24 in E, while R_ij phi_j alone would
// lose the ratio |phi| / (|E| h) to cancellation.
// dev_gate (re-check passes only): run only if the recursion has stopped;
// workgroup 0 records the decision for the start pass that follows.
__device__ inline void k_cg_resfield_body(const CgArgs& a, int reset, VB vb,
                                          int dev_gate = 0) {
  if (dev_gate) {
    const bool on = a.ctrl->state == CG_RECHECK;
    if (vb.id == 0 && threadIdx.x == 0) a.ctrl->rc_gate = on ? 1 : 0;
    if (!on) return;
  }
  const DevMesh& m = a.m;
  if (reset && vb.id == 0 && threadIdx.x == 0) ctrl_reset(a.ctrl);
  if (reset && a.acc_rows && vb.id < kStepCounters)
    step_counter_sum(a.acc_rows, a.acc_n, a.step_stats, vb.id);
  const int lane = threadIdx.x & (kSell - 1);
  const int sub = threadIdx.x / kSell;
  const int nsub = blockDim.x / kSell;
  const bool withE = a.E != nullptr && !(reset && a.keep_field);
  const bool e32 = a.e32 != 0;
  const int64_t np = m.k_np;
  double v[2] = {0.0, 0.0};
  {
    const Range sl = my_range(m.k_nslices, vb);
    for (int64_t s = sl.lo + sub; s < sl.hi; s += nsub) {
      const int64_t r = s * kSell + lane;
      const bool row = r < m.n_free;
      const int32_t nd = row ? m.free2node[r] : 0;
      const double pi = row ? a.phi[nd] : 0.0;
      const int32_t p0 = m.k_sptr[s], p1 = m.k_sptr[s + 1];
      double kx = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
      // four entries per trip where the slice allows (uniform across the
      // wave): their loads are in flight together; sums in entry order
      int32_t p = p0 + lane;
      if (!withE) {
        for (; p + 3 * kSell < p1; p += 4 * kSell) {
          int32_t c[4];
          double kv[4], xj[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            c[u] = m.k_ncol[p + u * kSell];
            kv[u] = m.k_sval[p + u * kSell];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) xj[u] = a.phi[c[u]];
#pragma unroll
          for (int u = 0; u < 4; ++u) kx += kv[u] * xj[u];
        }
        for (; p < p1; p += kSell)
          kx += m.k_sval[p] * a.phi[m.k_ncol[p]];
      } else if (!e32) {
        for (; p + 3 * kSell < p1; p += 4 * kSell) {
          int32_t c[4];
          double kv[4], rx[4], ry[4], rz[4], xj[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int32_t q = p + u * kSell;
            c[u] = m.k_ncol[q];
            kv[u] = m.k_sval[q];
            rx[u] = m.r_sval[q];
            ry[u] = m.r_sval[np + q];
            rz[u] = m.r_sval[2 * np + q];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) xj[u] = a.phi[c[u]];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            kx += kv[u] * xj[u];
            ex += rx[u] * xj[u];
            ey += ry[u] * xj[u];
            ez += rz[u] * xj[u];
          }
        }
        for (; p < p1; p += kSell) {
          const double xj = a.phi[m.k_ncol[p]];
          kx += m.k_sval[p] * xj;
          ex += m.r_sval[p] * xj;
          ey += m.r_sval[np + p] * xj;
          ez += m.r_sval[2 * np + p] * xj;
        }
      } else {
        for (; p + 3 * kSell < p1; p += 4 * kSell) {
          int32_t c[4];
          double kv[4], xj[4];
          float rx[4], ry[4], rz[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int32_t q = p + u * kSell;
            c[u] = m.k_ncol[q];
            kv[u] = m.k_sval[q];
            rx[u] = m.r_sval32[q];
            ry[u] = m.r_sval32[np + q];
            rz[u] = m.r_sval32[2 * np + q];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) xj[u] = a.phi[c[u]];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            kx += kv[u] * xj[u];
            const double d = xj[u] - pi;
            ex += (double)rx[u] * d;
            ey += (double)ry[u] * d;
            ez += (double)rz[u] * d;
          }
        }
        for (; p < p1; p += kSell) {
          const double xj = a.phi[m.k_ncol[p]];
          kx += m.k_sval[p] * xj;
          const double d = xj - pi;
          ex += (double)m.r_sval32[p] * d;
          ey += (double)m.r_sval32[np + p] * d;
          ez += (double)m.r_sval32[2 * np + p] * d;
        }
      }
      if (!row) continue;
      double bi;
      if (a.rhs) {
        bi = a.rhs[r];
      } else if (a.b_saved) {
        bi = a.bprev[r];  // the same value, formed by the solve's first pass
      } else {
        const double c = a.charge ? (double)a.charge[nd] : 0.0;
        bi = a.coef * c + a.E0 * m.g_unit[r];
      }
      const double ri = bi - kx;
      a.x[r] = pi;
      if (a.bprev) a.bprev[r] = bi;
      if (a.mixed) {
        a.r[r] = ri;  // (kept for an incremental next pass)
        a.r32[r] = (float)ri;
        a.u32[r] = (float)(ri * m.invdiag[r]);
      } else {
        a.r[r] = ri;
        a.u[r] = ri * m.invdiag[r];
      }
      v[0] += bi * bi;
      v[1] += ri * ri;
      if (withE) {
        if (e32) {
          const double4 S = m.f_rowsum[nd];
          reinterpret_cast<float4*>(a.E)[nd] =
              make_float4((float)(ex + S.x * pi), (float)(ey + S.y * pi),
                          (float)(ez + S.z * pi), 0.0f);
        } else {
          reinterpret_cast<double4*>(a.E)[nd] = make_double4(ex, ey, ez, 0.0);
        }
      }
    }
  }
  // Dirichlet rows: phi = 0 there (never read above: columns are free
  // nodes), E = R phi
  {
    const Range dr = my_range(a.n_dir, vb);
    for (int64_t i = dr.lo + threadIdx.x; i < dr.hi; i += blockDim.x)
      a.phi[a.dir_nodes[i]] = 0.0;
  }
  if (withE) {
    const int64_t dnp = m.d_np;
    const Range sl = my_range(m.d_nslices, vb);
    for (int64_t s = sl.lo + sub; s < sl.hi; s += nsub) {
      const int64_t r = s * kSell + lane;
      const int32_t p0 = m.d_sptr[s], p1 = m.d_sptr[s + 1];
      double ex = 0.0, ey = 0.0, ez = 0.0;
      if (!e32) {
        for (int32_t p = p0 + lane; p < p1; p += kSell) {
          const double xj = a.phi[m.d_ncol[p]];
          ex += m.d_sval[p] * xj;
          ey += m.d_sval[dnp + p] * xj;
          ez += m.d_sval[2 * dnp + p] * xj;
        }
      } else {
        for (int32_t p = p0 + lane; p < p1; p += kSell) {
          const double xj = a.phi[m.d_ncol[p]];
          ex += (double)m.d_sval32[p] * xj;
          ey += (double)m.d_sval32[dnp + p] * xj;
          ez += (double)m.d_sval32[2 * dnp + p] * xj;
        }
      }
      if (r >= a.n_dir) continue;
      const int32_t nd = a.dir_nodes[r];
      if (e32)
        reinterpret_cast<float4*>(a.E)[nd] =
            make_float4((float)ex, (float)ey, (float)ez, 0.0f);
      else
        reinterpret_cast<double4*>(a.E)[nd] = make_double4(ex, ey, ez, 0.0);
    }
  }
  write_partials<2>(slot(a, 0), a.G, v, vb);
}

// x = phi and u = D^-1 r of free row i (node nd) with residual ri: FP32
// copies of r and u for the mixed-precision recursion.
__device__ inline void cg_prep_row(const CgArgs& a, int64_t i, int32_t nd,
                                   double ri) {
  a.x[i] = a.phi[nd];
  if (a.mixed) {
    a.r32[i] = (float)ri;
    a.u32[i] = (float)(ri * a.m.invdiag[i]);
  } else {
    a.u[i] = ri * a.m.invdiag[i];
  }
}

// First pass of a solve whose previous solve (same system, phi unchanged
// since) ended with the true residual r and right-hand side b_prev: r =
// (b - b_prev) + r, the same quantity as b - K phi without the product with
// K; x = phi, u = D^-1 r, (b,b), (r,r) as in the full pass.  The field is
// that of phi already.
__device__ inline void k_cg_resinc_body(const CgArgs& a, VB vb) {
  const DevMesh& m = a.m;
  if (vb.id == 0 && threadIdx.x == 0) ctrl_reset(a.ctrl);
  if (a.acc_rows && vb.id < kStepCounters)
    step_counter_sum(a.acc_rows, a.acc_n, a.step_stats, vb.id);
  const Range rows = my_range(m.n_free, vb);
  double v[2] = {0.0, 0.0};
  for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x) {
    const int32_t nd = m.free2node[i];
    const double c = a.charge ? (double)a.charge[nd] : 0.0;
    const double bi = a.coef * c + a.E0 * m.g_unit[i];
    const double ri = (bi - a.bprev[i]) + a.r[i];
    a.r[i] = ri;
    a.bprev[i] = bi;
    if (a.lean) {
      a.clear_charge[nd] = 0;  // (read above; b stays in bprev)
    } else {
      cg_prep_row(a, i, nd, ri);
    }
    v[0] += bi * bi;
    v[1] += ri * ri;
  }
  if (a.lean) {
    // the Dirichlet nodes' charges (never part of b) cleared as well
    const Range dr = my_range(a.n_dir, vb);
    for (int64_t i = dr.lo + threadIdx.x; i < dr.hi; i += blockDim.x)
      a.clear_charge[a.dir_nodes[i]] = 0;
  }
  write_partials<2>(slot(a, 0), a.G, v, vb);
}

// x and u of a lean first pass whose test asked for iterations (the same
// values as the full first pass writes).
__device__ inline void k_cg_prep_body(const CgArgs& a, VB vb) {
  const DevMesh& m = a.m;
  const Range rows = my_range(m.n_free, vb);
  for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x)
    cg_prep_row(a, i, m.free2node[i], a.r[i]);
}

// phi = x on the free nodes (before a re-check pass; dev_gate: only if the
// recursion has stopped).
__device__ inline void k_cg_scatter_body(const CgArgs& a, VB vb, int dev_gate = 0) {
  if (dev_gate && a.ctrl->state != CG_RECHECK) return;
  const DevMesh& m = a.m;
  const Range rows = my_range(m.n_free, vb);
  for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x)
    a.phi[m.free2node[i]] = a.x[i];
}

// The first product w = K u of a (re)started CG and its two sums.
__device__ inline void start_product(const CgArgs& a, VB vb) {
  const DevMesh& m = a.m;
  double v[2] = {0.0, 0.0};
  if (a.mixed) {
    spmv_sell(m.k_sptr, m.k_scol, m.k_sval32, a.u32, m.k_nslices, m.n_free, vb,
              [&](int64_t i, float s) {
                a.w32[i] = s;
                const double ui = a.u32[i];
                v[0] += (double)a.r32[i] * ui;
                v[1] += (double)s * ui;
              });
  } else {
    spmv_sell(m.k_sptr, m.k_scol, m.k_sval, a.u, m.k_nslices, m.n_free, vb,
              [&](int64_t i, double s) {
                a.w[i] = s;
                const double ui = a.u[i];
                v[0] += a.r[i] * ui;
                v[1] += s * ui;
              });
  }
  write_partials<2>(slot(a, 2), a.G, v, vb);
}

// Convergence test on the true residual of the last resfield pass; when the
// solve ends, its statistics; when not converged, the first product w = K u
// of a (re)started CG.  Fields written here by workgroup 0 (state, iters,
// bb, relres, rstart, restarts) are never read by other workgroups of this
// launch; they read iters_final, which is stable here.  A zero right-hand
// side gives phi = 0 and E = 0, written by every workgroup.
// dev_gate 1: only where the resfield pass before it ran (rc_gate; the
// state itself is rewritten by workgroup 0 here); 2: the product only,
// after a lean first pass's test (state CG_ITER) and k_cg_prep; 3: the test
// of a lean first pass only (one workgroup).
__device__ inline void k_cg_start_body(const CgArgs& a, int64_t seq, VB vb,
                                       int dev_gate = 0) {
  CgCtrl* c = a.ctrl;
  if (dev_gate == 1 && !c->rc_gate) return;
  if (dev_gate == 2) {
    if (c->state == CG_ITER && !a.amg) start_product(a, vb);
    return;
  }
  double t[2];
  totals<2>(slot(a, 0), a.G, a.G, t);
  const double bn = sqrt(t[0]);
  const double rn = sqrt(t[1]);
  const int64_t done_iters = c->iters_final;
  const double bs = a.bref ? fmax(bn, *a.bref) : bn;
  const bool done = bn == 0.0 || rn <= a.tol * bs;
  const bool noconv = !done && done_iters >= a.max_iter;
  if (vb.id == 0 && threadIdx.x == 0) {
    c->bb = t[0];
    c->iters = done_iters;
    const double relres = bn > 0.0 ? rn / bn : 0.0;
    c->relres = relres;
    c->rstart = rn;
    const int32_t state = done ? CG_DONE : (noconv ? CG_NOCONV : CG_ITER);
    c->state = state;
    c->it_a = 0;
    if (!done && !noconv) c->restarts += 1;
    if (bn == 0.0) c->zero_rhs = 1;
    if (done || noconv) {
      const int64_t st = noconv ? PIC_E_NOCONV : 0;
      if (a.stats) {
        a.stats->iters = done_iters;
        a.stats->status = st;
        a.stats->restarts = c->restarts;
        a.stats->relres = relres;
        a.stats->bnorm = bn;
      }
      if (a.step_stats) {
        a.step_stats->cg_iters = done_iters;
        a.step_stats->cg_relres = relres;
        if (st != 0 && a.step_stats->status == 0) a.step_stats->status = st;
      }
    }
    if (seq) {
      __threadfence_system();
      report(c, a.report, seq, state);
    }
  }
  if (bn == 0.0) {
    const DevMesh& m = a.m;
    // phi = 0 solves it; its residual (b = 0) is 0, which is what the next
    // solve's incremental first pass builds on
    const Range fr = my_range(m.n_free, vb);
    for (int64_t i = fr.lo + threadIdx.x; i < fr.hi; i += blockDim.x) a.r[i] = 0.0;
    const Range nr = my_range(m.n_nodes, vb);
    for (int64_t i = nr.lo + threadIdx.x; i < nr.hi; i += blockDim.x) {
      a.phi[i] = 0.0;
      if (a.E && a.e32)
        reinterpret_cast<float4*>(a.E)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      else if (a.E)
        reinterpret_cast<double4*>(a.E)[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    }
  }
  if ((done || noconv) && a.next_stats) {
    // the start of the next step (as k_begin does it)
    if (vb.id == 0) {
      int64_t* s64 = reinterpret_cast<int64_t*>(a.next_stats);
      const int ns = (int)(sizeof(pic_step_stats) / sizeof(int64_t));
      if (threadIdx.x < ns) s64[threadIdx.x] = 0;
      int32_t* c32 = reinterpret_cast<int32_t*>(a.next_scratch);
      const int nc = (int)(sizeof(StepScratch) / sizeof(int32_t));
      if (threadIdx.x < nc) c32[threadIdx.x] = 0;
      __syncthreads();
      if (threadIdx.x == 0) a.next_scratch->inj_base = *a.n_slots;
    }
    if (!a.b_saved) {  // (else the lean first pass cleared them)
      const Range cr = my_range(a.n_clear, vb);
      for (int64_t i = cr.lo + threadIdx.x; i < cr.hi; i += blockDim.x)
        a.clear_charge[i] = 0;
    }
  }
  if (done || noconv) return;
  if (dev_gate == 3) return;  // the test of a lean first pass only
  if (a.amg) return;  // its iterations start with the V-cycle
  start_product(a, vb);
}

// Iteration it (0-based since the last (re)start): scalars from the
// previous products, then the row-local updates.
// it < 0: take the iteration index from the control word (batched launch).
__device__ inline void k_cg_upd_body(const CgArgs& a, int it, VB vb) {
  CgCtrl* c = a.ctrl;
  if (c->state != CG_ITER) return;
  if (it < 0) {
    it = c->it_a;
    if (vb.id == 0 && threadIdx.x == 0) c->it_b = it;
  }
  double alpha, beta, gamma;
  if (it == 0) {
    double t[2];
    totals<2>(slot(a, 2), a.G, a.G, t);
    gamma = t[0];
    alpha = gamma / t[1];
    beta = 0.0;
  } else {
    const int pb = (it - 1) & 1;
    double t3[3];
    {
      double t2[2];
      totals<2>(slot(a, 4 + 2 * pb), a.G, a.G, t2);
      double t1[1];
      totals<1>(slot(a, 8 + pb), a.G, 1, t1);
      t3[0] = t2[0];
      t3[1] = t2[1];
      t3[2] = t1[0];
    }
    // it iterations done since the (re)start; c->iters is stable while
    // iterating, so every workgroup takes the same decision
    const double rn = sqrt(t3[0]);
    const double bn = sqrt(c->bb);
    double thr = a.tol * (a.bref ? fmax(bn, *a.bref) : bn);
    if (a.mixed) thr = fmax(thr, a.inner_tol * c->rstart);
    if (rn <= thr || c->iters + it >= a.max_iter) {
      if (vb.id == 0 && threadIdx.x == 0) {
        c->state = CG_RECHECK;
        c->iters_final = c->iters + it;
      }
      return;
    }
    const double g_prev = c->gamma[pb];
    const double a_prev = c->alpha[pb];
    gamma = t3[1];
    beta = gamma / g_prev;
    alpha = gamma / (t3[2] - beta * gamma / a_prev);
  }
  if (vb.id == 0 && threadIdx.x == 0) {
    c->gamma[it & 1] = gamma;
    c->alpha[it & 1] = alpha;
  }
  const DevMesh& m = a.m;
  const Range rows = my_range(m.n_free, vb);
  double v[2] = {0.0, 0.0};
  const bool first = it == 0;
  if (a.mixed) {
    const float al = (float)alpha, be = (float)beta;
    for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x) {
      const float pi = first ? a.u32[i] : a.u32[i] + be * a.p32[i];
      const float si = first ? a.w32[i] : a.w32[i] + be * a.s32[i];
      a.p32[i] = pi;
      a.s32[i] = si;
      a.x[i] += alpha * (double)pi;
      const float ri = a.r32[i] - al * si;
      a.r32[i] = ri;
      const float ui = ri * m.invdiag32[i];
      a.u32[i] = ui;
      v[0] += (double)ri * ri;
      v[1] += (double)ri * ui;
    }
    write_partials<2>(slot(a, 4 + 2 * (it & 1)), a.G, v, vb);
    return;
  }
  for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x) {
    const double pi = first ? a.u[i] : a.u[i] + beta * a.p[i];
    const double si = first ? a.w[i] : a.w[i] + beta * a.s[i];
    a.p[i] = pi;
    a.s[i] = si;
    a.x[i] += alpha * pi;
    const double ri = a.r[i] - alpha * si;
    a.r[i] = ri;
    const double ui = ri * m.invdiag[i];
    a.u[i] = ui;
    v[0] += ri * ri;
    v[1] += ri * ui;
  }
  write_partials<2>(slot(a, 4 + 2 * (it & 1)), a.G, v, vb);
}

__device__ inline void k_cg_spmv_body(const CgArgs& a, int it,
                                                int64_t seq, VB vb) {
  const int32_t state = a.ctrl->state;
  if (seq && vb.id == 0 && threadIdx.x == 0) report(a.ctrl, a.report, seq, state);
  if (state != CG_ITER) return;
  if (it < 0) {
    it = a.ctrl->it_b;
    if (vb.id == 0 && threadIdx.x == 0) a.ctrl->it_a = it + 1;
  }
  const DevMesh& m = a.m;
  double v[1] = {0.0};
  if (a.mixed) {
    spmv_sell(m.k_sptr, m.k_scol, m.k_sval32, a.u32, m.k_nslices, m.n_free, vb,
              [&](int64_t i, float s) {
                a.w32[i] = s;
                v[0] += (double)s * a.u32[i];
              });
  } else {
    spmv_sell(m.k_sptr, m.k_scol, m.k_sval, a.u, m.k_nslices, m.n_free, vb,
              [&](int64_t i, double s) {
                a.w[i] = s;
                v[0] += s * a.u[i];
              });
  }
  write_partials<1>(slot(a, 8 + (it & 1)), a.G, v, vb);
}

// Single-instance kernels.
__global__ void __launch_bounds__(kCgBlock) k_cg_resfield(CgArgs a, int reset,
                                                         int dev_gate) {
  k_cg_resfield_body(a, reset, VB{(int)blockIdx.x, (int)gridDim.x}, dev_gate);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_scatter(CgArgs a, int dev_gate) {
  k_cg_scatter_body(a, VB{(int)blockIdx.x, (int)gridDim.x}, dev_gate);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_resinc(CgArgs a) {
  k_cg_resinc_body(a, VB{(int)blockIdx.x, (int)gridDim.x});
}
__global__ void __launch_bounds__(kCgBlock) k_cg_prep(CgArgs a) {
  k_cg_prep_body(a, VB{(int)blockIdx.x, (int)gridDim.x});
}
__global__ void __launch_bounds__(kCgBlock) k_cg_start(CgArgs a, int64_t seq,
                                                      int dev_gate) {
  k_cg_start_body(a, seq, VB{(int)blockIdx.x, (int)gridDim.x}, dev_gate);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_upd(CgArgs a, int it) {
  k_cg_upd_body(a, it, VB{(int)blockIdx.x, (int)gridDim.x});
}
__global__ void __launch_bounds__(kCgBlock) k_cg_spmv(CgArgs a, int it,
                                                     int64_t seq) {
  k_cg_spmv_body(a, it, seq, VB{(int)blockIdx.x, (int)gridDim.x});
}

__global__ void k_cg_report(CgArgs a, int64_t seq) {
  if (threadIdx.x != 0) return;
  __threadfence_system();
  report(a.ctrl, a.report, seq, a.ctrl->state);
}

// Batched kernels: block -> (instance, virtual block) by the schedule.
// gated (re-check launches): 1 skips the instances outside the mask, 2
// leaves the decision to each instance's state (conditional re-check).
__global__ void __launch_bounds__(kCgBlock) k_cg_resfield_b(CgBatch b, int reset,
                                                           int gated) {
  int i;
  const VB vb = batch_block(b.map, i);
  if (gated == 1 && !((b.mask >> i) & 1ull)) return;
  const CgArgs a = b.args[i];  // a private copy: no aliasing with the stores
  k_cg_resfield_body(a, reset, vb, gated == 2);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_resinc_b(CgBatch b) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  k_cg_resinc_body(a, vb);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_scatter_b(CgBatch b, int gated) {
  int i;
  const VB vb = batch_block(b.map, i);
  if (gated == 1 && !((b.mask >> i) & 1ull)) return;
  const CgArgs a = b.args[i];
  k_cg_scatter_body(a, vb, gated == 2);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_start_b(CgBatch b, int gated) {
  int i;
  const VB vb = batch_block(b.map, i);
  if (gated == 1 && !((b.mask >> i) & 1ull)) return;
  const CgArgs a = b.args[i];
  k_cg_start_body(a, 0, vb, gated == 2);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_upd_b(CgBatch b) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  k_cg_upd_body(a, -1, vb);
}
__global__ void __launch_bounds__(kCgBlock) k_cg_spmv_b(CgBatch b) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  k_cg_spmv_body(a, -1, 0, vb);
}
// One thread per instance: report the control state with sequence seq.
__global__ void k_cg_report_b(CgBatch b, int n, int64_t seq) {
  const int i = threadIdx.x;
  if (i >= n) return;
  const CgArgs& a = b.args[i];
  __threadfence_system();
  report(a.ctrl, a.report, seq, a.ctrl->state);
}

// ---------------------------------------------------------------------------
// CG preconditioned by one smoothed-aggregation V(1,1)-cycle (FP64).  Each
// iteration is [V-cycle u = M r, w = K u, update], the Chronopoulos-Gear
// recurrences being the same for any symmetric positive definite M.
// Partial-sum slots of parity p = it & 1: 4 + 2p (r,r) from the update,
// 5 + 2p (r,u) from the last V-cycle kernel, 8 + p (w,u) from the product.
// Counters: the V-cycle and the product read it_a, the product copies it to
// it_b, the update reads it_b and sets it_a = it_b + 1.  The first V-cycle
// kernel of every iteration after the first applies the stopping test to
// the recursive residual.  Every kernel returns at once unless the state is
// ITER.
// ---------------------------------------------------------------------------
namespace {

// emit(r, sum_j val_rj g(col_rj)) for every row r of M in this workgroup's
// share, in the arithmetic of T (the values of M in T: val or val32).
// SELL (lpr = 1): one lane per row, entries in order, four loads in flight
// per trip.  CSR (lpr > 1): lpr lanes per row, each summing every lpr-th
// entry, then a fixed shuffle tree; every group of a workgroup makes the
// same number of trips, so the shuffles run on whole waves.
template <typename T>
__device__ inline const T* mat_val(const SellMat& M) {
  if constexpr (std::is_same<T, float>::value) return M.val32;
  else return M.val;
}

template <typename T, typename Gf, typename Ef>
__device__ inline void amg_rows(const SellMat& M, VB vb, Gf&& g, Ef&& emit) {
  const T* __restrict__ val = mat_val<T>(M);
  if (M.lpr == 1) {
    const Range sl = my_range(M.nslices, vb);
    const int lane = threadIdx.x & (kSell - 1);
    for (int64_t s = sl.lo + threadIdx.x / kSell; s < sl.hi;
         s += blockDim.x / kSell) {
      const int32_t p1 = M.sptr[s + 1];
      int32_t p = M.sptr[s] + lane;
      T acc = 0;
      for (; p + 3 * kSell < p1; p += 4 * kSell) {
        int32_t c[4];
        T v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = M.col[p + u * kSell];
          v[u] = val[p + u * kSell];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = g(c[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u] * xv[u];
      }
      for (; p < p1; p += kSell) acc += val[p] * g(M.col[p]);
      const int64_t r = s * kSell + lane;
      if (r < M.nrows) emit(r, acc);
    }
    return;
  }
  const int lpr = M.lpr;
  const Range rows = my_range(M.nrows, vb);
  const int sub = threadIdx.x & (lpr - 1);
  const int grp = threadIdx.x / lpr, ngrp = blockDim.x / lpr;
  for (int64_t r0 = rows.lo; r0 < rows.hi; r0 += ngrp) {
    const int64_t r = r0 + grp;
    T acc = 0;
    if (r < rows.hi) {
      // four entries per trip with their loads in flight together, summed
      // in the lane's entry order
      const int32_t p1 = M.sptr[r + 1];
      int32_t p = M.sptr[r] + sub;
      for (; p + 3 * lpr < p1; p += 4 * lpr) {
        int32_t c[4];
        T v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = M.col[p + u * lpr];
          v[u] = val[p + u * lpr];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = g(c[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u] * xv[u];
      }
      for (; p < p1; p += lpr) acc += val[p] * g(M.col[p]);
    }
    for (int off = lpr >> 1; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, lpr);
    if (r < rows.hi && sub == 0) emit(r, acc);
  }
}

// The stopping test on the recursive residual of the previous update
// (iterations after the first of a (re)start); true when the solve leaves
// the iteration (every workgroup decides alike).
__device__ inline bool amg_stop(const CgArgs& a, VB vb) {
  CgCtrl* c = a.ctrl;
  const int it = c->it_a;
  if (it == 0) return false;
  double t[1];
  totals<1>(slot(a, 4 + 2 * ((it - 1) & 1)), a.G, 1, t);
  const double rn = sqrt(t[0]);
  const double bn = sqrt(c->bb);
  const double thr = a.tol * (a.bref ? fmax(bn, *a.bref) : bn);
  if (rn <= thr || c->iters + it >= a.max_iter) {
    if (vb.id == 0 && threadIdx.x == 0) {
      c->state = CG_RECHECK;
      c->iters_final = c->iters + it;
    }
    return true;
  }
  return false;
}

// Vectors and diagonal of a level in the arithmetic of T.
template <typename T>
struct LevelVecs {
  const T* dinv;
  T *b, *x, *r, *t;
};
template <typename T>
__host__ __device__ inline LevelVecs<T> level_vecs(const AmgLevel& L) {
  if constexpr (std::is_same<T, float>::value)
    return LevelVecs<T>{L.invdiag32, L.b32, L.x32, L.r32, L.t32};
  else
    return LevelVecs<T>{L.invdiag, L.b, L.x, L.r, L.t};
}

}  // namespace

// Pre-smoothing from zero and the residual: x = w D^-1 b,
// r = b - A x = b - w sum_j a_ij d_j^-1 b_j.  On the finest level b is the
// CG residual (FP64; rounded once to T).
template <typename T>
__device__ inline void amg_down_body(const CgArgs& a, const AmgLevel& L,
                                     int level, VB vb) {
  if (a.ctrl->state != CG_ITER) return;
  if (level == 0 && amg_stop(a, vb)) return;
  const LevelVecs<T> V = level_vecs<T>(L);
  const double* __restrict__ r64 = a.r;
  const T* __restrict__ bl = V.b;
  const T* __restrict__ dinv = V.dinv;
  const T omega = (T)L.omega;
  auto B = [&](int64_t c) -> T { return level == 0 ? (T)r64[c] : bl[c]; };
  amg_rows<T>(L.A, vb, [&](int32_t c) { return B(c) * dinv[c]; },
              [&](int64_t r, T ax) {
                const T br = B(r);
                V.x[r] = omega * (dinv[r] * br);
                V.r[r] = br - omega * ax;
              });
}

// y = M x for the rows of M (restriction and prolongation; add: y += M x).
template <typename T>
__device__ inline void amg_apply_body(const CgArgs& a, const SellMat& M,
                                      const T* x, T* y, int add, VB vb) {
  if (a.ctrl->state != CG_ITER) return;
  amg_rows<T>(M, vb, [&](int32_t c) { return x[c]; },
              [&](int64_t r, T v) { y[r] = add ? y[r] + v : v; });
}

// Coarsest level: x = A^-1 b with the dense inverse, one wave per row.
template <typename T>
__device__ inline void amg_coarse_body(const CgArgs& a, int64_t n, const T* inv,
                                       const T* b, T* x, VB vb) {
  if (a.ctrl->state != CG_ITER) return;
  const Range rows = my_range(n, vb);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t i0 = rows.lo; i0 < rows.hi; i0 += blockDim.x >> 6) {
    const int64_t i = i0 + wave;
    T s = 0;
    if (i < rows.hi)
      for (int64_t j = lane; j < n; j += 64) s += inv[i * n + j] * b[j];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (i < rows.hi && lane == 0) x[i] = s;
  }
}

// Post-smoothing: out = x + w D^-1 (b - A x); on the finest level out is
// the CG vector u (FP64) and the workgroups write their share of (r,u).
template <typename T>
__device__ inline void amg_post_body(const CgArgs& a, const AmgLevel& L,
                                     int level, VB vb) {
  if (a.ctrl->state != CG_ITER) return;
  const LevelVecs<T> V = level_vecs<T>(L);
  const double* __restrict__ r64 = a.r;
  const T* __restrict__ x = V.x;
  const T omega = (T)L.omega;
  double v[1] = {0.0};
  amg_rows<T>(L.A, vb, [&](int32_t c) { return x[c]; },
              [&](int64_t r, T ax) {
                const T br = level == 0 ? (T)r64[r] : V.b[r];
                const T o = x[r] + omega * (V.dinv[r] * (br - ax));
                if (level == 0) {
                  a.u[r] = (double)o;
                  v[0] += r64[r] * (double)o;
                } else {
                  V.t[r] = o;
                }
              });
  if (level == 0) write_partials<1>(slot(a, 5 + 2 * (a.ctrl->it_a & 1)), a.G, v, vb);
}

// w = K u and (w,u); it_b = it_a.
__device__ inline void amg_spmv_body(const CgArgs& a, VB vb) {
  CgCtrl* c = a.ctrl;
  if (c->state != CG_ITER) return;
  const int it = c->it_a;
  if (vb.id == 0 && threadIdx.x == 0) c->it_b = it;
  const DevMesh& m = a.m;
  double v[1] = {0.0};
  spmv_sell(m.k_sptr, m.k_scol, m.k_sval, a.u, m.k_nslices, m.n_free, vb,
            [&](int64_t i, double s) {
              a.w[i] = s;
              v[0] += s * a.u[i];
            });
  write_partials<1>(slot(a, 8 + (it & 1)), a.G, v, vb);
}

// Scalars of iteration it from (r,u) and (w,u), then p, s, x, r and (r,r);
// it_a = it + 1.
__device__ inline void amg_upd_body(const CgArgs& a, VB vb) {
  CgCtrl* c = a.ctrl;
  if (c->state != CG_ITER) return;
  const int it = c->it_b;
  const int pb = it & 1;
  double t1[1], t2[1];
  totals<1>(slot(a, 5 + 2 * pb), a.G, 1, t1);
  totals<1>(slot(a, 8 + pb), a.G, 1, t2);
  const double gamma = t1[0];
  double alpha, beta;
  if (it == 0) {
    beta = 0.0;
    alpha = gamma / t2[0];
  } else {
    beta = gamma / c->gamma[pb ^ 1];
    alpha = gamma / (t2[0] - beta * gamma / c->alpha[pb ^ 1]);
  }
  if (vb.id == 0 && threadIdx.x == 0) {
    c->gamma[pb] = gamma;
    c->alpha[pb] = alpha;
    c->it_a = it + 1;
  }
  const Range rows = my_range(a.m.n_free, vb);
  double v[1] = {0.0};
  for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x) {
    const double pi = it == 0 ? a.u[i] : a.u[i] + beta * a.p[i];
    const double si = it == 0 ? a.w[i] : a.w[i] + beta * a.s[i];
    a.p[i] = pi;
    a.s[i] = si;
    a.x[i] += alpha * pi;
    const double ri = a.r[i] - alpha * si;
    a.r[i] = ri;
    v[0] += ri * ri;
  }
  write_partials<1>(slot(a, 4 + 2 * pb), a.G, v, vb);
}

// One instance: the level, matrix and vectors come as kernel arguments.
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_down(CgArgs a, AmgLevel L,
                                                       int level) {
  amg_down_body<T>(a, L, level, VB{(int)blockIdx.x, (int)gridDim.x});
}
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_apply(CgArgs a, SellMat M,
                                                        const T* x, T* y,
                                                        int add) {
  amg_apply_body<T>(a, M, x, y, add, VB{(int)blockIdx.x, (int)gridDim.x});
}
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_coarse(CgArgs a, int64_t n,
                                                         const T* inv,
                                                         const T* b, T* x) {
  amg_coarse_body<T>(a, n, inv, b, x, VB{(int)blockIdx.x, (int)gridDim.x});
}
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_post(CgArgs a, AmgLevel L,
                                                       int level) {
  amg_post_body<T>(a, L, level, VB{(int)blockIdx.x, (int)gridDim.x});
}
__global__ void __launch_bounds__(kCgBlock) k_amg_spmv(CgArgs a) {
  amg_spmv_body(a, VB{(int)blockIdx.x, (int)gridDim.x});
}
__global__ void __launch_bounds__(kCgBlock) k_amg_upd(CgArgs a) {
  amg_upd_body(a, VB{(int)blockIdx.x, (int)gridDim.x});
}

// Several instances: block -> (instance, virtual block) by the schedule;
// each instance's hierarchy is read from the device copy of its AmgDev.
struct AmgBatch {
  const CgArgs* args;
  BatchMap map;
};

template <typename T>
__device__ inline T* coarse_vec(const AmgDev& D, int which) {
  if constexpr (std::is_same<T, float>::value)
    return which ? D.coarse_x32 : D.coarse_b32;
  else
    return which ? D.coarse_x : D.coarse_b;
}

template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_down_b(AmgBatch b, int level) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  const AmgLevel L = ((const AmgDev*)a.amg_dev)->lv[level];
  amg_down_body<T>(a, L, level, vb);
}
// restriction of level l's residual into the next level's right-hand side
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_restrict_b(AmgBatch b, int level) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  const AmgDev* D = (const AmgDev*)a.amg_dev;
  const AmgLevel& L = D->lv[level];
  T* nb = level + 1 < D->n_levels ? level_vecs<T>(D->lv[level + 1]).b
                                  : coarse_vec<T>(*D, 0);
  amg_apply_body<T>(a, L.R, (const T*)level_vecs<T>(L).r, nb, 0, vb);
}
// the coarse correction of level l added to its pre-smoothed iterate
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_prolong_b(AmgBatch b, int level) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  const AmgDev* D = (const AmgDev*)a.amg_dev;
  const AmgLevel& L = D->lv[level];
  const T* y = level + 1 < D->n_levels ? level_vecs<T>(D->lv[level + 1]).t
                                       : coarse_vec<T>(*D, 1);
  amg_apply_body<T>(a, L.P, y, level_vecs<T>(L).x, 1, vb);
}
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_coarse_b(AmgBatch b) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  const AmgDev* D = (const AmgDev*)a.amg_dev;
  const T* inv;
  if constexpr (std::is_same<T, float>::value) inv = D->coarse_inv32;
  else inv = D->coarse_inv;
  amg_coarse_body<T>(a, D->n_coarse, inv, coarse_vec<T>(*D, 0),
                     coarse_vec<T>(*D, 1), vb);
}
template <typename T>
__global__ void __launch_bounds__(kCgBlock) k_amg_post_b(AmgBatch b, int level) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  const AmgLevel L = ((const AmgDev*)a.amg_dev)->lv[level];
  amg_post_body<T>(a, L, level, vb);
}
__global__ void __launch_bounds__(kCgBlock) k_amg_spmv_b(AmgBatch b) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  amg_spmv_body(a, vb);
}
__global__ void __launch_bounds__(kCgBlock) k_amg_upd_b(AmgBatch b) {
  int i;
  const VB vb = batch_block(b.map, i);
  const CgArgs a = b.args[i];
  amg_upd_body(a, vb);
}

namespace {

// Workgroups for a level kernel over n rows: the full solver grid on the
// finest level (its kernels also reduce over that grid), fewer below, so
// that the small coarse passes do not launch and drain hundreds of idle
// workgroups.
template <typename T>
struct CoarseVecs {
  const T* inv;
  T *b, *x;
};
template <typename T>
CoarseVecs<T> coarse_host(const AmgDev& d) {
  if constexpr (std::is_same<T, float>::value)
    return CoarseVecs<T>{d.coarse_inv32, d.coarse_b32, d.coarse_x32};
  else
    return CoarseVecs<T>{d.coarse_inv, d.coarse_b, d.coarse_x};
}

// Workgroups for a level kernel over the rows of M: one lane of work per
// thread (a row takes M.lpr lanes; the rows of a SELL slice share a lane
// column), at most the solver grid, so that the small coarse passes neither
// loop over row groups in one workgroup nor launch and drain hundreds of
// idle workgroups.  The finest level's smoothing kernels keep the solver
// grid (they also reduce over it).
int amg_grid(const CgArgs& a, const SellMat& M) {
  const int64_t lanes = M.nrows * (int64_t)M.lpr;
  const int64_t want = (lanes + kCgBlock - 1) / kCgBlock;
  int g = (int)std::min<int64_t>(a.G, std::max<int64_t>(8, want));
  return g >= 8 ? g - g % 8 : g;
}

template <typename T>
hipError_t amg_iters_t(const CgArgs& a, const AmgDev& d, int n, hipStream_t s) {
  const dim3 b(kCgBlock);
  const int L = d.n_levels;
  auto vec = [](const AmgLevel& lv) { return level_vecs<T>(lv); };
  const auto cv = coarse_host<T>(d);
  // one wave per row of the dense coarsest inverse
  const int gc = (int)std::min<int64_t>(
      a.G, std::max<int64_t>(8, (d.n_coarse + kCgBlock / 64 - 1) / (kCgBlock / 64)));
  for (int k = 0; k < n; ++k) {
    for (int l = 0; l < L; ++l) {
      const AmgLevel& lv = d.lv[l];
      hipLaunchKernelGGL(k_amg_down<T>, dim3(l == 0 ? a.G : amg_grid(a, lv.A)), b, 0,
                         s, a, lv, l);
      T* nb = l + 1 < L ? vec(d.lv[l + 1]).b : cv.b;
      hipLaunchKernelGGL(k_amg_apply<T>, dim3(amg_grid(a, lv.R)), b, 0, s, a, lv.R,
                         (const T*)vec(lv).r, nb, 0);
    }
    hipLaunchKernelGGL(k_amg_coarse<T>, dim3(gc), b, 0, s, a, d.n_coarse, cv.inv,
                       (const T*)cv.b, cv.x);
    for (int l = L - 1; l >= 0; --l) {
      const AmgLevel& lv = d.lv[l];
      const T* y = l + 1 < L ? vec(d.lv[l + 1]).t : cv.x;
      hipLaunchKernelGGL(k_amg_apply<T>, dim3(amg_grid(a, lv.P)), b, 0, s, a, lv.P, y,
                         vec(lv).x, 1);
      hipLaunchKernelGGL(k_amg_post<T>, dim3(l == 0 ? a.G : amg_grid(a, lv.A)), b, 0,
                         s, a, lv, l);
    }
    hipLaunchKernelGGL(k_amg_spmv, dim3(a.G), b, 0, s, a);
    hipLaunchKernelGGL(k_amg_upd, dim3(a.G), b, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t amg_launch_iters(const CgArgs& a, const AmgDev& d, int n,
                            hipStream_t s) {
  return a.amg32 ? amg_iters_t<float>(a, d, n, s) : amg_iters_t<double>(a, d, n, s);
}

namespace {

// Workgroups of one dense coarse solve: one wave per row.
int coarse_grid(const CgArgs& a, int64_t n_coarse) {
  return (int)std::min<int64_t>(
      a.G, std::max<int64_t>(8, (n_coarse + kCgBlock / 64 - 1) / (kCgBlock / 64)));
}

// Schedule over the instances with on[i] and count(i) > 0 workgroups.
template <typename F>
BatchMap sched(const std::vector<char>& on, F&& count) {
  BatchMap m;
  std::memset(&m, 0, sizeof m);
  int j = 0;
  for (size_t i = 0; i < on.size(); ++i) {
    if (!on[i]) continue;
    const int c = count((int)i);
    if (c <= 0) continue;
    m.inst[j] = (int8_t)i;
    m.off[j + 1] = m.off[j] + c;
    ++j;
  }
  m.n_seg = j;
  return m;
}

template <typename T>
hipError_t amg_batch_t(const CgArgs* dargs, const std::vector<const CgArgs*>& hargs,
                       const std::vector<char>& on, int n, hipStream_t s) {
  const dim3 blk(kCgBlock);
  auto hier = [&](int i) -> const AmgDev& { return *(const AmgDev*)hargs[i]->amg; };
  int L = 0;
  for (size_t i = 0; i < on.size(); ++i)
    if (on[i]) L = std::max(L, hier((int)i).n_levels);
  BatchMap mA[kAmgMaxLevels], mR[kAmgMaxLevels], mP[kAmgMaxLevels];
  for (int l = 0; l < L; ++l) {
    mA[l] = sched(on, [&](int i) {
      const AmgDev& d = hier(i);
      return l >= d.n_levels ? 0 : l == 0 ? hargs[i]->G : amg_grid(*hargs[i], d.lv[l].A);
    });
    mR[l] = sched(on, [&](int i) {
      const AmgDev& d = hier(i);
      return l >= d.n_levels ? 0 : amg_grid(*hargs[i], d.lv[l].R);
    });
    mP[l] = sched(on, [&](int i) {
      const AmgDev& d = hier(i);
      return l >= d.n_levels ? 0 : amg_grid(*hargs[i], d.lv[l].P);
    });
  }
  const BatchMap mC = sched(on, [&](int i) { return coarse_grid(*hargs[i], hier(i).n_coarse); });
  const BatchMap mG = sched(on, [&](int i) { return hargs[i]->G; });
  auto grid = [](const BatchMap& m) { return m.off[m.n_seg]; };
  auto B = [&](const BatchMap& m) { return AmgBatch{dargs, m}; };
  for (int k = 0; k < n; ++k) {
    for (int l = 0; l < L; ++l) {
      if (grid(mA[l])) hipLaunchKernelGGL(k_amg_down_b<T>, dim3(grid(mA[l])), blk, 0, s, B(mA[l]), l);
      if (grid(mR[l])) hipLaunchKernelGGL(k_amg_restrict_b<T>, dim3(grid(mR[l])), blk, 0, s, B(mR[l]), l);
    }
    if (grid(mC)) hipLaunchKernelGGL(k_amg_coarse_b<T>, dim3(grid(mC)), blk, 0, s, B(mC));
    for (int l = L - 1; l >= 0; --l) {
      if (grid(mP[l])) hipLaunchKernelGGL(k_amg_prolong_b<T>, dim3(grid(mP[l])), blk, 0, s, B(mP[l]), l);
      if (grid(mA[l])) hipLaunchKernelGGL(k_amg_post_b<T>, dim3(grid(mA[l])), blk, 0, s, B(mA[l]), l);
    }
    if (grid(mG)) {
      hipLaunchKernelGGL(k_amg_spmv_b, dim3(grid(mG)), blk, 0, s, B(mG));
      hipLaunchKernelGGL(k_amg_upd_b, dim3(grid(mG)), blk, 0, s, B(mG));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t amg_batch_iters(const CgArgs* dargs, const std::vector<const CgArgs*>& hargs,
                           const std::vector<char>& on, int n, hipStream_t s) {
  int f32 = -1;
  for (size_t i = 0; i < on.size(); ++i) {
    if (!on[i]) continue;
    if (!hargs[i]->amg || !hargs[i]->amg_dev) return hipErrorInvalidValue;
    if (f32 >= 0 && f32 != hargs[i]->amg32) return hipErrorInvalidValue;
    f32 = hargs[i]->amg32;
  }
  if (f32 < 0 || n <= 0) return hipSuccess;
  return f32 ? amg_batch_t<float>(dargs, hargs, on, n, s)
             : amg_batch_t<double>(dargs, hargs, on, n, s);
}

#define LAUNCH(kern, ...)                                                   \
  do {                                                                      \
    hipLaunchKernelGGL(kern, dim3(a.G), dim3(kCgBlock), 0, s, __VA_ARGS__); \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess) return e_;                                        \
  } while (0)

hipError_t cg_launch_begin(const CgArgs& a, int64_t seq, hipStream_t s) {
  const bool inc = a.incremental && !a.rhs && a.bprev;
  if (a.lean) {
    if (!inc || !a.next_stats || !a.charge ||
        (const int64_t*)a.clear_charge != a.charge)
      return hipErrorInvalidValue;
    LAUNCH(k_cg_resinc, a);
    // the test in one workgroup (no product to start)
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kCgBlock), 0, s, a, seq, 3);
    return hipGetLastError();
  }
  if (inc)
    LAUNCH(k_cg_resinc, a);
  else
    LAUNCH(k_cg_resfield, a, 1, 0);
  LAUNCH(k_cg_start, a, seq, 0);
  return hipSuccess;
}

hipError_t cg_launch_lean_iter(const CgArgs& a, hipStream_t s) {
  if (!a.lean) return hipErrorInvalidValue;
  LAUNCH(k_cg_prep, a);
  if (!a.amg) LAUNCH(k_cg_start, a, (int64_t)0, 2);
  return hipSuccess;
}

hipError_t cg_launch_iters(const CgArgs& a, int it0, int n, int64_t seq,
                           hipStream_t s) {
  for (int k = 0; k < n; ++k) {
    LAUNCH(k_cg_upd, a, it0 + k);
    LAUNCH(k_cg_spmv, a, it0 + k, k == n - 1 ? seq : (int64_t)0);
  }
  return hipSuccess;
}

hipError_t cg_launch_report(const CgArgs& a, int64_t seq, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_report, dim3(1), dim3(64), 0, s, a, seq);
  return hipGetLastError();
}

hipError_t cg_launch_iters_dev(const CgArgs& a, int n, hipStream_t s) {
  for (int k = 0; k < n; ++k) {
    LAUNCH(k_cg_upd, a, -1);
    LAUNCH(k_cg_spmv, a, -1, (int64_t)0);
  }
  return hipSuccess;
}

hipError_t cg_launch_recheck(const CgArgs& a, int64_t seq, hipStream_t s) {
  LAUNCH(k_cg_scatter, a, 0);
  LAUNCH(k_cg_resfield, a, 0, 0);
  LAUNCH(k_cg_start, a, seq, 0);
  return hipSuccess;
}

hipError_t cg_launch_recheck_if(const CgArgs& a, hipStream_t s) {
  LAUNCH(k_cg_scatter, a, 1);
  LAUNCH(k_cg_resfield, a, 0, 1);
  LAUNCH(k_cg_start, a, (int64_t)0, 1);
  return hipSuccess;
}

#define BLAUNCH(kern, ...)                                                    \
  do {                                                                        \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kCgBlock), 0, s, __VA_ARGS__);  \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess) return e_;                                          \
  } while (0)

hipError_t cg_batch_begin(const CgBatch& b, int grid, int incremental,
                          hipStream_t s) {
  if (incremental)
    BLAUNCH(k_cg_resinc_b, b);
  else
    BLAUNCH(k_cg_resfield_b, b, 1, 0);
  BLAUNCH(k_cg_start_b, b, 0);
  return hipSuccess;
}

hipError_t cg_batch_iters(const CgBatch& b, int grid, int n, hipStream_t s) {
  for (int k = 0; k < n; ++k) {
    BLAUNCH(k_cg_upd_b, b);
    BLAUNCH(k_cg_spmv_b, b);
  }
  return hipSuccess;
}

hipError_t cg_batch_recheck(const CgBatch& b, int grid, hipStream_t s) {
  BLAUNCH(k_cg_scatter_b, b, 1);
  BLAUNCH(k_cg_resfield_b, b, 0, 1);
  BLAUNCH(k_cg_start_b, b, 1);
  return hipSuccess;
}

hipError_t cg_batch_recheck_if(const CgBatch& b, int grid, hipStream_t s) {
  BLAUNCH(k_cg_scatter_b, b, 2);
  BLAUNCH(k_cg_resfield_b, b, 0, 2);
  BLAUNCH(k_cg_start_b, b, 2);
  return hipSuccess;
}

hipError_t cg_batch_report(const CgBatch& b, int n, int64_t seq, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_report_b, dim3(1), dim3(kMaxBatch), 0, s, b, n, seq);
  return hipGetLastError();
}

}  // namespace fp
