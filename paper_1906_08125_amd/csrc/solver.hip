// Poisson solve on the free nodes (Eq. poisson with Eq. poisson_bc in the
// Galerkin form of App. B) as one cooperative persistent kernel: Jacobi-
// preconditioned CG in the single-reduction (Chronopoulos-Gear) ordering,
// warm started, with the stopping test re-checked on the true residual, then
// the nodal field E = R phi for every node.
//
// Layout: every workgroup owns one contiguous block of rows; block indices
// are assigned so that the 8 XCDs each sweep one contiguous eighth of the
// rows (workgroup g runs on XCD g mod 8), which keeps the SpMV's neighbour
// gathers inside one XCD's L2.  Reductions are deterministic: each
// workgroup writes a partial in a fixed order and every workgroup sums all
// partials in the same fixed order after the grid barrier.
#include <hip/hip_cooperative_groups.h>

#include "common.h"
#include "solver.h"

namespace cgs = cooperative_groups;

namespace fp {

namespace {

constexpr int kLPR = 8;  // lanes per CSR row in the SpMV

struct Rows {
  int64_t lo, hi;
};

__device__ inline Rows my_rows(int64_t n) {
  const int G = gridDim.x;
  const int g = blockIdx.x;
  int chunk = g;
  if ((G & 7) == 0) chunk = (g & 7) * (G >> 3) + (g >> 3);
  const int64_t per = (n + G - 1) / G;
  Rows r;
  r.lo = (int64_t)chunk * per;
  r.hi = r.lo + per < n ? r.lo + per : n;
  if (r.lo > n) r.lo = n;
  return r;
}

// Deterministic block sum of up to 3 values per thread; result valid in all
// threads.  Fixed shuffle pattern inside a wave, fixed wave order in LDS.
template <int NQ>
__device__ inline void block_sum(double (&v)[NQ], double* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) lds[q * 16 + wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[q * 16 + w];
    v[q] = s;
  }
  __syncthreads();
}

// Sum of the per-workgroup partials part[q*G + j] over j, identical in every
// workgroup (same data, same order).
template <int NQ>
__device__ inline void grid_total(const double* part, int G, double (&tot)[NQ],
                                  double* lds) {
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int j = threadIdx.x; j < G; j += blockDim.x) s += part[q * G + j];
    v[q] = s;
  }
  block_sum<NQ>(v, lds);
#pragma unroll
  for (int q = 0; q < NQ; ++q) tot[q] = v[q];
}

// y_i = sum_k val[k] x[col[k]] for the rows of this workgroup; returns via
// callback on the first lane of each row group.
template <typename F>
__device__ inline void spmv_rows(const DevMesh& m, const double* __restrict__ x,
                                 Rows rows, F&& emit) {
  const int sub = threadIdx.x % kLPR;
  const int grp = threadIdx.x / kLPR;
  const int ngrp = blockDim.x / kLPR;
  for (int64_t i0 = rows.lo; i0 < rows.hi; i0 += ngrp) {
    const int64_t i = i0 + grp;
    double s = 0.0;
    if (i < rows.hi) {
      const int k1 = m.rowptr[i + 1];
      for (int k = m.rowptr[i] + sub; k < k1; k += kLPR)
        s += m.val[k] * x[m.col[k]];
    }
#pragma unroll
    for (int off = kLPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, kLPR);
    if (i < rows.hi && sub == 0) emit(i, s);
  }
}

}  // namespace

__global__ void __launch_bounds__(512)
k_pcg_fp64(CgArgs a) {
  cgs::grid_group grid = cgs::this_grid();
  __shared__ double lds[64];
  const DevMesh& m = a.m;
  const int64_t n = m.n_free;
  const int G = gridDim.x;
  const Rows rows = my_rows(n);
  double* part = a.part;  // [2][4][G]
  auto P = [&](int buf, int q) { return part + ((size_t)buf * 4 + q) * G; };

  // right-hand side and warm start
  {
    double v[1] = {0.0};
    for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x) {
      const int32_t nd = m.free2node[i];
      const double c = a.charge ? (double)a.charge[nd] : 0.0;
      const double bi = a.coef * c + a.E0 * m.g_unit[i];
      a.b[i] = bi;
      a.x[i] = a.phi[nd];
      v[0] += bi * bi;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) P(0, 0)[blockIdx.x] = v[0];
  }
  grid.sync();
  double bn;
  {
    double t[1];
    grid_total<1>(P(0, 0), G, t, lds);
    bn = sqrt(t[0]);
  }
  int64_t it = 0;
  int64_t restarts = 0;
  int status = 0;
  double relres = 0.0;
  int buf = 1;
  if (bn == 0.0) {
    for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x)
      a.x[i] = 0.0;
    grid.sync();
  } else {
    const double thr = a.tol * bn;
    for (;;) {
      // true residual r = b - K x, u = D^-1 r
      {
        double v[1] = {0.0};
        spmv_rows(m, a.x, rows, [&](int64_t i, double s) {
          const double ri = a.b[i] - s;
          a.r[i] = ri;
          a.u[i] = ri * m.invdiag[i];
          v[0] += ri * ri;
        });
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) P(buf, 0)[blockIdx.x] = v[0];
      }
      grid.sync();
      double t1[1];
      grid_total<1>(P(buf, 0), G, t1, lds);
      buf ^= 1;
      relres = sqrt(t1[0]) / bn;
      if (sqrt(t1[0]) <= thr) break;
      if (it >= a.max_iter) {
        status = PIC_E_NOCONV;
        break;
      }
      ++restarts;
      // w = K u, gamma = (r, u), delta = (w, u)
      {
        double v[2] = {0.0, 0.0};
        spmv_rows(m, a.u, rows, [&](int64_t i, double s) {
          a.w[i] = s;
          const double ui = a.u[i];
          v[0] += a.r[i] * ui;
          v[1] += s * ui;
        });
        block_sum<2>(v, lds);
        if (threadIdx.x == 0) {
          P(buf, 0)[blockIdx.x] = v[0];
          P(buf, 1)[blockIdx.x] = v[1];
        }
      }
      grid.sync();
      double t2[2];
      grid_total<2>(P(buf, 0), G, t2, lds);
      buf ^= 1;
      double gamma = t2[0];
      double alpha = gamma / t2[1];
      double beta = 0.0;
      bool first = true;
      bool recheck = false;
      while (!recheck) {
        // row-local: p = u + beta p; s = w + beta s; x += alpha p;
        // r -= alpha s; u = D^-1 r; partial (r, r), (r, u)
        double v[3] = {0.0, 0.0, 0.0};
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
        first = false;
        grid.sync();
        ++it;
        // w = K u; partial (w, u)
        spmv_rows(m, a.u, rows, [&](int64_t i, double s) {
          a.w[i] = s;
          v[2] += s * a.u[i];
        });
        block_sum<3>(v, lds);
        if (threadIdx.x == 0) {
          P(buf, 0)[blockIdx.x] = v[0];
          P(buf, 1)[blockIdx.x] = v[1];
          P(buf, 2)[blockIdx.x] = v[2];
        }
        grid.sync();
        double t3[3];
        grid_total<3>(P(buf, 0), G, t3, lds);
        buf ^= 1;
        if (sqrt(t3[0]) <= thr || it >= a.max_iter) {
          recheck = true;
          break;
        }
        const double g1 = t3[1];
        beta = g1 / gamma;
        alpha = g1 / (t3[2] - beta * g1 / alpha);
        gamma = g1;
      }
    }
  }
  // scatter the solution; Dirichlet nodes hold 0
  for (int64_t i = rows.lo + threadIdx.x; i < rows.hi; i += blockDim.x)
    a.phi[m.free2node[i]] = a.x[i];
  {
    const Rows dr = my_rows(a.n_dir);
    for (int64_t i = dr.lo + threadIdx.x; i < dr.hi; i += blockDim.x)
      a.phi[a.dir_nodes[i]] = 0.0;
  }
  // nodal field E_i = sum_j R_ij x_j (x is complete after the last barrier)
  if (a.E) {
    const Rows fr = my_rows(m.n_nodes);
    const int sub = threadIdx.x % kLPR;
    const int grp = threadIdx.x / kLPR;
    const int ngrp = blockDim.x / kLPR;
    const int64_t nf = m.nnz_field;
    for (int64_t i0 = fr.lo; i0 < fr.hi; i0 += ngrp) {
      const int64_t i = i0 + grp;
      double ex = 0.0, ey = 0.0, ez = 0.0;
      if (i < fr.hi) {
        const int k1 = m.frow[i + 1];
        for (int k = m.frow[i] + sub; k < k1; k += kLPR) {
          const double xj = a.x[m.fcol[k]];
          ex += m.fval[k] * xj;
          ey += m.fval[nf + k] * xj;
          ez += m.fval[2 * nf + k] * xj;
        }
      }
#pragma unroll
      for (int off = kLPR / 2; off >= 1; off >>= 1) {
        ex += __shfl_xor(ex, off, kLPR);
        ey += __shfl_xor(ey, off, kLPR);
        ez += __shfl_xor(ez, off, kLPR);
      }
      if (i < fr.hi && sub == 0) {
        double4 e;
        e.x = ex;
        e.y = ey;
        e.z = ez;
        e.w = 0.0;
        reinterpret_cast<double4*>(a.E)[i] = e;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (a.stats) {
      a.stats->iters = it;
      a.stats->status = status;
      a.stats->restarts = restarts;
      a.stats->relres = relres;
      a.stats->bnorm = bn;
    }
    if (a.step_stats) {
      a.step_stats->cg_iters = it;
      a.step_stats->cg_relres = relres;
      if (status != 0 && a.step_stats->status == 0) a.step_stats->status = status;
    }
  }
}

hipError_t launch_pcg_fp64(const CgArgs& args, int grid, int block,
                           hipStream_t s) {
  void* kargs[] = {(void*)&args};
  return hipLaunchCooperativeKernel((const void*)k_pcg_fp64, dim3(grid),
                                    dim3(block), kargs, 0, s);
}

hipError_t pcg_fp64_occupancy(int block, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, (const void*)k_pcg_fp64, block, 0);
}

}  // namespace fp
