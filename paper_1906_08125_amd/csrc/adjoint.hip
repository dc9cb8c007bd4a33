// Reverse of one PIC step (an addition to the paper, which has no adjoint).
//
// The step map is differentiated where it is smooth: the containing tets,
// the absorption events, the emission counts and the injection draws are
// held fixed, and the fixed-point rounding of the deposition is taken as
// exact (c = sum lambda w, scaled).  With rb, vb the adjoints of the
// post-step positions and velocities and Eb that of E_{k+1}:
//   Eb += objective term (mean |E| at the emitting-face centroids),
//   rhs = R^T Eb, K mu = rhs (K symmetric: the forward solver),
//   dJ/dE0 += g . mu, cb = (-e/eps0) w_sp mu,
//   kept superparticle at r' (tet t', map m'):
//     rb += w sum_j (cb[n_j] - cb[n_0]) m'_j,  sb[birth] += omega sum_i cb[n_i] lambda_i(r')
//   anode-collected: sb[birth] += wQ w_sp omega
//   pre-step superparticle (kick v' = v + 2Q E(r), drift r' = r + dt v'):
//     vt = vb + dt rb, a = 2Q vt, rb_prev = rb + sum_j m_j ((E_k[n_j] - E_k[n_0]) . a),
//     vb_prev = vt, Eb_k[n_i] += lambda_i(r) a
//   injected (r' = x_f + dt (1 + R) v0, v0 = (q/m) dt (0.5 + R) E_f):
//     v0b = vb + dt (1 + R) rb, Eb_k[face nodes] += (l0, R1, R2) (q/m) dt (0.5 + R) v0b
// with omega = w / s_birth the weight before the face multiplier.
//
// The scatters into nodes and faces are deterministic: every contribution
// is rounded to a 64-bit integer at a power-of-two scale chosen from the
// largest contribution (so no sum can overflow), added with integer
// atomics (exact, order-free) and converted back once.
#include "adjoint.h"

namespace fp {

namespace {

struct Range {
  int64_t lo, hi;
};

// contiguous, XCD-grouped share of [0, n) for this workgroup
__device__ inline Range my_range(int64_t n) {
  const int G = gridDim.x;
  const int g = blockIdx.x;
  int chunk = g;
  if ((G & 7) == 0) chunk = (g & 7) * (G >> 3) + (g >> 3);
  const int64_t per = (n + G - 1) / G;
  Range r;
  r.lo = (int64_t)chunk * per;
  if (r.lo > n) r.lo = n;
  r.hi = r.lo + per < n ? r.lo + per : n;
  return r;
}

__device__ inline void ld_pos(const void* x, const void* y, const void* z,
                              int f32, int64_t i, double& px, double& py,
                              double& pz) {
  if (f32) {
    px = ((const float*)x)[i];
    py = ((const float*)y)[i];
    pz = ((const float*)z)[i];
  } else {
    px = ((const double*)x)[i];
    py = ((const double*)y)[i];
    pz = ((const double*)z)[i];
  }
}

__device__ inline double4 ld_field(const void* E, int e32, int32_t node) {
  if (e32) {
    const float4 e = reinterpret_cast<const float4*>(E)[node];
    return make_double4(e.x, e.y, e.z, 0.0);
  }
  return reinterpret_cast<const double4*>(E)[node];
}

template <int NT>
__device__ inline double block_sum(double v) {
  __shared__ double lds[NT / 64];
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += lds[w];
  __syncthreads();
  return s;
}

template <int NT>
__device__ inline double block_max(double v) {
  __shared__ double lds[NT / 64];
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s = fmax(s, lds[w]);
  __syncthreads();
  return s;
}

// Power-of-two scale S with (n + 1) vmax S < 2^62.
__device__ inline double fx_scale(double vmax, int64_t n) {
  if (!(vmax > 0.0)) return 1.0;
  int ex = 0;
  frexp(vmax * (double)(n + 1), &ex);
  int e = 62 - ex;
  if (e > 1000) e = 1000;
  return ldexp(1.0, e);
}

// The scatter scales, written by k_adj_scales after the particle kernel.
__device__ inline void adj_scales(const AdjArgs& a, double& S_s, double& S_E) {
  S_s = a.part[a.G + 2 * a.Gp];
  S_E = a.part[a.G + 2 * a.Gp + 1];
}

}  // namespace

// Objective term of E_{k+1}: d(wE mean_f |e_f|) / dE, the mean over the
// emitting faces and the T post-solve fields of the window.  One thread per
// node of the emitting faces sums its faces in ascending order.
__global__ void __launch_bounds__(256) k_adj_obj(AdjArgs a) {
  const DevMesh& m = a.m;
  const int64_t F = m.n_emit;
  if (a.initial || a.wE == 0.0 || F == 0) return;
  const double scale = a.wE / (3.0 * (double)F * (double)a.T);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m.en_n;
       j += (int64_t)gridDim.x * blockDim.x) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t q = m.en_ptr[j]; q < m.en_ptr[j + 1]; ++q) {
      const int32_t* nd = m.e_nodes + 3 * (int64_t)m.en_face[q];
      const double4 A = ld_field(a.Ek1, a.e32, nd[0]);
      const double4 B = ld_field(a.Ek1, a.e32, nd[1]);
      const double4 C = ld_field(a.Ek1, a.e32, nd[2]);
      const double ex = ((A.x + B.x) + C.x) / 3.0;
      const double ey = ((A.y + B.y) + C.y) / 3.0;
      const double ez = ((A.z + B.z) + C.z) / 3.0;
      const double n = sqrt((ex * ex + ey * ey) + ez * ez);
      const double k = n > 0.0 ? scale / n : 0.0;
      sx += k * ex;
      sy += k * ey;
      sz += k * ez;
    }
    double* e = a.Eb + 4 * (int64_t)m.en_node[j];
    e[0] += sx;
    e[1] += sy;
    e[2] += sz;
  }
}

// rhs = R^T Eb on the free rows; clears the fixed-point accumulators.
__global__ void __launch_bounds__(512) k_adj_rt(AdjArgs a) {
  const DevMesh& m = a.m;
  {
    const Range r = my_range(3 * m.n_nodes);
    for (int64_t i = r.lo + threadIdx.x; i < r.hi; i += blockDim.x) a.acc_E[i] = 0;
    const Range f = my_range(m.n_emit);
    for (int64_t i = f.lo + threadIdx.x; i < f.hi; i += blockDim.x) a.acc_s[i] = 0;
  }
  const int lane = threadIdx.x & (kSell - 1);
  const int sub = threadIdx.x / kSell;
  const int nsub = blockDim.x / kSell;
  const int64_t np = m.k_np, tnp = m.t_np;
  const Range sl = my_range(m.k_nslices);
  for (int64_t s = sl.lo + sub; s < sl.hi; s += nsub) {
    const int64_t r = s * kSell + lane;
    double acc = 0.0;
    for (int32_t p = m.k_sptr[s] + lane; p < m.k_sptr[s + 1]; p += kSell) {
      const double* e = a.Eb + 4 * (int64_t)m.k_ncol[p];
      acc += (m.rt_sval[p] * e[0] + m.rt_sval[np + p] * e[1]) +
             m.rt_sval[2 * np + p] * e[2];
    }
    for (int32_t p = m.t_sptr[s] + lane; p < m.t_sptr[s + 1]; p += kSell) {
      const double* e = a.Eb + 4 * (int64_t)m.t_ncol[p];
      acc += (m.t_sval[p] * e[0] + m.t_sval[tnp + p] * e[1]) +
             m.t_sval[2 * tnp + p] * e[2];
    }
    if (r < m.n_free) a.rhs[r] = acc;
  }
}

// Partial sums of g . mu (slot 0 of part).
__global__ void __launch_bounds__(512) k_adj_mu(AdjArgs a) {
  const DevMesh& m = a.m;
  const Range r = my_range(m.n_free);
  double v = 0.0;
  for (int64_t i = r.lo + threadIdx.x; i < r.hi; i += blockDim.x)
    v += m.g_unit[i] * a.mu[m.free2node[i]];
  v = block_sum<512>(v);
  if (threadIdx.x == 0) a.part[blockIdx.x] = v;
}

// Per slot: the deposition, collection, kick and drift reverses (see the
// file comment); writes the adjoint of the pre-step state in place, the
// weight contribution sc and the gather-adjoint vector a (and the draws of
// an injected superparticle), and the block maxima used for the scales.
__global__ void __launch_bounds__(kAdjBlock) k_adj_particles(AdjArgs a) {
  const DevMesh& m = a.m;
  const int64_t npre = *a.n_pre;
  const int64_t n = a.initial ? npre : *a.n_post;
  const int64_t cap = a.cap;
  double msc = 0.0, ma = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int tq = a.qtet[i];
    const bool pre_live = !a.initial && i < npre && a.ptet[i] >= 0;
    const bool inj = !a.initial && i >= npre;
    double sc = 0.0, ax = 0.0, ay = 0.0, az = 0.0, R1 = 0.0, R2 = 0.0;
    double orb[3] = {0.0, 0.0, 0.0}, ovb[3] = {0.0, 0.0, 0.0};
    if (a.initial || pre_live || inj) {
      const double w = a.qw[i];
      const int f = a.qbirth[i];
      const double sf = a.s_face ? a.s_face[f] : 1.0;
      const double omega = w / sf;
      double qx, qy, qz;
      ld_pos(a.qx, a.qy, a.qz, a.f32, i, qx, qy, qz);
      if (tq >= 0) {
        const TetGeom G = m.tg[tq];
        double lam[4];
        barycentric(G, qx, qy, qz, lam);
        double c[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) c[l] = a.coef_real * a.mu[G.node[l]];
        sc = omega * (((c[0] * lam[0] + c[1] * lam[1]) + c[2] * lam[2]) +
                      c[3] * lam[3]);
        if (!a.initial) {
          double r[3] = {a.rb[i], a.rb[cap + i], a.rb[2 * cap + i]};
          const double v[3] = {a.vb[i], a.vb[cap + i], a.vb[2 * cap + i]};
          const double d1 = c[1] - c[0], d2 = c[2] - c[0], d3 = c[3] - c[0];
#pragma unroll
          for (int k = 0; k < 3; ++k)
            r[k] += w * ((d1 * G.m[k] + d2 * G.m[3 + k]) + d3 * G.m[6 + k]);
          if (pre_live) {
            double vt[3], av[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              vt[k] = v[k] + a.dt * r[k];
              av[k] = (a.qm * a.dt) * vt[k];
            }
            double px, py, pz;
            ld_pos(a.px, a.py, a.pz, a.f32, i, px, py, pz);
            const TetGeom G0 = m.tg[a.ptet[i]];
            const double4 E0 = ld_field(a.Ek, a.e32, G0.node[0]);
            double proj[3];
#pragma unroll
            for (int j = 1; j < 4; ++j) {
              const double4 Ej = ld_field(a.Ek, a.e32, G0.node[j]);
              proj[j - 1] = ((Ej.x - E0.x) * av[0] + (Ej.y - E0.y) * av[1]) +
                            (Ej.z - E0.z) * av[2];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              orb[k] = r[k] + ((proj[0] * G0.m[k] + proj[1] * G0.m[3 + k]) +
                               proj[2] * G0.m[6 + k]);
              ovb[k] = vt[k];
            }
            ax = av[0];
            ay = av[1];
            az = av[2];
          } else {
            const int64_t id = a.qid[i];
            const uint64_t o = (uint64_t)(id & ((1ll << 21) - 1));
            const uint64_t fi = (uint64_t)((id >> 21) & ((1ll << 21) - 1));
            uint64_t r4[4];
            philox4x64_10(a.seed, a.instance, (uint64_t)a.step, fi, o, 1, r4);
            R1 = unit_double(r4[0]);
            R2 = unit_double(r4[1]);
            const double Rf = unit_double(r4[2]);
            if (R1 + R2 > 1.0) {
              R1 = 1.0 - R1;
              R2 = 1.0 - R2;
            }
            const double k1 = a.dt * (1.0 + Rf);
            const double k2 = (a.qm * a.dt) * (0.5 + Rf);
            ax = k2 * (v[0] + k1 * r[0]);
            ay = k2 * (v[1] + k1 * r[1]);
            az = k2 * (v[2] + k1 * r[2]);
          }
        }
      } else if (!a.initial && qz >= m.z_top) {
        sc = a.wQ * a.w_sp * omega;
      }
    }
    if (!a.initial) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a.rb[k * cap + i] = orb[k];
        a.vb[k * cap + i] = ovb[k];
      }
    }
    a.sc[i] = sc;
    a.av[i] = ax;
    a.av[cap + i] = ay;
    a.av[2 * cap + i] = az;
    a.av[3 * cap + i] = R1;
    a.av[4 * cap + i] = R2;
    msc = fmax(msc, fabs(sc));
    ma = fmax(ma, fmax(fabs(ax), fmax(fabs(ay), fabs(az))));
  }
  msc = block_max<kAdjBlock>(msc);
  ma = block_max<kAdjBlock>(ma);
  if (threadIdx.x == 0) {
    a.part[a.G + blockIdx.x] = msc;
    a.part[a.G + a.Gp + blockIdx.x] = ma;
  }
}

// Scales of the weight (S_s) and field (S_E) scatters from the per-block
// maxima of the particle kernel (one workgroup).
__global__ void __launch_bounds__(256) k_adj_scales(AdjArgs a) {
  double ms = 0.0, ma = 0.0;
  for (int j = threadIdx.x; j < a.Gp; j += blockDim.x) {
    ms = fmax(ms, a.part[a.G + j]);
    ma = fmax(ma, a.part[a.G + a.Gp + j]);
  }
  ms = block_max<256>(ms);
  ma = block_max<256>(ma);
  if (threadIdx.x == 0) {
    const int64_t n = a.initial ? *a.n_pre : *a.n_post;
    a.part[a.G + 2 * a.Gp] = fx_scale(ms, n);
    a.part[a.G + 2 * a.Gp + 1] = fx_scale(ma, n);
  }
}

// Fixed-point scatters of the weight contributions (to faces) and of the
// gather-adjoint vectors (to nodes).
// Per-workgroup accumulation before the global integer atomics: thousands
// of superparticles add into the same face (born there) and, sorted by tet,
// into the same few nodes, and same-address atomics in L2 serialize.  A
// workgroup sums its contributions in LDS -- a node table (open addressing)
// and, when the faces fit, one slot per face -- and flushes one atomic per
// distinct node component and face.  Integer addition is exact and
// order-free, so the totals are unchanged.
constexpr int kAdjTable = 1024;  // > 4 nodes x the superparticles of a chunk
constexpr int kAdjFaces = 2048;

struct AdjTable {
  int32_t key[kAdjTable];
  unsigned long long v[3][kAdjTable];
  unsigned long long face[kAdjFaces];
};

__device__ inline void adj_node_add(AdjTable& T, int32_t node, const long long q[3],
                                    long long* acc) {
  uint32_t h = ((uint32_t)node * 2654435761u) >> 22;  // 10 bits
  // kept as a loop (unrolled at each call site it bloats the kernel and
  // spills scalar registers)
#pragma unroll 1
  for (int probe = 0; probe < 64; ++probe) {
    const int32_t old = atomicCAS(&T.key[h], -1, node);
    if (old == -1 || old == node) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (q[k]) atomicAdd(&T.v[k][h], (unsigned long long)q[k]);
      return;
    }
    h = (h + 1) & (kAdjTable - 1);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (q[k]) atomicAdd((unsigned long long*)(acc + 3 * (int64_t)node + k),
                        (unsigned long long)q[k]);
}

__global__ void __launch_bounds__(kAdjBlock) k_adj_scatter(AdjArgs a) {
  const DevMesh& m = a.m;
  __shared__ AdjTable T;
  const bool faces_lds = m.n_emit <= kAdjFaces;
  for (int k = threadIdx.x; k < kAdjTable; k += blockDim.x) {
    T.key[k] = -1;
    T.v[0][k] = T.v[1][k] = T.v[2][k] = 0ull;
  }
  for (int k = threadIdx.x; k < kAdjFaces; k += blockDim.x) T.face[k] = 0ull;
  __syncthreads();
  double S_s, S_E;
  adj_scales(a, S_s, S_E);
  const int64_t npre = *a.n_pre;
  const int64_t n = a.initial ? npre : *a.n_post;
  const int64_t cap = a.cap;
  const Range rg = my_range(n);
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += blockDim.x) {
    const double sc = a.sc[i];
    if (sc != 0.0) {
      const long long q = __double2ll_rn(sc * S_s);
      if (faces_lds)
        atomicAdd(&T.face[a.qbirth[i]], (unsigned long long)q);
      else
        atomicAdd((unsigned long long*)(a.acc_s + a.qbirth[i]), (unsigned long long)q);
    }
    if (a.initial || a.qtet[i] < 0) continue;
    const double av[3] = {a.av[i], a.av[cap + i], a.av[2 * cap + i]};
    if (i < npre) {
      if (a.ptet[i] < 0) continue;
      double px, py, pz;
      ld_pos(a.px, a.py, a.pz, a.f32, i, px, py, pz);
      const TetGeom G0 = m.tg[a.ptet[i]];
      double lam[4];
      barycentric(G0, px, py, pz, lam);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        long long q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = __double2ll_rn(lam[l] * av[k] * S_E);
        adj_node_add(T, G0.node[l], q, a.acc_E);
      }
    } else {
      const double R1 = a.av[3 * cap + i], R2 = a.av[4 * cap + i];
      const double wgt[3] = {(1.0 - R1) - R2, R1, R2};
      const int32_t* nd = m.e_nodes + 3 * (int64_t)a.qbirth[i];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        long long q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = __double2ll_rn(wgt[f] * av[k] * S_E);
        adj_node_add(T, nd[f], q, a.acc_E);
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kAdjTable; k += blockDim.x) {
    const int32_t node = T.key[k];
    if (node < 0) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned long long v = T.v[c][k];
      if (v) atomicAdd((unsigned long long*)(a.acc_E + 3 * (int64_t)node + c), v);
    }
  }
  if (faces_lds)
    for (int k = threadIdx.x; k < m.n_emit; k += blockDim.x) {
      const unsigned long long v = T.face[k];
      if (v) atomicAdd((unsigned long long*)(a.acc_s + k), v);
    }
}

// Eb = the field adjoint of E_k (from the accumulators); dJ/ds and dJ/dE0.
__global__ void __launch_bounds__(512) k_adj_finish(AdjArgs a) {
  const DevMesh& m = a.m;
  double S_s, S_E;
  adj_scales(a, S_s, S_E);
  if (!a.initial) {
    const Range r = my_range(m.n_nodes);
    for (int64_t i = r.lo + threadIdx.x; i < r.hi; i += blockDim.x) {
      double4 e;
      e.x = (double)a.acc_E[3 * i] / S_E;
      e.y = (double)a.acc_E[3 * i + 1] / S_E;
      e.z = (double)a.acc_E[3 * i + 2] / S_E;
      e.w = 0.0;
      reinterpret_cast<double4*>(a.Eb)[i] = e;
    }
  }
  const Range f = my_range(m.n_emit);
  for (int64_t i = f.lo + threadIdx.x; i < f.hi; i += blockDim.x)
    a.dJ_ds[i] += (double)a.acc_s[i] / S_s;
  if (blockIdx.x == 0) {
    double v = 0.0;
    for (int j = threadIdx.x; j < a.G; j += blockDim.x) v += a.part[j];
    v = block_sum<512>(v);
    if (threadIdx.x == 0) {
      *a.dJ_dE0 += v;
      // the solve's ||b||^2 sits in the solver's control word
      if (a.bref) *a.bref = fmax(*a.bref, sqrt(a.ctrl->bb));
    }
  }
}

hipError_t adj_launch_pre_solve(const AdjArgs& a, hipStream_t s) {
  const int gobj = (int)((a.m.en_n + 255) / 256);
  hipLaunchKernelGGL(k_adj_obj, dim3(gobj > 0 ? gobj : 1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_rt, dim3(a.G), dim3(512), 0, s, a);
  return hipGetLastError();
}

hipError_t adj_launch_post_solve(const AdjArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_mu, dim3(a.G), dim3(512), 0, s, a);
  hipLaunchKernelGGL(k_adj_particles, dim3(a.Gp), dim3(kAdjBlock), 0, s, a);
  hipLaunchKernelGGL(k_adj_scales, dim3(1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_scatter, dim3(a.Gp), dim3(kAdjBlock), 0, s, a);
  hipLaunchKernelGGL(k_adj_finish, dim3(a.G), dim3(512), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window objective and face weights (the forward side of the adjoint's
// objective, reading R15): one workgroup sums |E| at the emitting-face
// centroids ((E_a + E_b) + E_c) / 3 in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kAdjBlock) k_window_objective(
    DevMesh m, const void* E, int f32, const pic_step_stats* st, double w_sp,
    double inv_T, double wQ, double wE, double* J) {
  __shared__ double lds[kAdjBlock / 64];
  double acc = 0.0;
  for (int64_t f = threadIdx.x; f < m.n_emit; f += blockDim.x) {
    const int32_t* nd = m.e_nodes + 3 * f;
    double e[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (f32) {
        const float4 v = reinterpret_cast<const float4*>(E)[nd[k]];
        e[k][0] = v.x;
        e[k][1] = v.y;
        e[k][2] = v.z;
      } else {
        const double4 v = reinterpret_cast<const double4*>(E)[nd[k]];
        e[k][0] = v.x;
        e[k][1] = v.y;
        e[k][2] = v.z;
      }
    }
    double c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = ((e[0][d] + e[1][d]) + e[2][d]) / 3.0;
    acc += sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += lds[w];
    const double mean = m.n_emit ? sum / (double)m.n_emit : 0.0;
    J[0] += (double)st->q_anode * (w_sp * kFxInv);
    J[1] += mean * inv_T;
    J[2] = wQ * J[0] + wE * J[1];
  }
}

__global__ void __launch_bounds__(kAdjBlock) k_face_weights(
    int64_t cap, const int32_t* n_slots, const int32_t* tet,
    const int32_t* birth, const double* w_base, const double* s_face,
    double* w) {
  const int64_t n = *n_slots < cap ? *n_slots : cap;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = tet[i] >= 0 ? w_base[i] * s_face[birth[i]] : w_base[i];
}

hipError_t launch_window_objective(const DevMesh& m, const void* E, int f32,
                                   const pic_step_stats* st, double w_sp,
                                   int T, double wQ, double wE, double* J,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_window_objective, dim3(1), dim3(kAdjBlock), 0, s, m, E,
                     f32, st, w_sp, 1.0 / (double)T, wQ, wE, J);
  return hipGetLastError();
}

hipError_t launch_face_weights(int64_t cap, const int32_t* n_slots,
                               const int32_t* tet, const int32_t* birth,
                               const double* w_base, const double* s_face,
                               double* w, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_face_weights, dim3(grid), dim3(kAdjBlock), 0, s, cap,
                     n_slots, tet, birth, w_base, s_face, w);
  return hipGetLastError();
}

}  // namespace fp
