// Binary Monte Carlo collisions (App. F, after Takizuka and Abe) of the
// superparticles of each tet, on slots sorted by tet (as a re-sort leaves
// them):
//   k_coll_keys      a Philox key per superparticle, (step, id) counter;
//   k_coll_rank      each superparticle finds the run of its tet (a scan
//                    of its neighbours) and, in a short run, its rank by
//                    (key, id, slot); perm lists the run in rank order;
//   k_coll_rank_big  long runs (the tets at the emitter hold hundreds):
//                    a workgroup per run, keys staged through LDS;
//   k_coll_pair      the first member of every pair (in rank order)
//                    collides it (leaders queued per wave so that every
//                    lane computes); in a run of odd length the first three
//                    collide pairwise at half variance (one thread, in
//                    order).
// A collision (Eq. vel12, Eq. scat_vel, Eq. rot_mat, Eq. sin_theta,
// Eq. variance with the Landau logarithm 13): delta = tan(theta/2) normal
// with <delta^2> = (q/m)^2 (q/eps0)^2 n Lambda dt / (2 pi u^3 V), q and m
// the electron's, n = w_sp times the run's summed relative weight (summed
// in the fixed point of the charge, 2^-40 per unit, so that no order of
// atomic additions shows in the result); the relative velocity
// u = v2 - v1 turns to (I + M) u, so v1 -= dv/2 and v2 += dv/2 (energy and
// momentum conserved).  Draws: Philox at
// (step, id of the pair's first member, 4, j) for collision j of the pair
// leader; Box-Muller for the normal, a uniform azimuth.
#include "collide.h"

namespace fp {

namespace {

constexpr int kThreads = 256;
constexpr int kSmallRun = 62;    // runs ranked by their members alone
constexpr int kRankTile = 1024;  // keys per LDS tile of a long run
constexpr int kBigRuns = 1024;   // long runs ranked side by side
constexpr int kBigChunks = 4;    // member chunks of a run side by side
constexpr double kLandau = 13.0;
constexpr double kTwoPi = 6.283185307179586;

__device__ inline double3 ld_v(const CollideArgs& a, int32_t i) {
  if (a.f32)
    return make_double3(((const float*)a.v[0])[i], ((const float*)a.v[1])[i],
                        ((const float*)a.v[2])[i]);
  return make_double3(((const double*)a.v[0])[i], ((const double*)a.v[1])[i],
                      ((const double*)a.v[2])[i]);
}

__device__ inline void st_v(const CollideArgs& a, int32_t i, double3 v) {
  if (a.f32) {
    ((float*)a.v[0])[i] = (float)v.x;
    ((float*)a.v[1])[i] = (float)v.y;
    ((float*)a.v[2])[i] = (float)v.z;
  } else {
    ((double*)a.v[0])[i] = v.x;
    ((double*)a.v[1])[i] = v.y;
    ((double*)a.v[2])[i] = v.z;
  }
}

// Tet volume from the stored inverse map: V = 1 / (6 |det m|).
__device__ inline double tet_volume(const TetGeom& g) {
  const double* r = g.m;
  const double det = r[0] * (r[4] * r[8] - r[5] * r[7]) -
                     r[1] * (r[3] * r[8] - r[5] * r[6]) +
                     r[2] * (r[3] * r[7] - r[4] * r[6]);
  return 1.0 / (6.0 * fabs(det));
}

// One elastic collision of a and b; nv = n Lambda dt / V times the variance
// factor; the draws of collision j of the pair led by id lead.
__device__ void collide_pair(const CollideArgs& a, int32_t ia, int32_t ib,
                             double nv, int64_t lead, int j) {
  double3 va = ld_v(a, ia), vb = ld_v(a, ib);
  const double ux = vb.x - va.x, uy = vb.y - va.y, uz = vb.z - va.z;
  const double u = sqrt(ux * ux + uy * uy + uz * uz);
  if (!(u > 0.0)) return;
  const double var = a.c_var * nv / (u * u * u);
  uint64_t r[4];
  philox4x64_10(a.seed, a.instance, (uint64_t)a.step, (uint64_t)lead, 4,
                (uint64_t)j, r);
  const double U1 = 1.0 - unit_double(r[0]), U2 = unit_double(r[1]),
               U3 = unit_double(r[2]);
  const double g = sqrt(-2.0 * log(U1)) * cos(kTwoPi * U2);
  double delta = sqrt(var) * g;
  double st, omc;  // sin theta, 1 - cos theta
  if (delta != delta) delta = 0.0;  // infinite variance times g = 0
  if (fabs(delta) < 1e100) {
    st = 2.0 * delta / (1.0 + delta * delta);
    omc = 2.0 * delta * delta / (1.0 + delta * delta);
  } else {  // the same limits without overflow: theta -> pi
    const double r = 1.0 / delta;
    st = 2.0 * r;
    omc = 2.0 - 2.0 * r * r;
  }
  const double phi = kTwoPi * U3;
  double sp, cp;
  sincos(phi, &sp, &cp);
  const double up = sqrt(ux * ux + uy * uy);
  double dx, dy, dz;
  if (up > 0.0) {
    const double A = st * sp * u / up;
    const double bx = st * cp * ux / up, by = st * cp * uy / up;
    dx = -omc * ux + A * uy + bx * uz;
    dy = -A * ux - omc * uy + by * uz;
    dz = -bx * ux - by * uy - omc * uz;
  } else {
    dx = u * st * cp;
    dy = u * st * sp;
    dz = -omc * uz;
  }
  va.x -= 0.5 * dx;
  va.y -= 0.5 * dy;
  va.z -= 0.5 * dz;
  vb.x += 0.5 * dx;
  vb.y += 0.5 * dy;
  vb.z += 0.5 * dz;
  st_v(a, ia, va);
  st_v(a, ib, vb);
}

__global__ void __launch_bounds__(kThreads) k_coll_keys(CollideArgs a) {
  const int32_t n = *a.n_slots;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_big = 0;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gridDim.x * blockDim.x) {
    uint64_t r[4];
    philox4x64_10(a.seed, a.instance, (uint64_t)a.step, (uint64_t)a.id[i], 3,
                  0, r);
    a.key[i] = r[0];
    a.seg_q[i] = 0;
  }
}

// (key, id, slot) order: a permutation of the run even if ids repeat
// (branch-free, so that unrolled loops keep their loads in flight).
__device__ inline int before(uint64_t kj, int64_t dj, int32_t j, uint64_t ki,
                             int64_t di, int32_t i) {
  return (int)(kj < ki) |
         ((int)(kj == ki) & ((int)(dj < di) | ((int)(dj == di) & (int)(j < i))));
}

// Every wave stages the tets, keys, ids and weights of the slots
// [i0 - 64, i0 + 128) around its 64 slots in LDS; each slot scans its
// neighbours there (at most kSmallRun + 1 each way) for the run of its
// tet.  A run of up to kSmallRun is ranked here (each member counts the
// members before it; the first member sums the weights); the first member
// of a longer run finds its end by binary search and lists it for
// k_coll_rank_big.
constexpr int kWin = 192;    // staged slots per wave
constexpr int kWinLo = 64;   // of them before the wave's first slot
// the backward scan reads down to li - kSmallRun - 1 >= 0, the forward
// scan up to li + kSmallRun + 1 < kWin (li = kWinLo + lane)
static_assert(kSmallRun + 1 <= kWinLo, "the backward scan stays staged");
static_assert(kWinLo + 63 + kSmallRun + 1 < kWin, "the forward scan too");

__global__ void __launch_bounds__(kThreads) k_coll_rank(CollideArgs a) {
  __shared__ int32_t s_tet[kThreads / 64][kWin];
  __shared__ uint64_t s_key[kThreads / 64][kWin];
  __shared__ int64_t s_id[kThreads / 64][kWin];
  __shared__ double s_w[kThreads / 64][kWin];
  const int32_t n = *a.n_slots;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int32_t stride = gridDim.x * blockDim.x;
  // wave-uniform loop over blocks of 64 slots
  for (int32_t i0 = blockIdx.x * blockDim.x + (threadIdx.x - lane); i0 < n;
       i0 += stride) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < kWin / 64; ++k) {
      const int32_t j = i0 - kWinLo + 64 * k + lane;
      const bool in = j >= 0 && j < n;
      s_tet[wv][64 * k + lane] = in ? a.tet[j] : -2;
      s_key[wv][64 * k + lane] = in ? a.key[j] : 0;
      s_id[wv][64 * k + lane] = in ? a.id[j] : 0;
      s_w[wv][64 * k + lane] = in ? a.w[j] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int32_t i = i0 + lane;
    const int li = kWinLo + lane;  // this slot in the window
    const int32_t t = i < n ? s_tet[wv][li] : -2;
    if (i >= n) continue;
    if (t < 0) {
      a.seg_n[i] = 0;
      continue;
    }
    int ls = li, le = li + 1;
    while (li - ls <= kSmallRun && s_tet[wv][ls - 1] == t) --ls;
    while (le - ls <= kSmallRun && s_tet[wv][le] == t) ++le;
    const int32_t s = i0 - kWinLo + ls, e = i0 - kWinLo + le;
    if (le - ls > kSmallRun) {
      // a long run: its members are handled by k_coll_rank_big
      if (ls == li && s_tet[wv][li - 1] != t) {
        int32_t lo = e, hi = n;  // first slot past the run
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (a.tet[mid] == t) lo = mid + 1; else hi = mid;
        }
        a.seg_n[i] = lo - i;
        a.big[atomicAdd(a.n_big, 1)] = i;
      }
      continue;
    }
    a.seg_s[i] = s;
    a.seg_n[i] = e - s;
    const uint64_t ki = s_key[wv][li];
    const int64_t di = s_id[wv][li];
    int32_t rank = 0;
#pragma unroll 4
    for (int j = ls; j < le; ++j)
      rank += before(s_key[wv][j], s_id[wv][j], i0 - kWinLo + j, ki, di, i);
    a.perm[s + rank] = i;
    if (ls == li) {
      long long q = 0;
      for (int j = ls; j < le; ++j) q += fx_round(s_w[wv][j] * kFx);
      a.seg_q[s] = q;
    }
  }
}

// Long runs: workgroup (x, y) takes member chunk y (kThreads members) of
// every gridDim.x-th listed run; the run's keys pass through LDS in tiles.
// It also records each member's run and adds the chunk's weights.
__global__ void __launch_bounds__(kThreads) k_coll_rank_big(CollideArgs a) {
  __shared__ uint64_t s_key[kRankTile];
  __shared__ int64_t s_id[kRankTile];
  __shared__ long long s_q[kThreads / 64];
  const int32_t nb = *a.n_big;
  for (int32_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int32_t s = a.big[b];
    const int32_t cnt = a.seg_n[s];
    for (int32_t m0 = blockIdx.y * kThreads; m0 < cnt;
         m0 += gridDim.y * kThreads) {
      const int32_t m = m0 + threadIdx.x;
      const bool mine = m < cnt;
      const int32_t i = s + (mine ? m : 0);
      const uint64_t ki = a.key[i];
      const int64_t di = a.id[i];
      int32_t rank = 0;
      for (int32_t t0 = 0; t0 < cnt; t0 += kRankTile) {
        const int32_t tn = cnt - t0 < kRankTile ? cnt - t0 : kRankTile;
        __syncthreads();
        for (int32_t j = threadIdx.x; j < tn; j += blockDim.x) {
          s_key[j] = a.key[s + t0 + j];
          s_id[j] = a.id[s + t0 + j];
        }
        __syncthreads();
#pragma unroll 8
        for (int32_t j = 0; j < tn; ++j)
          rank += before(s_key[j], s_id[j], s + t0 + j, ki, di, i);
      }
      long long q = mine ? fx_round(a.w[i] * kFx) : 0;
      if (mine) {
        a.perm[s + rank] = i;
        a.seg_s[i] = s;
        if (m > 0) a.seg_n[i] = cnt;
      }
      for (int off = 32; off >= 1; off >>= 1) q += __shfl_xor(q, off, 64);
      if ((threadIdx.x & 63) == 0) s_q[threadIdx.x >> 6] = q;
      __syncthreads();
      if (threadIdx.x == 0) {
        long long tq = 0;
        for (int k = 0; k < kThreads / 64; ++k) tq += s_q[k];
        atomicAdd((unsigned long long*)&a.seg_q[s], (unsigned long long)tq);
      }
    }
  }
}

// The collision(s) led by position p of a run (rank p - s): the pair
// (p, p + 1), or the odd run's triple at p = s.
__device__ void collide_at(const CollideArgs& a, int32_t p, int32_t n) {
  const int32_t cnt = a.seg_n[p];
  const int32_t s = a.seg_s[p];
  const bool triple = (cnt & 1) != 0 && p == s;
  // (range checks: with tets out of order a run's perm entries may be
  // stale; the result is then wrong but stays inside the arrays)
  const int32_t i0 = a.perm[p];
  const int32_t i1 = a.perm[triple ? s + 1 : p + 1];
  const int32_t i2 = triple ? a.perm[s + 2] : 0;
  if ((uint32_t)i0 >= (uint32_t)n || (uint32_t)i1 >= (uint32_t)n ||
      (uint32_t)i2 >= (uint32_t)n || a.tet[i0] < 0)
    return;
  const double V = tet_volume(a.m.tg[a.tet[i0]]);
  const double ws = (double)a.seg_q[s] * (1.0 / kFx);
  const double nv = (a.w_sp * ws) * kLandau * a.dt_coll / V;
  const int64_t lead = a.id[i0];
  if (triple) {
    collide_pair(a, i0, i1, 0.5 * nv, lead, 0);
    collide_pair(a, i1, i2, 0.5 * nv, lead, 1);
    collide_pair(a, i2, i0, 0.5 * nv, lead, 2);
  } else {
    collide_pair(a, i0, i1, nv, lead, 0);
  }
}

// Leaders are about 45 % of the positions: every wave queues the leading
// positions of its blocks in LDS and collides them 64 at a time, all lanes
// busy in the arithmetic.
__global__ void __launch_bounds__(kThreads) k_coll_pair(CollideArgs a) {
  __shared__ int32_t s_lead[kThreads / 64][128];
  const int32_t n = *a.n_slots;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  int qn = 0;  // queued leaders (wave-uniform), < 64 between blocks
  for (int32_t i0 = blockIdx.x * blockDim.x + (threadIdx.x - lane); i0 < n;
       i0 += gridDim.x * blockDim.x) {
    const int32_t p = i0 + lane;
    bool lead = false;
    if (p < n) {
      const int32_t cnt = a.seg_n[p];
      if (cnt >= 2) {
        const int32_t r = p - a.seg_s[p];
        if (r >= 0 && r < cnt) {  // (only out-of-order tets fail this)
          const bool odd = (cnt & 1) != 0;
          lead = odd ? (r == 0 || (r >= 3 && ((r - 3) & 1) == 0 && r + 1 < cnt))
                     : ((r & 1) == 0);
        }
      }
    }
    const uint64_t m = __ballot(lead);
    if (lead) s_lead[wv][qn + __popcll(m & below)] = p;
    qn += __popcll(m);
    if (qn >= 64) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      collide_at(a, s_lead[wv][lane], n);
      const int rest = qn - 64;
      const int32_t mv = lane < rest ? s_lead[wv][64 + lane] : 0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane < rest) s_lead[wv][lane] = mv;
      qn = rest;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < qn) collide_at(a, s_lead[wv][lane], n);
}

}  // namespace

hipError_t collide_particles(const CollideArgs& a, int n_cu, hipStream_t s) {
  const int grid = n_cu * 4;
  hipLaunchKernelGGL(k_coll_keys, dim3(grid), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_coll_rank, dim3(grid), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_coll_rank_big, dim3(kBigRuns, kBigChunks), dim3(kThreads),
                     0, s, a);
  hipLaunchKernelGGL(k_coll_pair, dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace fp
