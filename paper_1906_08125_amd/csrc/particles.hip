// Particle side of the PIC cycle (Sec. II B 1-3): gather + leapfrog kick +
// drift + lateral wrap + absorption + neighbour-walk location + fixed-point
// deposition for the live particles; FN emission counts per face; injection
// of new particles; exact canonical location for the few particles the walk
// cannot certify.
//
// Particles are SoA arrays; every kernel runs a fixed grid-stride over the
// slot range read from device memory, so the host never waits for counts.
// Block b of the grid sweeps a contiguous slot range chosen so that the 8
// XCDs (block b runs on XCD b mod 8) each see one contiguous eighth of the
// slots; with particles sorted by tet, neighbouring tets then share an L2.
#include "common.h"
#include "particles.h"
#include "solver.h"

namespace fp {

namespace {

constexpr int kMaxWalk = 256;
constexpr int kBlock = 256;

struct Span {
  int64_t lo, hi;
};

// contiguous, XCD-grouped slot span of workgroup g of G
__device__ inline Span block_span(int64_t n, int G, int g) {
  int chunk = g;
  if ((G & 7) == 0) chunk = (g & 7) * (G >> 3) + (g >> 3);
  const int64_t per = (n + G - 1) / G;
  Span s;
  s.lo = (int64_t)chunk * per;
  s.hi = s.lo + per < n ? s.lo + per : n;
  if (s.lo > n) s.lo = n;
  return s;
}

// A launch gated on a solve whose outcome was not known when it was
// enqueued runs only if that solve has ended.
__device__ inline bool gate_closed(const int32_t* gate) {
  if (!gate) return false;
  const int32_t st = *gate;
  return st != CG_DONE && st != CG_NOCONV;
}

// Per-thread counters of one kernel, flushed once per block.
struct Acc {
  long long n_before, q_before, n_anode, q_anode, n_after, q_after;
  long long n_cathode, q_cathode, n_inj, q_inj, walk_steps;
  int walk_max;
};

__device__ inline void acc_zero(Acc& a) {
  a.n_before = a.q_before = a.n_anode = a.q_anode = a.n_after = a.q_after = 0;
  a.n_cathode = a.q_cathode = a.n_inj = a.q_inj = a.walk_steps = 0;
  a.walk_max = 0;
}

__device__ inline long long wave_sum(long long v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline int wave_max(int v) {
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Block totals of the counters written to this block's row of the partials
// (no atomics: thousands of same-address atomics per step serialize); the
// stats kernel sums the rows at the end of the step.
__device__ inline void acc_flush(const Acc& a, int64_t* rows, int row,
                                 int stride) {
  __shared__ long long lds[kAccFields][kBlock / 64];
  const long long v[kAccFields] = {a.n_before, a.q_before, a.n_anode,
                                   a.q_anode,  a.n_after,  a.q_after,
                                   a.n_cathode, a.q_cathode, a.n_inj,
                                   a.q_inj,    a.walk_steps, a.walk_max};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kAccFields; ++k) {
    long long s = v[k];
    if (k == kAccFields - 1) {
      s = wave_max((int)s);
    } else {
      s = wave_sum(s);
    }
    if (lane == 0) lds[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < kAccFields) {
    const int k = threadIdx.x;
    long long s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
      s = k == kAccFields - 1 ? (lds[k][w] > s ? lds[k][w] : s) : s + lds[k][w];
    rows[(int64_t)k * stride + row] = s;  // field-major: coalesced sums
  }
}

// Nodal field at one node, widened to double when stored in float.
__device__ inline double4 ld_E(const void* E, int f32, int32_t node) {
  if (f32) {
    const float4 e = reinterpret_cast<const float4*>(E)[node];
    return make_double4(e.x, e.y, e.z, e.w);
  }
  return reinterpret_cast<const double4*>(E)[node];
}

// Field at p inside tet g: sum_i lambda_i E_i in a fixed order.
__device__ inline void gather_field(const TetGeom& g, const void* E,
                                    double x, double y, double z,
                                    double& ex, double& ey, double& ez) {
  double lam[4];
  barycentric(g, x, y, z, lam);
  const double4 e0 = ld_E(E, 0, g.node[0]);
  const double4 e1 = ld_E(E, 0, g.node[1]);
  const double4 e2 = ld_E(E, 0, g.node[2]);
  const double4 e3 = ld_E(E, 0, g.node[3]);
  ex = ((lam[0] * e0.x + lam[1] * e1.x) + lam[2] * e2.x) + lam[3] * e3.x;
  ey = ((lam[0] * e0.y + lam[1] * e1.y) + lam[2] * e2.y) + lam[3] * e3.y;
  ez = ((lam[0] * e0.z + lam[1] * e1.z) + lam[2] * e2.z) + lam[3] * e3.z;
}

// Cell field of a tet (cell mode): E = -(grad phi)_t with grad lambda_k the
// rows m_k (k = 1..3) and grad lambda_0 = -(m_1 + m_2 + m_3), summed in a
// fixed order.
__device__ inline void cell_field(const TetGeom& g, const double* phi,
                                  double& ex, double& ey, double& ez) {
  const double p0 = phi[g.node[0]], p1 = phi[g.node[1]], p2 = phi[g.node[2]],
               p3 = phi[g.node[3]];
  double e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double g0 = -((g.m[k] + g.m[3 + k]) + g.m[6 + k]);
    e[k] = -(((p0 * g0 + p1 * g.m[k]) + p2 * g.m[3 + k]) + p3 * g.m[6 + k]);
  }
  ex = e[0];
  ey = e[1];
  ez = e[2];
}

__device__ inline void deposit_one(const TetGeom& g, double x, double y,
                                   double z, double w, int64_t* charge) {
  double lam[4];
  barycentric(g, x, y, z, lam);
  int64_t q[4];
  charge_split(lam, w, q);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    atomicAdd(reinterpret_cast<unsigned long long*>(charge + g.node[k]),
              (unsigned long long)q[k]);
}

// The seed tet of p's bucket (lowest-index tet whose centroid lies in the
// bucket), or -1: a walk start within about one cell of p.
__device__ inline int bucket_guess(const DevMesh& m, double x, double y,
                                   double z) {
  if (!(x >= m.b0[0] && x <= m.b1[0] && y >= m.b0[1] && y <= m.b1[1] &&
        z >= m.b0[2] && z <= m.b1[2]))
    return -1;
  const int bx = bucket_axis(x, m.b0[0], m.binv[0], m.nb[0]);
  const int by = bucket_axis(y, m.b0[1], m.binv[1], m.nb[1]);
  const int bz = bucket_axis(z, m.b0[2], m.binv[2], m.nb[2]);
  const int64_t id = ((int64_t)bx * m.nb[1] + by) * m.nb[2] + bz;
  return m.bseed[id];
}

// The fine-grid seed of p (the tet holding the centre of p's sub-cell).
__device__ inline int fine_seed(const DevMesh& m, double x, double y,
                                double z) {
  if (!(x >= m.b0[0] && x <= m.b1[0] && y >= m.b0[1] && y <= m.b1[1] &&
        z >= m.b0[2] && z <= m.b1[2]))
    return -1;
  const int bx = bucket_axis(x, m.b0[0], m.finv[0], m.fnb[0]);
  const int by = bucket_axis(y, m.b0[1], m.finv[1], m.fnb[1]);
  const int bz = bucket_axis(z, m.b0[2], m.finv[2], m.fnb[2]);
  return m.fseed[((int64_t)bx * m.fnb[1] + by) * m.fnb[2] + bz];
}

// Barycentric coordinates of p in tet g (the fixed arithmetic of
// barycentric()) with a certificate.  With d = p - v0 and
// M_k = max_j |m_kj|, each computed lambda_k (k = 1..3) lies within
// B_k = lam_c M_k |d|_1 of the exact barycentric coordinate of p in the tet
// of the exact vertices (lam_c bounds the rounding of the stored map, of d
// and of the dot product; it is set up with the mesh), and lambda_0 within
// B_0 = 3.01 u (1 + sum_k |lambda_k|) + sum_k B_k.  Returns true when every
// lambda_k > B_k, i.e. p is certainly strictly inside.  Otherwise exitf is
// the face (opposite vertex k) with the most negative lambda_k among those
// certainly negative (lambda_k < -B_k), or -1 when there is none.
__device__ inline bool lam_test(const TetGeom& g, double x, double y, double z,
                                double C, double lam[4], int& exitf) {
  barycentric(g, x, y, z, lam);
  const double dx = x - g.v0[0], dy = y - g.v0[1], dz = z - g.v0[2];
  const double dn = (fabs(dx) + fabs(dy)) + fabs(dz);
  double B[4];
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const double* r = g.m + 3 * (k - 1);
    const double M = fmax(fmax(fabs(r[0]), fabs(r[1])), fabs(r[2]));
    B[k] = (C * M) * dn;
  }
  B[0] = 3.01 * 1.1102230246251565e-16 *
             (((1.0 + fabs(lam[1])) + fabs(lam[2])) + fabs(lam[3])) +
         1.0001 * ((B[1] + B[2]) + B[3]);
  bool inside = true;
  exitf = -1;
  double worst = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (lam[k] > B[k]) continue;
    inside = false;
    if (lam[k] < -B[k] && lam[k] < worst) {
      worst = lam[k];
      exitf = k;
    }
  }
  return inside;
}

// Neighbour walk from tet t with the point's frame offset (sx, sy) relative
// to t; G holds the record of t on entry.  A point that moved far (far =
// true), or is not in t, restarts from the fine-grid seed of its sub-cell.
// Returns the tet when the point is certified strictly inside it in its own
// frame (then no other tet holds it, so it is the canonical answer), with
// lam its barycentric coordinates there and G its record, or -1 when the
// exact bucket scan must decide.
__device__ inline int walk(const DevMesh& m, double x, double y, double z,
                           int t, int sx, int sy, int& steps, bool far,
                           TetGeom& G, double lam[4], bool have_G = true) {
  bool jumped = false;
  for (steps = 0; steps < kMaxWalk; ++steps) {
    bool reload = steps > 0 || !have_G;
    if (!jumped && (far || steps == 1)) {
      jumped = true;
      int g = fine_seed(m, x, y, z);
      if (g < 0) g = bucket_guess(m, x, y, z);
      if (g >= 0 && !(g == t && sx == 0 && sy == 0)) {
        t = g;
        sx = 0;
        sy = 0;
        reload = true;
      }
    }
    if (reload) G = m.tg[t];
    int exitf;
    if (lam_test(G, x + (double)sx * m.Lx, y + (double)sy * m.Ly, z, m.lam_c,
                 lam, exitf))
      return (sx == 0 && sy == 0) ? t : -1;
    if (exitf < 0) return -1;
    // (selects, not an indexed load: G stays in registers)
    const uint32_t nb = exitf == 0 ? G.nbr[0]
                        : exitf == 1 ? G.nbr[1]
                        : exitf == 2 ? G.nbr[2]
                                     : G.nbr[3];
    if ((nb & kNoNbr) == kNoNbr) return -1;
    sx += (int)((nb >> 28) & 3u) - 1;
    sy += (int)(nb >> 30) - 1;
    t = (int)(nb & kNoNbr);
  }
  return -1;
}

// Canonical location by exact predicates over the bucket's candidates
// (listed in ascending tet order, so the first hit is the lowest index).
__device__ int scan_locate(const DevMesh& m, double x, double y, double z) {
  if (!(x >= m.b0[0] && x <= m.b1[0] && y >= m.b0[1] && y <= m.b1[1] &&
        z >= m.b0[2] && z <= m.b1[2]))
    return -1;
  const int bx = bucket_axis(x, m.b0[0], m.binv[0], m.nb[0]);
  const int by = bucket_axis(y, m.b0[1], m.binv[1], m.nb[1]);
  const int bz = bucket_axis(z, m.b0[2], m.binv[2], m.nb[2]);
  const int64_t id = ((int64_t)bx * m.nb[1] + by) * m.nb[2] + bz;
  const double p[3] = {x, y, z};
  for (int q = m.bstart[id]; q < m.bstart[id + 1]; ++q) {
    const int t = m.bitem[q];
    const double* v = m.tw[t].v;
    if (vol6_sign(p, v + 3, v + 6, v + 9) < 0) continue;
    if (vol6_sign(v, p, v + 6, v + 9) < 0) continue;
    if (vol6_sign(v, v + 3, p, v + 9) < 0) continue;
    if (vol6_sign(v, v + 3, v + 6, p) < 0) continue;
    return t;
  }
  return -1;
}

// The same canonical location with the 64 lanes of a wave testing 64
// candidates at a time (the point is uniform across the wave; every lane
// must call it).  The lowest lane holding the point gives the lowest index.
__device__ int scan_locate_wave(const DevMesh& m, double x, double y,
                                double z) {
  if (!(x >= m.b0[0] && x <= m.b1[0] && y >= m.b0[1] && y <= m.b1[1] &&
        z >= m.b0[2] && z <= m.b1[2]))
    return -1;
  const int bx = bucket_axis(x, m.b0[0], m.binv[0], m.nb[0]);
  const int by = bucket_axis(y, m.b0[1], m.binv[1], m.nb[1]);
  const int bz = bucket_axis(z, m.b0[2], m.binv[2], m.nb[2]);
  const int64_t id = ((int64_t)bx * m.nb[1] + by) * m.nb[2] + bz;
  const double p[3] = {x, y, z};
  const int lane = threadIdx.x & 63;
  const int q1 = m.bstart[id + 1];
  for (int base = m.bstart[id]; base < q1; base += 64) {
    const int q = base + lane;
    bool hit = false;
    if (q < q1) {
      const double* v = m.tw[m.bitem[q]].v;
      hit = vol6_sign(p, v + 3, v + 6, v + 9) >= 0 &&
            vol6_sign(v, p, v + 6, v + 9) >= 0 &&
            vol6_sign(v, v + 3, p, v + 9) >= 0 &&
            vol6_sign(v, v + 3, v + 6, p) >= 0;
    }
    const unsigned long long mask = __ballot(hit);
    if (mask) return m.bitem[base + __ffsll((long long)mask) - 1];
  }
  return -1;
}

// After the drift: wrap, absorb at the anode, locate, deposit.
// Per-workgroup node-charge table in LDS (open addressing on the node id).
// Particles of one workgroup share few nodes, so accumulating their int64
// charges here and flushing one global atomic per distinct node removes
// the same-address contention of per-particle global atomics.  Integer
// addition is exact and order-free, so the result is unchanged.
constexpr int kTable = 2048;  // > 4 nodes x the particles of one block

struct ChargeTable {
  int32_t key[kTable];
  unsigned long long val[kTable];
};

__device__ inline void table_clear(ChargeTable& T) {
  for (int k = threadIdx.x; k < kTable; k += blockDim.x) {
    T.key[k] = -1;
    T.val[k] = 0ull;
  }
  __syncthreads();
}

// 64-bit add into LDS.  The table reaches the helpers by reference, and
// through it the compiler emits a generic (flat) atomic, which takes the
// vector-memory path; the explicit LDS address space gives ds_add_u64.
__device__ inline void lds_add_u64(unsigned long long* p, unsigned long long v) {
  __atomic_fetch_add((__attribute__((address_space(3))) unsigned long long*)p, v,
                     __ATOMIC_RELAXED);
}

__device__ inline void table_add(ChargeTable& T, int32_t node, int64_t q,
                                 int64_t* charge) {
  uint32_t h = ((uint32_t)node * 2654435761u) >> 21;  // 11 bits
  // kept as a loop: unrolled at every inlined call site, the 64 probes
  // made the particle kernel tens of thousands of instructions long (an
  // instruction-cache and scalar-register-spill cost paid by every wave)
#pragma unroll 1
  for (int probe = 0; probe < 64; ++probe) {
    const int32_t old = atomicCAS(&T.key[h], -1, node);
    if (old == -1 || old == node) {
      lds_add_u64(&T.val[h], (unsigned long long)q);
      return;
    }
    h = (h + 1) & (kTable - 1);
  }
  atomicAdd(reinterpret_cast<unsigned long long*>(charge + node),
            (unsigned long long)q);
}

__device__ inline void table_flush(ChargeTable& T, int64_t* charge) {
  __syncthreads();
  for (int k = threadIdx.x; k < kTable; k += blockDim.x) {
    const int32_t node = T.key[k];
    const unsigned long long v = T.val[k];
    if (node >= 0 && v != 0ull)
      atomicAdd(reinterpret_cast<unsigned long long*>(charge + node), v);
  }
}

__device__ inline void deposit_table(const TetGeom& g, const double lam[4],
                                     double w, ChargeTable& T,
                                     int64_t* charge) {
  int64_t q[4];
  charge_split(lam, w, q);
#pragma unroll
  for (int k = 0; k < 4; ++k) table_add(T, g.node[k], q[k], charge);
}

// G: the record of the hint tet (have_G), or to be loaded when needed.
__device__ inline void settle(const DevMesh& m, const StepArgs& a, int64_t i,
                              double x, double y, double z, int sx, int sy,
                              int hint, TetGeom& G, double w, long long qfx,
                              Acc& acc, ChargeTable& T, bool far,
                              bool have_G = true) {
  if (z >= m.z_top) {
    a.tet[i] = -1;
    acc.n_anode += 1;
    acc.q_anode += qfx;
    return;
  }
  int steps = 0;
  double lam[4];
  const int t = walk(m, x, y, z, hint, sx, sy, steps, far, G, lam, have_G);
  acc.walk_steps += steps;
  if (steps > acc.walk_max) acc.walk_max = steps;
  if (t >= 0) {
    a.tet[i] = t;
    deposit_table(G, lam, w, T, a.charge);
    acc.n_after += 1;
    acc.q_after += qfx;
  } else {
    a.tet[i] = hint;
    const int slot = atomicAdd(&a.scratch->n_fallback, 1);
    a.queue[slot] = (int32_t)i;
  }
}

__device__ inline void wrap(const DevMesh& m, double& x, double& y, int& sx,
                            int& sy) {
  sx = 0;
  sy = 0;
  if (x >= m.Lx) {
    x = x - m.Lx;
    sx = 1;
  } else if (x < 0.0) {
    x = x + m.Lx;
    sx = -1;
  }
  if (y >= m.Ly) {
    y = y - m.Ly;
    sy = 1;
  } else if (y < 0.0) {
    y = y + m.Ly;
    sy = -1;
  }
}

}  // namespace

__device__ inline double fn_current(double F, double phi, const EmitConsts& c,
                                    int& clamped) {
  if (!(F > 1e-3)) return 0.0;
  double f = c.c_s * F / (phi * phi);
  if (f >= 1.0) {
    f = 1.0 - 1e-9;
    clamped = 1;
  }
  const double lf = log(f);
  const double v = 1.0 - f + (f / 6.0) * lf;
  const double t = 1.0 + f / 9.0 - (f / 18.0) * lf;
  const double Fsi = F * 1e9;
  return c.a_fn * Fsi * Fsi / (phi * t * t) *
         exp(-v * c.b_fn * (phi * sqrt(phi)) / F);
}

__device__ inline void face_field(const DevMesh& m, const void* E, int f32,
                                  int64_t f, double& ex, double& ey,
                                  double& ez) {
  const int32_t* nd = m.e_nodes + 3 * f;
  const double4 a = ld_E(E, f32, nd[0]);
  const double4 b = ld_E(E, f32, nd[1]);
  const double4 c = ld_E(E, f32, nd[2]);
  ex = ((a.x + b.x) + c.x) / 3.0;
  ey = ((a.y + b.y) + c.y) / 3.0;
  ez = ((a.z + b.z) + c.z) / 3.0;
}


// ---------------------------------------------------------------------------
// Emission counts (one workgroup): per emitting face the centroid field
// ((E_a + E_b) + E_c)/3, the FN current when the field pulls electrons out of
// the metal, Eq. nsp and the rounding of Eq. rnd_nsp; an exclusive scan of
// the counts gives every new particle its slot.
// ---------------------------------------------------------------------------
template <int NT>
__device__ void emit_block(const EmitArgs& a) {
  const DevMesh& m = a.m;
  __shared__ long long s_scan[NT / 64];
  __shared__ double s_red[3][NT / 64];
  __shared__ long long s_cl[NT / 64];
  long long offset = 0;
  double cur_sum = 0.0, F_sum = 0.0, F_max = 0.0;
  long long n_clamp = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t f0 = 0; f0 < m.n_emit; f0 += NT) {
    const int64_t f = f0 + threadIdx.x;
    long long cnt = 0;
    double cur = 0.0, F = 0.0;
    int clamped = 0;
    if (f < m.n_emit) {
      double ex, ey, ez;
      if (a.cell)
        cell_field(m.tg[m.e_tet[f]], a.phi, ex, ey, ez);
      else
        face_field(m, a.E, a.f32, f, ex, ey, ez);
      F = sqrt((ex * ex + ey * ey) + ez * ez);
      const double* nr = m.e_nrm + 3 * f;
      const double en = (ex * nr[0] + ey * nr[1]) + ez * nr[2];
      double jd = 0.0;
      if (en < 0.0)
        jd = fn_current(F, a.phi_w, a.c, clamped) * a.c.j_unit;
      jd = jd * a.j_scale;
      cur = jd * m.e_area[f];
      if (a.counts) {
        const double nsp = cur * a.dt / a.w_sp;
        uint64_t r4[4];
        philox4x64_10(a.seed, a.instance, (uint64_t)a.step, (uint64_t)f, 0, 0,
                      r4);
        const double R = unit_double(r4[0]);
        const double fl = floor(nsp);
        double c = (R >= nsp - fl) ? fl : ceil(nsp);
        if (c > 2097152.0) c = 2097152.0;
        cnt = (long long)c;
        if (a.counts_in) {
          const int32_t ci = a.counts_in[f];
          cnt = ci < 0 ? 0 : (ci > 2097152 ? 2097152 : ci);
        }
        if (a.counts_out) a.counts_out[f] = (int32_t)cnt;
      }
      if (a.face_F) a.face_F[f] = F;
    }
    // exclusive scan of the counts: shuffle scan per wave, then waves
    long long inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    if (lane == 63) s_scan[wave] = inc;
    // sums of current and |E|, max |E|, clamp count (fixed order)
    double v0 = cur, v1 = F, v2 = F;
    long long vc = clamped;
    for (int off = 32; off >= 1; off >>= 1) {
      v0 += __shfl_xor(v0, off, 64);
      v1 += __shfl_xor(v1, off, 64);
      const double o2 = __shfl_xor(v2, off, 64);
      v2 = o2 > v2 ? o2 : v2;
      vc += __shfl_xor(vc, off, 64);
    }
    if (lane == 0) {
      s_red[0][wave] = v0;
      s_red[1][wave] = v1;
      s_red[2][wave] = v2;
      s_cl[wave] = vc;
    }
    __syncthreads();
    long long before = 0, chunk = 0;
    for (int w = 0; w < NT / 64; ++w) {
      if (w < wave) before += s_scan[w];
      chunk += s_scan[w];
      cur_sum += s_red[0][w];
      F_sum += s_red[1][w];
      F_max = s_red[2][w] > F_max ? s_red[2][w] : F_max;
      n_clamp += s_cl[w];
    }
    if (f < m.n_emit && a.counts) {
      a.counts[f] = (int32_t)cnt;
      a.offsets[f] = (int32_t)(offset + before + inc - cnt);
    }
    offset += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (a.rate) *a.rate = cur_sum;
    if (a.stats) {
      pic_step_stats* st = a.stats;
      st->emit_current = cur_sum;
      st->mean_face_E = m.n_emit ? F_sum / (double)m.n_emit : 0.0;
      st->max_face_E = F_max;
      st->n_clamp = n_clamp;
    }
    if (a.counts) {
      a.offsets[m.n_emit] = (int32_t)offset;
      const long long base = *a.n_slots;
      long long fit = a.capacity - base;
      if (fit > offset) fit = offset;
      if (fit < 0) fit = 0;
      a.scratch->inj_base = (int32_t)base;
      a.scratch->inj_total = (int32_t)offset;
      a.scratch->inj_fit = (int32_t)fit;
      *a.n_slots = (int32_t)(base + fit);
      if (a.stats) {
        a.stats->n_trunc = offset - fit;
        if (offset > fit) a.stats->status = PIC_E_CAPACITY;
        a.stats->n_slots = base + fit;
      }
    }
  }
}

constexpr int kBeginBlock = 512;  // 1024 would cap registers below the emission path's needs

__global__ void __launch_bounds__(kBlock) k_emit(EmitArgs a) {
  emit_block<kBlock>(a);
}

// Start of a step: workgroup 0 clears the step's stats and counters and
// computes the emission counts; the others clear the node charges.
__device__ inline void begin_body(const EmitArgs& a, VB vb) {
  if (gate_closed(a.gate)) return;
  if (vb.id == 0) {  // dispatched first: the emission path is the longest
    int64_t* s64 = reinterpret_cast<int64_t*>(a.stats);
    const int ns = (int)(sizeof(pic_step_stats) / sizeof(int64_t));
    if (threadIdx.x < ns) s64[threadIdx.x] = 0;
    int32_t* c32 = reinterpret_cast<int32_t*>(a.scratch);
    const int nc = (int)(sizeof(StepScratch) / sizeof(int32_t));
    if (threadIdx.x < nc) c32[threadIdx.x] = 0;
    __syncthreads();
    if (a.defer) {
      // the particle kernel emits; its pushing workgroups need the slot
      // count before injection now
      if (threadIdx.x == 0) a.scratch->inj_base = *a.n_slots;
      return;
    }
    emit_block<kBeginBlock>(a);
    return;
  }
  const int64_t G = vb.n - 1;
  for (int64_t i = (vb.id - 1) * (int64_t)blockDim.x + threadIdx.x;
       i < a.n_clear; i += G * blockDim.x)
    a.clear[i] = 0;
}

__global__ void __launch_bounds__(kBeginBlock) k_begin(EmitArgs a) {
  begin_body(a, VB{(int)blockIdx.x, (int)gridDim.x});
}

__global__ void __launch_bounds__(kBeginBlock) k_begin_b(const EmitArgs* E,
                                                         BatchMap map) {
  int i;
  const VB vb = batch_block(map, i);
  const EmitArgs a = E[i];  // a private copy: no aliasing with the stores
  begin_body(a, vb);
}

// ---------------------------------------------------------------------------
// The particle kernel of a step.  Workgroups [0, g_push) advance the live
// particles (gather E_k, kick (v + QE) + QE, drift, wrap, absorb, walk,
// deposit); the remaining workgroups inject the new ones (Sec. II B 3,
// App. E: sample the face, Eq. sp_velocity, Eq. sp_displacement, drift,
// wrap, absorb, walk, deposit).  Both halves only read the slots below the
// pre-injection count, so they run side by side.
// ---------------------------------------------------------------------------
// Live particles, FP64 storage: the fixed arithmetic shared with the oracle.
// Element o of a stream read from the workgroup's base: the streams' bases
// advanced to the start of the workgroup's span are uniform (scalar
// registers), and one 32-bit byte offset per lane then addresses every
// stream (scalar base + vector offset) instead of a 64-bit address per
// stream and lane.  The FP64 push needed 142 VGPRs with per-stream
// addresses and spilled 9 dwords per lane at its 128-register bound; with
// the shared offset it fits in 124 (83.6 against 86.6 us per launch).
template <typename T>
__device__ inline T& at_off(const void* base, uint32_t bytes) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<void*>(base)) + bytes);
}

__device__ inline void push_role64(const StepArgs& a, int g, int G, Acc& acc,
                                   ChargeTable& T) {
  const DevMesh& m = a.m;
  const int64_t n = a.scratch->inj_base;
  const Span sp = block_span(n, G, g);
  const double Q = a.Q;
  const double dt = a.dt;
  // the span's streams (see at_off)
  double* X = (double*)a.x + sp.lo;
  double* Y = (double*)a.y + sp.lo;
  double* Z = (double*)a.z + sp.lo;
  double* VX = (double*)a.vx + sp.lo;
  double* VY = (double*)a.vy + sp.lo;
  double* VZ = (double*)a.vz + sp.lo;
  const double* W = a.w + sp.lo;
  const int32_t* TT = a.tet + sp.lo;
  const uint32_t len = (uint32_t)(sp.hi - sp.lo);
  for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) {
    const uint32_t o8 = j * 8u;
    const int t = at_off<const int32_t>(TT, j * 4u);
    if (t < 0) continue;
    const int64_t i = sp.lo + j;
    const double w = at_off<const double>(W, o8);
    const long long qfx = fx_round(w * kFx);
    acc.n_before += 1;
    acc.q_before += qfx;
    double x = at_off<double>(X, o8), y = at_off<double>(Y, o8), z = at_off<double>(Z, o8);
    double vx = at_off<double>(VX, o8), vy = at_off<double>(VY, o8),
           vz = at_off<double>(VZ, o8);
    TetGeom G = m.tg[t];
    double ex, ey, ez;
    if (a.cell)
      cell_field(G, a.phi, ex, ey, ez);
    else
      gather_field(G, a.E, x, y, z, ex, ey, ez);
    const double qx = Q * ex, qy = Q * ey, qz = Q * ez;
    vx = (vx + qx) + qx;
    vy = (vy + qy) + qy;
    vz = (vz + qz) + qz;
    const double dx = dt * vx, dy = dt * vy, dz = dt * vz;
    const bool far = (dx * dx + dy * dy) + dz * dz > m.jump_len2;
    x = x + dx;
    y = y + dy;
    z = z + dz;
    int sx, sy;
    wrap(m, x, y, sx, sy);
    at_off<double>(X, o8) = x;
    at_off<double>(Y, o8) = y;
    at_off<double>(Z, o8) = z;
    at_off<double>(VX, o8) = vx;
    at_off<double>(VY, o8) = vy;
    at_off<double>(VZ, o8) = vz;
    settle(m, a, i, x, y, z, sx, sy, t, G, w, qfx, acc, T, far);
  }
}

// Live particles, mixed precision: FP32 position, velocity, field gather,
// kick and drift; the barycentric weights, the walk and the deposition take
// the stored FP32 position widened exactly to FP64.
__device__ inline void push_role32(const StepArgs& a, int g, int G, Acc& acc,
                                   ChargeTable& T) {
  const DevMesh& m = a.m;
  const int64_t n = a.scratch->inj_base;
  const Span sp = block_span(n, G, g);
  const float Q = (float)a.Q;
  const float dt = (float)a.dt;
  const float Lx = (float)m.Lx, Ly = (float)m.Ly;
  const float4* E = reinterpret_cast<const float4*>(a.E);
  // the span's streams (see at_off)
  float* X = (float*)a.x + sp.lo;
  float* Y = (float*)a.y + sp.lo;
  float* Z = (float*)a.z + sp.lo;
  float* VX = (float*)a.vx + sp.lo;
  float* VY = (float*)a.vy + sp.lo;
  float* VZ = (float*)a.vz + sp.lo;
  const double* W = a.w + sp.lo;
  const int32_t* TT = a.tet + sp.lo;
  const uint32_t len = (uint32_t)(sp.hi - sp.lo);
  for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) {
    const uint32_t o4 = j * 4u;
    const int t = at_off<const int32_t>(TT, o4);
    if (t < 0) continue;
    const int64_t i = sp.lo + j;
    const double w = at_off<const double>(W, j * 8u);
    const long long qfx = fx_round(w * kFx);
    acc.n_before += 1;
    acc.q_before += qfx;
    float x = at_off<float>(X, o4), y = at_off<float>(Y, o4), z = at_off<float>(Z, o4);
    float vx = at_off<float>(VX, o4), vy = at_off<float>(VY, o4), vz = at_off<float>(VZ, o4);
    // FP32 gather from the FP32 record (half the bytes of the FP64 one,
    // which the walk loads only when it needs the hint tet itself)
    const TetGeom32 G32 = m.tg32[t];
    float ex, ey, ez;
    if (a.cell) {
      // -(grad phi)_t from the potential differences to vertex 0 (FP64
      // differences, FP32 products: no cancellation of the potential's size)
      const double p0 = a.phi[G32.node[0]];
      const float d1 = (float)(a.phi[G32.node[1]] - p0);
      const float d2 = (float)(a.phi[G32.node[2]] - p0);
      const float d3 = (float)(a.phi[G32.node[3]] - p0);
      ex = -((d1 * G32.m[0] + d2 * G32.m[3]) + d3 * G32.m[6]);
      ey = -((d1 * G32.m[1] + d2 * G32.m[4]) + d3 * G32.m[7]);
      ez = -((d1 * G32.m[2] + d2 * G32.m[5]) + d3 * G32.m[8]);
    } else {
      const float dx0 = x - G32.v0[0], dy0 = y - G32.v0[1], dz0 = z - G32.v0[2];
      const float l1 = (G32.m[0] * dx0 + G32.m[1] * dy0) + G32.m[2] * dz0;
      const float l2 = (G32.m[3] * dx0 + G32.m[4] * dy0) + G32.m[5] * dz0;
      const float l3 = (G32.m[6] * dx0 + G32.m[7] * dy0) + G32.m[8] * dz0;
      const float l0 = ((1.0f - l1) - l2) - l3;
      const float4 e0 = E[G32.node[0]], e1 = E[G32.node[1]],
                   e2 = E[G32.node[2]], e3 = E[G32.node[3]];
      ex = ((l0 * e0.x + l1 * e1.x) + l2 * e2.x) + l3 * e3.x;
      ey = ((l0 * e0.y + l1 * e1.y) + l2 * e2.y) + l3 * e3.y;
      ez = ((l0 * e0.z + l1 * e1.z) + l2 * e2.z) + l3 * e3.z;
    }
    const float qx = Q * ex, qy = Q * ey, qz = Q * ez;
    vx = (vx + qx) + qx;
    vy = (vy + qy) + qy;
    vz = (vz + qz) + qz;
    const float dx = dt * vx, dy = dt * vy, dz = dt * vz;
    const bool far = (double)((dx * dx + dy * dy) + dz * dz) > m.jump_len2;
    x = x + dx;
    y = y + dy;
    z = z + dz;
    int sx = 0, sy = 0;
    if (x >= Lx) {
      x = x - Lx;
      sx = 1;
    } else if (x < 0.0f) {
      x = x + Lx;
      sx = -1;
    }
    if (y >= Ly) {
      y = y - Ly;
      sy = 1;
    } else if (y < 0.0f) {
      y = y + Ly;
      sy = -1;
    }
    at_off<float>(X, o4) = x;
    at_off<float>(Y, o4) = y;
    at_off<float>(Z, o4) = z;
    at_off<float>(VX, o4) = vx;
    at_off<float>(VY, o4) = vy;
    at_off<float>(VZ, o4) = vz;
    TetGeom G4;
    settle(m, a, i, x, y, z, sx, sy, t, G4, w, qfx, acc, T, far, false);
  }
}

__device__ inline void inject_role(const StepArgs& a, int g, int G, Acc& acc,
                                   ChargeTable& T) {
  const DevMesh& m = a.m;
  const int64_t n = a.scratch->inj_fit;
  const int64_t base = a.scratch->inj_base;
  const double dt = a.dt;
  const int32_t* off = a.offsets;
  for (int64_t s = g * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)G * blockDim.x) {
    // face: last f with off[f] <= s
    int lo = 0, hi = (int)m.n_emit - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const int f = lo;
    const int64_t o = s - off[f];
    uint64_t r4[4];
    philox4x64_10(a.seed, a.instance, (uint64_t)a.step, (uint64_t)f,
                  (uint64_t)o, 1, r4);
    double R1 = unit_double(r4[0]), R2 = unit_double(r4[1]);
    const double R = unit_double(r4[2]);
    if (R1 + R2 > 1.0) {
      R1 = 1.0 - R1;
      R2 = 1.0 - R2;
    }
    const double l0 = (1.0 - R1) - R2;
    const double* A = m.e_abc + 9 * (int64_t)f;
    const double px = (A[0] + R1 * (A[3] - A[0])) + R2 * (A[6] - A[0]);
    const double py = (A[1] + R1 * (A[4] - A[1])) + R2 * (A[7] - A[1]);
    const double pz = (A[2] + R1 * (A[5] - A[2])) + R2 * (A[8] - A[2]);
    double Ex, Ey, Ez;
    if (a.cell) {
      cell_field(m.tg[m.e_tet[f]], a.phi, Ex, Ey, Ez);
    } else {
      const int32_t* nd = m.e_nodes + 3 * (int64_t)f;
      const double4 ea = ld_E(a.E, a.f32, nd[0]);
      const double4 eb = ld_E(a.E, a.f32, nd[1]);
      const double4 ec = ld_E(a.E, a.f32, nd[2]);
      Ex = (l0 * ea.x + R1 * eb.x) + R2 * ec.x;
      Ey = (l0 * ea.y + R1 * eb.y) + R2 * ec.y;
      Ez = (l0 * ea.z + R1 * eb.z) + R2 * ec.z;
    }
    const double cv = a.qm_dt * (0.5 + R);
    const double vx = cv * Ex, vy = cv * Ey, vz = cv * Ez;
    double x = px + (vx * dt) * R;
    double y = py + (vy * dt) * R;
    double z = pz + (vz * dt) * R;
    x = x + dt * vx;
    y = y + dt * vy;
    z = z + dt * vz;
    int sx, sy;
    wrap(m, x, y, sx, sy);
    const int64_t i = base + s;
    const double w = a.s_face ? a.s_face[f] : 1.0;
    const long long qfx = fx_round(w * kFx);
    if (a.f32) {
      // stored in FP32; the walk and deposition use the stored values
      const float xf = (float)x, yf = (float)y, zf = (float)z;
      ((float*)a.x)[i] = xf;
      ((float*)a.y)[i] = yf;
      ((float*)a.z)[i] = zf;
      ((float*)a.vx)[i] = (float)vx;
      ((float*)a.vy)[i] = (float)vy;
      ((float*)a.vz)[i] = (float)vz;
      x = xf;
      y = yf;
      z = zf;
    } else {
      ((double*)a.x)[i] = x;
      ((double*)a.y)[i] = y;
      ((double*)a.z)[i] = z;
      ((double*)a.vx)[i] = vx;
      ((double*)a.vy)[i] = vy;
      ((double*)a.vz)[i] = vz;
    }
    a.w[i] = w;
    a.birth[i] = f;
    a.id[i] = (a.step << 42) | ((int64_t)f << 21) | o;
    acc.n_inj += 1;
    acc.q_inj += qfx;
    const int h = m.e_tet[f];
    TetGeom G = m.tg[h];
    settle(m, a, i, x, y, z, sx, sy, h, G, w, qfx, acc, T, false);
  }
}

// The emission of the step computed inside the particle kernel: workgroup 0
// (dispatched first, so resident before any workgroup that waits for it)
// computes the counts and offsets, then publishes them; the injecting
// workgroups (dispatched last) wait for the flag.  The wait is bounded: a
// flag not seen in time (never expected) skips the injection and marks the
// step with a device error.
__device__ inline void emit_publish(const EmitArgs& e) {
  emit_block<kBlock>(e);
  __threadfence();  // every thread's counts and offsets reach L2
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&e.scratch->emitted, 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline bool emit_wait(const StepArgs& a) {
  __shared__ int seen;
  if (threadIdx.x == 0) {
    int ok = 0;
    for (int it = 0; it < (1 << 22); ++it) {
      if (__hip_atomic_load(&a.scratch->emitted, __ATOMIC_ACQUIRE,
                            __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ok && a.stats) a.stats->status = PIC_E_DEVICE;
    seen = ok;
  }
  __syncthreads();
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  return seen != 0;
}

// One instance per storage precision, so that only one push is compiled in.
// wait: the injecting workgroups wait for the emission (see emit_wait).
template <bool F32>
__device__ inline void particles_body(const StepArgs& a, VB vb, bool wait) {
  Acc acc;
  acc_zero(acc);
  __shared__ ChargeTable T;
  table_clear(T);
  const int g_push = a.g_push;
  if (vb.id < g_push) {
    if (F32)
      push_role32(a, vb.id, g_push, acc, T);
    else
      push_role64(a, vb.id, g_push, acc, T);
  } else if (!wait || emit_wait(a)) {
    inject_role(a, vb.id - g_push, vb.n - g_push, acc, T);
  }
  table_flush(T, a.charge);
  acc_flush(acc, a.acc_rows, vb.id, a.acc_stride);
}

// With the emission inside (e.defer), workgroup 0 only emits and the
// particle workgroups are 1 .. gridDim.x - 1 (virtual index one less: the
// XCD grouping of the slot spans is a fixed rotation of the hardware's).
// At most 128 VGPRs (4 waves per SIMD): the FP64 push needs 142 unbounded
// and spills 9 dwords per lane at this bound, which the fourth wave's latency
// hiding more than pays for (86.6 against 90.4 us per push at 1e6
// superparticles); the FP32 push fits in 124 either way.
template <bool F32>
__global__ void __launch_bounds__(kBlock, 4) k_particles(StepArgs a, EmitArgs e) {
  if (gate_closed(a.gate)) return;
  if (!e.defer) {
    particles_body<F32>(a, VB{(int)blockIdx.x, (int)gridDim.x}, false);
  } else if (blockIdx.x == 0) {
    emit_publish(e);
  } else {
    particles_body<F32>(a, VB{(int)blockIdx.x - 1, (int)gridDim.x - 1}, true);
  }
}

template <bool F32>
__global__ void __launch_bounds__(kBlock) k_particles_b(const StepArgs* A,
                                                        BatchMap map) {
  int i;
  const VB vb = batch_block(map, i);
  const StepArgs a = A[i];  // a private copy: no aliasing with the stores
  particles_body<F32>(a, vb, false);
}

// ---------------------------------------------------------------------------
// Particles the walk could not certify: exact canonical location; those
// outside every tet (below the top plane) are absorbed by the cathode.
// ---------------------------------------------------------------------------
__device__ inline void fallback_body(const StepArgs& a, VB vb) {
  if (gate_closed(a.gate)) return;
  const DevMesh& m = a.m;
  const int64_t n = a.scratch->n_fallback;
  Acc acc;
  acc_zero(acc);
  // one wave per queued particle
  const int64_t waves = (int64_t)vb.n * (blockDim.x >> 6);
  const bool lead = (threadIdx.x & 63) == 0;
  for (int64_t j = vb.id * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
       j < n; j += waves) {
    const int64_t i = a.queue[j];
    double x, y, z;
    if (a.f32) {
      x = ((const float*)a.x)[i];
      y = ((const float*)a.y)[i];
      z = ((const float*)a.z)[i];
    } else {
      x = ((const double*)a.x)[i];
      y = ((const double*)a.y)[i];
      z = ((const double*)a.z)[i];
    }
    const double w = a.w[i];
    const long long qfx = fx_round(w * kFx);
    const int t = scan_locate_wave(m, x, y, z);
    if (!lead) continue;
    if (t >= 0) {
      a.tet[i] = t;
      deposit_one(m.tg[t], x, y, z, w, a.charge);
      acc.n_after += 1;
      acc.q_after += qfx;
    } else {
      a.tet[i] = -1;
      acc.n_cathode += 1;
      acc.q_cathode += qfx;
    }
  }
  // counter rows after those of the particle kernel
  acc_flush(acc, a.acc_rows, a.n_blocks + vb.id, a.acc_stride);
  if (vb.id == 0 && threadIdx.x == 0) a.stats->n_fallback = n;
}

__global__ void __launch_bounds__(kBlock) k_fallback(StepArgs a) {
  fallback_body(a, VB{(int)blockIdx.x, (int)gridDim.x});
}

__global__ void __launch_bounds__(kBlock) k_fallback_b(const StepArgs* A,
                                                       BatchMap map) {
  int i;
  const VB vb = batch_block(map, i);
  const StepArgs a = A[i];
  fallback_body(a, vb);
}

__global__ void __launch_bounds__(kBlock) k_stats(const int64_t* rows,
                                                  int n_rows,
                                                  pic_step_stats* st,
                                                  const int32_t* gate) {
  if (gate_closed(gate)) return;
  step_counter_sum(rows, n_rows, st, (int)blockIdx.x);
}

// Batched: kAccFields workgroups per instance (schedule of 16 per instance).
__global__ void __launch_bounds__(kBlock) k_stats_b(const StepArgs* A,
                                                    BatchMap map) {
  int i;
  const VB vb = batch_block(map, i);
  if (vb.id >= kAccFields) return;
  const StepArgs& a = A[i];
  step_counter_sum(a.acc_rows, a.acc_stride, a.stats, vb.id);
}

// ---------------------------------------------------------------------------
// Stand-alone location and deposition entry points.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_locate(LocateArgs a) {
  const DevMesh& m = a.m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = a.x[i], y = a.y[i], z = a.z[i];
    if (z >= m.z_top) {
      a.tet[i] = -1;
      a.where[i] = PIC_WHERE_ANODE;
      continue;
    }
    const int h = a.tet[i];
    int t = -1, steps = 0;
    if (h >= 0 && h < m.n_tets) {
      TetGeom G = m.tg[h];
      double lam[4];
      t = walk(m, x, y, z, h, 0, 0, steps, false, G, lam);
    }
    if (t >= 0) {
      a.tet[i] = t;
      a.where[i] = PIC_WHERE_INSIDE;
    } else {
      const int slot = atomicAdd(a.n_queue, 1);
      a.queue[slot] = (int32_t)i;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_locate_scan(LocateArgs a) {
  const DevMesh& m = a.m;
  const int64_t n = *a.n_queue;
  // one wave per queued point
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t j = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
       j < n; j += waves) {
    const int64_t i = a.queue[j];
    const int t = scan_locate_wave(m, a.x[i], a.y[i], a.z[i]);
    if ((threadIdx.x & 63) == 0) {
      a.tet[i] = t;
      a.where[i] = t >= 0 ? PIC_WHERE_INSIDE : PIC_WHERE_OUTSIDE;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_deposit(DepositArgs a) {
  const DevMesh& m = a.m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int t = a.tet[i];
    if (t < 0 || t >= m.n_tets) continue;
    deposit_one(m.tg[t], a.x[i], a.y[i], a.z[i], a.w[i], a.charge);
  }
}

// Fine walk seeds: the canonical tet of every sub-cell centre (exact scan),
// or the coarse seed where the centre lies in the metal.
__global__ void __launch_bounds__(kBlock) k_seed_build(DevMesh m) {
  const int64_t n = (int64_t)m.fnb[0] * m.fnb[1] * m.fnb[2];
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t iz = id % m.fnb[2];
    const int64_t iy = (id / m.fnb[2]) % m.fnb[1];
    const int64_t ix = id / ((int64_t)m.fnb[2] * m.fnb[1]);
    const double x = m.b0[0] + ((double)ix + 0.5) / m.finv[0];
    const double y = m.b0[1] + ((double)iy + 0.5) / m.finv[1];
    const double z = m.b0[2] + ((double)iz + 0.5) / m.finv[2];
    int t = scan_locate(m, x, y, z);
    if (t < 0) t = bucket_guess(m, x, y, z);
    m.fseed[id] = t;
  }
}


// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_begin(const EmitArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_begin, dim3(grid + 1), dim3(kBeginBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_begin_b(const EmitArgs* E, const BatchMap& map, int grid,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_begin_b, dim3(grid), dim3(kBeginBlock), 0, s, E, map);
  return hipGetLastError();
}
hipError_t launch_particles_b(const StepArgs* A, const BatchMap& map, int grid,
                              int f32, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(k_particles_b<true>, dim3(grid), dim3(kBlock), 0, s, A, map);
  else
    hipLaunchKernelGGL(k_particles_b<false>, dim3(grid), dim3(kBlock), 0, s, A, map);
  return hipGetLastError();
}
hipError_t launch_fallback_b(const StepArgs* A, const BatchMap& map, int grid,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_fallback_b, dim3(grid), dim3(kBlock), 0, s, A, map);
  return hipGetLastError();
}
hipError_t launch_stats_b(const StepArgs* A, const BatchMap& map, int grid,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_stats_b, dim3(grid), dim3(kBlock), 0, s, A, map);
  return hipGetLastError();
}
int particle_blocks_per_cu(int f32) {
  int n = 0;
  const hipError_t e =
      f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_particles<true>, kBlock, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_particles<false>, kBlock, 0);
  return e == hipSuccess ? n : 0;
}

hipError_t launch_particles(const StepArgs& a, const EmitArgs* e, int g_push,
                            int g_inj, hipStream_t s) {
  StepArgs b = a;
  b.g_push = g_push;
  EmitArgs ee;
  if (e) {
    ee = *e;
  } else {
    ee = EmitArgs{};
  }
  const int grid = g_push + g_inj + (ee.defer ? 1 : 0);
  if (a.f32)
    hipLaunchKernelGGL(k_particles<true>, dim3(grid), dim3(kBlock), 0, s, b, ee);
  else
    hipLaunchKernelGGL(k_particles<false>, dim3(grid), dim3(kBlock), 0, s, b, ee);
  return hipGetLastError();
}
hipError_t launch_seed_build(const DevMesh& m, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_build, dim3(grid), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}
hipError_t launch_stats(const int64_t* rows, int n_rows, pic_step_stats* st,
                        const int32_t* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(kAccFields), dim3(kBlock), 0, s, rows, n_rows, st, gate);
  return hipGetLastError();
}
hipError_t launch_emit(const EmitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_fallback(const StepArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_fallback, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_locate(const LocateArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_locate, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_locate_scan, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_deposit(const DepositArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_deposit, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace fp
