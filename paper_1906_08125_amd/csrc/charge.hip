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
// k_face_charge: one workgroup per face (Q_f, d_f,min, the sum);
// k_atom_charge: one thread per (atom, range of faces), the faces in LDS
// tiles, summed in face order; k_atom_reduce adds the ranges in order (no
// atomics: the result does not depend on scheduling).
#include "charge.h"

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
        const double d = dist_mi(m, c, at);
        q += (s_Q[k] * exp(-(d - s_min[k]) / a.r_c)) / s_S[k];
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

}  // namespace

int charge_splits(int64_t n_emit, int64_t n_atoms, int n_cu) {
  const int64_t blocks = (n_atoms + kThreads - 1) / kThreads;
  int64_t k = ((int64_t)n_cu * 4 + blocks - 1) / (blocks > 0 ? blocks : 1);
  const int64_t tiles = (n_emit + kFaceTile - 1) / kFaceTile;
  if (k > tiles * 4) k = tiles * 4;  // at least a quarter tile per range
  if (k > 1024) k = 1024;
  return (int)(k < 1 ? 1 : k);
}

hipError_t surface_charge_launch(const ChargeArgs& a, int n_cu, hipStream_t s) {
  if (a.m.n_emit == 0) {
    // no faces: every atom's charge is the empty sum
    if (a.n_atoms > 0) {
      ChargeArgs z = a;
      z.n_split = 0;
      const int ga = (int)((a.n_atoms + kThreads - 1) / kThreads);
      hipLaunchKernelGGL(k_atom_reduce, dim3(ga), dim3(kThreads), 0, s, z);
    }
    return hipGetLastError();
  }
  const int gf = (int)(a.m.n_emit < (int64_t)n_cu * 16 ? a.m.n_emit : (int64_t)n_cu * 16);
  hipLaunchKernelGGL(k_face_charge, dim3(gf), dim3(kThreads), 0, s, a);
  if (a.n_atoms > 0) {
    const int ga = (int)((a.n_atoms + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_atom_charge, dim3(ga, a.n_split), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_atom_reduce, dim3(ga), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace fp
