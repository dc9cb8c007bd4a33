// Launch interface of the adjoint kernels (reverse of one PIC step).
#pragma once
#include "common.h"
#include "solver.h"

namespace fp {

constexpr int kAdjBlock = 256;

struct AdjArgs {
  DevMesh m;
  // pre-step (checkpoint) particles
  const void *px, *py, *pz;
  const int32_t* ptet;
  const int32_t* n_pre;     // device scalar
  // post-step particles (the same slots, then the injected ones)
  const void *qx, *qy, *qz;
  const int32_t* qtet;
  const double* qw;
  const int32_t* qbirth;
  const int64_t* qid;
  const int32_t* n_post;    // device scalar
  int f32;                  // positions stored in FP32
  const void* Ek;           // E_k [4 n_nodes]
  const void* Ek1;          // E_{k+1}
  int e32;                  // fields stored in FP32
  const double* s_face;     // weight multipliers or null (all 1)
  int64_t cap;
  double* rb;               // [3][cap] adjoint of positions
  double* vb;               // [3][cap] adjoint of velocities
  double* Eb;               // [4 n_nodes] adjoint of the field
  const double* mu;         // [n_nodes] adjoint potential (0 on Dirichlet)
  double* rhs;              // [n_free] R^T Eb
  double* sc;               // [cap] weight-adjoint contribution per slot
  double* av;               // [5][cap] gather-adjoint vector a, then R1, R2
  long long* acc_E;         // [3 n_nodes] fixed-point accumulators
  long long* acc_s;         // [n_emit]
  double* part;             // [G + 2 Gp + 2]: g.mu partials, maxima, scales
  int G;                    // workgroups of the node kernels
  int Gp;                   // workgroups of the particle kernels
  double dt, qm, w_sp, coef_real, wQ, wE;
  int32_t T, initial;
  uint64_t seed, instance;
  int64_t step;
  double* dJ_dE0;           // device scalar (+=)
  double* dJ_ds;            // device [n_emit] (+=)
  double* bref;             // running max of the solves' ||b||, or null
  const CgCtrl* ctrl;       // the solver's control word (||b||^2 of the solve)
};

// objective term of E_{k+1} into Eb, then R^T Eb into rhs; clears the
// accumulators
hipError_t adj_launch_pre_solve(const AdjArgs& a, hipStream_t s);
// after the solve of K mu = rhs: the particle reverse and the scatters
hipError_t adj_launch_post_solve(const AdjArgs& a, hipStream_t s);
// J[0] += w_sp q_anode 2^-40, J[1] += (mean emitting-face |E|) / T,
// J[2] = wQ J[0] + wE J[1] (one workgroup).
hipError_t launch_window_objective(const DevMesh& m, const void* E, int f32,
                                   const pic_step_stats* st, double w_sp,
                                   int T, double wQ, double wE, double* J,
                                   hipStream_t s);
// w[i] = w_base[i] s_face[birth[i]] for live slots, w_base[i] otherwise.
hipError_t launch_face_weights(int64_t cap, const int32_t* n_slots,
                               const int32_t* tet, const int32_t* birth,
                               const double* w_base, const double* s_face,
                               double* w, int grid, hipStream_t s);

}  // namespace fp
