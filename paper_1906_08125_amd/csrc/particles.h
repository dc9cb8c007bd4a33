// Launch interface of the particle kernels.
#pragma once
#include "common.h"

namespace fp {

constexpr int kAccFields = kStepCounters;  // counters per block row (see acc_flush)

struct EmitConsts {
  double a_fn, b_fn, c_s, j_unit;
};

struct StepArgs {
  DevMesh m;
  void *x, *y, *z, *vx, *vy, *vz;  // double, or float when f32
  double* w;
  int32_t *tet, *birth;
  int64_t* id;
  int32_t* n_slots;
  const void* E;        // nodal field [4 n_nodes], double or float (f32)
  int f32;              // mixed precision: float particles and field
  int64_t* charge;      // [n_nodes]
  const double* s_face; // [n_emit] or null
  const int32_t* offsets;  // [n_emit + 1] exclusive scan of counts
  int32_t* queue;       // [capacity] fallback queue
  StepScratch* scratch;
  pic_step_stats* stats;
  int64_t* acc_rows;    // [kAccFields][acc_stride] per-block counters
  int acc_stride;       // rows of both kernels (field-major layout)
  double Q, dt, qm_dt;
  uint64_t seed;
  uint64_t instance;
  int64_t step;
  int g_push;           // workgroups of the push role (the rest inject)
  int n_blocks;         // workgroups of the particle kernel (the fallback
                        // kernel's counter rows follow theirs)
  // null, or the previous solve's control state: a launch enqueued before
  // that solve's outcome is known does nothing unless the solve has ended
  // (CG_DONE or CG_NOCONV)
  const int32_t* gate;
  // cell field mode: the field in tet t is -(grad phi)_t, from phi
  int cell;
  const double* phi;
};

struct EmitArgs {
  DevMesh m;
  const void* E;        // double [4 n_nodes], or float when f32
  int f32;
  EmitConsts c;
  double phi_w, j_scale, dt, w_sp;
  uint64_t seed, instance;
  int64_t step;
  int64_t capacity;
  int32_t* counts;   // [n_emit] or null (rate only)
  int32_t* offsets;  // [n_emit + 1]
  int32_t* n_slots;
  StepScratch* scratch;
  pic_step_stats* stats;  // or null
  double* rate;           // or null
  double* face_F;         // or null
  int64_t* clear;         // node charges cleared by k_begin, or null
  int64_t n_clear;
  const int32_t* gate;    // as StepArgs::gate
  // the emission counts are computed by the first workgroup of the particle
  // kernel (launch_particles with these arguments), not by k_begin
  int defer;
  int cell;               // as StepArgs::cell (face field of the face's tet)
  const double* phi;
  const int32_t* counts_in;  // frozen per-face counts (replace the rounding) or null
  int32_t* counts_out;       // the counts used, or null
};

struct LocateArgs {
  DevMesh m;
  int64_t n;
  const double *x, *y, *z;
  int32_t* tet;
  uint8_t* where;
  int32_t* queue;
  int32_t* n_queue;
};

struct DepositArgs {
  DevMesh m;
  int64_t n;
  const double *x, *y, *z, *w;
  const int32_t* tet;
  int64_t* charge;
};

hipError_t launch_begin(const EmitArgs& a, int grid, hipStream_t s);
// Workgroups of the particle kernel (FP64 or FP32 storage) resident on one
// compute unit at once, by the runtime's occupancy calculator (0 on error).
int particle_blocks_per_cu(int f32);
// e: the step's emission, computed by workgroup 0 while the others push
// (e.defer set; the injecting workgroups wait for it), or null
hipError_t launch_particles(const StepArgs& a, const EmitArgs* e, int g_push,
                            int g_inj, hipStream_t s);
hipError_t launch_stats(const int64_t* rows, int n_rows, pic_step_stats* st,
                        const int32_t* gate, hipStream_t s);
hipError_t launch_seed_build(const DevMesh& m, int grid, hipStream_t s);
hipError_t launch_emit(const EmitArgs& a, hipStream_t s);
hipError_t launch_fallback(const StepArgs& a, int grid, hipStream_t s);
hipError_t launch_locate(const LocateArgs& a, int grid, hipStream_t s);
hipError_t launch_deposit(const DepositArgs& a, int grid, hipStream_t s);

// Batched launches over the instances of device arrays E[] / A[] with the
// block schedules given (one schedule per kernel kind).
hipError_t launch_begin_b(const EmitArgs* E, const BatchMap& map, int grid,
                          hipStream_t s);
hipError_t launch_particles_b(const StepArgs* A, const BatchMap& map, int grid,
                              int f32, hipStream_t s);
hipError_t launch_fallback_b(const StepArgs* A, const BatchMap& map, int grid,
                             hipStream_t s);
hipError_t launch_stats_b(const StepArgs* A, const BatchMap& map, int grid,
                          hipStream_t s);

}  // namespace fp
