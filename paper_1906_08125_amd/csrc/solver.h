// Launch interface of the Poisson solver kernels.
#pragma once
#include "common.h"

namespace fp {

enum { CG_ITER = 0, CG_RECHECK = 1, CG_DONE = 2, CG_NOCONV = 3 };

// Solver control word (device memory; mirrored to pinned host memory).
struct CgCtrl {
  int32_t state;
  int32_t zero_rhs;
  int64_t iters;        // iterations completed before the current (re)start
  int64_t iters_final;  // iterations completed when the recursive test fired
  int64_t restarts;
  double bb;            // ||b||^2
  double relres;        // last true relative residual
  double rstart;        // ||r|| at the last (re)start (mixed inner target)
  double alpha[2], gamma[2];
  // iteration counters of batched launches (the host does not track each
  // instance): it_a is read by upd and written by spmv, it_b the reverse,
  // so no kernel reads a counter that the same launch writes
  int32_t it_a, it_b;
  // set by the resfield pass of a conditional re-check (1: the recursion
  // had stopped, the re-check runs) and read by the start pass after it
  int32_t rc_gate, pad;
};

// Host-visible report of the control word (pinned, device-mapped memory).
struct CgReport {
  int64_t seq;     // written last; the host waits for its value
  int32_t state;
  int32_t pad;
  int64_t iters;
};

constexpr int kCgBlock = 512;
constexpr int kCgSlots = 10;

struct CgArgs {
  DevMesh m;
  const int64_t* charge;  // [n_nodes] or null
  const double* rhs;      // [n_free] right-hand side replacing the load, or null
  // optional reference norm: the stopping test becomes
  // ||r|| <= tol max(||b||, *bref) (a scale shared by a sequence of solves)
  const double* bref;
  double coef;            // (-e/eps0) w_sp 2^-40
  double E0;
  double tol;
  int64_t max_iter;
  double* phi;            // [n_nodes] in: guess, out: solution
  void* E;                // [4 n_nodes] double (float if mixed) or null
  double *x, *r, *u, *w, *p, *s;  // [n_free]
  // Mixed precision: the CG recursion runs in FP32 (r, u, w, p, s below)
  // against K in FP32, while x, b, the true residual, every reduction and
  // the stopping tests stay FP64.  The recursion stops once its residual
  // falls below max(tol ||b||, inner_tol ||r_start||); the true residual is
  // then recomputed in FP64 and the FP32 recursion restarted from it
  // (iterative refinement) until tol is met.
  int mixed;
  int e32;                // E in FP32 from R in FP32 (difference form)
  double inner_tol;
  float *r32, *u32, *w32, *p32, *s32;  // [n_free]
  double* part;           // [kCgSlots][G]
  int G;                  // workgroups of every solver kernel
  // E already equals R phi for the incoming phi (the previous solve of the
  // same fields ended with it and nothing has changed phi since): the first
  // pass of the solve computes the residual only
  int keep_field;
  // The first pass forms the residual from the previous one instead of a
  // product with K: b - K phi = (b - b_prev) + r_prev, where r_prev (in r)
  // is the true residual that the previous solve of the same system ended
  // with (every solve ends with a residual pass over its final phi) and
  // b_prev its right-hand side; valid while phi is unchanged since.
  int incremental;
  double* bprev;          // [n_free] right-hand side of the last pass
  CgCtrl* ctrl;
  // host address of the AMG hierarchy (AmgDev) when the solve is
  // preconditioned by it, else null (Jacobi); the CG recursion is then FP64
  // (mixed = 0), and amg32 runs the V-cycle in FP32
  const void* amg;
  int amg32;
  const void* amg_dev;    // device copy of that AmgDev (batched launches)
  CgReport* report;       // host-mapped report record (device address)
  const int32_t* dir_nodes;
  int64_t n_dir;
  pic_solve_stats* stats;      // or null
  pic_step_stats* step_stats;  // or null
  // the particle kernels' per-workgroup counter rows of the step (or null):
  // the first pass of the solve sums them into step_stats (workgroups
  // 0 .. kStepCounters - 1), in place of a launch of its own
  const int64_t* acc_rows;
  int acc_n;
  // the start of the next step of a pic_step call, done by the kernel that
  // ends this solve instead of a launch of its own: the node charges
  // cleared, the next step's stats record and the particle counters reset,
  // inj_base taken from *n_slots.  next_stats null: no next step (the
  // charges of the last step stay for the caller).
  pic_step_stats* next_stats;
  StepScratch* next_scratch;
  const int32_t* n_slots;
  int64_t* clear_charge;
  int64_t n_clear;
  // lean: the incremental first pass of a step whose warm start is expected
  // to meet the tolerance (no iterations in the step before).  It leaves x
  // and u (r32 and u32 in mixed precision) to k_cg_prep, launched only if
  // the test asks for iterations, and clears the node charges as it reads
  // them (the next step's clear); the later passes of the solve take b
  // from bprev (b_saved).  The test then runs in one workgroup and does
  // not start the product, which k_cg_start with dev_gate 2 does after
  // k_cg_prep.  Requires a next step (next_stats) and clear_charge ==
  // charge.
  int lean;
  int b_saved;
};

// seq != 0: the last kernel of the launch writes the state with this
// sequence number into args.report (host-mapped).
hipError_t cg_launch_begin(const CgArgs& a, int64_t seq, hipStream_t s);
// after a lean first pass whose test asks for iterations: x and u, then the
// start pass's product (none for AMG)
hipError_t cg_launch_lean_iter(const CgArgs& a, hipStream_t s);
hipError_t cg_launch_iters(const CgArgs& a, int it0, int n, int64_t seq,
                           hipStream_t s);
hipError_t cg_launch_recheck(const CgArgs& a, int64_t seq, hipStream_t s);
// the same re-check, done only if the recursion has stopped (state
// CG_RECHECK; decided on the device, no report): ends a round of
// iterations so that a solve whose recursion stopped in it comes out of the
// round with its true-residual test done
hipError_t cg_launch_recheck_if(const CgArgs& a, hipStream_t s);
// n iterations numbered by the device counters (no report)
hipError_t cg_launch_iters_dev(const CgArgs& a, int n, hipStream_t s);
// the control state with sequence number seq into a.report
hipError_t cg_launch_report(const CgArgs& a, int64_t seq, hipStream_t s);

// Batched launches: one launch per solver kernel covers every instance of
// args[] (device array) with the block schedule map; mask selects the
// instances a re-check applies to.  Reports are written by cg_batch_report.
struct CgBatch {
  const CgArgs* args;
  BatchMap map;
  uint64_t mask;
};
// incremental: every instance's first pass forms its residual from its
// previous solve (CgArgs::incremental; all instances alike)
hipError_t cg_batch_begin(const CgBatch& b, int grid, int incremental,
                          hipStream_t s);
hipError_t cg_batch_iters(const CgBatch& b, int grid, int n, hipStream_t s);
hipError_t cg_batch_recheck(const CgBatch& b, int grid, hipStream_t s);
// cg_launch_recheck_if for every instance of the map
hipError_t cg_batch_recheck_if(const CgBatch& b, int grid, hipStream_t s);
// reports instances 0 .. n - 1 (all of the batch, whatever the map)
hipError_t cg_batch_report(const CgBatch& b, int n, int64_t seq, hipStream_t s);

}  // namespace fp
