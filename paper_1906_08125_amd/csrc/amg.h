// Smoothed-aggregation algebraic multigrid as a CG preconditioner for the
// FP64 solve (an alternative to Jacobi; the paper names no preconditioner).
#pragma once
#include <vector>

#include "common.h"
#include "solver.h"

namespace fp {

constexpr int kAmgMaxLevels = 8;
constexpr int kAmgCoarseMax = 512;  // the coarsest operator is inverted densely

// A sparse matrix of the hierarchy.  lpr = 1: the sliced ELLPACK layout of
// the solver (kSell rows per slice, column-major inside a slice, padding
// entries 0 with column 0; one lane per row), for short rows.  lpr > 1
// (a power of two up to 64): CSR with lpr lanes per row and a shuffle
// reduction, for the long rows of the Galerkin operators and restrictions.
struct SellMat {
  int64_t nrows, nslices;  // (nslices: SELL only)
  int lpr;
  const int32_t* sptr;     // SELL slice offsets, or CSR row offsets [nrows+1]
  const int32_t* col;
  const double* val;
  const float* val32;      // the same values rounded to FP32
};

// One level of the hierarchy.  Level 0 is K on the free nodes; b of level 0
// is the CG residual and its smoothed output is the CG vector u.
struct AmgLevel {
  SellMat A;
  const double* invdiag;
  double omega;   // Jacobi weight 4 / (3 lambda_max(D^-1 A))
  SellMat P;      // prolongation from the next level (rows: this level)
  SellMat R;      // restriction P^T (rows: the next level)
  double* b;      // right-hand side (levels > 0)
  double* x;      // pre-smoothed iterate, then corrected
  double* r;      // residual after pre-smoothing
  double* t;      // post-smoothed iterate (levels > 0)
  // FP32 copies for the FP32 V-cycle (mixed precision)
  const float* invdiag32;
  float *b32, *x32, *r32, *t32;
};

struct AmgDev {
  int n_levels;   // levels with a smoother; the dense coarsest level follows
  AmgLevel lv[kAmgMaxLevels];
  int64_t n_coarse;
  const double* coarse_inv;  // [n_coarse][n_coarse] inverse, row-major
  double* coarse_b;
  double* coarse_x;
  const float* coarse_inv32;
  float* coarse_b32;
  float* coarse_x32;
  int64_t rows[kAmgMaxLevels + 1];  // rows per level (the coarsest last)
  // device copy of this descriptor (written last by amg_build), read by
  // the batched launches, which find each instance's hierarchy through
  // CgArgs::amg_dev
  const AmgDev* dev;
};

// Builds the hierarchy of the FP64 stiffness of m on the host (strength of
// connection, three-phase aggregation, Jacobi-smoothed prolongation,
// Galerkin products, dense inverse of the coarsest operator) and uploads it
// with alloc().  Returns hipSuccess and fills d, or an error.
hipError_t amg_build(const DevMesh& m, hipStream_t s,
                     void* (*alloc)(void* ctx, size_t bytes), void* ctx,
                     AmgDev& d, std::string& msg);

// n iterations of CG preconditioned by one V(1,1)-cycle, in the
// Chronopoulos-Gear ordering [V-cycle, w = K u, update], numbered by the
// device counters of the control word; no report.  The first V-cycle
// kernel of every iteration after the first tests the recursive residual.
// With a.amg32 the V-cycle runs in FP32 (level matrices, diagonals and
// vectors; the CG recursion stays FP64).  Levels below the finest launch
// grids sized to their rows.
hipError_t amg_launch_iters(const CgArgs& a, const AmgDev& d, int n,
                            hipStream_t s);

// n such iterations of several instances at once: every V-cycle stage (a
// level's smoothing, restriction, prolongation; the coarse solve; the
// product; the update) is one launch over all instances i with on[i], each
// getting the workgroups its own launch would have.  dargs: the instances'
// solver arguments in device memory (index i), hargs: the same on the host
// (their amg set, all alike in amg32).
hipError_t amg_batch_iters(const CgArgs* dargs, const std::vector<const CgArgs*>& hargs,
                           const std::vector<char>& on, int n, hipStream_t s);

}  // namespace fp
