// Launch interface of the cooperative Poisson solver.
#pragma once
#include "common.h"

namespace fp {

struct CgArgs {
  DevMesh m;
  const int64_t* charge;  // [n_nodes] or null
  double coef;            // (-e/eps0) w_sp 2^-40
  double E0;
  double tol;
  int64_t max_iter;
  double* phi;            // [n_nodes] in: guess, out: solution
  double* E;              // [4 n_nodes] or null
  double *b, *x, *r, *u, *w, *p, *s;  // [n_free]
  double* part;           // [2][4][grid]
  const int32_t* dir_nodes;
  int64_t n_dir;
  pic_solve_stats* stats;      // or null
  pic_step_stats* step_stats;  // or null
};

hipError_t launch_pcg_fp64(const CgArgs& args, int grid, int block,
                           hipStream_t s);
hipError_t pcg_fp64_occupancy(int block, int* blocks_per_cu);

}  // namespace fp
