// Binary Monte Carlo collisions of the superparticles of each tet.
#pragma once
#include "common.h"

namespace fp {

struct CollideArgs {
  DevMesh m;
  const int32_t* n_slots;  // slots [0, *n_slots) grouped by tet
  void* v[3];              // vx, vy, vz (FP64, or FP32 when f32)
  int f32;
  const double* w;         // relative weights
  const int32_t* tet;
  const int64_t* id;
  double dt_coll, w_sp;
  double c_var;            // (q/m)^2 (q/eps0)^2 / (2 pi), nm^6 fs^-4
  uint64_t seed, instance;
  int64_t step;
  // scratch, capacity entries each
  uint64_t* key;
  int32_t* perm;
  int32_t* seg_s;   // first slot of the slot's run
  int32_t* seg_n;   // length of the slot's run (0: dead slot)
  long long* seg_q; // summed relative weight in 2^-40 units, at the run's
                    // first slot (integer atomics: order-free)
  int32_t* big;     // first slots of the runs ranked by a workgroup
  int32_t* n_big;   // scalar
};

// Pairing keys, ranks within the runs of equal tet, then one thread per
// pair (or per odd triple) colliding it.
hipError_t collide_particles(const CollideArgs& a, int n_cu, hipStream_t s);

}  // namespace fp
