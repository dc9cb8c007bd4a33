// Face charge and its distribution to surface atoms.
#pragma once
#include "common.h"

namespace fp {

struct ChargeArgs {
  DevMesh m;
  const void* E;       // nodal field (f64, or f32 when f32)
  int f32;
  const double* phi;   // potential (cell field mode)
  int cell;
  double e_eps;        // e / eps0, V nm
  int64_t n_atoms;
  const double* atoms; // [3 * n_atoms]
  double r_c;
  double* face_Q;      // out [n_emit]
  double* atom_q;      // out [n_atoms]
  double* f_min;       // scratch [n_emit]: nearest-atom distance
  double* f_sum;       // scratch [n_emit]: weight normalisation
  double* part;        // scratch [n_split][n_atoms]: per face-range sums
  int n_split;
};

// Face ranges of the atom pass: enough workgroups to fill the chip.
int charge_splits(int64_t n_emit, int64_t n_atoms, int n_cu);

hipError_t surface_charge_launch(const ChargeArgs& a, int n_cu, hipStream_t s);

}  // namespace fp
