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
  // Cutoff path (cut = 1).  A pair (f, j) enters the weights only if
  // d_fj - d_f,min <= kCutRc r_c: the pairs left out carry, per face, less
  // than n_atoms e^-kCutRc of its charge (< 1e-13 of it for 2e4 atoms).
  // Atoms and face centroids are binned into a grid of nx x ny x nz cells
  // (periodic in x and y, sizes cx, cy, cz >= c_min; z from z0, the end
  // cells open beyond the box) and copied in cell order.  A face's nearest
  // atom is looked up in the 27 cells around it (exact when within c_min),
  // its kept atoms and an atom's kept faces in the cells within reach
  // (at most K cells away).  A face without an atom within c_min (a "far"
  // face) scans every atom, and then the atom pass takes every face.
  int cut;
  int nx, ny, nz, K;
  double cx, cy, cz, z0, c_min;
  int64_t n_cells_pad; // n_cells + 1: the tile totals of the scan follow
  int32_t* a_cnt;      // [n_cells + 1] atoms per cell, then cell starts;
                       // then [ceil(n_cells / 1024)] scan tile totals
  int32_t* a_idx;      // [n_atoms] atom at each position (cell order,
                       // ascending inside a cell)
  int32_t* a_tmp;      // [n_atoms] the same in arrival order
  int32_t* a_cell;     // [n_atoms] cell of each atom
  int32_t* a_rank;     // [n_atoms] arrival slot inside its cell
  double* a_xyz;       // [3 n_atoms] atom coordinates by position
  int32_t* f_cnt;      // the same for the face centroids
  int32_t* f_idx;
  int32_t* f_tmp;
  int32_t* f_cell;
  int32_t* f_rank;
  double* f_cen;       // [3 n_emit] face centroids by position
  double* f_Q_s;       // [n_emit] Q_f, d_f,min and the weight sum by position
  double* f_min_s;
  double* f_sum_s;
  int32_t* n_far;      // [1] far faces
};

constexpr double kCutRc = 40.0;

// The cell grid of the cutoff path for mesh m and r_c: false when the
// cutoff sphere does not fit the periodic box (2 K + 1 cells per axis) --
// the all-pairs path is then taken.
bool charge_cut_plan(const DevMesh& m, double r_c, ChargeArgs& a);
// int32 and double scratch of the cutoff path
size_t charge_cut_ints(const ChargeArgs& a, int64_t n_atoms, int64_t n_emit);

// Face ranges of the atom pass: enough workgroups to fill the chip.
int charge_splits(int64_t n_emit, int64_t n_atoms, int n_cu);

hipError_t surface_charge_launch(const ChargeArgs& a, int n_cu, hipStream_t s);

}  // namespace fp
