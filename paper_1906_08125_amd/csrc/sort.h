// Launch interface of the particle re-sort (by tet, with compaction).
#pragma once
#include "common.h"

namespace fp {

constexpr int kSortBins = 256;   // 8-bit digits
constexpr int kSortTile = 4096;  // items per workgroup of a pass

struct SortArgs {
  int64_t n_tets;
  int32_t* n_slots;       // in: slots in use, out: live particles
  int32_t* n_live;        // scratch scalar
  pic_step_stats* stats;  // or null
  // particle arrays (x, y, z, vx, vy, vz of real_bytes each)
  void* real[6];
  int real_bytes;
  double* w;
  int32_t* tet;
  int32_t* birth;
  int64_t* id;
  // scratch
  uint32_t* key[2];
  uint32_t* val[2];
  uint32_t* hist;         // [kSortBins][sort_tiles(capacity)]
  uint32_t* total;        // [kSortBins]
  void* s_real[6];
  double* s_w;
  int32_t* s_tet;
  int32_t* s_birth;
  int64_t* s_id;
};

// copyback: the sorted particles are copied back into the arrays they came
// from (real, w, ...); else they stay in the scratch arrays (s_real, s_w,
// ...), which the caller then uses as the particle arrays, and only the
// slot count is set.
hipError_t sort_particles(const SortArgs& a, int64_t capacity, int n_cu,
                          hipStream_t s, bool copyback = true);
// the s_* arrays copied into real, w, ... for the *n_slots slots in use
hipError_t copy_particles(const SortArgs& a, int n_cu, hipStream_t s);
size_t sort_scratch_bytes(int64_t capacity, int real_bytes);
int sort_tiles(int64_t capacity);

}  // namespace fp
