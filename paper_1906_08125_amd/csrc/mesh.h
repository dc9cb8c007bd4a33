// Host handle of one mesh: device records plus the per-handle scratch.
#pragma once
#include <string>
#include <vector>

#include "common.h"

struct pic_mesh {
  fp::DevMesh dm{};
  pic_mesh_info info{};
  std::vector<void*> allocs;
  int device = 0;
  int n_cu = 0;
  // solver scratch: b, x, r, u, w, p, s (f64) and the partial sums
  double* cg_vec[7] = {};
  double* cg_part = nullptr;
  int cg_grid = 0;
  int cg_block = 512;
  const int32_t* dir_nodes = nullptr;
  int64_t n_dir = 0;
  // step scratch
  fp::StepScratch* scratch = nullptr;
  int32_t* offsets = nullptr;
  int32_t* counts = nullptr;
  pic_solve_stats* solve_stats = nullptr;
  int32_t* locate_count = nullptr;
  // particle-capacity scratch (grown on demand)
  int64_t pcap = 0;
  int32_t* queue = nullptr;
  void* sort_mem = nullptr;
  size_t sort_bytes = 0;
  // host copies of the emitting faces
  std::vector<int32_t> h_e_tet, h_e_nodes;
  std::vector<double> h_e_area;
};

namespace fp {
pic_status build_mesh(const pic_mesh_desc* d, pic_mesh* h, std::string& msg);
void free_mesh(pic_mesh* h);
void* dev_alloc(pic_mesh* h, size_t bytes, hipError_t& err);
}  // namespace fp
