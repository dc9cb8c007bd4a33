// Host handle of one mesh: device records plus the per-handle scratch.
#pragma once
#include <string>
#include <vector>

#include "amg.h"
#include "common.h"
#include "solver.h"

struct pic_mesh {
  fp::DevMesh dm{};
  pic_mesh_info info{};
  std::vector<void*> allocs;
  // caller workspace of mesh_create_in: the persistent device arrays are
  // carved from it (256-byte aligned) instead of allocated; ws_dry only
  // adds up their sizes (mesh_workspace_bytes: no device memory touched)
  char* ws_base = nullptr;
  size_t ws_size = 0, ws_used = 0;
  bool ws_dry = false;
  int device = 0;
  int n_cu = 0;
  // solver scratch: b, x, r, u, w, p, s (f64) and the partial sums
  double* cg_vec[7] = {};
  double* cg_bprev = nullptr;          // right-hand side of the last pass
  float* cg_vec32[5] = {};             // r, u, w, p, s of the FP32 recursion
  double* cg_part = nullptr;
  int cg_grid = 0;
  fp::CgCtrl* cg_ctrl = nullptr;       // device control word
  fp::CgReport* cg_report_host = nullptr;  // pinned, device-mapped report
  fp::CgReport* cg_report_dev = nullptr;   // its device address
  int64_t cg_seq = 0;
  hipEvent_t rb_event = nullptr;
  int step_spec = 0;                   // iterations speculated per step solve
  const int32_t* dir_nodes = nullptr;
  int64_t n_dir = 0;
  // step scratch
  fp::StepScratch* scratch = nullptr;
  int32_t* offsets = nullptr;
  int32_t* counts = nullptr;
  pic_solve_stats* solve_stats = nullptr;
  int32_t* locate_count = nullptr;
  // particle kernel grids and their per-block counter rows: grid_push and
  // grid_inj are the most any launch may use (the counter rows are sized
  // for them; a batch schedule may ask up to them); pic_step launches
  // step_push[f32] push workgroups (as many as are resident at once) and
  // step_inj injecting ones
  int grid_push = 0, grid_inj = 0, grid_fb = 0;
  int step_push[2] = {0, 0}, step_inj = 0;
  int64_t* acc_rows = nullptr;
  // particle-capacity scratch (grown on demand)
  int64_t pcap = 0;
  int32_t* queue = nullptr;
  void* sort_mem = nullptr;
  size_t sort_bytes = 0;
  void* adj_mem = nullptr;             // adjoint scratch (grown on demand)
  size_t adj_bytes = 0;
  double* charge_mem = nullptr;        // surface-charge scratch (grown on demand)
  size_t charge_cap = 0;               // its size in doubles
  // CG iteration batches captured as HIP graphs (kernel arguments, count)
  struct IterGraph {
    fp::CgArgs key;
    int count;
    hipGraphExec_t exec;
  };
  std::vector<IterGraph> graphs;
  hipStream_t cap_stream = nullptr;    // private stream used only to capture
  // AMG hierarchy of K (built on the first solve that asks for it)
  fp::AmgDev amg{};
  bool amg_ready = false;
  // host copies of the emitting faces
  std::vector<int32_t> h_e_tet, h_e_nodes;
  std::vector<double> h_e_area;
  // kernel timing: (class, start, stop) per launch while enabled
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_class;
  uint32_t prof_mask = 0;   // classes timed (1 << PIC_K_*)
  bool prof_open = false;   // the last prof_begin recorded an event
  int32_t prof_every = 1;   // pic_step times its steps k = 0, every, 2 every, ...
  hipEvent_t prof_settle = nullptr;  // untimed event before each bracket
  int64_t prof_step = -1;   // the step k of the call pic_step is enqueuing (-1: none)
};

namespace fp {
pic_status build_mesh(const pic_mesh_desc* d, pic_mesh* h, std::string& msg);
void free_mesh(pic_mesh* h);
void* dev_alloc(pic_mesh* h, size_t bytes, hipError_t& err);
}  // namespace fp
