// The C ABI (include/femocs_pic.h): argument checks, scratch management and
// the per-step kernel sequence.  Every entry point only enqueues work on the
// caller's stream.
#include <cmath>
#include <cstring>
#include <string>

#include "mesh.h"
#include "particles.h"
#include "solver.h"

namespace {

thread_local std::string g_err;

pic_status fail(pic_status s, const std::string& m) {
  g_err = m;
  return s;
}

pic_status hip_fail(hipError_t e, const char* where) {
  return fail(PIC_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Grow the particle-capacity scratch (fallback queue) of a handle.
hipError_t ensure_capacity(pic_mesh* h, int64_t cap) {
  if (cap <= h->pcap) return hipSuccess;
  if (h->queue) {
    hipError_t e = hipFree(h->queue);
    if (e != hipSuccess) return e;
    h->queue = nullptr;
  }
  hipError_t e = hipMalloc(&h->queue, sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1));
  if (e != hipSuccess) return e;
  h->pcap = cap;
  return hipSuccess;
}

fp::CgArgs cg_args(const pic_mesh* h, const int64_t* charge, double w_sp,
                   double E0, double* phi, double* E,
                   const pic_solve_params* prm) {
  const fp::Phys ph = fp::phys_constants();
  fp::CgArgs a;
  std::memset(&a, 0, sizeof a);
  a.m = h->dm;
  a.charge = charge;
  a.coef = ((-ph.e_eps) * w_sp) * fp::kFxInv;
  a.E0 = E0;
  a.tol = prm->tol;
  a.max_iter = prm->max_iter;
  a.phi = phi;
  a.E = E;
  a.b = h->cg_vec[0];
  a.x = h->cg_vec[1];
  a.r = h->cg_vec[2];
  a.u = h->cg_vec[3];
  a.w = h->cg_vec[4];
  a.p = h->cg_vec[5];
  a.s = h->cg_vec[6];
  a.part = h->cg_part;
  a.dir_nodes = h->dir_nodes;
  a.n_dir = h->n_dir;
  return a;
}

pic_status check_solve(const pic_solve_params* p) {
  if (!p) return fail(PIC_E_ARG, "solve params are null");
  if (!finite_pos(p->tol) || p->max_iter < 0)
    return fail(PIC_E_ARG, "solve params: tol must be > 0, max_iter >= 0");
  if (p->precision != PIC_FP64)
    return fail(PIC_E_ARG, "solve params: unsupported precision");
  return PIC_OK;
}

}  // namespace

extern "C" {

const char* pic_last_error(void) { return g_err.c_str(); }

pic_status mesh_create(const pic_mesh_desc* desc, void* stream, pic_mesh** out) {
  if (!desc || !out) return fail(PIC_E_ARG, "mesh_create: null argument");
  *out = nullptr;
  pic_mesh* h = new pic_mesh();
  (void)hipGetDevice(&h->device);
  std::string msg;
  const pic_status s = fp::build_mesh(desc, h, msg);
  if (s != PIC_OK) {
    fp::free_mesh(h);
    delete h;
    return fail(s, msg);
  }
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    fp::free_mesh(h);
    delete h;
    return hip_fail(e, "mesh_create");
  }
  *out = h;
  return PIC_OK;
}

pic_status mesh_destroy(pic_mesh* h) {
  if (!h) return PIC_OK;
  (void)hipDeviceSynchronize();
  fp::free_mesh(h);
  if (h->queue) (void)hipFree(h->queue);
  if (h->sort_mem) (void)hipFree(h->sort_mem);
  delete h;
  return PIC_OK;
}

pic_status mesh_query(const pic_mesh* h, pic_mesh_info* info) {
  if (!h || !info) return fail(PIC_E_ARG, "mesh_query: null argument");
  *info = h->info;
  return PIC_OK;
}

pic_status mesh_emit_faces(const pic_mesh* h, int32_t* tet, int32_t* nodes3,
                           double* area) {
  if (!h) return fail(PIC_E_ARG, "mesh_emit_faces: null mesh");
  const size_t F = h->h_e_tet.size();
  if (tet) std::memcpy(tet, h->h_e_tet.data(), F * sizeof(int32_t));
  if (nodes3) std::memcpy(nodes3, h->h_e_nodes.data(), 3 * F * sizeof(int32_t));
  if (area) std::memcpy(area, h->h_e_area.data(), F * sizeof(double));
  return PIC_OK;
}

pic_status locate(const pic_mesh* hc, int64_t n, const double* x,
                  const double* y, const double* z, int32_t* tet_inout,
                  uint8_t* where_out, void* stream) {
  pic_mesh* h = const_cast<pic_mesh*>(hc);
  if (!h || n < 0) return fail(PIC_E_ARG, "locate: bad mesh or count");
  if (n == 0) return PIC_OK;
  if (!x || !y || !z || !tet_inout || !where_out)
    return fail(PIC_E_ARG, "locate: null array");
  if (n >= (1ll << 31)) return fail(PIC_E_ARG, "locate: n >= 2^31");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ensure_capacity(h, n);
  if (e != hipSuccess) return hip_fail(e, "locate");
  e = hipMemsetAsync(h->locate_count, 0, sizeof(int32_t), s);
  if (e != hipSuccess) return hip_fail(e, "locate");
  fp::LocateArgs a;
  a.m = h->dm;
  a.n = n;
  a.x = x;
  a.y = y;
  a.z = z;
  a.tet = tet_inout;
  a.where = where_out;
  a.queue = h->queue;
  a.n_queue = h->locate_count;
  const int64_t want = (n + 255) / 256;
  const int grid = (int)std::min<int64_t>(want, (int64_t)h->n_cu * 8);
  e = fp::launch_locate(a, std::max(grid, 1), s);
  if (e != hipSuccess) return hip_fail(e, "locate");
  return PIC_OK;
}

pic_status deposit(const pic_mesh* h, int64_t n, const double* x,
                   const double* y, const double* z, const int32_t* tet,
                   const double* w, int64_t* charge, void* stream) {
  if (!h || n < 0) return fail(PIC_E_ARG, "deposit: bad mesh or count");
  if (n == 0) return PIC_OK;
  if (!x || !y || !z || !tet || !w || !charge)
    return fail(PIC_E_ARG, "deposit: null array");
  fp::DepositArgs a;
  a.m = h->dm;
  a.n = n;
  a.x = x;
  a.y = y;
  a.z = z;
  a.w = w;
  a.tet = tet;
  a.charge = charge;
  const int64_t want = (n + 255) / 256;
  const int grid = (int)std::min<int64_t>(want, (int64_t)h->n_cu * 8);
  hipError_t e = fp::launch_deposit(a, std::max(grid, 1), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "deposit");
  return PIC_OK;
}

pic_status poisson_solve(const pic_mesh* h, const int64_t* charge,
                         double w_sp, double E0, double* phi, double* E_out,
                         const pic_solve_params* params,
                         pic_solve_stats* stats, void* stream) {
  if (!h || !phi) return fail(PIC_E_ARG, "poisson_solve: null mesh or phi");
  if (!std::isfinite(w_sp) || !std::isfinite(E0))
    return fail(PIC_E_ARG, "poisson_solve: non-finite w_sp or E0");
  pic_status ps = check_solve(params);
  if (ps != PIC_OK) return ps;
  fp::CgArgs a = cg_args(h, charge, w_sp, E0, phi, E_out, params);
  a.stats = stats;
  hipError_t e = fp::launch_pcg_fp64(a, h->cg_grid, h->cg_block, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "poisson_solve");
  return PIC_OK;
}

pic_status emission_rate(const pic_mesh* h, const double* E, double phi_w,
                         double* rate, double* face_F, void* stream) {
  if (!h || !E || !rate) return fail(PIC_E_ARG, "emission_rate: null argument");
  if (!finite_pos(phi_w)) return fail(PIC_E_ARG, "emission_rate: phi_w <= 0");
  const fp::Phys ph = fp::phys_constants();
  fp::EmitArgs a;
  std::memset(&a, 0, sizeof a);
  a.m = h->dm;
  a.E = E;
  a.c = {ph.a_fn, ph.b_fn, ph.c_s, ph.j_unit};
  a.phi_w = phi_w;
  a.j_scale = 1.0;
  a.rate = rate;
  a.face_F = face_F;
  hipError_t e = fp::launch_emit(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "emission_rate");
  return PIC_OK;
}

pic_status pic_step(pic_mesh* h, const pic_particles* P, const pic_fields* F,
                    const pic_step_params* prm, int32_t n_steps,
                    pic_step_stats* stats, void* stream) {
  if (!h || !P || !F || !prm || !stats)
    return fail(PIC_E_ARG, "pic_step: null argument");
  if (n_steps < 0) return fail(PIC_E_ARG, "pic_step: n_steps < 0");
  if (n_steps == 0) return PIC_OK;
  if (P->precision != PIC_FP64)
    return fail(PIC_E_ARG, "pic_step: unsupported particle precision");
  if (P->capacity <= 0 || P->capacity >= (1ll << 31))
    return fail(PIC_E_ARG, "pic_step: capacity must be in [1, 2^31)");
  if (!P->x || !P->y || !P->z || !P->vx || !P->vy || !P->vz || !P->w ||
      !P->tet || !P->birth || !P->id || !P->n_slots)
    return fail(PIC_E_ARG, "pic_step: null particle array");
  if (!F->phi || !F->E || !F->charge)
    return fail(PIC_E_ARG, "pic_step: null field array");
  if (!finite_pos(prm->dt) || !std::isfinite(prm->E0) || !finite_pos(prm->w_sp) ||
      !finite_pos(prm->phi_w) || !std::isfinite(prm->j_scale) || prm->j_scale < 0 ||
      prm->step0 < 0 || prm->step0 + n_steps >= (1ll << 21) || prm->resort_every < 0)
    return fail(PIC_E_ARG, "pic_step: invalid step parameters");
  pic_status ps = check_solve(&prm->solve);
  if (ps != PIC_OK) return ps;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ensure_capacity(h, P->capacity);
  if (e != hipSuccess) return hip_fail(e, "pic_step");

  const fp::Phys ph = fp::phys_constants();
  fp::StepArgs a;
  std::memset(&a, 0, sizeof a);
  a.m = h->dm;
  a.x = (double*)P->x;
  a.y = (double*)P->y;
  a.z = (double*)P->z;
  a.vx = (double*)P->vx;
  a.vy = (double*)P->vy;
  a.vz = (double*)P->vz;
  a.w = P->w;
  a.tet = P->tet;
  a.birth = P->birth;
  a.id = P->id;
  a.n_slots = P->n_slots;
  a.E = F->E;
  a.charge = F->charge;
  a.s_face = prm->s_face;
  a.offsets = h->offsets;
  a.queue = h->queue;
  a.scratch = h->scratch;
  a.dt = prm->dt;
  a.qm_dt = ph.qm * prm->dt;
  a.Q = (ph.qm * prm->dt) * 0.5;
  a.seed = prm->seed;
  a.instance = (uint64_t)prm->instance;

  fp::EmitArgs ea;
  std::memset(&ea, 0, sizeof ea);
  ea.m = h->dm;
  ea.E = F->E;
  ea.c = {ph.a_fn, ph.b_fn, ph.c_s, ph.j_unit};
  ea.phi_w = prm->phi_w;
  ea.j_scale = prm->j_scale;
  ea.dt = prm->dt;
  ea.w_sp = prm->w_sp;
  ea.seed = prm->seed;
  ea.instance = (uint64_t)prm->instance;
  ea.capacity = P->capacity;
  ea.counts = h->counts;
  ea.offsets = h->offsets;
  ea.n_slots = P->n_slots;
  ea.scratch = h->scratch;

  fp::CgArgs ca = cg_args(h, F->charge, prm->w_sp, prm->E0, F->phi, F->E, &prm->solve);

  const int grid_push = h->n_cu * 8;
  const int grid_inj = h->n_cu * 2;
  const int grid_fb = 64;
  for (int32_t k = 0; k < n_steps; ++k) {
    const int64_t step = prm->step0 + k;
    pic_step_stats* st = stats + k;
    a.step = step;
    a.stats = st;
    ea.step = step;
    ea.stats = st;
    ca.step_stats = st;
    if ((e = hipMemsetAsync(st, 0, sizeof(pic_step_stats), s)) != hipSuccess ||
        (e = hipMemsetAsync(h->scratch, 0, sizeof(fp::StepScratch), s)) != hipSuccess ||
        (e = hipMemsetAsync(F->charge, 0, sizeof(int64_t) * (size_t)h->dm.n_nodes, s)) != hipSuccess)
      return hip_fail(e, "pic_step");
    if ((e = fp::launch_push(a, grid_push, s)) != hipSuccess) return hip_fail(e, "pic_step push");
    if ((e = fp::launch_emit(ea, s)) != hipSuccess) return hip_fail(e, "pic_step emit");
    if ((e = fp::launch_inject(a, grid_inj, s)) != hipSuccess) return hip_fail(e, "pic_step inject");
    if ((e = fp::launch_fallback(a, grid_fb, s)) != hipSuccess) return hip_fail(e, "pic_step fallback");
    if ((e = fp::launch_pcg_fp64(ca, h->cg_grid, h->cg_block, s)) != hipSuccess)
      return hip_fail(e, "pic_step solve");
  }
  return PIC_OK;
}

}  // extern "C"
