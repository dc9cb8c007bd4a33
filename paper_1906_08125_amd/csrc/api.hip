// The C ABI (include/femocs_pic.h): argument checks, scratch management and
// the per-step kernel sequence.  Every entry point only enqueues work on the
// caller's stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "adjoint.h"
#include "collide.h"
#include "charge.h"
#include "mesh.h"
#include "metal.h"
#include "particles.h"
#include "solver.h"
#include "sort.h"

struct pic_batch {
  std::vector<pic_mesh*> h;
  void* d_args = nullptr;   // per-step argument arrays (device)
  void* h_args = nullptr;   // their pinned staging copy
  size_t args_bytes = 0;
  hipEvent_t uploaded = nullptr;  // staging copy consumed
  hipEvent_t reported = nullptr;  // liveness of the report waits
  int64_t seq = 0;
};

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

// Grow the particle-capacity scratch (fallback queue, sort buffers) of a
// handle; later calls with the same or a smaller capacity allocate nothing.
hipError_t ensure_capacity(pic_mesh* h, int64_t cap, bool sort,
                           int real_bytes) {
  if (cap > h->pcap) {
    if (h->queue) {
      hipError_t e = hipFree(h->queue);
      if (e != hipSuccess) return e;
      h->queue = nullptr;
    }
    hipError_t e = hipMalloc(&h->queue, sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1));
    if (e != hipSuccess) return e;
    h->pcap = cap;
  }
  if (sort) {
    const size_t need = fp::sort_scratch_bytes(cap, real_bytes);
    if (need > h->sort_bytes) {
      if (h->sort_mem) {
        hipError_t e = hipFree(h->sort_mem);
        if (e != hipSuccess) return e;
        h->sort_mem = nullptr;
        h->sort_bytes = 0;
      }
      hipError_t e = hipMalloc(&h->sort_mem, need);
      if (e != hipSuccess) return e;
      h->sort_bytes = need;
    }
  }
  return hipSuccess;
}

// Carve the sort scratch into its arrays.
fp::SortArgs sort_args(pic_mesh* h, const pic_particles* P, int real_bytes) {
  fp::SortArgs a;
  std::memset(&a, 0, sizeof a);
  const int64_t cap = P->capacity;
  char* p = (char*)h->sort_mem;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~(size_t)255;
    return (void*)q;
  };
  a.n_tets = h->dm.n_tets;
  a.n_slots = P->n_slots;
  a.n_live = (int32_t*)take(256);
  void* real[6] = {P->x, P->y, P->z, P->vx, P->vy, P->vz};
  for (int f = 0; f < 6; ++f) {
    a.real[f] = real[f];
    a.s_real[f] = take((size_t)cap * real_bytes);
  }
  a.real_bytes = real_bytes;
  a.w = P->w;
  a.tet = P->tet;
  a.birth = P->birth;
  a.id = P->id;
  for (int k = 0; k < 2; ++k) {
    a.key[k] = (uint32_t*)take((size_t)cap * 4);
    a.val[k] = (uint32_t*)take((size_t)cap * 4);
  }
  a.s_w = (double*)take((size_t)cap * 8);
  a.s_tet = (int32_t*)take((size_t)cap * 4);
  a.s_birth = (int32_t*)take((size_t)cap * 4);
  a.s_id = (int64_t*)take((size_t)cap * 8);
  a.hist = (uint32_t*)take((size_t)fp::kSortBins * fp::sort_tiles(cap) * 4);
  a.total = (uint32_t*)take((size_t)fp::kSortBins * 4);
  return a;
}

// Collision arguments over the sort scratch (free between re-sorts).
fp::CollideArgs collide_args(pic_mesh* h, const pic_particles* P,
                             double dt_coll, double w_sp, uint64_t seed,
                             int64_t step, int64_t instance) {
  const bool f32 = P->precision == PIC_MIXED;
  const fp::SortArgs sa = sort_args(h, P, f32 ? 4 : 8);
  const fp::Phys ph = fp::phys_constants();
  const double qe = ph.qm * ph.e_eps;
  fp::CollideArgs c;
  std::memset(&c, 0, sizeof c);
  c.m = h->dm;
  c.n_slots = P->n_slots;
  c.v[0] = P->vx;
  c.v[1] = P->vy;
  c.v[2] = P->vz;
  c.f32 = f32;
  c.w = P->w;
  c.tet = P->tet;
  c.id = P->id;
  c.dt_coll = dt_coll;
  c.w_sp = w_sp;
  c.c_var = qe * qe / (2.0 * 3.14159265358979323846);
  c.seed = seed;
  c.instance = (uint64_t)instance;
  c.step = step;
  c.key = (uint64_t*)sa.s_id;
  c.perm = (int32_t*)sa.key[0];
  c.seg_s = (int32_t*)sa.key[1];
  c.seg_n = (int32_t*)sa.val[0];
  c.seg_q = (long long*)sa.s_w;
  c.big = (int32_t*)sa.val[1];
  c.n_big = sa.n_live;
  return c;
}

fp::CgArgs cg_args(const pic_mesh* h, const int64_t* charge, double w_sp,
                   double E0, double* phi, void* E, bool e32,
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
  a.x = h->cg_vec[1];
  a.r = h->cg_vec[2];
  a.u = h->cg_vec[3];
  a.w = h->cg_vec[4];
  a.p = h->cg_vec[5];
  a.s = h->cg_vec[6];
  a.bprev = h->cg_bprev;
  a.mixed = prm->precision == PIC_MIXED;
  a.e32 = e32;
  a.inner_tol = prm->inner_tol;
  a.r32 = h->cg_vec32[0];
  a.u32 = h->cg_vec32[1];
  a.w32 = h->cg_vec32[2];
  a.p32 = h->cg_vec32[3];
  a.s32 = h->cg_vec32[4];
  a.part = h->cg_part;
  a.G = h->cg_grid;
  a.ctrl = h->cg_ctrl;
  a.dir_nodes = h->dir_nodes;
  a.n_dir = h->n_dir;
  return a;
}

// Wait (spinning on the host) for the solver report with sequence number seq,
// written by a kernel already enqueued on s.  Liveness: a report still
// missing after 2 ms gets an event recorded behind everything enqueued so
// far; once that event has completed, the report must be visible or never
// comes.  (An event per solve instead would cost every step: each event is
// a packet of its own, and the GPU idles ~5 us at it.)
hipError_t cg_wait(pic_mesh* h, int64_t seq, hipStream_t s, fp::CgReport& out) {
  const auto t0 = std::chrono::steady_clock::now();
  bool armed = false;
  for (long spin = 0;; ++spin) {
    if (__atomic_load_n(&h->cg_report_host->seq, __ATOMIC_ACQUIRE) == seq) break;
    if ((spin & 1023) == 1023) {
      if (!armed) {
        if (std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(2))
          continue;
        const hipError_t r = hipEventRecord(h->rb_event, s);
        if (r != hipSuccess) return r;
        armed = true;
        continue;
      }
      // once the event has completed, the report kernel before it has too
      const hipError_t q = hipEventQuery(h->rb_event);
      if (q == hipSuccess) {
        if (__atomic_load_n(&h->cg_report_host->seq, __ATOMIC_ACQUIRE) == seq) break;
        return hipErrorUnknown;
      }
      if (q != hipErrorNotReady) return q;
    }
  }
  out.state = h->cg_report_host->state;
  out.iters = h->cg_report_host->iters;
  out.seq = seq;
  return hipSuccess;
}

void drop_graphs(pic_mesh* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

// n CG iterations (numbered by the device counters) as replays of captured
// graphs of 2^j iterations: a launch chain of short kernels is bound by the
// host's submission rate, a graph is submitted at once.  The graphs are
// kept per handle, keyed by the kernel arguments (the fields the iteration
// kernels do not read are cleared so that every step of a run shares them).
hipError_t iterate_graphs(pic_mesh* h, const fp::CgArgs& a0, int n, hipStream_t s) {
  fp::CgArgs a = a0;
  a.stats = nullptr;
  a.step_stats = nullptr;
  a.acc_rows = nullptr;
  a.acc_n = 0;
  a.next_stats = nullptr;
  a.next_scratch = nullptr;
  a.n_slots = nullptr;
  a.clear_charge = nullptr;
  a.n_clear = 0;
  a.report = nullptr;
  a.charge = nullptr;
  a.rhs = nullptr;
  a.E = nullptr;
  a.keep_field = 0;
  a.incremental = 0;
  a.lean = a.b_saved = 0;
  a.coef = a.E0 = 0.0;
  hipError_t e;
  if (!h->cap_stream &&
      (e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return e;
  for (int bit = 8; bit >= 0; --bit) {
    const int cnt = 1 << bit;
    while (n >= cnt) {
      hipGraphExec_t exec = nullptr;
      for (auto& g : h->graphs)
        if (g.count == cnt && std::memcmp(&g.key, &a, sizeof a) == 0) {
          exec = g.exec;
          break;
        }
      if (!exec) {
        if (h->graphs.size() >= 64) drop_graphs(h);
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return e;
        const hipError_t le =
            a.amg ? fp::amg_launch_iters(a, *(const fp::AmgDev*)a.amg, cnt, h->cap_stream)
                  : fp::cg_launch_iters_dev(a, cnt, h->cap_stream);
        if ((e = hipStreamEndCapture(h->cap_stream, &graph)) != hipSuccess) return e;
        if (le != hipSuccess) {
          (void)hipGraphDestroy(graph);
          return le;
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        pic_mesh::IterGraph ig;
        std::memcpy(&ig.key, &a, sizeof a);
        ig.count = cnt;
        ig.exec = exec;
        h->graphs.push_back(ig);
      }
      if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return e;
      n -= cnt;
    }
  }
  return hipSuccess;
}

// One Poisson solve: the resfield pass (residual of the warm start and the
// field of phi) and the convergence test, then -- before waiting -- a first
// batch of `spec` CG iterations (they return at once if the test passed).
// While the report says "not converged", further batches follow, and a
// re-check (scatter + resfield + test) when the recursive residual has
// converged.  The field is always that of the final phi.  Blocks the calling
// thread at the waits.  Returns the iterations done.
// First round of a solve: the residual pass and convergence test, spec
// speculated iterations, and the report of the state; *seq_out receives the
// report's sequence number.  Nothing waits here.
hipError_t solve_start(pic_mesh* h, fp::CgArgs& a, int spec, hipStream_t s,
                       int64_t* seq_out) {
  a.report = h->cg_report_dev;
  const int64_t seq = ++h->cg_seq;
  // A step solve after one that needed no iteration: its warm start is
  // expected to meet the tolerance at once, so the first pass leaves x and
  // u to a launch made only if it does not (and clears the charges for the
  // next step as it reads them).
  a.lean = spec <= 0 && a.incremental && !a.rhs && a.bprev && a.next_stats &&
                   a.charge && (const int64_t*)a.clear_charge == a.charge
               ? 1
               : 0;
  a.b_saved = a.lean;
  hipError_t e = fp::cg_launch_begin(a, spec > 0 ? 0 : seq, s);
  if (e != hipSuccess) return e;
  if (spec > 0) {
    if ((e = iterate_graphs(h, a, spec, s)) != hipSuccess ||
        (e = fp::cg_launch_recheck_if(a, s)) != hipSuccess ||
        (e = fp::cg_launch_report(a, seq, s)) != hipSuccess)
      return e;
  }
  *seq_out = seq;
  return hipSuccess;
}

void prof_begin(pic_mesh* h, int cls, hipStream_t s);
void prof_end(pic_mesh* h, hipStream_t s);
constexpr int kProfNoCount = 0x100;  // time the bracket, count no launch

// Waits for the report of the first round and enqueues further rounds (a
// true-residual re-check, or twice as many iterations as the last round)
// until the solve has ended.  *first_state: the state the first report
// carried.  Further rounds are timed as solve time while profiling.
hipError_t solve_finish(pic_mesh* h, const fp::CgArgs& a, int spec,
                        int64_t seq, hipStream_t s, int64_t* iters_out,
                        int32_t* first_state) {
  fp::CgReport r;
  hipError_t e = cg_wait(h, seq, s, r);
  if (e != hipSuccess) return e;
  if (first_state) *first_state = r.state;
  // a lean first pass has left x, u and the start's product undone
  bool prep = a.lean && r.state == fp::CG_ITER;
  int batch = spec, rounds = 0;
  for (int guard = 0; guard < (1 << 20); ++guard) {
    if (r.state == fp::CG_DONE || r.state == fp::CG_NOCONV) break;
    seq = ++h->cg_seq;
    prof_begin(h, PIC_K_SOLVE | kProfNoCount, s);
    if (r.state == fp::CG_RECHECK) {
      if ((e = fp::cg_launch_recheck(a, seq, s)) != hipSuccess) return e;
      batch = 16;
    } else {
      // Every round ends with the conditional re-check, so a recursion that
      // stops inside it comes back tested.  An AMG iteration is some fifteen
      // dependent launches and a solve needs few: after a speculated round
      // the next ones run 1, 2, 4, ... iterations (launches past the stop
      // cost as much as working ones); Jacobi rounds start at 8.
      if (a.amg)
        batch = rounds == 0 ? (spec > 0 ? 1 : 4) : std::min(2 * batch, 32);
      else
        batch = batch < 8 ? 8 : std::min(2 * batch, 256);
      ++rounds;
      if (prep) {
        if ((e = fp::cg_launch_lean_iter(a, s)) != hipSuccess) return e;
        prep = false;
      }
      if ((e = iterate_graphs(h, a, batch, s)) != hipSuccess ||
          (e = fp::cg_launch_recheck_if(a, s)) != hipSuccess ||
          (e = fp::cg_launch_report(a, seq, s)) != hipSuccess)
        return e;
    }
    prof_end(h, s);
    if ((e = cg_wait(h, seq, s, r)) != hipSuccess) return e;
  }
  if (iters_out) *iters_out = r.iters;
  return hipSuccess;
}

hipError_t run_solve(pic_mesh* h, const fp::CgArgs& a0, int spec, hipStream_t s,
                     int64_t* iters_out) {
  fp::CgArgs a = a0;
  int64_t seq = 0;
  hipError_t e = solve_start(h, a, spec, s, &seq);
  if (e != hipSuccess) return e;
  return solve_finish(h, a, spec, seq, s, iters_out, nullptr);
}

pic_status check_solve(const pic_solve_params* p) {
  if (!p) return fail(PIC_E_ARG, "solve params are null");
  if (!finite_pos(p->tol) || p->max_iter < 0)
    return fail(PIC_E_ARG, "solve params: tol must be > 0, max_iter >= 0");
  if (p->precision != PIC_FP64 && p->precision != PIC_MIXED)
    return fail(PIC_E_ARG, "solve params: unknown precision");
  if (p->precision == PIC_MIXED &&
      !(p->inner_tol >= 1e-7 && p->inner_tol <= 0.5))
    return fail(PIC_E_ARG, "solve params: inner_tol must be in [1e-7, 0.5]");
  if (p->precond != PIC_PRECOND_JACOBI && p->precond != PIC_PRECOND_AMG)
    return fail(PIC_E_ARG, "solve params: unknown preconditioner");
  return PIC_OK;
}

void* amg_alloc(void* ctx, size_t bytes) {
  hipError_t err = hipSuccess;
  void* p = fp::dev_alloc((pic_mesh*)ctx, bytes, err);
  return err == hipSuccess ? p : nullptr;
}

// Points a.amg at the handle's hierarchy when the parameters ask for AMG,
// building it on first use.
pic_status use_precond(pic_mesh* h, const pic_solve_params* p, fp::CgArgs& a,
                       hipStream_t s, const char* who) {
  a.amg = nullptr;
  a.amg_dev = nullptr;
  if (p->precond != PIC_PRECOND_AMG) return PIC_OK;
  if (!h->amg_ready) {
    std::string msg;
    const hipError_t e = fp::amg_build(h->dm, s, amg_alloc, h, h->amg, msg);
    if (e != hipSuccess)
      return fail(PIC_E_DEVICE, std::string(who) + ": " +
                                    (msg.empty() ? hipGetErrorString(e) : msg));
    h->amg_ready = true;
  }
  a.amg = &h->amg;
  a.amg_dev = h->amg.dev;
  // mixed precision with AMG: the CG recursion stays FP64, the V-cycle runs
  // in FP32 (no refinement restarts)
  a.amg32 = a.mixed;
  a.mixed = 0;
  return PIC_OK;
}

pic_status check_step(const pic_particles* P, const pic_fields* F,
                      const pic_step_params* prm, int32_t n_steps,
                      const char* who) {
  const std::string w(who);
  if (P->precision != PIC_FP64 && P->precision != PIC_MIXED)
    return fail(PIC_E_ARG, w + ": unknown particle precision");
  if (P->capacity <= 0 || P->capacity >= (1ll << 31))
    return fail(PIC_E_ARG, w + ": capacity must be in [1, 2^31)");
  if (!P->x || !P->y || !P->z || !P->vx || !P->vy || !P->vz || !P->w ||
      !P->tet || !P->birth || !P->id || !P->n_slots)
    return fail(PIC_E_ARG, w + ": null particle array");
  if (!F->phi || !F->E || !F->charge)
    return fail(PIC_E_ARG, w + ": null field array");
  if (!finite_pos(prm->dt) || !std::isfinite(prm->E0) || !finite_pos(prm->w_sp) ||
      !finite_pos(prm->phi_w) || !std::isfinite(prm->j_scale) || prm->j_scale < 0 ||
      prm->step0 < 0 || prm->step0 + n_steps >= (1ll << 21) || prm->resort_every < 0)
    return fail(PIC_E_ARG, w + ": invalid step parameters");
  if (prm->field_mode != PIC_FIELD_NODAL && prm->field_mode != PIC_FIELD_CELL)
    return fail(PIC_E_ARG, w + ": unknown field mode");
  if (prm->collide != 0 && (prm->collide != 1 || prm->resort_every <= 0))
    return fail(PIC_E_ARG, w + ": collide must be 0, or 1 with resort_every > 0");
  return check_solve(&prm->solve);
}

// The kernel arguments of one instance's step (the per-step fields -- step
// index and stats record -- are set by the caller).
struct StepSet {
  fp::StepArgs a;
  fp::EmitArgs ea;
  fp::CgArgs ca;
};

StepSet step_set(pic_mesh* h, const pic_particles* P, const pic_fields* F,
                 const pic_step_params* prm, int g_push, int g_inj, int g_fb) {
  const bool f32 = P->precision == PIC_MIXED;
  const fp::Phys ph = fp::phys_constants();
  StepSet ss;
  fp::StepArgs& a = ss.a;
  std::memset(&a, 0, sizeof a);
  a.m = h->dm;
  a.x = P->x;
  a.y = P->y;
  a.z = P->z;
  a.vx = P->vx;
  a.vy = P->vy;
  a.vz = P->vz;
  a.f32 = f32;
  a.w = P->w;
  a.tet = P->tet;
  a.birth = P->birth;
  a.id = P->id;
  a.n_slots = P->n_slots;
  a.E = F->E;
  a.cell = prm->field_mode == PIC_FIELD_CELL;
  a.phi = F->phi;
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
  a.acc_rows = h->acc_rows;
  a.acc_stride = g_push + g_inj + g_fb;
  a.g_push = g_push;
  a.n_blocks = g_push + g_inj;

  fp::EmitArgs& ea = ss.ea;
  std::memset(&ea, 0, sizeof ea);
  ea.m = h->dm;
  ea.E = F->E;
  ea.f32 = f32;
  ea.cell = a.cell;
  ea.phi = F->phi;
  ea.counts_in = prm->counts_in;
  ea.counts_out = prm->counts_out;
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
  ea.clear = F->charge;
  ea.n_clear = h->dm.n_nodes;

  ss.ca = cg_args(h, F->charge, prm->w_sp, prm->E0, F->phi, F->E, f32, &prm->solve);
  return ss;
}

// Kernel timing: an event before and after each launch while enabled.
void prof_mark(pic_mesh* h, hipStream_t s) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) {
      h->profiling = false;
      return;
    }
    h->ev_pool.push_back(ev);
  }
  (void)hipEventRecord(h->ev_pool[h->ev_used++], s);
}

// The first event after kernels stalls the stream while the caches are
// written back for the host (~5 us after a kernel that wrote much); an
// untimed event just before the bracket takes that stall, so that the
// bracket times the kernels inside it.
void prof_begin(pic_mesh* h, int cls, hipStream_t s) {
  const bool sampled = h->prof_every <= 1 || h->prof_step < 0 ||
                       h->prof_step % h->prof_every == 0;
  h->prof_open = h->profiling && sampled && ((h->prof_mask >> (cls & 0xff)) & 1u);
  if (!h->prof_open) return;
  if (!h->prof_settle &&
      hipEventCreateWithFlags(&h->prof_settle, hipEventDisableTiming) != hipSuccess) {
    h->prof_settle = nullptr;
    h->profiling = h->prof_open = false;
    return;
  }
  (void)hipEventRecord(h->prof_settle, s);
  h->ev_class.push_back(cls);
  prof_mark(h, s);
}

void prof_end(pic_mesh* h, hipStream_t s) {
  if (!h->prof_open) return;
  h->prof_open = false;
  prof_mark(h, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of locate_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends.  Element 0 is the counter of the exact-scan
// queue, elements [kNoallocHead, kNoallocHead + n) the queue itself.  Host
// code never uses the array's name as an address: each device's copy is
// looked up once (hipGetSymbolAddress with that device current) and only
// that address is passed to kernels.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNoallocHead = 64;  // counter, padded to 256 bytes
constexpr int64_t kNoallocInts = kNoallocHead + PIC_LOCATE_NOALLOC_MAX;
static_assert(kNoallocInts == (1 << 20), "4 MiB of scratch");

}  // namespace

static __device__ __align__(256) int32_t scratch[kNoallocInts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_dev[kMaxDevices] = {};

// The address of the current device's copy of scratch (looked up on the
// first call on that device), or null with *err set.
int32_t* noalloc_scratch(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_dev[device] = (int32_t*)ptr;
  }
  *err = hipSuccess;
  return g_scratch_dev[device];
}

// Clears the queue counter with a kernel (no memset node where the caller
// captures the stream into a graph).
__global__ void k_noalloc_clear(int32_t* head) {
  if (threadIdx.x < kNoallocHead) head[threadIdx.x] = 0;
}

}  // namespace

extern "C" {

pic_status pic_profile(pic_mesh* h, int32_t classes) {
  if (!h) return fail(PIC_E_ARG, "pic_profile: null mesh");
  h->prof_mask = (uint32_t)classes & PIC_PROFILE_ALL;
  h->profiling = h->prof_mask != 0;
  h->prof_open = false;
  h->ev_used = 0;
  h->ev_class.clear();
  return PIC_OK;
}

pic_status pic_profile_every(pic_mesh* h, int32_t every) {
  if (!h) return fail(PIC_E_ARG, "pic_profile_every: null mesh");
  if (every < 1) return fail(PIC_E_ARG, "pic_profile_every: every must be >= 1");
  h->prof_every = every;
  return PIC_OK;
}

pic_status pic_profile_read(pic_mesh* h, pic_kernel_times* out) {
  if (!h || !out) return fail(PIC_E_ARG, "pic_profile_read: null argument");
  std::memset(out, 0, sizeof *out);
  const size_t pairs = std::min(h->ev_class.size(), h->ev_used / 2);
  if (pairs == 0) return PIC_OK;
  hipError_t e = hipEventSynchronize(h->ev_pool[2 * pairs - 1]);
  if (e != hipSuccess) return hip_fail(e, "pic_profile_read");
  for (size_t i = 0; i < pairs; ++i) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, h->ev_pool[2 * i], h->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "pic_profile_read");
    const int c = h->ev_class[i];
    if (c < 0) continue;  // a gated launch that did not run
    out->ms[c & 0xff] += ms;
    if (!(c & kProfNoCount)) out->launches[c & 0xff] += 1;
  }
  return PIC_OK;
}

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

pic_status mesh_workspace_bytes(const pic_mesh_desc* desc, size_t* bytes) {
  if (!desc || !bytes) return fail(PIC_E_ARG, "mesh_workspace_bytes: null argument");
  *bytes = 0;
  pic_mesh* h = new pic_mesh();
  (void)hipGetDevice(&h->device);
  h->ws_dry = true;
  std::string msg;
  const pic_status s = fp::build_mesh(desc, h, msg);
  const size_t need = h->ws_used;
  fp::free_mesh(h);
  delete h;
  if (s != PIC_OK) return fail(s, msg);
  *bytes = need;
  return PIC_OK;
}

pic_status mesh_create_in(const pic_mesh_desc* desc, void* workspace, size_t ws_bytes,
                          void* stream, pic_mesh** out) {
  if (!desc || !out || !workspace)
    return fail(PIC_E_ARG, "mesh_create_in: null argument");
  if (((uintptr_t)workspace & 255u) != 0)
    return fail(PIC_E_ARG, "mesh_create_in: workspace not 256-byte aligned");
  *out = nullptr;
  pic_mesh* h = new pic_mesh();
  (void)hipGetDevice(&h->device);
  h->ws_base = (char*)workspace;
  h->ws_size = ws_bytes;
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
    return hip_fail(e, "mesh_create_in");
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
  if (h->adj_mem) (void)hipFree(h->adj_mem);
  if (h->charge_mem) (void)hipFree(h->charge_mem);
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (hipEvent_t ev : h->ev_pool) (void)hipEventDestroy(ev);
  if (h->prof_settle) (void)hipEventDestroy(h->prof_settle);
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
  hipError_t e = ensure_capacity(h, n, false, 8);
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

pic_status locate_noalloc(const pic_mesh* h, int64_t n, const double* x,
                          const double* y, const double* z, int32_t* tet_inout,
                          uint8_t* where_out, void* stream) {
  if (!h || n < 0) return fail(PIC_E_ARG, "locate_noalloc: bad mesh or count");
  if (n > PIC_LOCATE_NOALLOC_MAX)
    return fail(PIC_E_ARG, "locate_noalloc: n exceeds PIC_LOCATE_NOALLOC_MAX");
  if (n == 0) return PIC_OK;
  if (!x || !y || !z || !tet_inout || !where_out)
    return fail(PIC_E_ARG, "locate_noalloc: null array");
  int device = -1;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, "locate_noalloc");
  if (device != h->device || device < 0 || device >= kMaxDevices)
    return fail(PIC_E_ARG, "locate_noalloc: the mesh lives on another device");
  int32_t* sc = noalloc_scratch(device, &e);
  if (!sc) return hip_fail(e, "locate_noalloc");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(kNoallocHead), 0, s, sc);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "locate_noalloc");
  fp::LocateArgs a;
  a.m = h->dm;
  a.n = n;
  a.x = x;
  a.y = y;
  a.z = z;
  a.tet = tet_inout;
  a.where = where_out;
  a.queue = sc + kNoallocHead;
  a.n_queue = sc;
  const int64_t want = (n + 255) / 256;
  const int grid = (int)std::min<int64_t>(want, (int64_t)h->n_cu * 8);
  e = fp::launch_locate(a, std::max(grid, 1), s);
  if (e != hipSuccess) return hip_fail(e, "locate_noalloc");
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
                         double w_sp, double E0, double* phi, void* E_out,
                         const pic_solve_params* params,
                         pic_solve_stats* stats, void* stream) {
  if (!h || !phi) return fail(PIC_E_ARG, "poisson_solve: null mesh or phi");
  if (!std::isfinite(w_sp) || !std::isfinite(E0))
    return fail(PIC_E_ARG, "poisson_solve: non-finite w_sp or E0");
  pic_status ps = check_solve(params);
  if (ps != PIC_OK) return ps;
  fp::CgArgs a = cg_args(h, charge, w_sp, E0, phi, E_out,
                         params->precision == PIC_MIXED, params);
  a.stats = stats;
  pic_mesh* hm = const_cast<pic_mesh*>(h);
  if ((ps = use_precond(hm, params, a, (hipStream_t)stream, "poisson_solve")) != PIC_OK)
    return ps;
  prof_begin(hm, PIC_K_SOLVE, (hipStream_t)stream);
  hipError_t e = run_solve(hm, a, 0, (hipStream_t)stream, nullptr);
  if (e != hipSuccess) return hip_fail(e, "poisson_solve");
  prof_end(hm, (hipStream_t)stream);
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

pic_status collide(pic_mesh* h, const pic_particles* P,
                   const pic_collide_params* prm, void* stream) {
  if (!h || !P || !prm) return fail(PIC_E_ARG, "collide: null argument");
  if (P->precision != PIC_FP64 && P->precision != PIC_MIXED)
    return fail(PIC_E_ARG, "collide: unknown particle precision");
  if (P->capacity <= 0 || P->capacity >= (1ll << 31))
    return fail(PIC_E_ARG, "collide: capacity must be in [1, 2^31)");
  if (!P->vx || !P->vy || !P->vz || !P->w || !P->tet || !P->id || !P->n_slots)
    return fail(PIC_E_ARG, "collide: null particle array");
  if (!finite_pos(prm->dt_coll) || !finite_pos(prm->w_sp))
    return fail(PIC_E_ARG, "collide: dt_coll and w_sp must be positive");
  const bool f32 = P->precision == PIC_MIXED;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ensure_capacity(h, P->capacity, true, f32 ? 4 : 8);
  if (e != hipSuccess) return hip_fail(e, "collide");
  prof_begin(h, PIC_K_COLLIDE, s);
  const fp::CollideArgs cl = collide_args(h, P, prm->dt_coll, prm->w_sp,
                                          prm->seed, prm->step, prm->instance);
  if ((e = fp::collide_particles(cl, h->n_cu, s)) != hipSuccess)
    return hip_fail(e, "collide");
  prof_end(h, s);
  return PIC_OK;
}

pic_status metal_create(const pic_metal_desc* desc, void* stream, pic_metal** out) {
  if (!desc || !out) return fail(PIC_E_ARG, "metal_create: null argument");
  *out = nullptr;
  std::string err;
  const pic_status rc = fp::metal_build(desc, (hipStream_t)stream, out, &err);
  return rc == PIC_OK ? rc : fail(rc, err);
}

pic_status metal_destroy(pic_metal* metal) {
  fp::metal_free(metal);
  return PIC_OK;
}

pic_status continuity_solve(pic_metal* metal, const double* sigma, const double* flux,
                            double tol, int64_t max_iter, double* Phi, double* P_J,
                            pic_metal_stats* stats, void* stream) {
  if (!metal || !sigma || !Phi) return fail(PIC_E_ARG, "continuity_solve: null argument");
  if (!flux && fp::metal_n_faces(metal) > 0)
    return fail(PIC_E_ARG, "continuity_solve: null flux");
  if (!finite_pos(tol) || max_iter < 0 || max_iter >= (1ll << 31))
    return fail(PIC_E_ARG, "continuity_solve: tol must be > 0, max_iter in [0, 2^31)");
  std::string err;
  const pic_status rc = fp::metal_continuity(metal, sigma, flux, tol, max_iter, Phi, P_J,
                                             stats, (hipStream_t)stream, &err);
  return rc == PIC_OK ? rc : fail(rc, err);
}

pic_status heat_step(pic_metal* metal, const pic_heat_params* p, const double* sigma,
                     const double* P_J, const double* P_N, double* T,
                     pic_metal_stats* stats, void* stream) {
  if (!metal || !p || !sigma || !T) return fail(PIC_E_ARG, "heat_step: null argument");
  if (!P_N && fp::metal_n_faces(metal) > 0) return fail(PIC_E_ARG, "heat_step: null P_N");
  if (!finite_pos(p->Cv) || !(std::isfinite(p->L) && p->L >= 0.0) || !finite_pos(p->dt) ||
      !(p->theta >= 0.0 && p->theta <= 1.0) || !std::isfinite(p->T_amb) ||
      !finite_pos(p->tol) || p->max_iter < 0 || p->max_iter >= (1ll << 31))
    return fail(PIC_E_ARG, "heat_step: invalid parameters");
  std::string err;
  const pic_status rc = fp::metal_heat(metal, p, sigma, P_J, P_N, T, stats,
                                       (hipStream_t)stream, &err);
  return rc == PIC_OK ? rc : fail(rc, err);
}

pic_status surface_charge(pic_mesh* h, const pic_fields* F,
                          const pic_charge_params* prm, double* face_Q,
                          double* atom_q, void* stream) {
  if (!h || !F || !prm || !face_Q)
    return fail(PIC_E_ARG, "surface_charge: null argument");
  if (prm->n_atoms < 0 || prm->n_atoms >= (1ll << 31))
    return fail(PIC_E_ARG, "surface_charge: n_atoms must be in [0, 2^31)");
  if (prm->n_atoms > 0 && (!prm->atoms || !atom_q))
    return fail(PIC_E_ARG, "surface_charge: null atom array");
  if (!finite_pos(prm->r_c))
    return fail(PIC_E_ARG, "surface_charge: r_c must be positive");
  if (prm->field_mode != PIC_FIELD_NODAL && prm->field_mode != PIC_FIELD_CELL)
    return fail(PIC_E_ARG, "surface_charge: unknown field mode");
  if (prm->precision != PIC_FP64 && prm->precision != PIC_MIXED)
    return fail(PIC_E_ARG, "surface_charge: unknown precision");
  if (prm->field_mode == PIC_FIELD_CELL ? !F->phi : !F->E)
    return fail(PIC_E_ARG, "surface_charge: null field array");
  hipStream_t s = (hipStream_t)stream;
  const int n_split = fp::charge_splits(h->dm.n_emit, prm->n_atoms, h->n_cu);
  fp::ChargeArgs a;
  std::memset(&a, 0, sizeof a);
  // the cutoff path when there are atoms and faces and the box holds the
  // cutoff sphere (else every pair)
  if (prm->n_atoms > 0 && h->dm.n_emit > 0) (void)fp::charge_cut_plan(h->dm, prm->r_c, a);
  const size_t n_dbl = 2 * (size_t)h->dm.n_emit + (size_t)n_split * (size_t)prm->n_atoms;
  // (cutoff path: sorted atom coordinates, face centroids and three face
  // results by position)
  const size_t n_cen = a.cut ? 3 * (size_t)prm->n_atoms + 6 * (size_t)h->dm.n_emit : 0;
  const size_t n_int = a.cut ? fp::charge_cut_ints(a, prm->n_atoms, h->dm.n_emit) : 0;
  const size_t need = n_dbl + n_cen + (n_int + 1) / 2;
  if (need > h->charge_cap) {
    if (h->charge_mem) {
      hipError_t e = hipFree(h->charge_mem);
      h->charge_mem = nullptr;
      h->charge_cap = 0;
      if (e != hipSuccess) return hip_fail(e, "surface_charge");
    }
    hipError_t e = hipMalloc(&h->charge_mem, sizeof(double) * need);
    if (e != hipSuccess) return hip_fail(e, "surface_charge");
    h->charge_cap = need;
  }
  a.m = h->dm;
  a.E = F->E;
  a.f32 = prm->precision == PIC_MIXED;
  a.phi = F->phi;
  a.cell = prm->field_mode == PIC_FIELD_CELL;
  a.e_eps = fp::phys_constants().e_eps;
  a.n_atoms = prm->n_atoms;
  a.atoms = prm->atoms;
  a.r_c = prm->r_c;
  a.face_Q = face_Q;
  a.atom_q = atom_q;
  a.f_min = h->charge_mem;
  a.f_sum = h->charge_mem ? h->charge_mem + h->dm.n_emit : nullptr;
  a.part = h->charge_mem ? h->charge_mem + 2 * h->dm.n_emit : nullptr;
  a.n_split = n_split;
  if (a.cut) {
    const int64_t n_cells = (int64_t)a.nx * a.ny * a.nz;
    const int64_t na = prm->n_atoms, nf = h->dm.n_emit;
    double* dp = h->charge_mem + n_dbl;
    a.a_xyz = dp;
    dp += 3 * na;
    a.f_cen = dp;
    dp += 3 * nf;
    a.f_Q_s = dp;
    dp += nf;
    a.f_min_s = dp;
    dp += nf;
    a.f_sum_s = dp;
    int32_t* ip = reinterpret_cast<int32_t*>(h->charge_mem + n_dbl + n_cen);
    const int64_t tiles = (n_cells + 1023) / 1024;
    a.a_cnt = ip;
    ip += n_cells + 1 + tiles;
    a.f_cnt = ip;
    ip += n_cells + 1 + tiles;
    a.a_idx = ip;
    ip += na;
    a.a_tmp = ip;
    ip += na;
    a.a_cell = ip;
    ip += na;
    a.a_rank = ip;
    ip += na;
    a.f_idx = ip;
    ip += nf;
    a.f_tmp = ip;
    ip += nf;
    a.f_cell = ip;
    ip += nf;
    a.f_rank = ip;
    ip += nf;
    a.n_far = ip;
  }
  const hipError_t e = fp::surface_charge_launch(a, h->n_cu, s);
  if (e != hipSuccess) return hip_fail(e, "surface_charge");
  return PIC_OK;
}

pic_status pic_step(pic_mesh* h, const pic_particles* P, const pic_fields* F,
                    const pic_step_params* prm, int32_t n_steps,
                    pic_step_stats* stats, void* stream) {
  if (!h || !P || !F || !prm || !stats)
    return fail(PIC_E_ARG, "pic_step: null argument");
  if (n_steps < 0) return fail(PIC_E_ARG, "pic_step: n_steps < 0");
  if (n_steps == 0) return PIC_OK;
  pic_status ps = check_step(P, F, prm, n_steps, "pic_step");
  if (ps != PIC_OK) return ps;
  const bool f32 = P->precision == PIC_MIXED;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ensure_capacity(h, P->capacity, prm->resort_every > 0, f32 ? 4 : 8);
  if (e != hipSuccess) return hip_fail(e, "pic_step");

  StepSet ss = step_set(h, P, F, prm, h->step_push[f32 ? 1 : 0], h->step_inj, h->grid_fb);
  if ((ps = use_precond(h, &prm->solve, ss.ca, s, "pic_step")) != PIC_OK) return ps;
  const fp::StepArgs& a = ss.a;
  const fp::EmitArgs& ea = ss.ea;
  fp::CgArgs& ca = ss.ca;
  const int grid_push = h->step_push[f32 ? 1 : 0];
  const int grid_inj = h->step_inj;
  const int grid_fb = h->grid_fb;
  // The kernels of step k before its solve: clears + emission counts, the
  // live and new particles in one launch, the exact fallback, the counters.
  // gate: null, or the control state of the previous solve (see below).
  // *prof0 receives the first profile slot of these launches.
  // (the step whose kernels are being enqueued, for the timing sample; reset
  // on every return)
  struct ProfStep {
    pic_mesh* h;
    ~ProfStep() { h->prof_step = -1; }
  } prof_step_guard{h};
  // The particle arrays alternate between the caller's and the re-sort's
  // scratch: a re-sort within the call gathers into the other set and the
  // kernels after it take that one (no copy back per re-sort); a call that
  // ends on the scratch set copies it back once.  Not with collisions,
  // which use the sort scratch themselves.
  const bool alternate = prm->resort_every > 0 && !prm->collide;
  const fp::SortArgs base_sort =
      prm->resort_every > 0 ? sort_args(h, P, f32 ? 4 : 8) : fp::SortArgs{};
  int on_scratch = 0;
  auto use_set = [&](fp::StepArgs& x) {
    if (!on_scratch) return;
    x.x = base_sort.s_real[0];
    x.y = base_sort.s_real[1];
    x.z = base_sort.s_real[2];
    x.vx = base_sort.s_real[3];
    x.vy = base_sort.s_real[4];
    x.vz = base_sort.s_real[5];
    x.w = base_sort.s_w;
    x.tet = base_sort.s_tet;
    x.birth = base_sort.s_birth;
    x.id = base_sort.s_id;
  };
  // the re-sort (or final copy) from the current set into the other one
  auto sort_from_current = [&]() {
    fp::SortArgs sa = base_sort;
    if (on_scratch) {
      for (int f = 0; f < 6; ++f) std::swap(sa.real[f], sa.s_real[f]);
      std::swap(sa.w, sa.s_w);
      std::swap(sa.tet, sa.s_tet);
      std::swap(sa.birth, sa.s_birth);
      std::swap(sa.id, sa.s_id);
    }
    return sa;
  };
  auto pre_solve = [&](int32_t k, const int32_t* gate, size_t* prof0) -> hipError_t {
    h->prof_step = k;
    fp::StepArgs ak = a;
    use_set(ak);
    fp::EmitArgs ek = ea;
    ak.step = ek.step = prm->step0 + k;
    ak.stats = ek.stats = stats + k;
    ak.gate = ek.gate = gate;
    ek.defer = 1;  // the emission runs inside the particle kernel
    *prof0 = h->ev_class.size();
    hipError_t e;
    // the first step of a call clears the charges and counters itself;
    // later steps find them cleared by the solve before them
    if (k == 0) {
      prof_begin(h, PIC_K_EMIT, s);
      if ((e = fp::launch_begin(ek, h->n_cu * 2, s)) != hipSuccess) return e;
      prof_end(h, s);
    }
    prof_begin(h, PIC_K_PUSH, s);
    if ((e = fp::launch_particles(ak, &ek, grid_push, grid_inj, s)) != hipSuccess) return e;
    prof_end(h, s);
    prof_begin(h, PIC_K_FALLBACK, s);
    if ((e = fp::launch_fallback(ak, grid_fb, s)) != hipSuccess) return e;
    prof_end(h, s);
    // (the step's counter rows are summed by the first pass of its solve)
    return hipSuccess;
  };
  // The host learns the outcome of a solve from its report.  Rather than
  // leave the GPU idle meanwhile, the next step's pre-solve kernels are
  // enqueued right behind the first report, gated on the solve's state:
  // they run if that round ended the solve (the usual case: a warm start
  // that already meets the tolerance) and do nothing otherwise, in which
  // case they are enqueued again once the solve has ended.
  bool pre_done = false;
  for (int32_t k = 0; k < n_steps; ++k) {
    const int64_t step = prm->step0 + k;
    pic_step_stats* st = stats + k;
    size_t p0 = 0;
    if (!pre_done && (e = pre_solve(k, nullptr, &p0)) != hipSuccess)
      return hip_fail(e, "pic_step particles");
    h->prof_step = k;
    // the re-sort touches only particles and the solve only the charge:
    // the sort goes first so that the next step's kernels can follow the
    // solve directly
    if (prm->resort_every > 0 && (step + 1) % prm->resort_every == 0) {
      prof_begin(h, PIC_K_SORT, s);
      fp::SortArgs sa = alternate ? sort_from_current() : base_sort;
      sa.stats = st;
      if ((e = fp::sort_particles(sa, P->capacity, h->n_cu, s, !alternate)) != hipSuccess)
        return hip_fail(e, "pic_step sort");
      if (alternate) on_scratch ^= 1;
      prof_end(h, s);
      if (prm->collide) {
        prof_begin(h, PIC_K_COLLIDE, s);
        const fp::CollideArgs cl = collide_args(
            h, P, prm->dt * prm->resort_every, prm->w_sp, prm->seed, step,
            prm->instance);
        if ((e = fp::collide_particles(cl, h->n_cu, s)) != hipSuccess)
          return hip_fail(e, "pic_step collide");
        prof_end(h, s);
      }
    }
    ca.step_stats = st;
    ca.acc_rows = h->acc_rows;
    ca.acc_n = grid_push + grid_inj + grid_fb;
    const bool next = k + 1 < n_steps;
    ca.next_stats = next ? stats + k + 1 : nullptr;
    ca.next_scratch = h->scratch;
    ca.n_slots = P->n_slots;
    ca.clear_charge = F->charge;
    ca.n_clear = h->dm.n_nodes;
    // after the first step of this call, E = R phi still holds from the
    // previous solve (every solve ends with a field pass over its final phi)
    ca.keep_field = k > 0 ? 1 : 0;
    // and its true residual and right-hand side: the first pass of this
    // solve needs no product with K
    ca.incremental = k > 0 ? 1 : 0;
    const int spec = h->step_spec;
    int64_t seq = 0;
    prof_begin(h, PIC_K_SOLVE, s);
    if ((e = solve_start(h, ca, spec, s, &seq)) != hipSuccess)
      return hip_fail(e, "pic_step solve");
    prof_end(h, s);
    const bool ahead = k + 1 < n_steps;
    size_t p1 = 0;
    if (ahead && (e = pre_solve(k + 1, &ca.ctrl->state, &p1)) != hipSuccess)
      return hip_fail(e, "pic_step particles");
    h->prof_step = k;  // (further rounds of this step's solve)
    const size_t p1e = h->ev_class.size();
    int64_t iters = 0;
    int32_t first = fp::CG_ITER;
    if ((e = solve_finish(h, ca, spec, seq, s, &iters, &first)) != hipSuccess)
      return hip_fail(e, "pic_step solve");
    pre_done = ahead && (first == fp::CG_DONE || first == fp::CG_NOCONV);
    if (ahead && !pre_done)
      for (size_t i = p1; i < p1e; ++i) h->ev_class[i] = -1;
    // speculate this many iterations in the next step's first round
    h->step_spec = (int)std::min<int64_t>(iters, 256);
  }
  if (on_scratch) {  // the caller's arrays hold the state again
    if ((e = fp::copy_particles(base_sort, h->n_cu, s)) != hipSuccess)
      return hip_fail(e, "pic_step copy");
  }
  return PIC_OK;
}

pic_status adjoint_step(pic_mesh* h, const pic_particles* pre,
                        const pic_particles* post, const pic_fields* Fk,
                        const pic_fields* Fk1, const pic_step_params* prm,
                        const pic_adjoint* adj, pic_solve_stats* stats,
                        void* stream) {
  if (!h || !pre || !Fk || !prm || !adj)
    return fail(PIC_E_ARG, "adjoint_step: null argument");
  const bool initial = adj->mode == PIC_ADJ_INITIAL;
  if (adj->mode != PIC_ADJ_STEP && !initial)
    return fail(PIC_E_ARG, "adjoint_step: unknown mode");
  if (!initial && (!post || !Fk1 || !Fk1->E || !Fk->E))
    return fail(PIC_E_ARG, "adjoint_step: a step needs post, E_k and E_{k+1}");
  if (!adj->rb || !adj->vb || !adj->Eb || !adj->mu || !adj->dJ_dE0 || !adj->dJ_ds)
    return fail(PIC_E_ARG, "adjoint_step: null adjoint array");
  if (adj->T <= 0 || !std::isfinite(adj->wQ) || !std::isfinite(adj->wE))
    return fail(PIC_E_ARG, "adjoint_step: T must be > 0 and the weights finite");
  if (pre->precision != PIC_FP64 && pre->precision != PIC_MIXED)
    return fail(PIC_E_ARG, "adjoint_step: unknown particle precision");
  if (!initial && (post->precision != pre->precision || post->capacity != pre->capacity))
    return fail(PIC_E_ARG, "adjoint_step: pre and post differ in precision or capacity");
  if (pre->capacity <= 0 || pre->capacity >= (1ll << 31))
    return fail(PIC_E_ARG, "adjoint_step: capacity must be in [1, 2^31)");
  if (!finite_pos(prm->dt) || !finite_pos(prm->w_sp))
    return fail(PIC_E_ARG, "adjoint_step: invalid step parameters");
  if (prm->field_mode != PIC_FIELD_NODAL || prm->collide != 0)
    return fail(PIC_E_ARG, "adjoint_step: only the nodal field mode without collisions has an adjoint");
  pic_status ps = check_solve(&prm->solve);
  if (ps != PIC_OK) return ps;
  const pic_particles* Q = initial ? pre : post;
  if (!pre->x || !pre->tet || !pre->n_slots || !Q->x || !Q->y || !Q->z ||
      !Q->w || !Q->tet || !Q->birth || !Q->id || !Q->n_slots)
    return fail(PIC_E_ARG, "adjoint_step: null particle array");
  hipStream_t s = (hipStream_t)stream;
  const int64_t cap = pre->capacity;
  const int64_t N = h->dm.n_nodes, F = h->dm.n_emit;
  const int Gp = h->n_cu * 4;
  const int G = h->cg_grid;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t need = al(8 * (size_t)cap) + al(40 * (size_t)cap) + al(24 * (size_t)N) +
                      al(8 * (size_t)std::max<int64_t>(F, 1)) + al(8 * (size_t)(G + 2 * Gp + 2));
  if (need > h->adj_bytes) {
    if (h->adj_mem) {
      hipError_t e = hipFree(h->adj_mem);
      if (e != hipSuccess) return hip_fail(e, "adjoint_step");
      h->adj_mem = nullptr;
      h->adj_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->adj_mem, need);
    if (e != hipSuccess) return hip_fail(e, "adjoint_step");
    h->adj_bytes = need;
  }
  char* p = (char*)h->adj_mem;
  auto take = [&](size_t b) {
    char* q = p;
    p += al(b);
    return (void*)q;
  };
  const fp::Phys ph = fp::phys_constants();
  fp::AdjArgs a;
  std::memset(&a, 0, sizeof a);
  a.m = h->dm;
  a.px = pre->x;
  a.py = pre->y;
  a.pz = pre->z;
  a.ptet = pre->tet;
  a.n_pre = pre->n_slots;
  a.qx = Q->x;
  a.qy = Q->y;
  a.qz = Q->z;
  a.qtet = Q->tet;
  a.qw = Q->w;
  a.qbirth = Q->birth;
  a.qid = Q->id;
  a.n_post = Q->n_slots;
  a.f32 = pre->precision == PIC_MIXED;
  a.Ek = Fk->E;
  a.Ek1 = initial ? nullptr : Fk1->E;
  a.e32 = a.f32;
  a.s_face = prm->s_face;
  a.cap = cap;
  a.rb = adj->rb;
  a.vb = adj->vb;
  a.Eb = adj->Eb;
  a.mu = adj->mu;
  a.rhs = h->cg_vec[0];
  a.sc = (double*)take(8 * (size_t)cap);
  a.av = (double*)take(40 * (size_t)cap);
  a.acc_E = (long long*)take(24 * (size_t)N);
  a.acc_s = (long long*)take(8 * (size_t)std::max<int64_t>(F, 1));
  a.part = (double*)take(8 * (size_t)(G + 2 * Gp + 2));
  a.G = G;
  a.Gp = Gp;
  a.dt = prm->dt;
  a.qm = ph.qm;
  a.w_sp = prm->w_sp;
  a.coef_real = (-ph.e_eps) * prm->w_sp;
  a.wQ = adj->wQ;
  a.wE = adj->wE;
  a.T = adj->T;
  a.initial = initial ? 1 : 0;
  a.seed = prm->seed;
  a.instance = (uint64_t)prm->instance;
  a.step = prm->step0;
  a.dJ_dE0 = adj->dJ_dE0;
  a.dJ_ds = adj->dJ_ds;
  a.bref = adj->bref;
  a.ctrl = h->cg_ctrl;
  prof_begin(h, PIC_K_ADJOINT, s);
  hipError_t e = fp::adj_launch_pre_solve(a, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint_step");
  fp::CgArgs ca = cg_args(h, nullptr, 0.0, 0.0, adj->mu, nullptr, false, &prm->solve);
  {
    const pic_status pq = use_precond(h, &prm->solve, ca, s, "adjoint_step");
    if (pq != PIC_OK) return pq;
  }
  ca.rhs = a.rhs;
  ca.bref = adj->bref;
  ca.stats = stats;
  int64_t iters = 0;
  if ((e = run_solve(h, ca, 0, s, &iters)) != hipSuccess) return hip_fail(e, "adjoint_step solve");
  if ((e = fp::adj_launch_post_solve(a, s)) != hipSuccess) return hip_fail(e, "adjoint_step");
  prof_end(h, s);
  return PIC_OK;
}

pic_status window_objective(const pic_mesh* h, const void* E, int32_t precision,
                            const pic_step_stats* stats, double w_sp, int32_t T,
                            double wQ, double wE, double* J, void* stream) {
  if (!h || !E || !stats || !J) return fail(PIC_E_ARG, "window_objective: null argument");
  if (precision != PIC_FP64 && precision != PIC_MIXED)
    return fail(PIC_E_ARG, "window_objective: unknown precision");
  if (T <= 0 || !finite_pos(w_sp) || !std::isfinite(wQ) || !std::isfinite(wE))
    return fail(PIC_E_ARG, "window_objective: T > 0, w_sp > 0 and finite weights required");
  const hipError_t e = fp::launch_window_objective(h->dm, E, precision == PIC_MIXED ? 1 : 0,
                                                   stats, w_sp, T, wQ, wE, J,
                                                   (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "window_objective");
  return PIC_OK;
}

pic_status apply_face_weights(const pic_mesh* h, const pic_particles* P,
                              const double* w_base, const double* s_face,
                              void* stream) {
  if (!h || !P || !w_base || !s_face)
    return fail(PIC_E_ARG, "apply_face_weights: null argument");
  if (P->capacity <= 0 || P->capacity >= (1ll << 31))
    return fail(PIC_E_ARG, "apply_face_weights: capacity must be in [1, 2^31)");
  if (!P->w || !P->tet || !P->birth || !P->n_slots)
    return fail(PIC_E_ARG, "apply_face_weights: null particle array");
  if (h->dm.n_emit == 0) return fail(PIC_E_ARG, "apply_face_weights: no emitting faces");
  const int64_t want = (P->capacity + 255) / 256;
  const int grid = (int)std::min<int64_t>(want, (int64_t)h->n_cu * 8);
  const hipError_t e = fp::launch_face_weights(P->capacity, P->n_slots, P->tet, P->birth,
                                               w_base, s_face, P->w, std::max(grid, 1),
                                               (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "apply_face_weights");
  return PIC_OK;
}

pic_status pic_batch_create(pic_mesh* const* meshes, int32_t n,
                            pic_batch** out, int32_t* limits) {
  if (!meshes || !out || n < 1 || n > PIC_MAX_BATCH)
    return fail(PIC_E_ARG, "pic_batch_create: need 1..PIC_MAX_BATCH meshes");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!meshes[i]) return fail(PIC_E_ARG, "pic_batch_create: null mesh");
    for (int j = 0; j < i; ++j)
      if (meshes[j] == meshes[i])
        return fail(PIC_E_ARG, "pic_batch_create: a mesh appears twice");
  }
  pic_batch* b = new pic_batch();
  b->h.assign(meshes, meshes + n);
  hipError_t e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->reported, hipEventDisableTiming);
  if (e != hipSuccess) {
    pic_batch_destroy(b);
    return hip_fail(e, "pic_batch_create");
  }
  if (limits)
    for (int i = 0; i < n; ++i) {
      limits[4 * i + 0] = meshes[i]->grid_push;
      limits[4 * i + 1] = meshes[i]->grid_inj;
      limits[4 * i + 2] = meshes[i]->cg_grid;
      limits[4 * i + 3] = meshes[i]->grid_fb;
    }
  *out = b;
  return PIC_OK;
}

pic_status pic_batch_destroy(pic_batch* b) {
  if (!b) return PIC_OK;
  (void)hipDeviceSynchronize();
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->h_args) (void)hipHostFree(b->h_args);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->reported) (void)hipEventDestroy(b->reported);
  delete b;
  return PIC_OK;
}

namespace {

int round8(int x) { return (x + 7) & ~7; }

// Map over the instances with active[i] (all when active is empty).
fp::BatchMap batch_map(const std::vector<int>& counts,
                       const std::vector<char>& active = {}) {
  fp::BatchMap m;
  std::memset(&m, 0, sizeof m);
  int j = 0;
  for (size_t i = 0; i < counts.size(); ++i) {
    if (!active.empty() && !active[i]) continue;
    m.inst[j] = (int8_t)i;
    m.off[j + 1] = m.off[j] + counts[i];
    ++j;
  }
  m.n_seg = j;
  return m;
}

// Wait until every instance's report carries seq (the liveness check of
// cg_wait: an event recorded on s once the reports are 2 ms late).
hipError_t batch_wait(pic_batch* b, int64_t seq, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  bool armed = false;
  for (pic_mesh* h : b->h) {
    for (long spin = 0;; ++spin) {
      if (__atomic_load_n(&h->cg_report_host->seq, __ATOMIC_ACQUIRE) == seq) break;
      if ((spin & 1023) == 1023) {
        if (!armed) {
          if (std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(2))
            continue;
          const hipError_t r = hipEventRecord(b->reported, s);
          if (r != hipSuccess) return r;
          armed = true;
          continue;
        }
        const hipError_t q = hipEventQuery(b->reported);
        if (q == hipSuccess) {
          if (__atomic_load_n(&h->cg_report_host->seq, __ATOMIC_ACQUIRE) == seq) break;
          return hipErrorUnknown;
        }
        if (q != hipErrorNotReady) return q;
      }
    }
  }
  return hipSuccess;
}

int64_t batch_next_seq(pic_batch* b) {
  int64_t s = b->seq;
  for (pic_mesh* h : b->h) s = std::max(s, h->cg_seq);
  b->seq = s + 1;
  for (pic_mesh* h : b->h) h->cg_seq = b->seq;
  return b->seq;
}

}  // namespace

pic_status pic_batch_step(pic_batch* b, const pic_particles* P,
                          const pic_fields* F, const pic_step_params* prm,
                          const pic_batch_schedule* sc, int32_t n_steps,
                          pic_step_stats* stats, void* stream) {
  if (!b || !P || !F || !prm || !sc || !stats)
    return fail(PIC_E_ARG, "pic_batch_step: null argument");
  if (n_steps < 0) return fail(PIC_E_ARG, "pic_batch_step: n_steps < 0");
  if (n_steps == 0) return PIC_OK;
  const int n = (int)b->h.size();
  const bool f32 = P[0].precision == PIC_MIXED;
  std::vector<int> c_push(n), c_inj(n), c_cg(n), c_clear(n), c_fb(n), c_stats(n, 16);
  const int fb = round8(std::max(sc->fallback_blocks, 8));
  for (int i = 0; i < n; ++i) {
    pic_mesh* h = b->h[i];
    pic_status ps = check_step(&P[i], &F[i], &prm[i], n_steps, "pic_batch_step");
    if (ps != PIC_OK) return ps;
    if ((P[i].precision == PIC_MIXED) != f32)
      return fail(PIC_E_ARG, "pic_batch_step: instances differ in precision");
    c_push[i] = round8(std::max(sc->push_blocks[i], 8));
    c_inj[i] = round8(std::max(sc->inject_blocks[i], 8));
    c_cg[i] = round8(std::max(sc->cg_blocks[i], 8));
    c_clear[i] = round8(std::max(sc->clear_blocks[i], 8));
    c_fb[i] = fb;
    if (c_push[i] > h->grid_push || c_inj[i] > h->grid_inj || c_cg[i] > h->cg_grid ||
        fb > h->grid_fb)
      return fail(PIC_E_ARG, "pic_batch_step: schedule beyond the instance's limits");
  }
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    hipError_t e = ensure_capacity(b->h[i], P[i].capacity, prm[i].resort_every > 0,
                                   f32 ? 4 : 8);
    if (e != hipSuccess) return hip_fail(e, "pic_batch_step");
  }
  // per-step argument arrays: [k][i] StepArgs, EmitArgs, CgArgs
  const size_t sa = sizeof(fp::StepArgs), se = sizeof(fp::EmitArgs), sg = sizeof(fp::CgArgs);
  const size_t per = (size_t)n * (sa + se + sg);
  const size_t need = per * (size_t)n_steps;
  hipError_t e = hipEventSynchronize(b->uploaded);  // staging free again
  if (e != hipSuccess) return hip_fail(e, "pic_batch_step");
  if (need > b->args_bytes) {
    if (b->d_args) (void)hipFree(b->d_args);
    if (b->h_args) (void)hipHostFree(b->h_args);
    b->d_args = b->h_args = nullptr;
    b->args_bytes = 0;
    if ((e = hipMalloc(&b->d_args, need)) != hipSuccess) return hip_fail(e, "pic_batch_step");
    if ((e = hipHostMalloc(&b->h_args, need, hipHostMallocDefault)) != hipSuccess)
      return hip_fail(e, "pic_batch_step");
    b->args_bytes = need;
  }
  char* hb = (char*)b->h_args;
  for (int i = 0; i < n; ++i) {
    StepSet ss = step_set(b->h[i], &P[i], &F[i], &prm[i], c_push[i], c_inj[i], fb);
    pic_status ps = use_precond(b->h[i], &prm[i].solve, ss.ca, s, "pic_batch_step");
    if (ps != PIC_OK) return ps;
    ss.ca.G = c_cg[i];
    ss.ca.report = b->h[i]->cg_report_dev;
    for (int32_t k = 0; k < n_steps; ++k) {
      const int64_t step = prm[i].step0 + k;
      pic_step_stats* st = stats + (size_t)k * n + i;
      char* base = hb + per * k;
      fp::StepArgs a = ss.a;
      a.step = step;
      a.stats = st;
      fp::EmitArgs ea = ss.ea;
      ea.step = step;
      ea.stats = st;
      fp::CgArgs ca = ss.ca;
      ca.step_stats = st;
      // as in pic_step: the field and the true residual of the previous
      // solve still hold, so the first pass needs no product with K or R
      ca.keep_field = k > 0 ? 1 : 0;
      ca.incremental = k > 0 ? 1 : 0;
      std::memcpy(base + sa * i, &a, sa);
      std::memcpy(base + sa * n + se * i, &ea, se);
      std::memcpy(base + (sa + se) * n + sg * i, &ca, sg);
    }
  }
  if ((e = hipMemcpyAsync(b->d_args, b->h_args, need, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "pic_batch_step");
  if ((e = hipEventRecord(b->uploaded, s)) != hipSuccess) return hip_fail(e, "pic_batch_step");
  std::vector<int> c_part(n);
  for (int i = 0; i < n; ++i) c_part[i] = c_push[i] + c_inj[i];
  const fp::BatchMap m_clear = batch_map(c_clear), m_part = batch_map(c_part),
                     m_fb = batch_map(c_fb), m_stats = batch_map(c_stats),
                     m_cg = batch_map(c_cg);
  const int g_clear = m_clear.off[n], g_part = m_part.off[n], g_fb = m_fb.off[n],
            g_stats = m_stats.off[n], g_cg = m_cg.off[n];
  (void)g_cg;
  pic_mesh* h0 = b->h[0];
  for (int32_t k = 0; k < n_steps; ++k) {
    char* base = (char*)b->d_args + per * k;
    const fp::StepArgs* A = (const fp::StepArgs*)base;
    const fp::EmitArgs* E = (const fp::EmitArgs*)(base + sa * n);
    fp::CgBatch cb;
    cb.args = (const fp::CgArgs*)(base + (sa + se) * n);
    cb.map = m_cg;
    cb.mask = 0;
    prof_begin(h0, PIC_K_EMIT, s);
    if ((e = fp::launch_begin_b(E, m_clear, g_clear, s)) != hipSuccess)
      return hip_fail(e, "pic_batch_step begin");
    prof_end(h0, s);
    prof_begin(h0, PIC_K_PUSH, s);
    if ((e = fp::launch_particles_b(A, m_part, g_part, f32 ? 1 : 0, s)) != hipSuccess)
      return hip_fail(e, "pic_batch_step particles");
    prof_end(h0, s);
    prof_begin(h0, PIC_K_FALLBACK, s);
    if ((e = fp::launch_fallback_b(A, m_fb, g_fb, s)) != hipSuccess ||
        (e = fp::launch_stats_b(A, m_stats, g_stats, s)) != hipSuccess)
      return hip_fail(e, "pic_batch_step fallback");
    prof_end(h0, s);
    // the solves of all instances, in shared launches: the first round
    // speculates as many iterations as the previous step needed; later
    // rounds launch only the instances still iterating
    prof_begin(h0, PIC_K_SOLVE, s);
    int64_t seq = batch_next_seq(b);
    // speculation: the instances that iterated in the previous step get as
    // many iterations before the first wait
    std::vector<char> spec_on(n, 0);
    std::vector<int> spec_n(n, 0);
    int spec = 0;
    for (int i = 0; i < n; ++i)
      if (b->h[i]->step_spec > 0) {
        spec_on[i] = 1;
        spec_n[i] = b->h[i]->step_spec;
        spec = std::max(spec, b->h[i]->step_spec);
      }
    // host copies of this step's solver arguments (a round with a single
    // active instance launches its own kernels: no batch indirection)
    auto host_cg = [&](int i) -> const fp::CgArgs& {
      return *(const fp::CgArgs*)(hb + per * k + (sa + se) * n + sg * i);
    };
    // One round of iterations over the instances act[i].  counts: per
    // instance (speculation), else count for the Jacobi instances and
    // amg_count for the AMG ones.  Instances in mask have a stopped
    // recursion and get their re-check alone this round.  Two or more AMG
    // instances iterating share the V-cycle launches (as many iterations as
    // the most any of them asks for, at most 16); a single one replays its
    // own graphs.  More than two Jacobi instances share batched launches,
    // fewer replay their own graphs.  The round ends with the conditional
    // re-check of every instance that iterated, so one whose recursion
    // stopped inside the round comes back tested.
    auto iterate = [&](const std::vector<char>& act, uint64_t mask, int count,
                       int amg_count, const std::vector<int>* counts) {
      auto want = [&](int i) {
        return counts ? (*counts)[i] : host_cg(i).amg ? amg_count : count;
      };
      std::vector<char> amg_on(n, 0), jac_on(n, 0), iterated(n, 0);
      int n_amg = 0, n_jac = 0, c_amg = 0, c_jac = 0;
      for (int i = 0; i < n; ++i) {
        if (!act[i] || ((mask >> i) & 1ull)) continue;
        if (host_cg(i).amg) {
          amg_on[i] = 1;
          ++n_amg;
          c_amg = std::max(c_amg, std::min(want(i), 16));
        } else {
          jac_on[i] = 1;
          ++n_jac;
          c_jac = std::max(c_jac, want(i));
        }
      }
      const bool amg_shared = n_amg >= 2, jac_shared = n_jac > 2;
      hipError_t r;
      // re-checks of stopped recursions
      std::vector<char> rc_on(n, 0);
      bool any_rc = false;
      for (int i = 0; i < n; ++i)
        if (act[i] && ((mask >> i) & 1ull)) rc_on[i] = any_rc = true;
      if (any_rc) {
        fp::CgBatch ca = cb;
        ca.map = batch_map(c_cg, rc_on);
        ca.mask = mask;
        if ((r = fp::cg_batch_recheck(ca, ca.map.off[ca.map.n_seg], s)) != hipSuccess)
          return r;
      }
      // iterations
      for (int i = 0; i < n; ++i) {
        const bool mine = (amg_on[i] && !amg_shared) || (jac_on[i] && !jac_shared);
        if (!mine) continue;
        const int c = host_cg(i).amg ? std::min(want(i), 16) : want(i);
        if (c <= 0) continue;
        if ((r = iterate_graphs(b->h[i], host_cg(i), c, s)) != hipSuccess) return r;
        iterated[i] = 1;
      }
      if (amg_shared && c_amg > 0) {
        std::vector<const fp::CgArgs*> hargs(n);
        for (int i = 0; i < n; ++i) hargs[i] = &host_cg(i);
        if ((r = fp::amg_batch_iters(cb.args, hargs, amg_on, c_amg, s)) != hipSuccess)
          return r;
        for (int i = 0; i < n; ++i)
          if (amg_on[i]) iterated[i] = 1;
      }
      if (jac_shared && c_jac > 0) {
        fp::CgBatch ca = cb;
        ca.map = batch_map(c_cg, jac_on);
        ca.mask = 0;
        if ((r = fp::cg_batch_iters(ca, ca.map.off[ca.map.n_seg], c_jac, s)) != hipSuccess)
          return r;
        for (int i = 0; i < n; ++i)
          if (jac_on[i]) iterated[i] = 1;
      }
      bool any_it = false;
      for (int i = 0; i < n; ++i) any_it = any_it || iterated[i];
      if (!any_it) return hipSuccess;
      fp::CgBatch ca = cb;
      ca.map = batch_map(c_cg, iterated);
      ca.mask = 0;
      return fp::cg_batch_recheck_if(ca, ca.map.off[ca.map.n_seg], s);
    };
    if ((e = fp::cg_batch_begin(cb, m_cg.off[m_cg.n_seg], k > 0 ? 1 : 0, s)) != hipSuccess ||
        (spec > 0 && (e = iterate(spec_on, 0, 0, 0, &spec_n)) != hipSuccess) ||
        (e = fp::cg_batch_report(cb, n, seq, s)) != hipSuccess ||
        (e = batch_wait(b, seq, s)) != hipSuccess)
      return hip_fail(e, "pic_batch_step solve");
    // later rounds: Jacobi 8, 16, 32, ... iterations; AMG (some fifteen
    // dependent launches per iteration, launches past the stop costing as
    // much as working ones) 1, 2, 4, ... after a speculated round, else from 4
    int batch = spec, amg_batch = 0;
    for (int guard = 0; guard < (1 << 20); ++guard) {
      uint64_t mask = 0;
      std::vector<char> active(n, 0);
      bool any = false;
      for (int i = 0; i < n; ++i) {
        const int32_t st = b->h[i]->cg_report_host->state;
        if (st == fp::CG_RECHECK) mask |= 1ull << i;
        if (st == fp::CG_RECHECK || st == fp::CG_ITER) active[i] = any = true;
      }
      if (!any) break;
      seq = batch_next_seq(b);
      batch = batch < 8 ? 8 : std::min(2 * batch, 256);
      if (mask) batch = std::min(batch, 16);
      amg_batch = guard == 0 ? (spec > 0 ? 1 : 4) : std::min(2 * amg_batch, 16);
      if ((e = iterate(active, mask, batch, amg_batch, nullptr)) != hipSuccess ||
          (e = fp::cg_batch_report(cb, n, seq, s)) != hipSuccess ||
          (e = batch_wait(b, seq, s)) != hipSuccess)
        return hip_fail(e, "pic_batch_step solve");
    }
    for (int i = 0; i < n; ++i)
      b->h[i]->step_spec = (int)std::min<int64_t>(b->h[i]->cg_report_host->iters, 256);
    prof_end(h0, s);
    for (int i = 0; i < n; ++i) {
      const int64_t step = prm[i].step0 + k;
      if (prm[i].resort_every > 0 && (step + 1) % prm[i].resort_every == 0) {
        prof_begin(h0, PIC_K_SORT, s);
        fp::SortArgs sa2 = sort_args(b->h[i], &P[i], f32 ? 4 : 8);
        sa2.stats = stats + (size_t)k * n + i;
        if ((e = fp::sort_particles(sa2, P[i].capacity, b->h[i]->n_cu, s)) != hipSuccess)
          return hip_fail(e, "pic_batch_step sort");
        prof_end(h0, s);
        if (prm[i].collide) {
          prof_begin(h0, PIC_K_COLLIDE, s);
          const fp::CollideArgs cl = collide_args(
              b->h[i], &P[i], prm[i].dt * prm[i].resort_every, prm[i].w_sp,
              prm[i].seed, step, prm[i].instance);
          if ((e = fp::collide_particles(cl, b->h[i]->n_cu, s)) != hipSuccess)
            return hip_fail(e, "pic_batch_step collide");
          prof_end(h0, s);
        }
      }
    }
  }
  return PIC_OK;
}

}  // extern "C"
