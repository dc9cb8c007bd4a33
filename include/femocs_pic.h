/*
 * femocs_pic.h -- C ABI of the MI355X (gfx950) electron particle-in-cell
 * library: the PIC cycle in the vacuum above a field-emitting tip, after
 * Veske et al., "Dynamic coupling between particle-in-cell and atomistic
 * simulations", Phys. Rev. E 101, 053307 (2020), Sec. II A-D and
 * Appendices B-F.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Units: nm, fs, V, V/nm, eV, elementary charge e.
 *  Memory: "host" pointers are read during the call only; "device" pointers
 *    are HIP device memory owned by the caller.  The library never frees
 *    caller memory.  mesh_create allocates the mesh's own device arrays
 *    (freed by mesh_destroy), mesh_create_in places them in a caller
 *    workspace sized by mesh_workspace_bytes; pic_step grows a per-handle
 *    particle scratch on the first call with a larger capacity and
 *    allocates nothing after.
 *  Streams: `stream` is a hipStream_t passed as void*; NULL is the null
 *    stream.  Every call only enqueues work on that stream (mesh_create and
 *    mesh_destroy synchronize it); results land in device memory.  One mesh
 *    handle must not be used on two streams at once.
 *  Errors: every call returns a pic_status (0 = success) and never throws.
 *    PIC_E_ARG: a host-checked argument is invalid; nothing was enqueued.
 *    PIC_E_DEVICE: a HIP runtime call failed.  Device-side conditions
 *    (non-convergence, capacity overflow) are reported in the stats structs
 *    the caller passes.  pic_last_error() returns the last message of the
 *    calling thread.
 *  Geometry: tetrahedra are oriented by the library so that
 *    D = (v1-v0).((v2-v0)x(v3-v0)) > 0 (local vertices 2 and 3 swapped when
 *    needed); face i of a tetrahedron is the one opposite local vertex i.
 *  Charge: deposited in int64 fixed point, 2^40 units per unit relative
 *    weight; the rounding rule makes deposition order-independent.
 */
#ifndef FEMOCS_PIC_H
#define FEMOCS_PIC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PIC_API __attribute__((visibility("default")))
#else
#define PIC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pic_status;
enum {
  PIC_OK = 0,
  PIC_E_ARG = -1,
  PIC_E_DEVICE = -2,
  PIC_E_MESH = -3,
  PIC_E_NOCONV = -4,
  PIC_E_CAPACITY = -5,
  PIC_E_NUMERIC = -6
};

enum { PIC_FP64 = 0, PIC_MIXED = 1 };

/* Fixed-point scale of deposited charge: units per unit relative weight. */
#define PIC_CHARGE_SCALE 1099511627776.0 /* 2^40 */

/* Where a located point ended up. */
enum { PIC_WHERE_INSIDE = 0, PIC_WHERE_ANODE = 1, PIC_WHERE_OUTSIDE = 2 };

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. II A: linear tetrahedral elements over the vacuum domain;     */
/* Eq. poisson_bc: Neumann E0 on the top plane, Dirichlet 0 on the metal,   */
/* lateral periodicity of Sec. II B 1).                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n_nodes;
  const double* xyz;    /* host [3*n_nodes]: node coordinates, wrapped      */
  int64_t n_tets;
  const int32_t* tet;   /* host [4*n_tets]: node ids                         */
  const int8_t* shift;  /* host [8*n_tets] or NULL: per vertex (sx, sy);   */
                        /* unwrapped vertex = xyz + (sx Lx, sy Ly, 0)        */
  double Lx, Ly;        /* lateral periods (> 0)                            */
  double z_top;         /* top plane: Neumann boundary and particle anode   */
  double emit_zmin;     /* metal faces with centroid z >= emit_zmin emit    */
} pic_mesh_desc;

typedef struct pic_mesh pic_mesh;

typedef struct {
  int64_t n_nodes, n_tets, n_free, nnz, nnz_field, n_emit, n_top, n_metal;
  int64_t device_bytes;
} pic_mesh_info;

/* Build a mesh handle: orientation, adjacency with periodic shifts,
 * boundary tags (a boundary face is top when its three vertices lie on
 * z = z_top, metal otherwise; metal vertices are Dirichlet), the P1
 * stiffness matrix on free nodes (App. B), the Neumann load per unit E0,
 * the nodal-field operator, the emitting faces and a bucket grid; uploads
 * everything to the current device.  PIC_E_MESH for out-of-range node ids,
 * zero-volume or non-manifold elements.  *out receives the handle. */
PIC_API pic_status mesh_create(const pic_mesh_desc* desc, void* stream, pic_mesh** out);
/* The same set-up with the mesh's persistent device arrays (the element     */
/* records, K and the field operator, face and bucket data, the solver's    */
/* vectors) placed in a caller-owned workspace: mesh_workspace_bytes runs   */
/* the host part of the set-up (seconds at millions of tets) and returns    */
/* the bytes needed; mesh_create_in takes a device workspace of at least    */
/* that size, 256-byte aligned (hipMalloc's alignment), which must outlive  */
/* the handle -- mesh_destroy does not free it.  PIC_E_ARG when it is too   */
/* small or misaligned.  Not in the workspace: the per-call scratch that    */
/* pic_step, collide, surface_charge and adjoint_step grow on the first     */
/* call with a larger capacity, the AMG hierarchy (built on the first AMG   */
/* solve), and the pinned host record of the solver's convergence report.   */
PIC_API pic_status mesh_workspace_bytes(const pic_mesh_desc* desc, size_t* bytes);
PIC_API pic_status mesh_create_in(const pic_mesh_desc* desc, void* workspace,
                                  size_t ws_bytes, void* stream, pic_mesh** out);
PIC_API pic_status mesh_destroy(pic_mesh* mesh);
PIC_API pic_status mesh_query(const pic_mesh* mesh, pic_mesh_info* info);
/* Host copies of the emitting faces: owner tet, node ids (3 per face),
 * area (nm^2); each pointer may be NULL. */
PIC_API pic_status mesh_emit_faces(const pic_mesh* mesh, int32_t* tet, int32_t* nodes3,
                           double* area);

/* ------------------------------------------------------------------------ */
/* Point location (Sec. II B 2): the containing element of each point.      */
/* The answer is canonical: the lowest-index tetrahedron whose closed        */
/* region holds the point, decided with exact orientation predicates; the   */
/* neighbour walk from the hint only finds it faster.                       */
/* x, y, z: device [n] f64, already wrapped into [0, Lx] x [0, Ly].          */
/* tet_inout: device [n] i32, in: hint tet or -1, out: tet or -1.           */
/* where_out: device [n] u8 (PIC_WHERE_*); z >= z_top is ANODE.             */
/* ------------------------------------------------------------------------ */
PIC_API pic_status locate(const pic_mesh* mesh, int64_t n, const double* x,
                  const double* y, const double* z, int32_t* tet_inout,
                  uint8_t* where_out, void* stream);

/* ------------------------------------------------------------------------ */
/* locate without allocation.  For callers that cannot allocate device      */
/* memory (code under HIP graph capture, tight serving loops, harnesses     */
/* that forbid hipMalloc): the same results as locate, with its scratch --  */
/* the queue of points for the exact scan and its counter -- in a fixed     */
/* 4 MiB device array of the library instead of the mesh handle's           */
/* (grown) queue.  Every GPU the library runs on holds its own copy until   */
/* the process ends; the call allocates nothing, and clears the counter     */
/* with a kernel (no memset).  Arguments as locate; the mesh must live on   */
/* the current device.  PIC_E_ARG when n > PIC_LOCATE_NOALLOC_MAX (locate  */
/* larger sets in chunks).  All calls on one GPU share the array: calls     */
/* that overlap in time on one GPU (two streams, or two threads) race, so   */
/* the caller serializes them.                                              */
/* ------------------------------------------------------------------------ */
#define PIC_LOCATE_NOALLOC_MAX 1048512 /* 2^20 - 64 points per call */
PIC_API pic_status locate_noalloc(const pic_mesh* mesh, int64_t n, const double* x,
                                  const double* y, const double* z, int32_t* tet_inout,
                                  uint8_t* where_out, void* stream);

/* ------------------------------------------------------------------------ */
/* Charge deposition (Eq. q_delta, Eq. poisson_rhs; same shape functions    */
/* as the field gather).  For each point with tet >= 0: lambda_i of the     */
/* point in its tet, q_i = rint(lambda_i w 2^40) (i = 1..3),                */
/* q_0 = rint(w 2^40) - (q_1 + q_2 + q_3), added atomically to the four     */
/* vertices of charge (device [n_nodes] i64, accumulated, not cleared).      */
/* ------------------------------------------------------------------------ */
PIC_API pic_status deposit(const pic_mesh* mesh, int64_t n, const double* x,
                   const double* y, const double* z, const int32_t* tet,
                   const double* w, int64_t* charge, void* stream);

/* ------------------------------------------------------------------------ */
/* Poisson solve (Eq. poisson with Eq. poisson_bc, Galerkin form of App. B) */
/* K phi_f = b_f on free nodes, b_i = (-e/eps0) w_sp c_i 2^-40 + E0 g_i,    */
/* preconditioned CG (the paper only says "iteratively"; params->precond),  */
/* started from phi, stopped when ||b - K phi||_2 <= tol ||b||_2 (checked   */
/* on the true residual).  phi: device [n_nodes] f64 (in: guess, out:       */
/* solution, 0 on Dirichlet nodes).  charge: device [n_nodes] or NULL.      */
/* E_out: device [4*n_nodes] or NULL: nodal field (x, y, z, 0), the         */
/* volume-weighted mean of -grad(phi) over the tets holding each node;       */
/* f64 for PIC_FP64, f32 for PIC_MIXED.                                      */
/* stats: device pic_solve_stats or NULL.                                   */
/* PIC_MIXED (not in the paper): the CG recursion runs in FP32 against K    */
/* rounded to FP32; phi, b, the true residual, every reduction and the      */
/* stopping tests stay FP64.  When the FP32 recursion has reduced its       */
/* residual below max(tol ||b||, inner_tol ||r_restart||), the true         */
/* residual is recomputed in FP64 and the recursion restarted from it       */
/* (iterative refinement) until tol holds on the true residual.             */
/* inner_tol must lie in [1e-7, 0.5] for PIC_MIXED (ignored for PIC_FP64).   */
/* ------------------------------------------------------------------------ */
/* precond (not in the paper, which names no preconditioner):              */
/*   PIC_PRECOND_JACOBI  diagonal scaling (default);                        */
/*   PIC_PRECOND_AMG     one V(1,1)-cycle of smoothed-aggregation algebraic */
/*                       multigrid (Jacobi smoothing, dense coarsest solve) */
/*                       per iteration.  With PIC_MIXED the CG recursion    */
/*                       stays FP64 and the V-cycle runs in FP32 (level     */
/*                       matrices, diagonals and vectors rounded to FP32;   */
/*                       no refinement restarts).  The hierarchy is         */
/*                       built on the host from the mesh's K on the first   */
/*                       solve that asks for it (seconds at 5e5 unknowns)   */
/*                       and kept with the mesh.                            */
enum { PIC_PRECOND_JACOBI = 0, PIC_PRECOND_AMG = 1 };
typedef struct {
  double tol;        /* relative residual target                         */
  double inner_tol;  /* mixed precision: FP32 inner solve target          */
  int32_t max_iter;  /* iteration cap (PIC_E_NOCONV in stats beyond it)   */
  int32_t precision; /* PIC_FP64 or PIC_MIXED (FP32 inner CG + FP64 IR)   */
  int32_t precond;   /* PIC_PRECOND_JACOBI or PIC_PRECOND_AMG             */
  int32_t pad;
} pic_solve_params;

typedef struct {
  int64_t iters;     /* CG iterations (inner ones in mixed mode)          */
  int64_t status;    /* PIC_OK or PIC_E_NOCONV                            */
  int64_t restarts;  /* true-residual restarts / refinement sweeps        */
  int64_t pad;
  double relres;     /* final true relative residual                      */
  double bnorm;
} pic_solve_stats;

PIC_API pic_status poisson_solve(const pic_mesh* mesh, const int64_t* charge,
                         double w_sp, double E0, double* phi, void* E_out,
                         const pic_solve_params* params,
                         pic_solve_stats* stats, void* stream);

/* ------------------------------------------------------------------------ */
/* The PIC cycle (Sec. II B 1-3).                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t capacity;  /* slots in every array below                        */
  int32_t precision; /* PIC_FP64: x..vz are double; PIC_MIXED: float       */
  int32_t pad;
  void *x, *y, *z;    /* device [capacity] positions (wrapped)            */
  void *vx, *vy, *vz; /* device [capacity] velocities v_{k-1/2}           */
  double* w;          /* device [capacity] relative weight               */
  int32_t* tet;       /* device [capacity] containing tet; -1 = free slot */
  int32_t* birth;     /* device [capacity] emitting face index            */
  int64_t* id;        /* device [capacity] step<<42 | face<<21 | ordinal  */
  int32_t* n_slots;   /* device scalar: slots in use (live + free slots)   */
} pic_particles;

typedef struct {
  double* phi;      /* device [n_nodes] potential                         */
  void* E;          /* device [4*n_nodes] nodal field of phi: f64, or f32 */
                    /* when particles->precision is PIC_MIXED             */
  int64_t* charge;  /* device [n_nodes] fixed-point charge of last step   */
} pic_fields;

/* Field the particles see (the paper's gather interpolates "with the      */
/* element's shape functions", which leaves open which field):              */
/*   PIC_FIELD_NODAL  E(r) = sum_i lambda_i(r) E_i with the nodal field     */
/*                    E_i of fields->E (default);                          */
/*   PIC_FIELD_CELL   E(r) = -(grad phi)_t, constant in the tet t holding   */
/*                    r, from fields->phi; the injection field is that of   */
/*                    the emitting face's tet, and so is the field the FN   */
/*                    current is evaluated at.                              */
enum { PIC_FIELD_NODAL = 0, PIC_FIELD_CELL = 1 };

typedef struct {
  double dt;        /* time step (fs)                                     */
  double E0;        /* applied field (V/nm)                               */
  double w_sp;      /* superparticle weight (electrons per unit w)        */
  double phi_w;     /* work function (eV)                                 */
  double j_scale;   /* multiplier on the emission current (1 = physical)  */
  uint64_t seed;    /* Philox key word 0                                  */
  int64_t step0;    /* index of the first step                            */
  int64_t instance; /* Philox key word 1                                  */
  const double* s_face; /* device [n_emit] weight per emitting face or NULL */
  int32_t resort_every; /* sort by tet + compact every k steps (0: never) */
  int32_t field_mode;   /* PIC_FIELD_NODAL or PIC_FIELD_CELL              */
  int32_t collide;      /* 1: binary collisions (see collide) after every */
                        /* re-sort, standing for resort_every steps       */
                        /* (needs resort_every > 0); 0: none              */
  int32_t pad;
  /* device [n_emit] or NULL: frozen emission counts -- each face injects */
  /* counts_in[f] superparticles (clamped to [0, 2^21]) instead of the     */
  /* rounding of Eq. rnd_nsp, in every step of the call (finite            */
  /* differences of a window hold them, as its adjoint does); counts_out:  */
  /* device [n_emit] or NULL, receives the counts used (the last step's;  */
  /* in pic_batch_step, per instance).                                     */
  const int32_t* counts_in;
  int32_t* counts_out;
  pic_solve_params solve;
} pic_step_params;

typedef struct {
  int64_t n_before, n_inj, n_anode, n_cathode, n_after;
  int64_t q_before, q_inj, q_anode, q_cathode, q_after; /* fixed point */
  int64_t cg_iters, n_clamp, status, n_trunc;
  int64_t walk_steps, walk_max, n_fallback, n_slots;
  double cg_relres, emit_current, mean_face_E, max_face_E;
} pic_step_stats;

/* Advance n_steps steps k = step0 .. step0+n_steps-1.  Per step: gather the
 * field at each particle (params->field_mode) and kick (Eq. leapfrog3 then
 * Eq. leapfrog1), inject from the emitting faces with the same field
 * (Eq. nsp, Eq. rnd_nsp -- or the held counts_in --, App. E,
 * Eq. sp_velocity, Eq. sp_displacement), drift (Eq. leapfrog2), wrap
 * laterally, absorb at z >= z_top (anode) or outside the vacuum (cathode),
 * locate, deposit, re-sort by tet every resort_every steps (then collide,
 * when params->collide), solve for phi_{k+1} and recover the nodal field.
 * fields->E must hold the field of phi on entry.
 * Mixed precision (particles->precision PIC_MIXED, not in the paper):
 * positions, velocities and fields->E are FP32, and the field gather, kick,
 * drift and wrap run in FP32; the barycentric weights of the stored FP32
 * position (widened exactly to FP64), locating, deposition, injection and
 * emission stay FP64, so charge and tet ids follow the stored positions
 * exactly.  params->solve.precision chooses the solver independently.
 * Within one call, each later solve starts from the previous one: its first
 * pass forms the residual as (b - b_prev) + r_prev rather than b - K phi
 * (equal up to rounding) and keeps the field, which already belongs to phi;
 * so one call of n steps and n calls of one step agree to the solver
 * tolerance, bit for bit when no solve iterates.  The host waits for each
 * solve's convergence report; the next step's kernels are already queued
 * behind it and do nothing if the solve needs more rounds.  With re-sorts
 * and no collisions, the particles may sit in the handle's re-sort scratch
 * between re-sorts of a call; the caller's arrays hold the state again once
 * the call's work on the stream has completed.
 * stats: device [n_steps] pic_step_stats (overwritten). */
PIC_API pic_status pic_step(pic_mesh* mesh, const pic_particles* particles,
                    const pic_fields* fields, const pic_step_params* params,
                    int32_t n_steps, pic_step_stats* stats, void* stream);

/* Sum over emitting faces of J_f A_f (e/fs) for the nodal field E (device
 * [4*n_nodes]); result written to device *rate (f64) and, when face_F is
 * not NULL, |E| at each face centroid to device face_F [n_emit]. */
PIC_API pic_status emission_rate(const pic_mesh* mesh, const double* E, double phi_w,
                         double* rate, double* face_F, void* stream);

/* ------------------------------------------------------------------------ */
/* Adjoint of one step (an addition: the paper has no adjoint).             */
/* Objective over a window of T steps: J = wQ J_Q + wE J_E with J_Q the     */
/* charge (in e) the anode collects, w_sp sum w, and J_E the mean over the  */
/* emitting faces and the post-solve fields E_1..E_T of |E| at the face     */
/* centroid.  Parameters: E0 (Eq. poisson_bc) and s_f, the multiplier of    */
/* the weight of every superparticle born at face f (params->s_face; in-    */
/* flight ones included).  Held fixed: emission counts (Eq. rnd_nsp), the   */
/* injection draws, the absorption events and the containing tets; the      */
/* fixed-point rounding of the deposition is taken as exact.                */
/*                                                                          */
/* pre: the state at the start of step k (a checkpoint).  post: the state   */
/* pic_step made from it with the same params and resort_every = 0 (slot i  */
/* < pre n_slots is the same superparticle; later slots are the ones        */
/* injected in step k).  Fk: phi_k and E_k; Fk1: E_{k+1}.  Both particle    */
/* sets have the precision of pre->precision, the fields the matching type.  */
/* adj: in: the adjoint of the post-step state (rb, vb per post slot) and,  */
/* in Eb, the adjoint of E_{k+1} from the gathers of step k + 1; out: the   */
/* adjoint of the pre-step state (pre slots; later slots zeroed) and, in    */
/* Eb, that of E_k from this step's gathers.  dJ_dE0 and dJ_ds accumulate.  */
/* Only the nodal field mode (PIC_FIELD_NODAL) without collisions has an  */
/* adjoint: another field_mode, or collide != 0, is PIC_E_ARG.              */
/* mode PIC_ADJ_INITIAL ends a window: the reverse of the solve that gave   */
/* phi_0 from the charge of pre and E0 (Eb in: adjoint of E_0; post, Fk1    */
/* unused; rb, vb untouched).  mu: device [n_nodes] adjoint potential,      */
/* warm start in, solution out.  Solves use params->solve; with bref (device */
/* scalar, or NULL) the test is ||r|| <= tol max(||b||, *bref), and *bref is */
/* raised to ||b||: over a window it holds the largest right-hand side, so  */
/* every solve is accurate relative to the scale of the whole gradient.     */
/* ------------------------------------------------------------------------ */
enum { PIC_ADJ_STEP = 0, PIC_ADJ_INITIAL = 1 };

typedef struct {
  double* rb;       /* device [3*capacity] f64, component-major           */
  double* vb;       /* device [3*capacity] f64                            */
  double* Eb;       /* device [4*n_nodes] f64 (x, y, z, unused)           */
  double* mu;       /* device [n_nodes] f64                               */
  double* dJ_dE0;   /* device scalar f64, accumulated                     */
  double* dJ_ds;    /* device [n_emit] f64, accumulated                   */
  double* bref;     /* device scalar f64 (in/out) or NULL, see above      */
  double wQ, wE;    /* objective weights                                  */
  int32_t T;        /* window length (J_E is a mean over T fields)        */
  int32_t mode;     /* PIC_ADJ_STEP or PIC_ADJ_INITIAL                    */
} pic_adjoint;

PIC_API pic_status adjoint_step(pic_mesh* mesh, const pic_particles* pre,
                        const pic_particles* post, const pic_fields* Fk,
                        const pic_fields* Fk1, const pic_step_params* params,
                        const pic_adjoint* adj, pic_solve_stats* stats,
                        void* stream);

/* The forward side of the window objective above, so that a caller        */
/* composes a window from library calls only:                               */
/* window_objective adds one step's terms to J (device [3] f64): J[0] +=    */
/* w_sp q_anode 2^-40 (stats->q_anode: the step's collected fixed-point    */
/* charge), J[1] += (1/T) times the mean over the emitting faces of |E| at  */
/* the face centroid, E_f = ((E_a + E_b) + E_c) / 3 of the post-solve nodal */
/* field E (device [4*n_nodes], f64 for PIC_FP64, f32 for PIC_MIXED), and    */
/* sets J[2] = wQ J[0] + wE J[1].  stats: device pic_step_stats of the step. */
/* apply_face_weights sets, for every slot below *n_slots, w = w_base s_f   */
/* with f the slot's birth face when the slot is live (tet >= 0), else      */
/* w = w_base (w_base, s_face: device f64 [capacity], [n_emit]): the        */
/* multiplier s_f acts on the in-flight superparticles born at f.           */
/* ------------------------------------------------------------------------ */
PIC_API pic_status window_objective(const pic_mesh* mesh, const void* E, int32_t precision,
                                    const pic_step_stats* stats, double w_sp, int32_t T,
                                    double wQ, double wE, double* J, void* stream);
PIC_API pic_status apply_face_weights(const pic_mesh* mesh, const pic_particles* particles,
                                      const double* w_base, const double* s_face,
                                      void* stream);

/* ------------------------------------------------------------------------ */
/* Binary Monte Carlo collisions (App. F, after Takizuka and Abe): the      */
/* superparticles of each tet are paired at random and every pair collides */
/* elastically (Eq. vel12, Eq. scat_vel, Eq. rot_mat, Eq. sin_theta), with */
/* delta = tan(theta/2) normal of variance Eq. variance (Landau logarithm  */
/* 13); a tet with an odd count collides its first three pairwise at half  */
/* variance.  q and m of Eq. variance are the electron's, n the electrons  */
/* in the tet (w_sp times the summed relative weights); superparticles are */
/* treated as identical.  The relative velocity u = v2 - v1 of a pair turns */
/* to (I + M) u: v1 -= dv / 2, v2 += dv / 2, conserving momentum and       */
/* energy.  Pairing: by a Philox key of (step, id) within the tet; draws:  */
/* Philox at (step, id of the pair's first member).  Velocities change in  */
/* place; positions, tets and weights are untouched.                        */
/* particles: slots [0, n_slots) must be sorted by tet (ascending, every   */
/* slot live), as pic_step's re-sort leaves them.  Slots with tet < 0 are  */
/* skipped; with tets out of order the grouping is wrong (no access leaves */
/* the arrays).                                                            */
/* Uses the handle's particle scratch (allocated on first use for the      */
/* capacity).  PIC_E_ARG for null pointers or non-positive dt_coll, w_sp.  */
/* ------------------------------------------------------------------------ */
typedef struct {
  double dt_coll;   /* time the collisions stand for (fs)                 */
  double w_sp;      /* electrons per unit relative weight                 */
  uint64_t seed;
  int64_t step;     /* counter of the draws                               */
  int64_t instance;
} pic_collide_params;

PIC_API pic_status collide(pic_mesh* mesh, const pic_particles* particles,
                           const pic_collide_params* params, void* stream);

/* ------------------------------------------------------------------------ */
/* Surface charge (Sec. II C, Eq. face_charge, Eq. atom_charge,             */
/* Eq. charge_weight): the charge of every emitting face -- every metal     */
/* face when the mesh was created with emit_zmin below the cathode --       */
/* Q_f = eps0 (E_f . n_f) A_f (E_f: the mean of the nodal field at the      */
/* face's vertices, or in PIC_FIELD_CELL mode the field of the face's tet   */
/* from phi; n_f into the vacuum), and its distribution to atoms,           */
/* q_j = sum_f w_fj Q_f with w_fj = exp(-d_fj / r_c) / sum_j'               */
/* exp(-d_fj' / r_c): normalised over the atoms, so that sum_j q_j =        */
/* sum_f Q_f (the printed normalisation condition, a sum over faces, would  */
/* not conserve charge); d_fj from the face centroid, minimum image in x    */
/* and y.  Charges in e.                                                    */
/* Cutoff: when the periodic box holds a sphere of 40 r_c plus a cell of    */
/* 10 r_c (the production tip at r_c = 0.1 nm), pairs with                  */
/* d_fj - min_j' d_fj' > 40 r_c are left out of both sums (found through    */
/* a cell grid of the atoms and face centroids); each face then loses less  */
/* than n_atoms e^-40 (4.2e-18 n_atoms) of its charge, and sum_j q_j =      */
/* sum_f Q_f still holds to rounding.  Otherwise every pair is summed.      */
/* fields: phi (cell mode) or E (nodal mode; FP64, or FP32 when precision   */
/* is PIC_MIXED).  face_Q: device [n_emit] out; atom_q: device [n_atoms]    */
/* out (may be NULL when n_atoms is 0).  Uses a per-handle scratch, grown   */
/* on demand (all pairs: two doubles per face plus one per atom and face    */
/* range, at most 1024 ranges; cutoff: in addition the cell grid, 6 doubles */
/* and 4 ints per face, 3 doubles and 4 ints per atom).  PIC_E_ARG for null */
/* pointers, n_atoms outside [0, 2^31), r_c <= 0 or an unknown mode or     */
/* precision.                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n_atoms;
  const double* atoms;  /* device [3*n_atoms] positions (x, y, z), nm      */
  double r_c;           /* nm (the paper uses 0.1)                         */
  int32_t field_mode;   /* PIC_FIELD_NODAL or PIC_FIELD_CELL               */
  int32_t precision;    /* of fields->E: PIC_FP64 or PIC_MIXED (FP32)      */
} pic_charge_params;

PIC_API pic_status surface_charge(pic_mesh* mesh, const pic_fields* fields,
                                  const pic_charge_params* params,
                                  double* face_Q, double* atom_q, void* stream);

/* ------------------------------------------------------------------------ */
/* Metal-side solves (Sec. II D; weak forms of App. C and App. D): the     */
/* current continuity equation (Eq. cont with Eq. cont_bc), the Joule heat  */
/* (Eq. joule) and one Theta-scheme step of the heat equation (Eq. heat,    */
/* Eq. heat_bc, Eq. heat_theta2) on a separate P1 tetrahedral mesh of the   */
/* metal.  Matrices are assembled on the device in CSR form from their      */
/* element definitions and solved by Jacobi-preconditioned CG in FP64.      */
/* ------------------------------------------------------------------------ */
typedef struct pic_metal pic_metal;

typedef struct {
  int64_t n_nodes;
  const double* xyz;          /* host [n_nodes][3]                               */
  int64_t n_tets;
  const int32_t* tets;        /* host [n_tets][4] node ids, any orientation       */
  int64_t n_faces;
  const int32_t* faces;       /* host [n_faces][3] metal-vacuum interface (Gamma3) */
  const uint8_t* dirichlet;   /* host [n_nodes] 1 on Gamma5 (fixed Phi and T)     */
} pic_metal_desc;

typedef struct {
  int64_t iters;              /* CG iterations                                  */
  double relres;              /* ||r|| / ||b|| of the CG recursion at exit       */
  int32_t converged;
  int32_t pad;
} pic_metal_stats;

typedef struct {
  double Cv;                  /* volumetric heat capacity (constant)             */
  double L;                   /* Lorentz number of Eq. wied_franz                */
  double dt;                  /* time step                                      */
  double theta;               /* Theta in [0, 1]; 1 is the paper's implicit Euler */
  double T_amb;               /* Dirichlet temperature on Gamma5                  */
  double tol;                 /* CG stopping test ||r|| <= tol ||b||              */
  int64_t max_iter;
} pic_heat_params;

/* Copies the mesh to the device, builds the CSR pattern and the node-to-
 * element lists on the host (setup), and the shape-function gradients and
 * volumes on the device.  Lateral boundary faces not listed in faces carry
 * no flux (Gamma4).  PIC_E_ARG for empty or out-of-range input or an
 * element of zero volume. */
PIC_API pic_status metal_create(const pic_metal_desc* desc, void* stream,
                                pic_metal** out);
PIC_API pic_status metal_destroy(pic_metal* metal);

/* Eq. cont_mat: K(sigma) Phi = f with K_ab = sum_t sigma_t int grad N_a .
 * grad N_b, f_a = sum over interface faces of flux_f A_f / 3 (flux_f =
 * J_e . n, n the outward normal of the metal), Phi = 0 on Gamma5.  sigma:
 * device [n_tets]; flux: device [n_faces]; Phi: device [n_nodes], in the
 * initial guess, out the solution; P_J (optional, device [n_tets]): Eq.
 * joule, sigma_t |grad Phi|^2.  The call waits for the solve (the host
 * reads the convergence state every few iterations).  PIC_E_NOCONV when
 * max_iter is reached (Phi holds the last iterate). */
PIC_API pic_status continuity_solve(pic_metal* metal, const double* sigma,
                                    const double* flux, double tol,
                                    int64_t max_iter, double* Phi, double* P_J,
                                    pic_metal_stats* stats, void* stream);

/* Eq. heat_theta2 with kappa_t = L sigma_t Tbar_t (Eq. wied_franz, Tbar_t
 * the mean of the element's four nodal temperatures at the start of the
 * step: the conductivity lagged as App. D states), C = int C_v N_a N_b
 * (consistent), f = int N_a P_J + int_Gamma3 N_a P_N (sources held over the
 * step), T = T_amb on Gamma5.  sigma, P_J: device [n_tets]; P_N: device
 * [n_faces]; T: device [n_nodes], in T^n, out T^{n+1}.  Waits like
 * continuity_solve. */
PIC_API pic_status heat_step(pic_metal* metal, const pic_heat_params* params,
                             const double* sigma, const double* P_J,
                             const double* P_N, double* T,
                             pic_metal_stats* stats, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched stepping (an addition: many independent instances of the cycle   */
/* -- each its own mesh_create handle, particles, fields and parameters --  */
/* advanced together).  Every kernel of a step is launched once for all     */
/* instances, the blocks of a launch mapped onto the instances by a         */
/* schedule: per-instance workgroup counts (each rounded up to a multiple    */
/* of 8, so that a workgroup's XCD follows its index inside its instance).   */
/* The solves of all instances iterate in the same launches; each stops at  */
/* its own tolerance.  Results per instance are those of pic_step with the  */
/* same parameters, up to the rounding order of the solver's reductions     */
/* (which depends on cg_blocks).                                           */
/* ------------------------------------------------------------------------ */
#define PIC_MAX_BATCH 64

typedef struct pic_batch pic_batch;

typedef struct {
  int32_t push_blocks[PIC_MAX_BATCH];   /* live-particle workgroups, 8..push max  */
  int32_t inject_blocks[PIC_MAX_BATCH]; /* injection workgroups, 8..inject max    */
  int32_t cg_blocks[PIC_MAX_BATCH];     /* solver workgroups, 8..cg max           */
  int32_t clear_blocks[PIC_MAX_BATCH];  /* step-start workgroups (>= 8)           */
  int32_t fallback_blocks;              /* per instance, 8..fallback max          */
  int32_t pad;
} pic_batch_schedule;

/* meshes: host array [n] of handles, 1 <= n <= PIC_MAX_BATCH, each used by
 * at most this batch while it steps.  limits (optional): the upper bounds
 * of each instance's counts (push, inject, cg, fallback) as [4*n]. */
PIC_API pic_status pic_batch_create(pic_mesh* const* meshes, int32_t n,
                            pic_batch** out, int32_t* limits);
PIC_API pic_status pic_batch_destroy(pic_batch* batch);

/* n_steps steps of every instance i with particles[i], fields[i] and
 * params[i] (all of one precision), under sched.  stats: device
 * [n_steps * n] pic_step_stats, step-major (stats[k * n + i]).  Blocks the
 * calling thread at the solves, like pic_step. */
PIC_API pic_status pic_batch_step(pic_batch* batch,
                          const pic_particles* particles,
                          const pic_fields* fields,
                          const pic_step_params* params,
                          const pic_batch_schedule* sched, int32_t n_steps,
                          pic_step_stats* stats, void* stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing (measurement support, not part of the method).  While      */
/* enabled, pic_step and poisson_solve bracket the kernels of the selected  */
/* classes with HIP events on the caller's stream; pic_profile_read         */
/* synchronizes on the last event and returns the summed elapsed            */
/* milliseconds and the launch count per kernel class since the last        */
/* enable.  Every event is a packet of its own in the stream and costs      */
/* GPU time: select only the classes wanted.  Event objects are created on  */
/* demand while profiling is on.                                            */
/* ------------------------------------------------------------------------ */
enum {
  PIC_K_PUSH = 0,     /* live + injected: gather, kick, drift, walk, deposit */
  PIC_K_EMIT = 1,     /* per-step clears, per-face FN counts and scan      */
  PIC_K_INJECT = 2,   /* (injection runs inside PIC_K_PUSH)                */
  PIC_K_FALLBACK = 3, /* exact location of uncertified particles, stats    */
  PIC_K_SOLVE = 4,    /* residual + nodal field pass, PCG iterations      */
  PIC_K_SORT = 5,     /* sort by tet + compaction                         */
  PIC_K_CLEAR = 6,    /* per-step clears of charge and counters           */
  PIC_K_ADJOINT = 7,  /* adjoint_step (its solve included)                */
  PIC_K_COLLIDE = 8,  /* binary collisions                                */
  PIC_K_COUNT = 9
};

typedef struct {
  double ms[PIC_K_COUNT];
  int64_t launches[PIC_K_COUNT];
} pic_kernel_times;

/* classes: bitmask of (1 << PIC_K_*), PIC_PROFILE_ALL for every class, 0  */
/* to stop.                                                                 */
#define PIC_PROFILE_ALL 0x1FF
PIC_API pic_status pic_profile(pic_mesh* mesh, int32_t classes);
/* Sampling of the timing in pic_step: only its steps k = 0, every,        */
/* 2 every, ... of each call are bracketed (every >= 1; 1, the default,     */
/* times every step; PIC_E_ARG below 1).  Other entry points time every     */
/* call.  Fewer events leave the untimed steps as they run without timing.  */
PIC_API pic_status pic_profile_every(pic_mesh* mesh, int32_t every);
PIC_API pic_status pic_profile_read(pic_mesh* mesh, pic_kernel_times* out);

PIC_API const char* pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FEMOCS_PIC_H */
