/*
 * FP64 CPU oracle of the electron particle-in-cell cycle (Veske et al.,
 * "Dynamic coupling between particle-in-cell and atomistic simulations",
 * Phys. Rev. E 101, 053307 (2020), Sec. II B-C and Appendices A, B, E).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library
 * against a plain, slow, obviously correct reading of the paper.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.  It shares no code with the HIP library.
 *
 * Conventions (both sides follow them, each in its own code):
 *   units nm, fs, V, V/nm, eV, elementary charge e;
 *   tetrahedra oriented so that D = (v1-v0).((v2-v0)x(v3-v0)) > 0
 *   (negative ones get local vertices 2 and 3 swapped);
 *   face i of a tetrahedron is the one opposite local vertex i, its vertices
 *   taken in ascending local order;
 *   charge is deposited in int64 fixed point, 2^40 units per unit weight.
 *
 * Parity unpinned: om_fn_current() follows the Murphy-Good form with Forbes'
 * approximation for the barrier functions; the paper takes its emission
 * current from an external tool (GETELEC) whose output is not available, so
 * only the formula itself is pinned.
 */
#ifndef FEMOCS_ORACLE_H
#define FEMOCS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct omesh omesh;

/* Build the mesh: orientation, geometry, adjacency, boundary tags,
 * stiffness matrix on free nodes, Neumann load, emitting faces, bucket grid.
 * Returns NULL on error (message in err). */
omesh* om_create(int64_t n_nodes, const double* xyz, int64_t n_tets,
                 const int32_t* tet, const int8_t* shift, double Lx, double Ly,
                 double z_top, double emit_zmin, char* err, int errlen);
void om_destroy(omesh* m);

enum {
  OM_N_NODES = 0, OM_N_TETS, OM_N_FREE, OM_NNZ, OM_N_EMIT, OM_N_TOP,
  OM_N_METAL, OM_N_FLIPPED
};
int64_t om_info(const omesh* m, int what);

/* Copies of derived arrays (for pins). */
void om_get_tets(const omesh* m, int32_t* tet4, double* vert12, double* mmat9,
                 double* D, int32_t* nbr4, int8_t* nbr_shift8);
void om_get_csr(const omesh* m, int64_t* rowptr, int32_t* col, double* val);
void om_get_free(const omesh* m, int32_t* free_id, double* g_unit);
void om_get_emit(const omesh* m, int32_t* tet, int32_t* local, double* area,
                 double* normal3, double* abc9, int32_t* nodes3);

/* Exact sign of vol6(a,b,c,d) = (b-a).((c-a)x(d-a)): -1, 0 or +1. */
int om_orient_sign(const double* a, const double* b, const double* c,
                   const double* d);
/* Barycentric coordinates of p in tetrahedron t (the fixed arithmetic). */
void om_lambda(const omesh* m, int32_t t, const double* p, double* lam4);

/* Canonical location: lowest-index tetrahedron whose closed region holds
 * p; where = 1 (anode) when z >= z_top, 2 when no tetrahedron holds p. */
void om_locate(const omesh* m, int64_t n, const double* x, const double* y,
               const double* z, const int32_t* hint, int32_t* tet_out,
               uint8_t* where_out);

/* Fixed-point deposition (adds into c, int64 per node). */
void om_deposit(const omesh* m, int64_t n, const double* x, const double* y,
                const double* z, const int32_t* tet, const double* w,
                int64_t* c);

/* Jacobi-PCG Poisson solve; phi holds all nodes (Dirichlet ones are 0).
 * Returns 0, or -4 on non-convergence. */
int om_poisson_solve(const omesh* m, const int64_t* c, double w_sp, double E0,
                     double* phi, double tol, int max_iter, int* iters,
                     double* relres);
void om_rhs(const omesh* m, const int64_t* c, double w_sp, double E0,
            double* b);
void om_spmv(const omesh* m, const double* x, double* y);

/* Nodal field: volume-weighted mean of -grad(phi) over incident tets. */
void om_field(const omesh* m, const double* phi, double* E3);

/* Transpose of om_field: phibar[j] = sum_i sum_k R_(i k),j Ebar3[3 i + k]
 * over all nodes j (the derivative of <Ebar, E(phi)> with respect to
 * phi_j).  Test infrastructure for the adjoint. */
void om_field_adj(const omesh* m, const double* Ebar3, double* phibar);

/* Murphy-Good Fowler-Nordheim current density in A/m^2 (F in V/nm, phi_w
 * in eV).  *clamped is set when the Schottky parameter had to be clamped. */
double om_fn_current(double F, double phi_w, int* clamped);
void om_constants(double* out8);

void om_philox4x64(uint64_t k0, uint64_t k1, const uint64_t* ctr,
                   uint64_t* out4);

/* Threads of the parallel loops: 1 in the plain build; in the -fopenmp
 * timing build, OpenMP's thread count. */
int om_threads(void);

typedef struct {
  int64_t cap, n;
  double *x, *y, *z, *vx, *vy, *vz, *w;
  int32_t *tet, *birth;
  int64_t *id;
} oparticles;

typedef struct {
  double dt, E0, w_sp, phi_w, j_scale, tol;
  uint64_t seed;
  int64_t step;
  int64_t instance;
  int32_t max_iter;
  int32_t field_mode;   /* 0 nodal field, 1 cell field (reading R2) */
  const double* s_face; /* per emitting face weight multiplier or NULL */
  /* frozen emission counts per emitting face (replace Eq. nsp and
   * Eq. rnd_nsp) or NULL; the counts used are written to counts_out */
  const int64_t* counts_in;
  int64_t* counts_out;
  /* per particle of the step, in the order of the pre-step particles then
   * the injected ones: fate (0 kept, 1 anode, 2 cathode) and, for the
   * injected ones (index - n_before), (R1, R2, R, face) */
  int8_t* fate_out;
  double* inj_out;
  /* the potential phi_k (cell field mode: the field of tet t is
   * -(grad phi_k)_t); om_pic_step sets it to its own phi */
  const double* phi;
  /* > 0: binary collisions (om_collide) at the end of every step k with
   * (k + 1) % collide_every == 0, standing for collide_every steps */
  int32_t collide_every;
  int32_t pad_c;
} ostep_params;

typedef struct {
  int64_t n_before, n_inj, n_anode, n_cathode, n_after;
  int64_t q_before, q_inj, q_anode, q_cathode, q_after;
  int64_t cg_iters, n_clamp, status, n_trunc;
  double cg_relres, emit_current, mean_face_E, max_face_E;
} ostep_stats;

int om_inject(const omesh* m, oparticles* P, const double* E3,
              const ostep_params* prm, ostep_stats* st, double* face_pts,
              int64_t* counts);

/* Binary Monte Carlo collisions of the superparticles of each tet (App. F
 * after Takizuka and Abe: group by cell, random pairing, Eq. vel12,
 * Eq. scat_vel, Eq. rot_mat, Eq. sin_theta, Eq. variance with Lambda = 13,
 * the odd-count rule).  Readings: delta is tan(theta/2) (the half-angle
 * forms of Eq. sin_theta); the pair's relative velocity u = v2 - v1 turns
 * to (I + M) u, i.e. v1 -= Delta v / 2 and v2 += Delta v / 2 (the signs
 * that conserve energy); q and m of Eq. variance are the electron's and n
 * is the number of electrons in the cell, w_sp times the sum of the
 * relative weights (superparticles are treated as identical).  Pairing:
 * the cell's superparticles ordered by a Philox key of (step, id), then
 * paired in that order; the draws of a collision are keyed by the id of
 * the pair's first member. */
typedef struct {
  double dt_coll;   /* time the collisions stand for (fs) */
  double w_sp;      /* electrons per unit relative weight */
  uint64_t seed;
  int64_t step;
  int64_t instance;
} ocollide_params;

void om_collide(const omesh* m, oparticles* P, const ocollide_params* prm);

/* Face charge (Eq. face_charge) on the emitting faces (every metal face
 * when emit_zmin lies below the cathode) and its distribution to atoms
 * (Eq. atom_charge, Eq. charge_weight).  Q_f = eps0 (E_f . n_f) A_f, E_f the
 * face field (field_mode 0: mean of the nodal field E3 at the face's
 * vertices; 1: the cell field of the face's tet from phi), n_f the normal
 * into the vacuum.  w_fj = exp(-d_fj / r_c) / sum_j' exp(-d_fj' / r_c),
 * normalised over the atoms so that sum_j q_j = sum_f Q_f (reading of
 * Eq. charge_cons), d_fj the distance from the face centroid to atom j,
 * minimum image in x and y; evaluated as exp(-(d_fj - d_f,min) / r_c) over
 * the same sum (an identity that keeps the terms representable).
 * faceQ [n_emit], atomq [n_atoms] (out). */
void om_surface_charge(const omesh* m, const double* E3, const double* phi,
                       int field_mode, int64_t n_atoms, const double* atoms,
                       double r_c, double* faceQ, double* atomq);

/* One step k -> k+1: kick with E_k, inject with E_k, drift, wrap, absorb,
 * locate, deposit, solve for phi_{k+1}, recover E_{k+1}.
 * E3 (in: E_k, out: E_{k+1}), phi (in: guess, out: phi_{k+1}), c (out). */
int om_pic_step(const omesh* m, oparticles* p, double* phi, double* E3,
                int64_t* c, const ostep_params* prm, ostep_stats* st);

/* Emission bookkeeping at a given field (for the weight rule): total
 * current sum_f J_f A_f in e/fs, per-face |E| at centroids. */
double om_emission_rate(const omesh* m, const double* E3, double phi_w,
                        double* faceF);
/* The same with phi non-null: the cell field mode (each face at the field
 * of its vacuum tet). */
double om_emission_rate_mode(const omesh* m, const double* E3,
                             const double* phi, double phi_w, double* faceF);

/* Cell field of every tet (reading R2, cell variant): E3t [T][3] =
 * -(grad phi)_t. */
void om_cell_field(const omesh* m, const double* phi, double* E3t);

#ifdef __cplusplus
}
#endif
#endif
