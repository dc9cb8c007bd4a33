/*
 * FP64 CPU oracle of the electron PIC cycle -- TEST INFRASTRUCTURE ONLY.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP library.
 *
 * Every function names the passage of Veske et al., Phys. Rev. E 101, 053307
 * (2020) it follows ("Sec." = section of the paper, "App." = appendix,
 * "Eq. name" = the equation label).  Readings where the paper is silent are
 * stated at the function.  Compile with -O2 -ffp-contract=off (no FMA
 * contraction, no fast-math): the barycentric and deposition arithmetic is
 * specified operation by operation and must not be re-associated.
 *
 * Parity unpinned: om_fn_current (see the header).
 *
 * Built twice: the plain build (the checker of the tests) and, with
 * -fopenmp, the timing build of the benchmark's CPU baseline.  The OpenMP
 * pragmas sit only on loops whose iterations are independent or add
 * integers (deposition), so both builds give bit-identical results.
 */
#include "femocs_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads of the parallel loops: 1 in the plain build */
int om_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Physical constants, derived from CODATA 2018 base values.                 */
/* ------------------------------------------------------------------------ */
static const double E_CHARGE = 1.602176634e-19;  /* C (exact)   */
static const double H_PLANCK = 6.62607015e-34;   /* J s (exact) */
static const double M_ELEC = 9.1093837015e-31;   /* kg          */
static const double EPS_0 = 8.8541878128e-12;    /* F/m         */
static const double PI_ = 3.14159265358979323846;

typedef struct {
  double qm;      /* q/m of an electron, nm fs^-2 per V/nm           */
  double e_eps;   /* e / eps0 in V nm per elementary charge         */
  double a_fn;    /* first FN constant, A eV V^-2                   */
  double b_fn;    /* second FN constant, eV^-3/2 V nm^-1            */
  double c_s;     /* Schottky constant e^3/(4 pi eps0), eV^2 V^-1 nm */
  double j_unit;  /* A/m^2 -> e nm^-2 fs^-1                          */
} consts_t;

static consts_t constants(void) {
  consts_t c;
  /* a = (-e/m) [C/kg = m s^-2 per V/m]; 1 V/nm = 1e9 V/m, 1 m s^-2 = 1e-21 nm fs^-2 */
  c.qm = -(E_CHARGE / M_ELEC) * 1e9 * 1e-21;
  /* e/eps0 in V m, times 1e9 for V nm */
  c.e_eps = (E_CHARGE / EPS_0) * 1e9;
  /* a_FN = e^3/(8 pi h) expressed with the work function in eV: e^2/(8 pi h) */
  c.a_fn = E_CHARGE * E_CHARGE / (8.0 * PI_ * H_PLANCK);
  /* b_FN = (8 pi/3) sqrt(2 m) / (e h) with phi in eV (x e^{3/2}) and F in V/nm (/1e9) */
  c.b_fn = (8.0 * PI_ / 3.0) * sqrt(2.0 * M_ELEC) / (E_CHARGE * H_PLANCK) *
           pow(E_CHARGE, 1.5) / 1e9;
  /* f = e^3 F / (4 pi eps0 phi^2) with phi in eV: e F/(4 pi eps0) [V m] -> V nm */
  c.c_s = E_CHARGE / (4.0 * PI_ * EPS_0) * 1e9;
  /* 1 A/m^2 = (1/e) e s^-1 m^-2 = (1/e) 1e-15 fs^-1 1e-18 nm^-2 */
  c.j_unit = 1.0 / E_CHARGE * 1e-33;
  return c;
}

void om_constants(double* out8) {
  consts_t c = constants();
  out8[0] = c.qm;
  out8[1] = c.e_eps;
  out8[2] = c.a_fn;
  out8[3] = c.b_fn;
  out8[4] = c.c_s;
  out8[5] = c.j_unit;
  out8[6] = 0x1p40;
  out8[7] = 0.0;
}

/* Murphy-Good FN current density (Sec. II B 3 takes J_e from GETELEC; this
 * closed form stands in for it).  J = a F^2/(phi t(f)^2) exp(-v(f) b phi^1.5/F),
 * f = c_s F/phi^2, v = 1 - f + (f/6) ln f, t = 1 + f/9 - (f/18) ln f. */
double om_fn_current(double F, double phi, int* clamped) {
  consts_t c = constants();
  if (!(F > 1e-3)) return 0.0;
  double f = c.c_s * F / (phi * phi);
  if (f >= 1.0) {
    f = 1.0 - 1e-9;
    if (clamped) *clamped = 1;
  }
  double lf = log(f);
  double v = 1.0 - f + (f / 6.0) * lf;
  double t = 1.0 + f / 9.0 - (f / 18.0) * lf;
  double Fsi = F * 1e9;
  return c.a_fn * Fsi * Fsi / (phi * t * t) *
         exp(-v * c.b_fn * (phi * sqrt(phi)) / F);
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based RNG.    */
/* ------------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void om_philox4x64(uint64_t k0, uint64_t k1, const uint64_t* ctr,
                   uint64_t* out4) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul128(M0, c0, &hi0, &lo0);
    mul128(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out4[0] = c0;
  out4[1] = c1;
  out4[2] = c2;
  out4[3] = c3;
}

static double u01(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

/* ------------------------------------------------------------------------ */
/* Exact orientation sign (point location, Sec. II B 2): the sign of the    */
/* 4x4 determinant |1 a; 1 b; 1 c; 1 d| = (b-a).((c-a)x(d-a)), by the       */
/* Leibniz formula with error-free products and expansion sums (Shewchuk,   */
/* "Adaptive precision floating-point arithmetic", 1997).  A floating-point */
/* filter with Shewchuk's static bound answers first when it can.           */
/* ------------------------------------------------------------------------ */
static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  *s = x;
  *e = (a - av) + (b - bv);
}

static void two_prod(double a, double b, double* p, double* e) {
  double x = a * b;
  *p = x;
  *e = fma(a, b, -x);
}

/* h <- e + b (exact), e nonoverlapping increasing; zero components dropped */
static int grow_expansion(int elen, const double* e, double b, double* h) {
  double q = b;
  int hl = 0;
  for (int i = 0; i < elen; ++i) {
    double s, err;
    two_sum(q, e[i], &s, &err);
    q = s;
    if (err != 0.0) h[hl++] = err;
  }
  if (q != 0.0 || hl == 0) h[hl++] = q;
  return hl;
}

static int exact_det4_sign(const double* a, const double* b, const double* c,
                           const double* d) {
  const double* P[4] = {a, b, c, d};
  static int perm_init = 0;
  static int perm[24][4];
  static int psign[24];
  if (!perm_init) {
    int k = 0;
    for (int s0 = 0; s0 < 4; ++s0)
      for (int s1 = 0; s1 < 4; ++s1)
        for (int s2 = 0; s2 < 4; ++s2)
          for (int s3 = 0; s3 < 4; ++s3) {
            int s[4] = {s0, s1, s2, s3};
            int ok = 1;
            for (int i = 0; i < 4; ++i)
              for (int j = i + 1; j < 4; ++j)
                if (s[i] == s[j]) ok = 0;
            if (!ok) continue;
            int inv = 0;
            for (int i = 0; i < 4; ++i)
              for (int j = i + 1; j < 4; ++j)
                if (s[i] > s[j]) ++inv;
            memcpy(perm[k], s, sizeof s);
            psign[k] = (inv & 1) ? -1 : 1;
            ++k;
          }
    perm_init = 1;
  }
  /* row r of the matrix is (1, P[r].x, P[r].y, P[r].z); sigma(r) = column */
  double e1[256], e2[256];
  double* cur = e1;
  double* nxt = e2;
  int len = 0;
  for (int k = 0; k < 24; ++k) {
    double f[3];
    int nf = 0;
    for (int r = 0; r < 4; ++r) {
      int col = perm[k][r];
      if (col == 0) continue;
      f[nf++] = P[r][col - 1];
    }
    /* exact f0*f1*f2 as four doubles */
    double p, e, p1, e1_, p2, e2_;
    two_prod(f[0], f[1], &p, &e);
    two_prod(p, f[2], &p1, &e1_);
    two_prod(e, f[2], &p2, &e2_);
    double t[4] = {p1, e1_, p2, e2_};
    for (int i = 0; i < 4; ++i) {
      double term = psign[k] > 0 ? t[i] : -t[i];
      if (term == 0.0) continue;
      len = grow_expansion(len, cur, term, nxt);
      double* sw = cur;
      cur = nxt;
      nxt = sw;
    }
  }
  for (int i = len - 1; i >= 0; --i) {
    if (cur[i] > 0) return 1;
    if (cur[i] < 0) return -1;
  }
  return 0;
}

int om_orient_sign(const double* a, const double* b, const double* c,
                   const double* d) {
  /* vol6(a,b,c,d) = det[b-a; c-a; d-a]; filter: differences w.r.t. a,
   * Shewchuk's orient3d stage-A bound (7 + 56 eps) eps * permanent. */
  double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
  double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
  double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
  double cydz = cy * dz, czdy = cz * dy;
  double czdx = cz * dx, cxdz = cx * dz;
  double cxdy = cx * dy, cydx = cy * dx;
  double det = bx * (cydz - czdy) + by * (czdx - cxdz) + bz * (cxdy - cydx);
  double perm = (fabs(cydz) + fabs(czdy)) * fabs(bx) +
                (fabs(czdx) + fabs(cxdz)) * fabs(by) +
                (fabs(cxdy) + fabs(cydx)) * fabs(bz);
  const double eps = 0x1p-53;
  double bound = (7.0 + 56.0 * eps) * eps * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return exact_det4_sign(a, b, c, d);
}

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. II A: linear elements; App. B: Galerkin stiffness and load).  */
/* ------------------------------------------------------------------------ */
struct omesh {
  int64_t n_nodes, n_tets, n_free, nnz, n_emit, n_top, n_metal, n_flipped;
  double Lx, Ly, z_top, emit_zmin;
  double* xyz;       /* [n][3] */
  int32_t* tet;      /* [T][4] oriented */
  int8_t* shift;     /* [T][4][2] oriented */
  double* vert;      /* [T][4][3] unwrapped */
  double* mm;        /* [T][3][3] rows m1, m2, m3 */
  double* D;         /* [T] */
  int32_t* nbr;      /* [T][4]: tet, -1 top, -2 metal */
  int8_t* nbr_shift; /* [T][4][2] */
  int32_t* free_id;  /* [n] free index or -1 */
  int64_t* rowptr;   /* [n_free+1] */
  int32_t* col;      /* [nnz] */
  double* val;       /* [nnz] */
  double* diag;      /* [n_free] */
  double* g_unit;    /* [n_free] */
  double* W;         /* [n] sum of incident tet volumes */
  /* emitting faces */
  int32_t* e_tet;
  int32_t* e_loc;
  double* e_area;
  double* e_nrm;  /* [F][3] into vacuum */
  double* e_abc;  /* [F][3][3] */
  int32_t* e_nodes; /* [F][3] */
  /* bucket grid */
  int nb[3];
  double b0[3], b1[3], binv[3];
  int64_t* bstart;
  int32_t* bitem;
};

static const int FACE_V[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

static void vsub(const double* a, const double* b, double* r) {
  r[0] = a[0] - b[0];
  r[1] = a[1] - b[1];
  r[2] = a[2] - b[2];
}
static void vcross(const double* a, const double* b, double* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static double vdot(const double* a, const double* b) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

typedef struct {
  int32_t n[3];
  int8_t d[4];
  int32_t tet;
  int8_t face;
  int8_t s1[2];
} fkey;

static int fkey_cmp(const void* pa, const void* pb) {
  const fkey* a = (const fkey*)pa;
  const fkey* b = (const fkey*)pb;
  for (int i = 0; i < 3; ++i)
    if (a->n[i] != b->n[i]) return a->n[i] < b->n[i] ? -1 : 1;
  for (int i = 0; i < 4; ++i)
    if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
  if (a->tet != b->tet) return a->tet < b->tet ? -1 : 1;
  return a->face - b->face;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static int bucket_of(const omesh* m, int ax, double x) {
  double f = floor((x - m->b0[ax]) * m->binv[ax]);
  int i = (int)f;
  if (f < 0) i = 0;
  if (f > m->nb[ax] - 1) i = m->nb[ax] - 1;
  return i;
}

void om_destroy(omesh* m) {
  if (!m) return;
  free(m->xyz); free(m->tet); free(m->shift); free(m->vert); free(m->mm);
  free(m->D); free(m->nbr); free(m->nbr_shift); free(m->free_id);
  free(m->rowptr); free(m->col); free(m->val); free(m->diag);
  free(m->g_unit); free(m->W); free(m->e_tet); free(m->e_loc);
  free(m->e_area); free(m->e_nrm); free(m->e_abc); free(m->e_nodes);
  free(m->bstart); free(m->bitem);
  free(m);
}

/* geometry of one oriented tet: m rows and D (the fixed arithmetic) */
static void tet_geometry(const double* v, double* mm, double* D) {
  double e1[3], e2[3], e3[3], c1[3], c2[3], c3[3];
  vsub(v + 3, v, e1);
  vsub(v + 6, v, e2);
  vsub(v + 9, v, e3);
  vcross(e2, e3, c1);
  vcross(e3, e1, c2);
  vcross(e1, e2, c3);
  double d = vdot(e1, c1);
  for (int k = 0; k < 3; ++k) {
    mm[0 + k] = c1[k] / d;
    mm[3 + k] = c2[k] / d;
    mm[6 + k] = c3[k] / d;
  }
  *D = d;
}

omesh* om_create(int64_t n_nodes, const double* xyz, int64_t n_tets,
                 const int32_t* tet_in, const int8_t* shift_in, double Lx,
                 double Ly, double z_top, double emit_zmin, char* err,
                 int errlen) {
  omesh* m = (omesh*)calloc(1, sizeof(omesh));
  m->n_nodes = n_nodes;
  m->n_tets = n_tets;
  m->Lx = Lx;
  m->Ly = Ly;
  m->z_top = z_top;
  m->emit_zmin = emit_zmin;
  m->xyz = (double*)malloc(sizeof(double) * 3 * n_nodes);
  memcpy(m->xyz, xyz, sizeof(double) * 3 * n_nodes);
  m->tet = (int32_t*)malloc(sizeof(int32_t) * 4 * n_tets);
  m->shift = (int8_t*)calloc(8 * n_tets, 1);
  m->vert = (double*)malloc(sizeof(double) * 12 * n_tets);
  m->mm = (double*)malloc(sizeof(double) * 9 * n_tets);
  m->D = (double*)malloc(sizeof(double) * n_tets);
  memcpy(m->tet, tet_in, sizeof(int32_t) * 4 * n_tets);
  if (shift_in) memcpy(m->shift, shift_in, 8 * n_tets);

  /* 1. orientation and geometry */
  for (int64_t t = 0; t < n_tets; ++t) {
    int32_t* tv = m->tet + 4 * t;
    int8_t* ts = m->shift + 8 * t;
    for (int i = 0; i < 4; ++i) {
      if (tv[i] < 0 || tv[i] >= n_nodes) {
        snprintf(err, errlen, "tet %lld: node index out of range", (long long)t);
        om_destroy(m);
        return NULL;
      }
    }
    double v[12];
    for (int i = 0; i < 4; ++i) {
      const double* p = xyz + 3 * (int64_t)tv[i];
      v[3 * i + 0] = p[0] + (double)ts[2 * i + 0] * Lx;
      v[3 * i + 1] = p[1] + (double)ts[2 * i + 1] * Ly;
      v[3 * i + 2] = p[2];
    }
    int s = om_orient_sign(v, v + 3, v + 6, v + 9);
    if (s == 0) {
      snprintf(err, errlen, "tet %lld has zero volume", (long long)t);
      om_destroy(m);
      return NULL;
    }
    if (s < 0) {
      int32_t a = tv[2]; tv[2] = tv[3]; tv[3] = a;
      int8_t b0 = ts[4], b1 = ts[5];
      ts[4] = ts[6]; ts[5] = ts[7]; ts[6] = b0; ts[7] = b1;
      for (int k = 0; k < 3; ++k) {
        double x = v[6 + k]; v[6 + k] = v[9 + k]; v[9 + k] = x;
      }
      m->n_flipped++;
    }
    memcpy(m->vert + 12 * t, v, sizeof v);
    tet_geometry(v, m->mm + 9 * t, m->D + t);
  }

  /* 2. adjacency by matching faces (node ids + relative lattice shifts) */
  int64_t nf = 4 * n_tets;
  fkey* keys = (fkey*)malloc(sizeof(fkey) * nf);
  for (int64_t t = 0; t < n_tets; ++t) {
    for (int f = 0; f < 4; ++f) {
      int32_t nn[3];
      int8_t ss[3][2];
      for (int j = 0; j < 3; ++j) {
        int l = FACE_V[f][j];
        nn[j] = m->tet[4 * t + l];
        ss[j][0] = m->shift[8 * t + 2 * l];
        ss[j][1] = m->shift[8 * t + 2 * l + 1];
      }
      /* sort by node id (3 elements) */
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2 - a; ++b)
          if (nn[b] > nn[b + 1]) {
            int32_t x = nn[b]; nn[b] = nn[b + 1]; nn[b + 1] = x;
            int8_t y0 = ss[b][0], y1 = ss[b][1];
            ss[b][0] = ss[b + 1][0]; ss[b][1] = ss[b + 1][1];
            ss[b + 1][0] = y0; ss[b + 1][1] = y1;
          }
      fkey* k = keys + 4 * t + f;
      k->n[0] = nn[0]; k->n[1] = nn[1]; k->n[2] = nn[2];
      k->d[0] = (int8_t)(ss[1][0] - ss[0][0]);
      k->d[1] = (int8_t)(ss[1][1] - ss[0][1]);
      k->d[2] = (int8_t)(ss[2][0] - ss[0][0]);
      k->d[3] = (int8_t)(ss[2][1] - ss[0][1]);
      k->tet = (int32_t)t;
      k->face = (int8_t)f;
      k->s1[0] = ss[0][0];
      k->s1[1] = ss[0][1];
    }
  }
  qsort(keys, nf, sizeof(fkey), fkey_cmp);
  m->nbr = (int32_t*)malloc(sizeof(int32_t) * 4 * n_tets);
  m->nbr_shift = (int8_t*)calloc(8 * n_tets, 1);
  for (int64_t i = 0; i < nf;) {
    int64_t j = i + 1;
    while (j < nf && memcmp(keys[j].n, keys[i].n, sizeof keys[i].n) == 0 &&
           memcmp(keys[j].d, keys[i].d, sizeof keys[i].d) == 0)
      ++j;
    if (j - i > 2) {
      snprintf(err, errlen, "non-manifold face shared by %lld tets",
               (long long)(j - i));
      free(keys);
      om_destroy(m);
      return NULL;
    }
    if (j - i == 2) {
      fkey* a = keys + i;
      fkey* b = keys + i + 1;
      m->nbr[4 * a->tet + a->face] = b->tet;
      m->nbr[4 * b->tet + b->face] = a->tet;
      m->nbr_shift[8 * a->tet + 2 * a->face] = (int8_t)(b->s1[0] - a->s1[0]);
      m->nbr_shift[8 * a->tet + 2 * a->face + 1] = (int8_t)(b->s1[1] - a->s1[1]);
      m->nbr_shift[8 * b->tet + 2 * b->face] = (int8_t)(a->s1[0] - b->s1[0]);
      m->nbr_shift[8 * b->tet + 2 * b->face + 1] = (int8_t)(a->s1[1] - b->s1[1]);
    } else {
      /* boundary: TOP when all three vertices lie on z = z_top, else metal */
      fkey* a = keys + i;
      const double* v = m->vert + 12 * (int64_t)a->tet;
      int top = 1;
      for (int q = 0; q < 3; ++q)
        if (v[3 * FACE_V[(int)a->face][q] + 2] != z_top) top = 0;
      m->nbr[4 * a->tet + a->face] = top ? -1 : -2;
      if (top) m->n_top++; else m->n_metal++;
    }
    i = j;
  }
  free(keys);

  /* 3. Dirichlet nodes (vertices of metal faces, Eq. poisson_bc on Gamma_3);
   *    free nodes numbered in ascending node order */
  char* dir = (char*)calloc(n_nodes, 1);
  for (int64_t t = 0; t < n_tets; ++t)
    for (int f = 0; f < 4; ++f)
      if (m->nbr[4 * t + f] == -2)
        for (int q = 0; q < 3; ++q) dir[m->tet[4 * t + FACE_V[f][q]]] = 1;
  m->free_id = (int32_t*)malloc(sizeof(int32_t) * n_nodes);
  m->n_free = 0;
  for (int64_t i = 0; i < n_nodes; ++i)
    m->free_id[i] = dir[i] ? -1 : (int32_t)(m->n_free++);
  free(dir);

  /* 4. node -> tet lists, sparsity of K on free nodes (App. B) */
  int64_t* nts = (int64_t*)calloc(n_nodes + 1, sizeof(int64_t));
  for (int64_t t = 0; t < n_tets; ++t)
    for (int i = 0; i < 4; ++i) nts[m->tet[4 * t + i] + 1]++;
  for (int64_t i = 0; i < n_nodes; ++i) nts[i + 1] += nts[i];
  int32_t* ntl = (int32_t*)malloc(sizeof(int32_t) * nts[n_nodes]);
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * n_nodes);
  memcpy(fill, nts, sizeof(int64_t) * n_nodes);
  for (int64_t t = 0; t < n_tets; ++t)
    for (int i = 0; i < 4; ++i) ntl[fill[m->tet[4 * t + i]]++] = (int32_t)t;
  free(fill);
  m->rowptr = (int64_t*)calloc(m->n_free + 1, sizeof(int64_t));
  int32_t tmp[4096];
  /* first pass: counts */
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t i = 0; i < n_nodes; ++i) {
      int32_t fi = m->free_id[i];
      if (fi < 0) continue;
      int nt = 0;
      for (int64_t q = nts[i]; q < nts[i + 1]; ++q) {
        int32_t t = ntl[q];
        for (int a = 0; a < 4; ++a) {
          int32_t fj = m->free_id[m->tet[4 * t + a]];
          if (fj >= 0 && nt < 4096) tmp[nt++] = fj;
        }
      }
      qsort(tmp, nt, sizeof(int32_t), cmp_i32);
      int u = 0;
      for (int q = 0; q < nt; ++q)
        if (u == 0 || tmp[q] != tmp[u - 1]) tmp[u++] = tmp[q];
      if (pass == 0) {
        m->rowptr[fi + 1] = u;
      } else {
        memcpy(m->col + m->rowptr[fi], tmp, sizeof(int32_t) * u);
      }
    }
    if (pass == 0) {
      for (int64_t i = 0; i < m->n_free; ++i) m->rowptr[i + 1] += m->rowptr[i];
      m->nnz = m->rowptr[m->n_free];
      m->col = (int32_t*)malloc(sizeof(int32_t) * m->nnz);
    }
  }
  /* 5. element stiffness V grad N_a . grad N_b, summed in tet order */
  m->val = (double*)calloc(m->nnz, sizeof(double));
  m->W = (double*)calloc(n_nodes, sizeof(double));
  for (int64_t t = 0; t < n_tets; ++t) {
    const double* mm = m->mm + 9 * t;
    double g[4][3];
    for (int k = 0; k < 3; ++k) {
      g[1][k] = mm[k];
      g[2][k] = mm[3 + k];
      g[3][k] = mm[6 + k];
      g[0][k] = -((mm[k] + mm[3 + k]) + mm[6 + k]);
    }
    double V = m->D[t] / 6.0;
    for (int a = 0; a < 4; ++a) m->W[m->tet[4 * t + a]] += V;
    for (int a = 0; a < 4; ++a) {
      int32_t fi = m->free_id[m->tet[4 * t + a]];
      if (fi < 0) continue;
      for (int b = 0; b < 4; ++b) {
        int32_t fj = m->free_id[m->tet[4 * t + b]];
        if (fj < 0) continue;
        double kab = V * vdot(g[a], g[b]);
        /* binary search column fj in row fi */
        int64_t lo = m->rowptr[fi], hi = m->rowptr[fi + 1] - 1;
        while (lo < hi) {
          int64_t mid = (lo + hi) / 2;
          if (m->col[mid] < fj) lo = mid + 1; else hi = mid;
        }
        m->val[lo] += kab;
      }
    }
  }
  m->diag = (double*)malloc(sizeof(double) * (m->n_free > 0 ? m->n_free : 1));
  for (int64_t i = 0; i < m->n_free; ++i)
    for (int64_t q = m->rowptr[i]; q < m->rowptr[i + 1]; ++q)
      if (m->col[q] == i) m->diag[i] = m->val[q];
  free(nts);
  free(ntl);

  /* 6. Neumann load per unit E0: integral of N_i over Gamma_1 = A/3 */
  m->g_unit = (double*)calloc(m->n_free > 0 ? m->n_free : 1, sizeof(double));
  for (int64_t t = 0; t < n_tets; ++t)
    for (int f = 0; f < 4; ++f) {
      if (m->nbr[4 * t + f] != -1) continue;
      const double* v = m->vert + 12 * t;
      const double* A = v + 3 * FACE_V[f][0];
      const double* B = v + 3 * FACE_V[f][1];
      const double* C = v + 3 * FACE_V[f][2];
      double ab[3], ac[3], cr[3];
      vsub(B, A, ab);
      vsub(C, A, ac);
      vcross(ab, ac, cr);
      double area = 0.5 * sqrt(vdot(cr, cr));
      for (int q = 0; q < 3; ++q) {
        int32_t fi = m->free_id[m->tet[4 * t + FACE_V[f][q]]];
        if (fi >= 0) m->g_unit[fi] += area / 3.0;
      }
    }

  /* 7. emitting faces: metal faces with centroid z >= emit_zmin, ordered by
   *    (owner tet, local face) (Sec. II B 3, reading: triangle faces) */
  int64_t ne = 0;
  for (int pass = 0; pass < 2; ++pass) {
    ne = 0;
    for (int64_t t = 0; t < n_tets; ++t)
      for (int f = 0; f < 4; ++f) {
        if (m->nbr[4 * t + f] != -2) continue;
        const double* v = m->vert + 12 * t;
        const double* A = v + 3 * FACE_V[f][0];
        const double* B = v + 3 * FACE_V[f][1];
        const double* C = v + 3 * FACE_V[f][2];
        if (!((A[2] + B[2]) + C[2] >= 3.0 * emit_zmin)) continue;
        if (pass == 1) {
          m->e_tet[ne] = (int32_t)t;
          m->e_loc[ne] = f;
          double ab[3], ac[3], cr[3], vo[3];
          vsub(B, A, ab);
          vsub(C, A, ac);
          vcross(ab, ac, cr);
          double len = sqrt(vdot(cr, cr));
          m->e_area[ne] = 0.5 * len;
          vsub(v + 3 * f, A, vo);
          double sg = vdot(cr, vo) < 0 ? -1.0 : 1.0;
          for (int k = 0; k < 3; ++k) {
            m->e_nrm[3 * ne + k] = sg * cr[k] / len;
            m->e_abc[9 * ne + k] = A[k];
            m->e_abc[9 * ne + 3 + k] = B[k];
            m->e_abc[9 * ne + 6 + k] = C[k];
          }
          for (int q = 0; q < 3; ++q)
            m->e_nodes[3 * ne + q] = m->tet[4 * t + FACE_V[f][q]];
        }
        ++ne;
      }
    if (pass == 0) {
      m->n_emit = ne;
      int64_t a = ne > 0 ? ne : 1;
      m->e_tet = (int32_t*)malloc(sizeof(int32_t) * a);
      m->e_loc = (int32_t*)malloc(sizeof(int32_t) * a);
      m->e_area = (double*)malloc(sizeof(double) * a);
      m->e_nrm = (double*)malloc(sizeof(double) * 3 * a);
      m->e_abc = (double*)malloc(sizeof(double) * 9 * a);
      m->e_nodes = (int32_t*)malloc(sizeof(int32_t) * 3 * a);
    }
  }

  /* 8. bucket grid over the unwrapped box; a tet is listed in every bucket
   *    its closed bounding box touches under the same monotone bucket map
   *    used for queries, so a query never misses a containing tet. */
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t q = 0; q < 4 * n_tets; ++q)
    for (int k = 0; k < 3; ++k) {
      double x = m->vert[3 * q + k];
      if (x < lo[k]) lo[k] = x;
      if (x > hi[k]) hi[k] = x;
    }
  double vol = 0;
  for (int64_t t = 0; t < n_tets; ++t) vol += m->D[t];
  double edge = cbrt(vol / (double)(n_tets > 0 ? n_tets : 1));
  for (int k = 0; k < 3; ++k) {
    double L = hi[k] - lo[k];
    int nb = (int)floor(L / edge);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    m->nb[k] = nb;
    m->b0[k] = lo[k];
    m->b1[k] = hi[k];
    m->binv[k] = (double)nb / L;
  }
  int64_t nbt = (int64_t)m->nb[0] * m->nb[1] * m->nb[2];
  m->bstart = (int64_t*)calloc(nbt + 1, sizeof(int64_t));
  for (int pass = 0; pass < 2; ++pass) {
    int64_t* pos = NULL;
    if (pass == 1) {
      pos = (int64_t*)malloc(sizeof(int64_t) * nbt);
      memcpy(pos, m->bstart, sizeof(int64_t) * nbt);
    }
    for (int64_t t = 0; t < n_tets; ++t) {
      const double* v = m->vert + 12 * t;
      int i0[3], i1[3];
      for (int k = 0; k < 3; ++k) {
        double a = v[k], b = v[k];
        for (int q = 1; q < 4; ++q) {
          if (v[3 * q + k] < a) a = v[3 * q + k];
          if (v[3 * q + k] > b) b = v[3 * q + k];
        }
        i0[k] = bucket_of(m, k, a);
        i1[k] = bucket_of(m, k, b);
      }
      for (int a = i0[0]; a <= i1[0]; ++a)
        for (int b = i0[1]; b <= i1[1]; ++b)
          for (int c = i0[2]; c <= i1[2]; ++c) {
            int64_t id = ((int64_t)a * m->nb[1] + b) * m->nb[2] + c;
            if (pass == 0) m->bstart[id + 1]++;
            else m->bitem[pos[id]++] = (int32_t)t;
          }
    }
    if (pass == 0) {
      for (int64_t i = 0; i < nbt; ++i) m->bstart[i + 1] += m->bstart[i];
      m->bitem = (int32_t*)malloc(sizeof(int32_t) * (m->bstart[nbt] + 1));
    } else {
      free(pos);
    }
  }
  return m;
}

int64_t om_info(const omesh* m, int what) {
  switch (what) {
    case OM_N_NODES: return m->n_nodes;
    case OM_N_TETS: return m->n_tets;
    case OM_N_FREE: return m->n_free;
    case OM_NNZ: return m->nnz;
    case OM_N_EMIT: return m->n_emit;
    case OM_N_TOP: return m->n_top;
    case OM_N_METAL: return m->n_metal;
    case OM_N_FLIPPED: return m->n_flipped;
  }
  return -1;
}

void om_get_tets(const omesh* m, int32_t* tet4, double* vert12, double* mmat9,
                 double* D, int32_t* nbr4, int8_t* nbr_shift8) {
  int64_t T = m->n_tets;
  if (tet4) memcpy(tet4, m->tet, sizeof(int32_t) * 4 * T);
  if (vert12) memcpy(vert12, m->vert, sizeof(double) * 12 * T);
  if (mmat9) memcpy(mmat9, m->mm, sizeof(double) * 9 * T);
  if (D) memcpy(D, m->D, sizeof(double) * T);
  if (nbr4) memcpy(nbr4, m->nbr, sizeof(int32_t) * 4 * T);
  if (nbr_shift8) memcpy(nbr_shift8, m->nbr_shift, 8 * T);
}

void om_get_csr(const omesh* m, int64_t* rowptr, int32_t* col, double* val) {
  memcpy(rowptr, m->rowptr, sizeof(int64_t) * (m->n_free + 1));
  memcpy(col, m->col, sizeof(int32_t) * m->nnz);
  memcpy(val, m->val, sizeof(double) * m->nnz);
}

void om_get_free(const omesh* m, int32_t* free_id, double* g_unit) {
  memcpy(free_id, m->free_id, sizeof(int32_t) * m->n_nodes);
  memcpy(g_unit, m->g_unit, sizeof(double) * m->n_free);
}

void om_get_emit(const omesh* m, int32_t* tet, int32_t* local, double* area,
                 double* normal3, double* abc9, int32_t* nodes3) {
  int64_t F = m->n_emit;
  memcpy(tet, m->e_tet, sizeof(int32_t) * F);
  memcpy(local, m->e_loc, sizeof(int32_t) * F);
  memcpy(area, m->e_area, sizeof(double) * F);
  memcpy(normal3, m->e_nrm, sizeof(double) * 3 * F);
  memcpy(abc9, m->e_abc, sizeof(double) * 9 * F);
  memcpy(nodes3, m->e_nodes, sizeof(int32_t) * 3 * F);
}

/* ------------------------------------------------------------------------ */
/* Point location and barycentric weights (Sec. II B 2).                    */
/* ------------------------------------------------------------------------ */

/* 1 if the closed tet t holds p, with *strict set when p is interior */
static int tet_contains(const omesh* m, int64_t t, const double* p,
                        int* strict) {
  const double* v = m->vert + 12 * t;
  const double* q[4] = {v, v + 3, v + 6, v + 9};
  int all_pos = 1;
  for (int i = 0; i < 4; ++i) {
    const double* r[4] = {q[0], q[1], q[2], q[3]};
    r[i] = p;
    int s = om_orient_sign(r[0], r[1], r[2], r[3]);
    if (s < 0) return 0;
    if (s == 0) all_pos = 0;
  }
  if (strict) *strict = all_pos;
  return 1;
}

static int32_t locate_one(const omesh* m, const double* p, int32_t hint) {
  if (hint >= 0 && hint < m->n_tets) {
    int strict = 0;
    /* interior of one tet: no other tet of a conforming mesh holds p */
    if (tet_contains(m, hint, p, &strict) && strict) return hint;
  }
  for (int k = 0; k < 3; ++k)
    if (!(p[k] >= m->b0[k] && p[k] <= m->b1[k])) return -1;
  int a = bucket_of(m, 0, p[0]);
  int b = bucket_of(m, 1, p[1]);
  int c = bucket_of(m, 2, p[2]);
  int64_t id = ((int64_t)a * m->nb[1] + b) * m->nb[2] + c;
  for (int64_t q = m->bstart[id]; q < m->bstart[id + 1]; ++q) {
    int32_t t = m->bitem[q]; /* ascending tet order: first hit is lowest */
    if (tet_contains(m, t, p, NULL)) return t;
  }
  return -1;
}

void om_locate(const omesh* m, int64_t n, const double* x, const double* y,
               const double* z, const int32_t* hint, int32_t* tet_out,
               uint8_t* where_out) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    if (p[2] >= m->z_top) {
      tet_out[i] = -1;
      where_out[i] = 1;
      continue;
    }
    int32_t t = locate_one(m, p, hint ? hint[i] : -1);
    tet_out[i] = t;
    where_out[i] = t >= 0 ? 0 : 2;
  }
}

/* lambda_i = m_i.(p - v0), i = 1..3; lambda_0 = ((1 - l1) - l2) - l3 */
void om_lambda(const omesh* m, int32_t t, const double* p, double* lam) {
  const double* v0 = m->vert + 12 * (int64_t)t;
  const double* mm = m->mm + 9 * (int64_t)t;
  double d[3];
  vsub(p, v0, d);
  double l1 = vdot(mm, d), l2 = vdot(mm + 3, d), l3 = vdot(mm + 6, d);
  lam[0] = ((1.0 - l1) - l2) - l3;
  lam[1] = l1;
  lam[2] = l2;
  lam[3] = l3;
}

/* ------------------------------------------------------------------------ */
/* Charge deposition (Eq. q_delta, Eq. poisson_rhs): each superparticle     */
/* adds N_i(r) = lambda_i of its tet to the four vertices, in int64 fixed   */
/* point with 2^40 units per unit relative weight.                          */
/* ------------------------------------------------------------------------ */
static void particle_charge(const double* lam, double w, int64_t* q) {
  const double S = 0x1p40;
  q[1] = llrint((lam[1] * w) * S);
  q[2] = llrint((lam[2] * w) * S);
  q[3] = llrint((lam[3] * w) * S);
  q[0] = llrint(w * S) - ((q[1] + q[2]) + q[3]);
}

void om_deposit(const omesh* m, int64_t n, const double* x, const double* y,
                const double* z, const int32_t* tet, const double* w,
                int64_t* c) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int32_t t = tet[i];
    if (t < 0) continue;
    double p[3] = {x[i], y[i], z[i]}, lam[4];
    om_lambda(m, t, p, lam);
    int64_t q[4];
    particle_charge(lam, w[i], q);
    for (int a = 0; a < 4; ++a) {
#pragma omp atomic
      c[m->tet[4 * (int64_t)t + a]] += q[a];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Poisson solve (Eq. poisson, Eq. poisson_bc, App. B): K phi_f = b_f with  */
/* b_i = (q w_sp/eps0) sum_j N_i(r_j) + E0 int_{Gamma_1} N_i; q = -e.        */
/* Jacobi-preconditioned CG (Saad, Iterative Methods, Alg. 9.1): the paper  */
/* only says the equation is solved iteratively.                            */
/* ------------------------------------------------------------------------ */
void om_rhs(const omesh* m, const int64_t* c, double w_sp, double E0,
            double* b) {
  consts_t k = constants();
  double coef = (-k.e_eps * w_sp) * 0x1p-40;
  for (int64_t i = 0; i < m->n_nodes; ++i) {
    int32_t fi = m->free_id[i];
    if (fi < 0) continue;
    double ci = c ? (double)c[i] : 0.0;
    b[fi] = coef * ci + E0 * m->g_unit[fi];
  }
}

void om_spmv(const omesh* m, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m->n_free; ++i) {
    double s = 0.0;
    for (int64_t q = m->rowptr[i]; q < m->rowptr[i + 1]; ++q)
      s += m->val[q] * x[m->col[q]];
    y[i] = s;
  }
}

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

int om_poisson_solve(const omesh* m, const int64_t* c, double w_sp, double E0,
                     double* phi, double tol, int max_iter, int* iters,
                     double* relres) {
  int64_t n = m->n_free;
  double* b = (double*)malloc(sizeof(double) * (n + 1));
  double* x = (double*)malloc(sizeof(double) * (n + 1));
  double* r = (double*)malloc(sizeof(double) * (n + 1));
  double* z = (double*)malloc(sizeof(double) * (n + 1));
  double* p = (double*)malloc(sizeof(double) * (n + 1));
  double* q = (double*)malloc(sizeof(double) * (n + 1));
  om_rhs(m, c, w_sp, E0, b);
  for (int64_t i = 0; i < m->n_nodes; ++i)
    if (m->free_id[i] >= 0) x[m->free_id[i]] = phi[i];
  double bn = sqrt(dot(n, b, b));
  int it = 0, status = 0;
  double rr = 0.0;
  if (bn == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
  } else {
    int converged = 0;
    while (!converged) {
      /* (re)start from the true residual */
      om_spmv(m, x, q);
      for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
      rr = sqrt(dot(n, r, r));
      if (rr <= tol * bn) break;
      if (it >= max_iter) {
        status = -4;
        break;
      }
      for (int64_t i = 0; i < n; ++i) z[i] = r[i] / m->diag[i];
      for (int64_t i = 0; i < n; ++i) p[i] = z[i];
      double rz = dot(n, r, z);
      while (it < max_iter) {
        om_spmv(m, p, q);
        double alpha = rz / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        ++it;
        if (sqrt(dot(n, r, r)) <= tol * bn) break; /* re-checked above */
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / m->diag[i];
        double rz2 = dot(n, r, z);
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      }
    }
  }
  for (int64_t i = 0; i < m->n_nodes; ++i)
    phi[i] = m->free_id[i] >= 0 ? x[m->free_id[i]] : 0.0;
  if (iters) *iters = it;
  if (relres) *relres = bn > 0 ? rr / bn : 0.0;
  free(b); free(x); free(r); free(z); free(p); free(q);
  return status;
}

/* Gradient of the linear-element potential in tet t: grad lambda_k are
 * the rows m_k (k = 1..3) and grad lambda_0 = -(m_1 + m_2 + m_3). */
static void tet_grad(const omesh* m, int64_t t, const double* phi,
                     double* grad) {
  const double* mm = m->mm + 9 * t;
  const int32_t* tv = m->tet + 4 * t;
  for (int k = 0; k < 3; ++k) {
    const double g0 = -((mm[k] + mm[3 + k]) + mm[6 + k]);
    grad[k] = ((phi[tv[0]] * g0 + phi[tv[1]] * mm[k]) +
               phi[tv[2]] * mm[3 + k]) + phi[tv[3]] * mm[6 + k];
  }
}

/* Cell field (reading R2, cell variant): E = -(grad phi)_t, constant in
 * tet t. */
static void cell_field(const omesh* m, int64_t t, const double* phi,
                       double* E) {
  double grad[3];
  tet_grad(m, t, phi, grad);
  for (int k = 0; k < 3; ++k) E[k] = -grad[k];
}

void om_cell_field(const omesh* m, const double* phi, double* E3t) {
  for (int64_t t = 0; t < m->n_tets; ++t) cell_field(m, t, phi, E3t + 3 * t);
}

/* Nodal field (reading of Sec. II B 2: the field interpolated with the
 * element's shape functions needs nodal values): E_i = sum_t V_t (-grad
 * phi)_t / sum_t V_t over the tets holding node i. */
void om_field(const omesh* m, const double* phi, double* E3) {
  double* acc = (double*)calloc(3 * m->n_nodes, sizeof(double));
  for (int64_t t = 0; t < m->n_tets; ++t) {
    const int32_t* tv = m->tet + 4 * t;
    double grad[3];
    tet_grad(m, t, phi, grad);
    double V = m->D[t] / 6.0;
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) acc[3 * (int64_t)tv[a] + k] += V * (-grad[k]);
  }
  for (int64_t i = 0; i < m->n_nodes; ++i)
    for (int k = 0; k < 3; ++k)
      E3[3 * i + k] = m->W[i] > 0 ? acc[3 * i + k] / m->W[i] : 0.0;
  free(acc);
}

void om_field_adj(const omesh* m, const double* Ebar3, double* phibar) {
  /* E_i = (1/W_i) sum_{t ∋ i} V_t (-grad phi_t), grad phi_t =
   * sum_b phi_(t,b) g_b: so d<Ebar, E>/d phi_j = sum_t sum_{b: node j}
   * -g_b . (V_t sum_{a in t} Ebar_(t,a) / W_(t,a)) */
  memset(phibar, 0, sizeof(double) * m->n_nodes);
  for (int64_t t = 0; t < m->n_tets; ++t) {
    const double* mm = m->mm + 9 * t;
    const int32_t* tv = m->tet + 4 * t;
    double g[4][3];
    for (int k = 0; k < 3; ++k) {
      g[1][k] = mm[k];
      g[2][k] = mm[3 + k];
      g[3][k] = mm[6 + k];
      g[0][k] = -((mm[k] + mm[3 + k]) + mm[6 + k]);
    }
    double V = m->D[t] / 6.0, A[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 4; ++a) {
      const double Wa = m->W[tv[a]];
      if (!(Wa > 0)) continue;
      for (int k = 0; k < 3; ++k) A[k] += Ebar3[3 * (int64_t)tv[a] + k] / Wa;
    }
    for (int b = 0; b < 4; ++b)
      phibar[tv[b]] -= V * ((g[b][0] * A[0] + g[b][1] * A[1]) + g[b][2] * A[2]);
  }
}

/* ------------------------------------------------------------------------ */
/* Injection (Sec. II B 3, Eq. nsp, Eq. rnd_nsp, Eq. sp_velocity,            */
/* Eq. sp_displacement, App. E).                                            */
/* ------------------------------------------------------------------------ */
static void face_centroid_field(const omesh* m, int64_t f, const double* E3,
                                double* Ec) {
  const int32_t* nd = m->e_nodes + 3 * f;
  for (int k = 0; k < 3; ++k)
    Ec[k] = ((E3[3 * (int64_t)nd[0] + k] + E3[3 * (int64_t)nd[1] + k]) +
             E3[3 * (int64_t)nd[2] + k]) / 3.0;
}

/* emission current density of face f in e nm^-2 fs^-1 (0 when the field
 * does not pull electrons out of the metal), and |E| at the centroid; the
 * centroid field is the nodal one, or with phi (cell mode) the field of the
 * face's vacuum tet */
static double face_emission(const omesh* m, int64_t f, const double* E3,
                            const double* phi, double phi_w, double* F_out,
                            int* clamped) {
  consts_t k = constants();
  double Ec[3];
  if (phi)
    cell_field(m, m->e_tet[f], phi, Ec);
  else
    face_centroid_field(m, f, E3, Ec);
  double F = sqrt(vdot(Ec, Ec));
  if (F_out) *F_out = F;
  if (!(vdot(Ec, m->e_nrm + 3 * f) < 0.0)) return 0.0;
  return om_fn_current(F, phi_w, clamped) * k.j_unit;
}

double om_emission_rate_mode(const omesh* m, const double* E3,
                             const double* phi, double phi_w, double* faceF) {
  double tot = 0.0;
  for (int64_t f = 0; f < m->n_emit; ++f) {
    int cl = 0;
    double F;
    double j = face_emission(m, f, E3, phi, phi_w, &F, &cl);
    if (faceF) faceF[f] = F;
    tot += j * m->e_area[f];
  }
  return tot;
}

double om_emission_rate(const omesh* m, const double* E3, double phi_w,
                        double* faceF) {
  return om_emission_rate_mode(m, E3, NULL, phi_w, faceF);
}

/* ------------------------------------------------------------------------ */
/* Surface charge (Eq. face_charge, Eq. atom_charge, Eq. charge_weight).     */
/* ------------------------------------------------------------------------ */
static double face_atom_dist(const omesh* m, const double* c, const double* a) {
  double dx = c[0] - a[0], dy = c[1] - a[1], dz = c[2] - a[2];
  if (dx > 0.5 * m->Lx) dx -= m->Lx;
  else if (dx < -0.5 * m->Lx) dx += m->Lx;
  if (dy > 0.5 * m->Ly) dy -= m->Ly;
  else if (dy < -0.5 * m->Ly) dy += m->Ly;
  return sqrt((dx * dx + dy * dy) + dz * dz);
}

void om_surface_charge(const omesh* m, const double* E3, const double* phi,
                       int field_mode, int64_t n_atoms, const double* atoms,
                       double r_c, double* faceQ, double* atomq) {
  consts_t K = constants();
  for (int64_t j = 0; j < n_atoms; ++j) atomq[j] = 0.0;
  for (int64_t f = 0; f < m->n_emit; ++f) {
    double Ef[3];
    if (field_mode == 1)
      cell_field(m, m->e_tet[f], phi, Ef);
    else
      face_centroid_field(m, f, E3, Ef);
    /* Eq. face_charge with the sign of E . n (eps0 = 1 / (e/eps0)) */
    double Q = (vdot(Ef, m->e_nrm + 3 * f) / K.e_eps) * m->e_area[f];
    faceQ[f] = Q;
    if (n_atoms == 0) continue;
    const double* abc = m->e_abc + 9 * f;
    double c[3];
    for (int k = 0; k < 3; ++k) c[k] = ((abc[k] + abc[3 + k]) + abc[6 + k]) / 3.0;
    double dmin = face_atom_dist(m, c, atoms);
    for (int64_t j = 1; j < n_atoms; ++j) {
      double d = face_atom_dist(m, c, atoms + 3 * j);
      if (d < dmin) dmin = d;
    }
    double S = 0.0;
    for (int64_t j = 0; j < n_atoms; ++j)
      S += exp(-(face_atom_dist(m, c, atoms + 3 * j) - dmin) / r_c);
    for (int64_t j = 0; j < n_atoms; ++j)
      atomq[j] += (Q * exp(-(face_atom_dist(m, c, atoms + 3 * j) - dmin) / r_c)) / S;
  }
}

/* ------------------------------------------------------------------------ */
/* Binary collisions (App. F).                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t tet;
  uint64_t key;
  int64_t id, idx;
} coll_key;

static int coll_cmp(const void* pa, const void* pb) {
  const coll_key* a = (const coll_key*)pa;
  const coll_key* b = (const coll_key*)pb;
  if (a->tet != b->tet) return a->tet < b->tet ? -1 : 1;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

/* One elastic collision of particles a and b (Eq. vel12 - Eq. variance):
 * nv = n Lambda dt_coll / V of the cell times the variance factor (1, or
 * 1/2 for the odd-count triple); draws from Philox at (step, lead, 4, j). */
static void collide_pair(oparticles* P, int64_t a, int64_t b, double nv,
                         const ocollide_params* prm, int64_t lead, int j) {
  consts_t K = constants();
  double ux = P->vx[b] - P->vx[a];
  double uy = P->vy[b] - P->vy[a];
  double uz = P->vz[b] - P->vz[a];
  double u = sqrt(ux * ux + uy * uy + uz * uz);
  if (!(u > 0.0)) return;
  /* Eq. variance: q^4 / (2 pi eps0^2 m^2) = (q/m)^2 (q/eps0)^2 / (2 pi) */
  double qe = K.qm * K.e_eps;
  double var = qe * qe / (2.0 * PI_) * nv / (u * u * u);
  uint64_t ctr[4] = {(uint64_t)prm->step, (uint64_t)lead, 4, (uint64_t)j}, w[4];
  om_philox4x64(prm->seed, (uint64_t)prm->instance, ctr, w);
  double U1 = 1.0 - u01(w[0]), U2 = u01(w[1]), U3 = u01(w[2]);
  double g = sqrt(-2.0 * log(U1)) * cos(2.0 * PI_ * U2); /* Box-Muller */
  double delta = sqrt(var) * g;
  double st, omc; /* sin theta, 1 - cos theta (Eq. sin_theta) */
  if (delta != delta) delta = 0.0; /* infinite variance times g = 0 */
  if (fabs(delta) < 1e100) {
    st = 2.0 * delta / (1.0 + delta * delta);
    omc = 2.0 * delta * delta / (1.0 + delta * delta);
  } else { /* the same limits without overflow: theta -> pi */
    double r = 1.0 / delta;
    st = 2.0 * r;
    omc = 2.0 - 2.0 * r * r;
  }
  double ph = 2.0 * PI_ * U3;
  double up = sqrt(ux * ux + uy * uy);
  double d[3];
  if (up > 0.0) {
    /* Eq. rot_mat applied to u (Eq. scat_vel) */
    double A = st * sin(ph) * u / up;
    double bx = st * cos(ph) * ux / up, by = st * cos(ph) * uy / up;
    d[0] = -omc * ux + A * uy + bx * uz;
    d[1] = -A * ux - omc * uy + by * uz;
    d[2] = -bx * ux - by * uy - omc * uz;
  } else {
    /* u along z: the azimuth is measured from the x axis */
    d[0] = u * st * cos(ph);
    d[1] = u * st * sin(ph);
    d[2] = -omc * uz;
  }
  P->vx[a] -= 0.5 * d[0];
  P->vy[a] -= 0.5 * d[1];
  P->vz[a] -= 0.5 * d[2];
  P->vx[b] += 0.5 * d[0];
  P->vy[b] += 0.5 * d[1];
  P->vz[b] += 0.5 * d[2];
}

void om_collide(const omesh* m, oparticles* P, const ocollide_params* prm) {
  const double lambda = 13.0; /* Landau logarithm of Eq. variance */
  coll_key* k = (coll_key*)malloc(sizeof(coll_key) * (P->n > 0 ? P->n : 1));
  int64_t n = 0;
  for (int64_t i = 0; i < P->n; ++i) {
    if (P->tet[i] < 0) continue;
    uint64_t ctr[4] = {(uint64_t)prm->step, (uint64_t)P->id[i], 3, 0}, w[4];
    om_philox4x64(prm->seed, (uint64_t)prm->instance, ctr, w);
    k[n].tet = P->tet[i];
    k[n].key = w[0];
    k[n].id = P->id[i];
    k[n].idx = i;
    ++n;
  }
  qsort(k, (size_t)n, sizeof(coll_key), coll_cmp);
  for (int64_t g0 = 0; g0 < n;) {
    int64_t g1 = g0 + 1;
    while (g1 < n && k[g1].tet == k[g0].tet) ++g1;
    int64_t cnt = g1 - g0;
    if (cnt >= 2) {
      double ws = 0.0;
      for (int64_t r = g0; r < g1; ++r) ws += P->w[k[r].idx];
      double V = m->D[k[g0].tet] / 6.0;
      double nv = (prm->w_sp * ws) * lambda * prm->dt_coll / V;
      int64_t r0 = g0;
      if (cnt & 1) {
        /* odd count: the first three collide pairwise at half variance */
        int64_t a = k[g0].idx, b = k[g0 + 1].idx, c = k[g0 + 2].idx;
        collide_pair(P, a, b, 0.5 * nv, prm, k[g0].id, 0);
        collide_pair(P, b, c, 0.5 * nv, prm, k[g0].id, 1);
        collide_pair(P, c, a, 0.5 * nv, prm, k[g0].id, 2);
        r0 = g0 + 3;
      }
      for (int64_t r = r0; r + 1 < g1; r += 2)
        collide_pair(P, k[r].idx, k[r + 1].idx, nv, prm, k[r].id, 0);
    }
    g0 = g1;
  }
  free(k);
}

/* ------------------------------------------------------------------------ */
/* One PIC step (Sec. II B 1-3; Fig. 3 ordering).                            */
/* ------------------------------------------------------------------------ */
static void gather(const omesh* m, int32_t t, const double* p,
                   const double* E3, const double* phi_cell, double* Ep) {
  if (phi_cell) {
    cell_field(m, t, phi_cell, Ep);
    return;
  }
  double lam[4];
  om_lambda(m, t, p, lam);
  const int32_t* tv = m->tet + 4 * (int64_t)t;
  for (int k = 0; k < 3; ++k)
    Ep[k] = ((lam[0] * E3[3 * (int64_t)tv[0] + k] +
              lam[1] * E3[3 * (int64_t)tv[1] + k]) +
             lam[2] * E3[3 * (int64_t)tv[2] + k]) +
            lam[3] * E3[3 * (int64_t)tv[3] + k];
}

static int64_t charge_of(double w) { return llrint(w * 0x1p40); }

/* Injection of one step (Sec. II B 3): per emitting face the FN current at
 * the centroid field, Eq. nsp, the unbiased rounding of Eq. rnd_nsp, then per
 * new superparticle a uniform point on the face (App. E, triangle reading),
 * the initial velocity of Eq. sp_velocity and the fractional push of
 * Eq. sp_displacement.  New particles are appended to P in (face, ordinal)
 * order; face_pts (optional, [cap][3]) receives the sampled face points and
 * counts (optional, [n_emit]) the rounded counts. */
int om_inject(const omesh* m, oparticles* P, const double* E3,
              const ostep_params* prm, ostep_stats* st, double* face_pts,
              int64_t* counts) {
  consts_t K = constants();
  const double dt = prm->dt;
  const double* phi_cell = prm->field_mode == 1 ? prm->phi : NULL;
  double Fsum = 0.0, Fmax = 0.0;
  int64_t n = P->n;
  for (int64_t f = 0; f < m->n_emit; ++f) {
    int cl = 0;
    double F;
    double jd = face_emission(m, f, E3, phi_cell, prm->phi_w, &F, &cl) * prm->j_scale;
    st->n_clamp += cl;
    Fsum += F;
    if (F > Fmax) Fmax = F;
    double cur = jd * m->e_area[f];
    st->emit_current += cur;
    double nsp = cur * dt / prm->w_sp; /* Eq. nsp in e units */
    uint64_t ctr[4] = {(uint64_t)prm->step, (uint64_t)f, 0, 0}, w4[4];
    om_philox4x64(prm->seed, (uint64_t)prm->instance, ctr, w4);
    double R = u01(w4[0]);
    double fl = floor(nsp);
    double cnt = (R >= nsp - fl) ? fl : ceil(nsp); /* Eq. rnd_nsp */
    if (cnt > (double)(1 << 21)) cnt = (double)(1 << 21);
    int64_t cnt_i = prm->counts_in ? prm->counts_in[f] : (int64_t)cnt;
    if (counts) counts[f] = cnt_i;
    if (prm->counts_out) prm->counts_out[f] = cnt_i;
    double s = prm->s_face ? prm->s_face[f] : 1.0;
    const double* A = m->e_abc + 9 * f;
    const double* B = A + 3;
    const double* C = A + 6;
    const int32_t* nd = m->e_nodes + 3 * f;
    for (int64_t o = 0; o < cnt_i; ++o) {
      if (n >= P->cap) {
        st->n_trunc++;
        st->status = -5;
        continue;
      }
      uint64_t c2[4] = {(uint64_t)prm->step, (uint64_t)f, (uint64_t)o, 1};
      om_philox4x64(prm->seed, (uint64_t)prm->instance, c2, w4);
      double R1 = u01(w4[0]), R2 = u01(w4[1]), Rf = u01(w4[2]);
      if (R1 + R2 > 1.0) {
        R1 = 1.0 - R1;
        R2 = 1.0 - R2;
      }
      double l0 = (1.0 - R1) - R2;
      double x[3], Ex[3], v0[3], r[3];
      for (int k = 0; k < 3; ++k) {
        x[k] = (A[k] + R1 * (B[k] - A[k])) + R2 * (C[k] - A[k]);
        Ex[k] = (l0 * E3[3 * (int64_t)nd[0] + k] + R1 * E3[3 * (int64_t)nd[1] + k]) +
                R2 * E3[3 * (int64_t)nd[2] + k];
      }
      if (phi_cell) cell_field(m, m->e_tet[f], phi_cell, Ex);
      double cv = (K.qm * dt) * (0.5 + Rf); /* Eq. sp_velocity */
      for (int k = 0; k < 3; ++k) {
        v0[k] = cv * Ex[k];
        r[k] = x[k] + (v0[k] * dt) * Rf; /* Eq. sp_displacement */
      }
      if (face_pts)
        for (int k = 0; k < 3; ++k) face_pts[3 * n + k] = x[k];
      if (prm->inj_out) {
        double* io = prm->inj_out + 4 * (n - P->n);
        io[0] = R1;
        io[1] = R2;
        io[2] = Rf;
        io[3] = (double)f;
      }
      P->x[n] = r[0];
      P->y[n] = r[1];
      P->z[n] = r[2];
      P->vx[n] = v0[0];
      P->vy[n] = v0[1];
      P->vz[n] = v0[2];
      P->w[n] = s;
      P->tet[n] = m->e_tet[f];
      P->birth[n] = (int32_t)f;
      P->id[n] = (prm->step << 42) | ((int64_t)f << 21) | o;
      st->n_inj++;
      st->q_inj += charge_of(s);
      ++n;
    }
  }
  st->mean_face_E = m->n_emit ? Fsum / (double)m->n_emit : 0.0;
  st->max_face_E = Fmax;
  P->n = n;
  return 0;
}

int om_pic_step(const omesh* m, oparticles* P, double* phi, double* E3,
                int64_t* c, const ostep_params* prm, ostep_stats* st) {
  consts_t K = constants();
  memset(st, 0, sizeof *st);
  const double dt = prm->dt;
  const double Q = (K.qm * dt) * 0.5;
  int64_t n0 = P->n;
  st->n_before = n0;
  for (int64_t i = 0; i < n0; ++i) st->q_before += charge_of(P->w[i]);

  /* 1. gather E_k at r_k and kick: v <- (v + Q E) + Q E (Eq. leapfrog3 of
   *    the previous step followed by Eq. leapfrog1 of this one) */
  ostep_params pr = *prm;  /* the potential of step k for the cell mode */
  pr.phi = phi;
  prm = &pr;
  const double* phi_cell = prm->field_mode == 1 ? phi : NULL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n0; ++i) {
    double p[3] = {P->x[i], P->y[i], P->z[i]}, Ep[3];
    gather(m, P->tet[i], p, E3, phi_cell, Ep);
    double qe0 = Q * Ep[0], qe1 = Q * Ep[1], qe2 = Q * Ep[2];
    P->vx[i] = (P->vx[i] + qe0) + qe0;
    P->vy[i] = (P->vy[i] + qe1) + qe1;
    P->vz[i] = (P->vz[i] + qe2) + qe2;
  }

  /* 2. injection between Eq. leapfrog1 and Eq. leapfrog2 */
  om_inject(m, P, E3, prm, st, NULL, NULL);
  int64_t n = P->n;

  /* 3. drift (Eq. leapfrog2), 4. lateral wrap, absorption, location: each
   *    particle on its own (fate -2: anode, -1: cathode, else its tet),
   *    then the survivors compacted in order */
  int32_t* fate = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    double x = P->x[i] + dt * P->vx[i];
    double y = P->y[i] + dt * P->vy[i];
    double z = P->z[i] + dt * P->vz[i];
    if (x >= m->Lx) x = x - m->Lx;
    else if (x < 0.0) x = x + m->Lx;
    if (y >= m->Ly) y = y - m->Ly;
    else if (y < 0.0) y = y + m->Ly;
    P->x[i] = x;
    P->y[i] = y;
    P->z[i] = z;
    if (z >= m->z_top) {
      fate[i] = -2;
      continue;
    }
    double p[3] = {x, y, z};
    int32_t t = locate_one(m, p, P->tet[i]);
    fate[i] = t < 0 ? -1 : t;
  }
  int64_t out = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t q = charge_of(P->w[i]);
    if (prm->fate_out) prm->fate_out[i] = fate[i] == -2 ? 1 : fate[i] == -1 ? 2 : 0;
    if (fate[i] == -2) {
      st->n_anode++;
      st->q_anode += q;
      continue;
    }
    if (fate[i] == -1) {
      st->n_cathode++;
      st->q_cathode += q;
      continue;
    }
    P->x[out] = P->x[i];
    P->y[out] = P->y[i];
    P->z[out] = P->z[i];
    P->vx[out] = P->vx[i];
    P->vy[out] = P->vy[i];
    P->vz[out] = P->vz[i];
    P->w[out] = P->w[i];
    P->tet[out] = fate[i];
    P->birth[out] = P->birth[i];
    P->id[out] = P->id[i];
    ++out;
  }
  free(fate);
  P->n = out;
  st->n_after = out;
  for (int64_t i = 0; i < out; ++i) st->q_after += charge_of(P->w[i]);

  /* 5. deposition, 6. solve, 7. nodal field */
  memset(c, 0, sizeof(int64_t) * m->n_nodes);
  om_deposit(m, out, P->x, P->y, P->z, P->tet, P->w, c);
  int it = 0;
  double rel = 0;
  int s = om_poisson_solve(m, c, prm->w_sp, prm->E0, phi, prm->tol,
                           prm->max_iter, &it, &rel);
  st->cg_iters = it;
  st->cg_relres = rel;
  if (s != 0 && st->status == 0) st->status = s;
  om_field(m, phi, E3);

  /* 8. binary collisions (App. F) standing for collide_every steps */
  if (prm->collide_every > 0 && (prm->step + 1) % prm->collide_every == 0) {
    ocollide_params cp;
    cp.dt_coll = dt * (double)prm->collide_every;
    cp.w_sp = prm->w_sp;
    cp.seed = prm->seed;
    cp.step = prm->step;
    cp.instance = prm->instance;
    om_collide(m, P, &cp);
  }
  return (int)st->status;
}
