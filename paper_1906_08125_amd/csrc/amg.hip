// Host setup of the smoothed-aggregation AMG hierarchy (Vanek, Mandel and
// Brezina 1996) used as a CG preconditioner for the FP64 Poisson solve:
//   strength  j is strongly coupled to i if |a_ij| >= theta sqrt(a_ii a_jj)
//             (theta = 0.08, halved on every coarser level);
//   aggregates three greedy phases in row order (root + its strong
//             neighbours when none of them is taken; leftovers join the
//             aggregate of a strong neighbour; the rest start new ones);
//   P         Jacobi-smoothed piecewise-constant prolongation
//             P = (I - omega D^-1 A) P0, omega = 4 / (3 lambda_max(D^-1 A))
//             with lambda_max from a power iteration;
//   coarse    A_c = P^T A P (symmetrized), down to at most kAmgCoarseMax
//             rows, whose dense inverse is applied exactly.
// Everything here runs once per mesh handle, on the first solve that asks
// for it; the V-cycle kernels are in solver.hip.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "amg.h"

namespace fp {

namespace {

struct HCsr {
  int64_t n = 0, m = 0;  // rows, columns
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

std::vector<double> diag_of(const HCsr& A) {
  std::vector<double> d(A.n, 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p)
      if (A.ci[p] == i) d[i] += A.v[p];
  return d;
}

HCsr transpose(const HCsr& A) {
  HCsr T;
  T.n = A.m;
  T.m = A.n;
  T.rp.assign(T.n + 1, 0);
  for (int64_t p = 0; p < A.rp[A.n]; ++p) T.rp[A.ci[p] + 1]++;
  for (int64_t i = 0; i < T.n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.rp[A.n]);
  T.v.resize(A.rp[A.n]);
  std::vector<int64_t> fill(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.n; ++i)  // rows in order: columns of T sorted
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      const int64_t q = fill[A.ci[p]]++;
      T.ci[q] = (int32_t)i;
      T.v[q] = A.v[p];
    }
  return T;
}

// C = A B (Gustavson, dense accumulator over the columns of B).
HCsr multiply(const HCsr& A, const HCsr& B) {
  HCsr C;
  C.n = A.n;
  C.m = B.m;
  C.rp.assign(C.n + 1, 0);
  std::vector<double> acc(B.m, 0.0);
  std::vector<int64_t> mark(B.m, -1);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < A.n; ++i) {
    cols.clear();
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      const int32_t k = A.ci[p];
      const double a = A.v[p];
      for (int64_t q = B.rp[k]; q < B.rp[k + 1]; ++q) {
        const int32_t j = B.ci[q];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += a * B.v[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      C.ci.push_back(j);
      C.v.push_back(acc[j]);
    }
    C.rp[i + 1] = (int64_t)C.ci.size();
  }
  return C;
}

// (A + A^T) / 2 for a structurally symmetric A (Galerkin products are).
HCsr symmetrize(const HCsr& A) {
  const HCsr T = transpose(A);
  HCsr S;
  S.n = A.n;
  S.m = A.m;
  S.rp.assign(S.n + 1, 0);
  for (int64_t i = 0; i < A.n; ++i) {
    int64_t p = A.rp[i], q = T.rp[i];
    const int64_t pe = A.rp[i + 1], qe = T.rp[i + 1];
    while (p < pe || q < qe) {
      int32_t j;
      double v = 0.0;
      if (q >= qe || (p < pe && A.ci[p] < T.ci[q])) {
        j = A.ci[p];
        v = 0.5 * A.v[p++];
      } else if (p >= pe || T.ci[q] < A.ci[p]) {
        j = T.ci[q];
        v = 0.5 * T.v[q++];
      } else {
        j = A.ci[p];
        v = 0.5 * (A.v[p++] + T.v[q++]);
      }
      S.ci.push_back(j);
      S.v.push_back(v);
    }
    S.rp[i + 1] = (int64_t)S.ci.size();
  }
  return S;
}

// Aggregate index of every row; nc receives the aggregate count.
std::vector<int32_t> aggregate(const HCsr& A, const std::vector<double>& d,
                               double theta, int64_t& nc) {
  const int64_t n = A.n;
  std::vector<int64_t> sp(n + 1, 0);
  std::vector<int32_t> sn;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      const int32_t j = A.ci[p];
      if (j != i && std::fabs(A.v[p]) >= theta * std::sqrt(std::fabs(d[i] * d[j])))
        sn.push_back(j);
    }
    sp[i + 1] = (int64_t)sn.size();
  }
  std::vector<int32_t> agg(n, -1);
  nc = 0;
  // 1: roots whose strong neighbourhood is untouched
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] != -1 || sp[i] == sp[i + 1]) continue;
    bool free = true;
    for (int64_t p = sp[i]; p < sp[i + 1] && free; ++p) free = agg[sn[p]] == -1;
    if (!free) continue;
    agg[i] = (int32_t)nc;
    for (int64_t p = sp[i]; p < sp[i + 1]; ++p) agg[sn[p]] = (int32_t)nc;
    ++nc;
  }
  // 2: join the phase-1 aggregate of the first strong neighbour
  const std::vector<int32_t> agg1 = agg;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] != -1) continue;
    for (int64_t p = sp[i]; p < sp[i + 1]; ++p)
      if (agg1[sn[p]] != -1) {
        agg[i] = agg1[sn[p]];
        break;
      }
  }
  // 3: the rest start aggregates with their untaken strong neighbours
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] != -1) continue;
    agg[i] = (int32_t)nc;
    for (int64_t p = sp[i]; p < sp[i + 1]; ++p)
      if (agg[sn[p]] == -1) agg[sn[p]] = (int32_t)nc;
    ++nc;
  }
  return agg;
}

// Largest eigenvalue of D^-1 A (power iteration from a fixed start).
double lambda_max(const HCsr& A, const std::vector<double>& d) {
  std::vector<double> x(A.n), y(A.n);
  for (int64_t i = 0; i < A.n; ++i)
    x[i] = 1.0 + (double)((uint32_t)(i * 2654435761u) % 1024u) / 1024.0;
  double lam = 0.0;
  for (int it = 0; it < 30; ++it) {
    double nx = 0.0, ny = 0.0;
    for (int64_t i = 0; i < A.n; ++i) {
      double s = 0.0;
      for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) s += A.v[p] * x[A.ci[p]];
      y[i] = s / d[i];
      nx += x[i] * x[i];
      ny += y[i] * y[i];
    }
    lam = std::sqrt(ny / nx);
    const double sc = 1.0 / std::sqrt(ny);
    for (int64_t i = 0; i < A.n; ++i) x[i] = y[i] * sc;
  }
  return lam;
}

// P = (I - omega D^-1 A) P0 with P0 the aggregate indicator.
HCsr smoothed_p(const HCsr& A, const std::vector<double>& d,
                const std::vector<int32_t>& agg, int64_t nc, double omega) {
  HCsr P;
  P.n = A.n;
  P.m = nc;
  P.rp.assign(A.n + 1, 0);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < A.n; ++i) {
    row.clear();
    row.push_back({agg[i], 1.0});
    const double s = omega / d[i];
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p)
      row.push_back({agg[A.ci[p]], -s * A.v[p]});
    std::stable_sort(row.begin(), row.end(),
              [](const std::pair<int32_t, double>& a,
                 const std::pair<int32_t, double>& b) { return a.first < b.first; });
    for (size_t k = 0; k < row.size();) {
      const int32_t j = row[k].first;
      double v = 0.0;
      while (k < row.size() && row[k].first == j) v += row[k++].second;
      if (v != 0.0) {
        P.ci.push_back(j);
        P.v.push_back(v);
      }
    }
    P.rp[i + 1] = (int64_t)P.ci.size();
  }
  return P;
}

struct HSell {
  int64_t nrows = 0, nslices = 0;
  std::vector<int32_t> sptr, col;
  std::vector<double> val;
};

HSell to_sell(const HCsr& A) {
  HSell S;
  S.nrows = A.n;
  S.nslices = (A.n + kSell - 1) / kSell;
  S.sptr.assign(S.nslices + 1, 0);
  for (int64_t s = 0; s < S.nslices; ++s) {
    int64_t w = 0;
    for (int64_t r = s * kSell; r < std::min<int64_t>(A.n, (s + 1) * kSell); ++r)
      w = std::max(w, A.rp[r + 1] - A.rp[r]);
    S.sptr[s + 1] = (int32_t)(S.sptr[s] + w * kSell);
  }
  const int64_t np = S.sptr[S.nslices];
  S.col.assign(np, 0);
  S.val.assign(np, 0.0);
  for (int64_t s = 0; s < S.nslices; ++s)
    for (int64_t r = s * kSell; r < std::min<int64_t>(A.n, (s + 1) * kSell); ++r)
      for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
        const int64_t p = S.sptr[s] + (k - A.rp[r]) * kSell + (r - s * kSell);
        S.col[p] = A.ci[k];
        S.val[p] = A.v[k];
      }
  return S;
}

// Inverse of a dense SPD matrix (Cholesky, then the inverse from the
// factor); false when a pivot is not positive.
bool spd_inverse(std::vector<double>& a, int64_t n) {
  std::vector<double> L(n * n, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    double s = a[j * n + j];
    for (int64_t k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    L[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double t = a[i * n + j];
      for (int64_t k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / ljj;
    }
  }
  // columns of A^-1: solve L L^T x = e_c
  std::vector<double> y(n);
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      double t = i == c ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; ++k) t -= L[i * n + k] * y[k];
      y[i] = t / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int64_t k = i + 1; k < n; ++k) t -= L[k * n + i] * y[k];
      y[i] = t / L[i * n + i];
    }
    for (int64_t i = 0; i < n; ++i) a[i * n + c] = y[i];
  }
  // exact symmetry of the applied operator
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      const double v = 0.5 * (a[i * n + j] + a[j * n + i]);
      a[i * n + j] = a[j * n + i] = v;
    }
  return true;
}

}  // namespace

hipError_t amg_build(const DevMesh& m, hipStream_t s,
                     void* (*alloc)(void* ctx, size_t bytes), void* ctx,
                     AmgDev& d, std::string& msg) {
  d = AmgDev{};
  hipError_t e;
  // level 0: K on the free nodes, from the device copy
  const int64_t ns = m.k_nslices;
  std::vector<int32_t> sptr(ns + 1);
  if ((e = hipMemcpyAsync(sptr.data(), m.k_sptr, sizeof(int32_t) * (ns + 1),
                          hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return e;
  const int64_t np = sptr[ns];
  std::vector<int32_t> scol(np);
  std::vector<double> sval(np);
  if ((e = hipMemcpyAsync(scol.data(), m.k_scol, sizeof(int32_t) * np,
                          hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(sval.data(), m.k_sval, sizeof(double) * np,
                          hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return e;
  std::vector<HCsr> A(1);
  A[0].n = A[0].m = m.n_free;
  A[0].rp.assign(m.n_free + 1, 0);
  for (int64_t r = 0; r < m.n_free; ++r) {
    const int64_t sl = r / kSell, lane = r % kSell;
    const int64_t w = (sptr[sl + 1] - sptr[sl]) / kSell;
    for (int64_t j = 0; j < w; ++j) {
      const int64_t p = sptr[sl] + j * kSell + lane;
      if (sval[p] != 0.0) {  // (padding entries are zeros)
        A[0].ci.push_back(scol[p]);
        A[0].v.push_back(sval[p]);
      }
    }
    A[0].rp[r + 1] = (int64_t)A[0].ci.size();
  }
  std::vector<HCsr> P, R;
  std::vector<std::vector<double>> diag;
  std::vector<double> omega;
  double theta = 0.08;
  // (at least one level with a smoother: its first kernel holds the
  // stopping test)
  while ((A.back().n > kAmgCoarseMax || P.empty()) &&
         (int)P.size() < kAmgMaxLevels) {
    const HCsr& Al = A.back();
    diag.push_back(diag_of(Al));
    const std::vector<double>& dl = diag.back();
    for (double v : dl)
      if (!(v > 0.0)) {
        msg = "amg: operator diagonal not positive";
        return hipErrorInvalidValue;
      }
    int64_t nc = 0;
    const std::vector<int32_t> agg = aggregate(Al, dl, theta, nc);
    if (nc >= Al.n) break;  // no coarsening possible
    omega.push_back(4.0 / (3.0 * lambda_max(Al, dl)));
    P.push_back(smoothed_p(Al, dl, agg, nc, omega.back()));
    R.push_back(transpose(P.back()));
    const HCsr AP = multiply(Al, P.back());
    A.push_back(symmetrize(multiply(R.back(), AP)));
    theta *= 0.5;
  }
  for (const auto* v : {&A, &P, &R})
    for (const HCsr& M : *v)
      if (M.rp[M.n] >= (int64_t)1 << 31) {
        msg = "amg: level matrix too large for 32-bit offsets";
        return hipErrorInvalidValue;
      }
  const int L = (int)P.size();
  const HCsr& Ac = A.back();
  if (L == 0 || Ac.n > 4 * kAmgCoarseMax) {
    msg = "amg: the operator does not coarsen";
    return hipErrorInvalidValue;
  }
  std::vector<double> dense(Ac.n * Ac.n, 0.0);
  for (int64_t i = 0; i < Ac.n; ++i)
    for (int64_t p = Ac.rp[i]; p < Ac.rp[i + 1]; ++p) dense[i * Ac.n + Ac.ci[p]] = Ac.v[p];
  if (!spd_inverse(dense, Ac.n)) {
    msg = "amg: coarsest operator not positive definite";
    return hipErrorInvalidValue;
  }
  // upload
  auto up = [&](const void* src, size_t bytes) -> void* {
    void* p = alloc(ctx, bytes);
    if (p && bytes &&
        hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
      return nullptr;
    return p;
  };
  // short rows: SELL, one lane per row; long rows: CSR with enough lanes
  // per row that each lane sums a handful of entries
  auto up_sell = [&](const HCsr& M, SellMat& out) -> bool {
    const double avg = M.n ? (double)M.rp[M.n] / (double)M.n : 0.0;
    out.nrows = M.n;
    out.lpr = avg <= 24.0 ? 1 : avg <= 96.0 ? 8 : avg <= 384.0 ? 32 : 64;
    if (out.lpr == 1) {
      const HSell S = to_sell(M);
      out.nslices = S.nslices;
      out.sptr = (const int32_t*)up(S.sptr.data(), sizeof(int32_t) * S.sptr.size());
      out.col = (const int32_t*)up(S.col.data(), sizeof(int32_t) * std::max<size_t>(S.col.size(), 1));
      out.val = (const double*)up(S.val.data(), sizeof(double) * std::max<size_t>(S.val.size(), 1));
      const std::vector<float> v32(S.val.begin(), S.val.end());
      out.val32 = (const float*)up(v32.data(), sizeof(float) * std::max<size_t>(v32.size(), 1));
      // (synchronized before the host copies go out of scope)
      return out.sptr && out.col && out.val && out.val32 &&
             hipStreamSynchronize(s) == hipSuccess;
    }
    std::vector<int32_t> rp(M.rp.begin(), M.rp.end());
    out.nslices = 0;
    out.sptr = (const int32_t*)up(rp.data(), sizeof(int32_t) * rp.size());
    out.col = (const int32_t*)up(M.ci.data(), sizeof(int32_t) * std::max<size_t>(M.ci.size(), 1));
    out.val = (const double*)up(M.v.data(), sizeof(double) * std::max<size_t>(M.v.size(), 1));
    const std::vector<float> v32(M.v.begin(), M.v.end());
    out.val32 = (const float*)up(v32.data(), sizeof(float) * std::max<size_t>(v32.size(), 1));
    return out.sptr && out.col && out.val && out.val32 &&
           hipStreamSynchronize(s) == hipSuccess;
  };
  d.n_levels = L;
  for (int l = 0; l <= L; ++l) d.rows[l] = A[l].n;
  for (int l = 0; l < L; ++l) {
    AmgLevel& lv = d.lv[l];
    if (l == 0) {
      lv.A = SellMat{m.n_free, m.k_nslices, 1, m.k_sptr, m.k_scol, m.k_sval,
                     m.k_sval32};
      lv.invdiag = m.invdiag;
      lv.invdiag32 = m.invdiag32;
    } else {
      if (!up_sell(A[l], lv.A)) return hipErrorOutOfMemory;
      std::vector<double> inv(A[l].n);
      for (int64_t i = 0; i < A[l].n; ++i) inv[i] = 1.0 / diag[l][i];
      const std::vector<float> inv32(inv.begin(), inv.end());
      lv.invdiag = (const double*)up(inv.data(), sizeof(double) * inv.size());
      lv.invdiag32 = (const float*)up(inv32.data(), sizeof(float) * inv32.size());
      if (!lv.invdiag || !lv.invdiag32 || hipStreamSynchronize(s) != hipSuccess)
        return hipErrorOutOfMemory;
    }
    lv.omega = omega[l];
    if (!up_sell(P[l], lv.P) || !up_sell(R[l], lv.R)) return hipErrorOutOfMemory;
    const size_t vb = sizeof(double) * (size_t)A[l].n;
    lv.b = l > 0 ? (double*)alloc(ctx, vb) : nullptr;
    lv.x = (double*)alloc(ctx, vb);
    lv.r = (double*)alloc(ctx, vb);
    lv.t = l > 0 ? (double*)alloc(ctx, vb) : nullptr;
    if (!lv.x || !lv.r || (l > 0 && (!lv.b || !lv.t))) return hipErrorOutOfMemory;
    lv.b32 = l > 0 ? (float*)alloc(ctx, vb / 2) : nullptr;
    lv.x32 = (float*)alloc(ctx, vb / 2);
    lv.r32 = (float*)alloc(ctx, vb / 2);
    lv.t32 = l > 0 ? (float*)alloc(ctx, vb / 2) : nullptr;
    if (!lv.x32 || !lv.r32 || (l > 0 && (!lv.b32 || !lv.t32))) return hipErrorOutOfMemory;
  }
  d.n_coarse = Ac.n;
  d.coarse_inv = (const double*)up(dense.data(), sizeof(double) * dense.size());
  const std::vector<float> dense32(dense.begin(), dense.end());
  d.coarse_inv32 = (const float*)up(dense32.data(), sizeof(float) * dense32.size());
  d.coarse_b = (double*)alloc(ctx, sizeof(double) * Ac.n);
  d.coarse_x = (double*)alloc(ctx, sizeof(double) * Ac.n);
  d.coarse_b32 = (float*)alloc(ctx, sizeof(float) * Ac.n);
  d.coarse_x32 = (float*)alloc(ctx, sizeof(float) * Ac.n);
  if (!d.coarse_inv || !d.coarse_b || !d.coarse_x || !d.coarse_inv32 ||
      !d.coarse_b32 || !d.coarse_x32)
    return hipErrorOutOfMemory;
  AmgDev* dd = (AmgDev*)alloc(ctx, sizeof(AmgDev));
  if (!dd) return hipErrorOutOfMemory;
  d.dev = dd;
  if ((e = hipMemcpyAsync(dd, &d, sizeof d, hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

}  // namespace fp
