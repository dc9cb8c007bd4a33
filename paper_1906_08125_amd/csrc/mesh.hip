// mesh_create / mesh_destroy: host preprocessing of the tetrahedral vacuum
// mesh (Sec. II A) and upload of the device records.
//
//  * orientation: exact sign of D, local vertices 2 and 3 swapped when
//    negative; the barycentric map m_k = c_k / D with c_1 = e2 x e3,
//    c_2 = e3 x e1, c_3 = e1 x e2, D = e1 . c_1 (fixed arithmetic);
//  * adjacency: faces matched by node triple plus relative lattice shift,
//    with the frame shift to apply when crossing a periodic face;
//  * boundary: unmatched faces on z = z_top are the Neumann top (Gamma_1),
//    all others metal (Gamma_3, Dirichlet) -- Eq. poisson_bc;
//  * P1 stiffness on free nodes (App. B), Jacobi inverse diagonal, Neumann
//    load per unit E0 (area/3 per top-face vertex), nodal-field operator R
//    (volume-weighted mean of -grad phi over the tets holding a node);
//  * emitting faces (metal faces with centroid z >= emit_zmin) in
//    (owner tet, local face) order, with vertices in ascending local order;
//  * a bucket grid listing every tet in each bucket its closed bounding box
//    touches under the monotone bucket map used by queries.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mesh.h"
#include "particles.h"
#include "solver.h"

namespace fp {

Phys phys_constants() {
  const double e = 1.602176634e-19;
  const double h = 6.62607015e-34;
  const double me = 9.1093837015e-31;
  const double eps0 = 8.8541878128e-12;
  const double pi = 3.14159265358979323846;
  Phys p;
  p.qm = -(e / me) * 1e9 * 1e-21;
  p.e_eps = (e / eps0) * 1e9;
  p.a_fn = e * e / (8.0 * pi * h);
  p.b_fn = (8.0 * pi / 3.0) * std::sqrt(2.0 * me) / (e * h) * std::pow(e, 1.5) / 1e9;
  p.c_s = e / (4.0 * pi * eps0) * 1e9;
  p.j_unit = 1.0 / e * 1e-33;
  return p;
}

namespace {

const int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

struct V3 {
  double x, y, z;
};
inline V3 sub(const double* a, const double* b) {
  return {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
}
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }

// Rounding-error bound of a computed barycentric map, as a multiple of
// u max_j |m_kj| (u = 2^-53): with e_i = v_i - v0, c = e x e and D = e1.c1
// all rounded, and m = c / D rounded, the exact map m* of the exact vertices
// satisfies |m_kj - m*_kj| <= eta_kj, where (standard model, first order
// terms with margin)
//   err(e)   <= u |e|,      err(c_kj) <= 4.01 u P_kj,  P = |a_y b_z| + |a_z b_y|...
//   err(D)   <= 4.02 u (sum_j |e1_j| |c1_j| + sum_j |e1_j| P1_j)
//   eta_kj    = 1.0001 u |m_kj| + (err(c_kj) + (|c_kj| + err(c_kj)) err(D) /
//               (|D| - err(D))) / |D|.
// Returns max_kj eta_kj / (u max_j |m_kj|), or a huge value for a tet whose
// determinant is not resolved (err(D) >= |D| / 2).
inline double lam_error_ratio(V3 e1, V3 e2, V3 e3, const V3 cs[3], double D,
                              const double* m) {
  const double u = 1.1102230246251565e-16;
  auto ab = [](V3 a) { return V3{std::fabs(a.x), std::fabs(a.y), std::fabs(a.z)}; };
  auto pcross = [](V3 a, V3 b) {
    return V3{a.y * b.z + a.z * b.y, a.z * b.x + a.x * b.z, a.x * b.y + a.y * b.x};
  };
  const V3 a1 = ab(e1), a2 = ab(e2), a3 = ab(e3);
  const V3 P[3] = {pcross(a2, a3), pcross(a3, a1), pcross(a1, a2)};
  const V3 c1 = ab(cs[0]);
  const double errD = 4.02 * u *
      ((a1.x * c1.x + a1.y * c1.y + a1.z * c1.z) +
       (a1.x * P[0].x + a1.y * P[0].y + a1.z * P[0].z));
  const double aD = std::fabs(D);
  if (!(errD < 0.5 * aD)) return 1e300;
  double worst = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double ck[3] = {std::fabs(cs[k].x), std::fabs(cs[k].y), std::fabs(cs[k].z)};
    const double pk[3] = {P[k].x, P[k].y, P[k].z};
    double M = 0.0;
    for (int j = 0; j < 3; ++j) M = std::max(M, std::fabs(m[3 * k + j]));
    for (int j = 0; j < 3; ++j) {
      const double ec = 4.01 * u * pk[j];
      const double eta = 1.0001 * u * std::fabs(m[3 * k + j]) +
                         (ec + (ck[j] + ec) * errD / (aD - errD)) / aD;
      worst = std::max(worst, 1.001 * eta / (u * M));
    }
  }
  return worst;
}

struct FaceKey {
  uint64_t hi, lo;
  int32_t tet;
  int8_t face, s0x, s0y, pad;
  bool operator<(const FaceKey& o) const {
    if (hi != o.hi) return hi < o.hi;
    if (lo != o.lo) return lo < o.lo;
    return tet < o.tet;
  }
  bool same(const FaceKey& o) const { return hi == o.hi && lo == o.lo; }
};

// Device memory for a persistent mesh array: from the caller's workspace
// when the handle has one (nothing when only sizes are being added up),
// else allocated and owned by the handle.
void* mesh_mem(pic_mesh* h, size_t bytes, hipError_t& err) {
  if (err != hipSuccess) return nullptr;
  bytes = std::max<size_t>(bytes, 16);
  const size_t at = (h->ws_used + 255) & ~(size_t)255;
  if (h->ws_dry || h->ws_base) {
    h->ws_used = at + bytes;
    h->info.device_bytes += (int64_t)bytes;
    if (h->ws_dry) return nullptr;
    if (h->ws_used > h->ws_size) {
      err = hipErrorOutOfMemory;
      return nullptr;
    }
    return h->ws_base + at;
  }
  void* p = nullptr;
  err = hipMalloc(&p, bytes);
  if (err != hipSuccess) return nullptr;
  h->allocs.push_back(p);
  h->info.device_bytes += (int64_t)bytes;
  return p;
}

template <typename T>
T* upload(pic_mesh* h, const std::vector<T>& v, hipError_t& err) {
  void* p = mesh_mem(h, v.size() * sizeof(T), err);
  if (p && !v.empty())
    err = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return (T*)p;
}

}  // namespace

void* dev_alloc(pic_mesh* h, size_t bytes, hipError_t& err) {
  return mesh_mem(h, bytes, err);
}

pic_status build_mesh(const pic_mesh_desc* d, pic_mesh* h, std::string& msg) {
  const int64_t N = d->n_nodes, T = d->n_tets;
  if (N <= 0 || T <= 0 || !d->xyz || !d->tet) {
    msg = "mesh_create: empty mesh or null arrays";
    return PIC_E_ARG;
  }
  if (!(d->Lx > 0) || !(d->Ly > 0) || !std::isfinite(d->z_top)) {
    msg = "mesh_create: lateral periods must be positive and z_top finite";
    return PIC_E_ARG;
  }
  if (N >= (1ll << 31) || T >= kMaxTets) {
    msg = "mesh_create: more than 2^31 nodes or 2^28 - 1 tets";
    return PIC_E_ARG;
  }
  const double Lx = d->Lx, Ly = d->Ly;
  std::vector<int32_t> tv(d->tet, d->tet + 4 * T);
  std::vector<int8_t> ts(8 * T, 0);
  if (d->shift) std::copy(d->shift, d->shift + 8 * T, ts.begin());
  std::vector<TetWalk> tw(T);
  std::vector<TetGeom> tg(T);
  std::vector<double> D(T);
  // 1. orientation, unwrapped vertices, barycentric maps
  double kappa = 0.0;
  for (int64_t t = 0; t < T; ++t) {
    double v[4][3];
    for (int k = 0; k < 4; ++k) {
      const int32_t nd = tv[4 * t + k];
      if (nd < 0 || nd >= N) {
        msg = "mesh_create: node id out of range in tet " + std::to_string(t);
        return PIC_E_MESH;
      }
      v[k][0] = d->xyz[3 * (int64_t)nd] + (double)ts[8 * t + 2 * k] * Lx;
      v[k][1] = d->xyz[3 * (int64_t)nd + 1] + (double)ts[8 * t + 2 * k + 1] * Ly;
      v[k][2] = d->xyz[3 * (int64_t)nd + 2];
    }
    const int s = vol6_sign(v[0], v[1], v[2], v[3]);
    if (s == 0) {
      msg = "mesh_create: zero-volume tet " + std::to_string(t);
      return PIC_E_MESH;
    }
    if (s < 0) {
      std::swap(tv[4 * t + 2], tv[4 * t + 3]);
      std::swap(ts[8 * t + 4], ts[8 * t + 6]);
      std::swap(ts[8 * t + 5], ts[8 * t + 7]);
      for (int k = 0; k < 3; ++k) std::swap(v[2][k], v[3][k]);
    }
    TetWalk& W = tw[t];
    TetGeom& G = tg[t];
    std::memset(&W, 0, sizeof W);
    std::memset(&G, 0, sizeof G);
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) W.v[3 * k + c] = v[k][c];
    const V3 e1 = sub(v[1], v[0]), e2 = sub(v[2], v[0]), e3 = sub(v[3], v[0]);
    const V3 c1 = cross(e2, e3), c2 = cross(e3, e1), c3 = cross(e1, e2);
    const double det = dot(e1, c1);
    D[t] = det;
    const V3 cs[3] = {c1, c2, c3};
    for (int r = 0; r < 3; ++r) {
      G.m[3 * r + 0] = cs[r].x / det;
      G.m[3 * r + 1] = cs[r].y / det;
      G.m[3 * r + 2] = cs[r].z / det;
    }
    for (int c = 0; c < 3; ++c) G.v0[c] = v[0][c];
    for (int k = 0; k < 4; ++k) G.node[k] = tv[4 * t + k];
    kappa = std::max(kappa, lam_error_ratio(e1, e2, e3, cs, det, G.m));
  }
  // 2. faces and neighbours
  {
    std::vector<FaceKey> keys(4 * T);
    for (int64_t t = 0; t < T; ++t)
      for (int f = 0; f < 4; ++f) {
        int32_t nn[3];
        int sx[3], sy[3];
        for (int j = 0; j < 3; ++j) {
          const int l = kFace[f][j];
          nn[j] = tv[4 * t + l];
          sx[j] = ts[8 * t + 2 * l];
          sy[j] = ts[8 * t + 2 * l + 1];
        }
        int ord[3] = {0, 1, 2};
        std::sort(ord, ord + 3, [&](int a, int b) { return nn[a] < nn[b]; });
        uint32_t code = 0;
        for (int j = 1; j < 3; ++j) {
          const int dx = sx[ord[j]] - sx[ord[0]] + 2;
          const int dy = sy[ord[j]] - sy[ord[0]] + 2;
          code = (code << 6) | (uint32_t)(dx << 3) | (uint32_t)dy;
        }
        FaceKey& k = keys[4 * t + f];
        k.hi = ((uint64_t)(uint32_t)nn[ord[0]] << 32) | (uint32_t)nn[ord[1]];
        k.lo = ((uint64_t)(uint32_t)nn[ord[2]] << 16) | code;
        k.tet = (int32_t)t;
        k.face = (int8_t)f;
        k.s0x = (int8_t)sx[ord[0]];
        k.s0y = (int8_t)sy[ord[0]];
      }
    std::sort(keys.begin(), keys.end());
    int64_t n_top = 0, n_metal = 0;
    for (size_t i = 0; i < keys.size();) {
      size_t j = i + 1;
      while (j < keys.size() && keys[j].same(keys[i])) ++j;
      if (j - i > 2) {
        msg = "mesh_create: non-manifold face";
        return PIC_E_MESH;
      }
      const FaceKey& a = keys[i];
      if (j - i == 2) {
        const FaceKey& b = keys[i + 1];
        tw[a.tet].nbr[a.face] = b.tet;
        tw[b.tet].nbr[b.face] = a.tet;
        tw[a.tet].nsh[2 * a.face] = (int8_t)(b.s0x - a.s0x);
        tw[a.tet].nsh[2 * a.face + 1] = (int8_t)(b.s0y - a.s0y);
        tw[b.tet].nsh[2 * b.face] = (int8_t)(a.s0x - b.s0x);
        tw[b.tet].nsh[2 * b.face + 1] = (int8_t)(a.s0y - b.s0y);
      } else {
        bool top = true;
        for (int q = 0; q < 3; ++q)
          if (tw[a.tet].v[3 * kFace[(int)a.face][q] + 2] != d->z_top) top = false;
        tw[a.tet].nbr[a.face] = top ? -1 : -2;
        if (top) ++n_top; else ++n_metal;
      }
      i = j;
    }
    h->info.n_top = n_top;
    h->info.n_metal = n_metal;
  }
  // neighbours with their frame offsets, packed into the barycentric record
  for (int64_t t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f) {
      const int32_t nb = tw[t].nbr[f];
      if (nb >= 0 && (std::abs(tw[t].nsh[2 * f]) > 1 || std::abs(tw[t].nsh[2 * f + 1]) > 1)) {
        msg = "mesh_create: neighbouring tets more than one period apart";
        return PIC_E_MESH;
      }
      tg[t].nbr[f] = nb < 0 ? kNoNbr
                            : ((uint32_t)nb | ((uint32_t)(tw[t].nsh[2 * f] + 1) << 28) |
                               ((uint32_t)(tw[t].nsh[2 * f + 1] + 1) << 30));
    }
  // 3. Dirichlet nodes and free numbering
  std::vector<char> dir(N, 0);
  for (int64_t t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f)
      if (tw[t].nbr[f] == -2)
        for (int q = 0; q < 3; ++q) dir[tv[4 * t + kFace[f][q]]] = 1;
  std::vector<int32_t> node2free(N, -1), free2node, dir_nodes;
  for (int64_t i = 0; i < N; ++i) {
    if (dir[i]) {
      dir_nodes.push_back((int32_t)i);
    } else {
      node2free[i] = (int32_t)free2node.size();
      free2node.push_back((int32_t)i);
    }
  }
  const int64_t NF = (int64_t)free2node.size();
  // 4. node -> tet lists
  std::vector<int64_t> nt_start(N + 1, 0);
  for (int64_t q = 0; q < 4 * T; ++q) nt_start[tv[q] + 1]++;
  for (int64_t i = 0; i < N; ++i) nt_start[i + 1] += nt_start[i];
  std::vector<int32_t> nt_list(4 * T);
  {
    std::vector<int64_t> fill(nt_start.begin(), nt_start.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int k = 0; k < 4; ++k) nt_list[fill[tv[4 * t + k]]++] = (int32_t)t;
  }
  // 5. rows: K on free rows (free columns), R on all rows (free columns)
  std::vector<int32_t> rowptr(NF + 1, 0), col;
  std::vector<double> val;
  std::vector<int32_t> frow(N + 1, 0), fcol;
  std::vector<double> fv[3];
  std::vector<double> invdiag(NF, 0.0), g_unit(NF, 0.0);
  std::vector<int32_t> nb;
  std::vector<double> kr, rx, ry, rz;
  for (int64_t i = 0; i < N; ++i) {
    nb.clear();
    for (int64_t q = nt_start[i]; q < nt_start[i + 1]; ++q) {
      const int32_t t = nt_list[q];
      for (int k = 0; k < 4; ++k) {
        const int32_t j = node2free[tv[4 * (int64_t)t + k]];
        if (j >= 0) nb.push_back(j);
      }
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    kr.assign(nb.size(), 0.0);
    rx.assign(nb.size(), 0.0);
    ry.assign(nb.size(), 0.0);
    rz.assign(nb.size(), 0.0);
    double Wi = 0.0;
    for (int64_t q = nt_start[i]; q < nt_start[i + 1]; ++q) {
      const int32_t t = nt_list[q];
      const TetGeom& G = tg[t];
      double g[4][3];
      for (int c = 0; c < 3; ++c) {
        g[1][c] = G.m[c];
        g[2][c] = G.m[3 + c];
        g[3][c] = G.m[6 + c];
        g[0][c] = -((G.m[c] + G.m[3 + c]) + G.m[6 + c]);
      }
      const double V = D[t] / 6.0;
      Wi += V;
      int a = 0;
      while (tv[4 * (int64_t)t + a] != i) ++a;
      for (int b = 0; b < 4; ++b) {
        const int32_t j = node2free[tv[4 * (int64_t)t + b]];
        if (j < 0) continue;
        const size_t pos = std::lower_bound(nb.begin(), nb.end(), j) - nb.begin();
        kr[pos] += V * ((g[a][0] * g[b][0] + g[a][1] * g[b][1]) + g[a][2] * g[b][2]);
        rx[pos] -= V * g[b][0];
        ry[pos] -= V * g[b][1];
        rz[pos] -= V * g[b][2];
      }
    }
    for (size_t p = 0; p < nb.size(); ++p) {
      fcol.push_back(nb[p]);
      fv[0].push_back(rx[p] / Wi);
      fv[1].push_back(ry[p] / Wi);
      fv[2].push_back(rz[p] / Wi);
    }
    frow[i + 1] = (int32_t)fcol.size();
    const int32_t fi = node2free[i];
    if (fi >= 0) {
      for (size_t p = 0; p < nb.size(); ++p) {
        col.push_back(nb[p]);
        val.push_back(kr[p]);
        if (nb[p] == fi) invdiag[fi] = 1.0 / kr[p];
      }
      rowptr[fi + 1] = (int32_t)col.size();
    }
  }
  if (col.size() >= (1ull << 31) || fcol.size() >= (1ull << 31)) {
    msg = "mesh_create: matrix too large for 32-bit row pointers";
    return PIC_E_ARG;
  }
  // sliced ELLPACK copies (slices of kSell rows, column-major inside a
  // slice): lane r of a wave reads entry j of row r at sptr[s] + j kSell + r,
  // so every load of a wave is one contiguous run.  Padding entries have
  // value 0 and a valid column.
  auto to_sell = [&](const std::vector<int32_t>& rp, const std::vector<int32_t>& cl,
                     const std::vector<const std::vector<double>*>& vs, int64_t nrows,
                     int32_t pad_col, std::vector<int32_t>& sptr,
                     std::vector<int32_t>& scol, std::vector<double>& sval) {
    const int64_t ns = (nrows + kSell - 1) / kSell;
    sptr.assign(ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) {
      int32_t w = 0;
      for (int64_t r = s * kSell; r < std::min<int64_t>(nrows, (s + 1) * kSell); ++r)
        w = std::max(w, rp[r + 1] - rp[r]);
      sptr[s + 1] = sptr[s] + w * kSell;
    }
    const int64_t np = sptr[ns];
    scol.assign(np, pad_col);
    sval.assign(np * vs.size(), 0.0);
    for (int64_t s = 0; s < ns; ++s)
      for (int64_t r = s * kSell; r < std::min<int64_t>(nrows, (s + 1) * kSell); ++r)
        for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
          const int64_t p = sptr[s] + (int64_t)(k - rp[r]) * kSell + (r - s * kSell);
          scol[p] = cl[k];
          for (size_t q = 0; q < vs.size(); ++q) sval[q * np + p] = (*vs[q])[k];
        }
    return np;
  };
  // R on the free rows in K's column order (both rows list the sorted free
  // neighbours of the node), and R on the Dirichlet rows
  std::vector<double> rf[3];
  for (int64_t fi = 0; fi < NF; ++fi) {
    const int32_t n = free2node[fi];
    for (int32_t p = frow[n]; p < frow[n + 1]; ++p)
      for (int c = 0; c < 3; ++c) rf[c].push_back(fv[c][p]);
  }
  std::vector<int32_t> ncol(col.size());
  for (size_t k = 0; k < col.size(); ++k) ncol[k] = free2node[col[k]];
  const int64_t ND = (int64_t)dir_nodes.size();
  std::vector<int32_t> drow(ND + 1, 0), dcol;
  std::vector<double> dv[3];
  for (int64_t di = 0; di < ND; ++di) {
    const int32_t n = dir_nodes[di];
    for (int32_t p = frow[n]; p < frow[n + 1]; ++p) {
      dcol.push_back(free2node[fcol[p]]);
      for (int c = 0; c < 3; ++c) dv[c].push_back(fv[c][p]);
    }
    drow[di + 1] = (int32_t)dcol.size();
  }
  // R^T: for free row j, the value R_ij at K's slot of (j, i) for free i,
  // and the entries of Dirichlet rows i in a CSR over the free rows j
  std::vector<double> rtv[3];
  for (int c = 0; c < 3; ++c) rtv[c].assign(col.size(), 0.0);
  std::vector<int32_t> trow(NF + 1, 0), tcol;
  std::vector<double> tv3[3];
  {
    for (int64_t i = 0; i < N; ++i) {
      const int32_t fi = node2free[i];
      for (int32_t p = frow[i]; p < frow[i + 1]; ++p) {
        const int32_t j = fcol[p];
        if (fi >= 0) {
          const int32_t* b = col.data() + rowptr[j];
          const int32_t* e = col.data() + rowptr[j + 1];
          const int32_t* hit = std::lower_bound(b, e, fi);
          if (hit == e || *hit != fi) {
            msg = "mesh_create: field operator and stiffness patterns differ";
            return PIC_E_MESH;
          }
          const size_t k = (size_t)(hit - col.data());
          for (int c = 0; c < 3; ++c) rtv[c][k] = fv[c][p];
        } else {
          trow[j + 1]++;
        }
      }
    }
    for (int64_t j = 0; j < NF; ++j) trow[j + 1] += trow[j];
    tcol.assign(trow[NF], 0);
    for (int c = 0; c < 3; ++c) tv3[c].assign(trow[NF], 0.0);
    std::vector<int32_t> fill(trow.begin(), trow.end() - 1);
    for (int64_t i = 0; i < N; ++i) {
      if (node2free[i] >= 0) continue;
      for (int32_t p = frow[i]; p < frow[i + 1]; ++p) {
        const int32_t j = fcol[p];
        const int32_t q = fill[j]++;
        tcol[q] = (int32_t)i;
        for (int c = 0; c < 3; ++c) tv3[c][q] = fv[c][p];
      }
    }
  }
  std::vector<int32_t> k_sptr, k_scol, k_ncol, d_sptr, d_ncol, k_sptr2, t_sptr, t_ncol;
  std::vector<double> rt_sval, t_sval;
  std::vector<double> k_sval, r_sval, d_sval;
  const int64_t k_np = to_sell(rowptr, col, {&val}, NF, 0, k_sptr, k_scol, k_sval);
  {
    to_sell(rowptr, ncol, {&rf[0], &rf[1], &rf[2]}, NF, free2node.empty() ? 0 : free2node[0],
            k_sptr2, k_ncol, r_sval);
  }
  const int64_t d_np = to_sell(drow, dcol, {&dv[0], &dv[1], &dv[2]}, ND,
                               free2node.empty() ? 0 : free2node[0], d_sptr, d_ncol, d_sval);
  {
    std::vector<int32_t> unused_cols;
    to_sell(rowptr, col, {&rtv[0], &rtv[1], &rtv[2]}, NF, 0, k_sptr2, unused_cols, rt_sval);
  }
  const int32_t pad_dir = dir_nodes.empty() ? 0 : dir_nodes[0];
  const int64_t t_np = to_sell(trow, tcol, {&tv3[0], &tv3[1], &tv3[2]}, NF, pad_dir,
                               t_sptr, t_ncol, t_sval);
  if (k_np >= (1ll << 31) || d_np >= (1ll << 31)) {
    msg = "mesh_create: padded matrix too large for 32-bit offsets";
    return PIC_E_ARG;
  }
  // 6. Neumann load per unit E0 on the top plane
  for (int64_t t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f) {
      if (tw[t].nbr[f] != -1) continue;
      const double* A = &tw[t].v[3 * kFace[f][0]];
      const double* B = &tw[t].v[3 * kFace[f][1]];
      const double* C = &tw[t].v[3 * kFace[f][2]];
      const V3 cr = cross(sub(B, A), sub(C, A));
      const double area = 0.5 * std::sqrt(dot(cr, cr));
      for (int q = 0; q < 3; ++q) {
        const int32_t fi = node2free[tv[4 * t + kFace[f][q]]];
        if (fi >= 0) g_unit[fi] += area / 3.0;
      }
    }
  // 7. emitting faces
  std::vector<int32_t> e_tet, e_nodes;
  std::vector<double> e_abc, e_area, e_nrm;
  for (int64_t t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f) {
      if (tw[t].nbr[f] != -2) continue;
      const double* A = &tw[t].v[3 * kFace[f][0]];
      const double* B = &tw[t].v[3 * kFace[f][1]];
      const double* C = &tw[t].v[3 * kFace[f][2]];
      if (!((A[2] + B[2]) + C[2] >= 3.0 * d->emit_zmin)) continue;
      const V3 cr = cross(sub(B, A), sub(C, A));
      const double len = std::sqrt(dot(cr, cr));
      const V3 to = sub(&tw[t].v[3 * f], A);
      const double sg = dot(cr, to) < 0 ? -1.0 : 1.0;
      e_tet.push_back((int32_t)t);
      for (int q = 0; q < 3; ++q) e_nodes.push_back(tv[4 * t + kFace[f][q]]);
      for (const double* P : {A, B, C})
        for (int c = 0; c < 3; ++c) e_abc.push_back(P[c]);
      e_area.push_back(0.5 * len);
      e_nrm.push_back(sg * cr.x / len);
      e_nrm.push_back(sg * cr.y / len);
      e_nrm.push_back(sg * cr.z / len);
    }
  // 8. bucket grid
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  double vol = 0.0;
  for (int64_t t = 0; t < T; ++t) {
    vol += D[t] / 6.0;
    for (int q = 0; q < 12; ++q) {
      lo[q % 3] = std::min(lo[q % 3], tw[t].v[q]);
      hi[q % 3] = std::max(hi[q % 3], tw[t].v[q]);
    }
  }
  DevMesh& M = h->dm;
  const double edge = std::cbrt(6.0 * vol / (double)T);
  for (int k = 0; k < 3; ++k) {
    const double L = hi[k] - lo[k];
    int n = (int)std::ceil(L / edge);
    n = std::max(1, std::min(n, 512));
    M.nb[k] = n;
    M.b0[k] = lo[k];
    M.b1[k] = hi[k];
    M.binv[k] = (double)n / L;
  }
  const int64_t NB = (int64_t)M.nb[0] * M.nb[1] * M.nb[2];
  std::vector<int32_t> bstart(NB + 1, 0), bitem;
  {
    std::vector<int32_t> box(6 * T);
    for (int64_t t = 0; t < T; ++t) {
      for (int k = 0; k < 3; ++k) {
        double a = tw[t].v[k], b = a;
        for (int q = 1; q < 4; ++q) {
          a = std::min(a, tw[t].v[3 * q + k]);
          b = std::max(b, tw[t].v[3 * q + k]);
        }
        box[6 * t + k] = bucket_axis(a, M.b0[k], M.binv[k], M.nb[k]);
        box[6 * t + 3 + k] = bucket_axis(b, M.b0[k], M.binv[k], M.nb[k]);
      }
    }
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int32_t> fill;
      if (pass == 1) fill.assign(bstart.begin(), bstart.end() - 1);
      for (int64_t t = 0; t < T; ++t) {
        const int32_t* b = &box[6 * t];
        for (int x = b[0]; x <= b[3]; ++x)
          for (int y = b[1]; y <= b[4]; ++y)
            for (int z = b[2]; z <= b[5]; ++z) {
              const int64_t id = ((int64_t)x * M.nb[1] + y) * M.nb[2] + z;
              if (pass == 0) bstart[id + 1]++;
              else bitem[fill[id]++] = (int32_t)t;
            }
      }
      if (pass == 0) {
        for (int64_t i = 0; i < NB; ++i) bstart[i + 1] += bstart[i];
        bitem.resize(bstart[NB]);
      }
    }
  }
  // 9. upload
  std::vector<float> invdiag32(invdiag.begin(), invdiag.end());
  std::vector<double4> f_rowsum(N);
  for (int64_t i = 0; i < N; ++i) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t p = frow[i]; p < frow[i + 1]; ++p) {
      sx += fv[0][p];
      sy += fv[1][p];
      sz += fv[2][p];
    }
    f_rowsum[i] = make_double4(sx, sy, sz, 0.0);
  }
  hipError_t err = hipSuccess;
  M.n_nodes = N;
  M.n_tets = T;
  M.n_free = NF;
  M.nnz = (int64_t)col.size();
  M.nnz_field = (int64_t)fcol.size();
  M.n_emit = (int64_t)e_tet.size();
  M.Lx = Lx;
  M.Ly = Ly;
  M.z_top = d->z_top;
  M.tw = upload(h, tw, err);
  M.tg = upload(h, tg, err);
  {
    std::vector<TetGeom32> tg32(T);
    for (int64_t t = 0; t < T; ++t) {
      for (int k = 0; k < 3; ++k) tg32[t].v0[k] = (float)tg[t].v0[k];
      for (int k = 0; k < 9; ++k) tg32[t].m[k] = (float)tg[t].m[k];
      for (int k = 0; k < 4; ++k) tg32[t].node[k] = tg[t].node[k];
    }
    M.tg32 = upload(h, tg32, err);
  }
  M.invdiag = upload(h, invdiag, err);
  M.invdiag32 = upload(h, invdiag32, err);
  M.g_unit = upload(h, g_unit, err);
  M.free2node = upload(h, free2node, err);
  M.node2free = upload(h, node2free, err);
  M.f_rowsum = upload(h, f_rowsum, err);
  M.e_tet = upload(h, e_tet, err);
  M.e_nodes = upload(h, e_nodes, err);
  M.e_abc = upload(h, e_abc, err);
  M.e_area = upload(h, e_area, err);
  {
    std::vector<std::pair<int32_t, int32_t>> nf;  // (node, face)
    for (size_t f = 0; f < e_tet.size(); ++f)
      for (int q = 0; q < 3; ++q) nf.emplace_back(e_nodes[3 * f + q], (int32_t)f);
    std::sort(nf.begin(), nf.end());
    std::vector<int32_t> en_node, en_ptr(1, 0), en_face;
    for (size_t i = 0; i < nf.size(); ++i) {
      if (i == 0 || nf[i].first != nf[i - 1].first) {
        if (i > 0) en_ptr.push_back((int32_t)en_face.size());
        en_node.push_back(nf[i].first);
      }
      en_face.push_back(nf[i].second);
    }
    if (!nf.empty()) en_ptr.push_back((int32_t)en_face.size());
    M.en_n = (int64_t)en_node.size();
    M.en_node = upload(h, en_node, err);
    M.en_ptr = upload(h, en_ptr, err);
    M.en_face = upload(h, en_face, err);
  }
  M.e_nrm = upload(h, e_nrm, err);
  M.bstart = upload(h, bstart, err);
  M.bitem = upload(h, bitem, err);
  {
    std::vector<float> k_sval32(k_sval.begin(), k_sval.end());
    std::vector<float> r_sval32(r_sval.begin(), r_sval.end());
    std::vector<float> d_sval32(d_sval.begin(), d_sval.end());
    M.k_nslices = (int64_t)k_sptr.size() - 1;
    M.k_np = k_np;
    M.k_sptr = upload(h, k_sptr, err);
    M.k_scol = upload(h, k_scol, err);
    M.k_ncol = upload(h, k_ncol, err);
    M.k_sval = upload(h, k_sval, err);
    M.k_sval32 = upload(h, k_sval32, err);
    M.r_sval = upload(h, r_sval, err);
    M.r_sval32 = upload(h, r_sval32, err);
    M.d_nslices = (int64_t)d_sptr.size() - 1;
    M.d_np = d_np;
    M.d_sptr = upload(h, d_sptr, err);
    M.d_ncol = upload(h, d_ncol, err);
    M.d_sval = upload(h, d_sval, err);
    M.d_sval32 = upload(h, d_sval32, err);
    M.rt_sval = upload(h, rt_sval, err);
    M.t_nslices = (int64_t)t_sptr.size() - 1;
    M.t_np = t_np;
    M.t_sptr = upload(h, t_sptr, err);
    M.t_ncol = upload(h, t_ncol, err);
    M.t_sval = upload(h, t_sval, err);
  }
  {
    // walk seeds: lowest-index tet whose centroid lies in each bucket
    std::vector<int32_t> bseed(NB, -1);
    for (int64_t t = 0; t < T; ++t) {
      int b[3];
      for (int k = 0; k < 3; ++k) {
        const double c = ((tw[t].v[k] + tw[t].v[3 + k]) + (tw[t].v[6 + k] + tw[t].v[9 + k])) * 0.25;
        b[k] = bucket_axis(c, M.b0[k], M.binv[k], M.nb[k]);
      }
      const int64_t id = ((int64_t)b[0] * M.nb[1] + b[1]) * M.nb[2] + b[2];
      if (bseed[id] < 0) bseed[id] = (int32_t)t;
    }
    M.bseed = upload(h, bseed, err);
  }
  h->dir_nodes = upload(h, dir_nodes, err);
  h->n_dir = (int64_t)dir_nodes.size();
  // solver scratch
  const size_t vb = sizeof(double) * (size_t)std::max<int64_t>(NF, 1);
  for (int k = 0; k < 7; ++k) h->cg_vec[k] = (double*)dev_alloc(h, vb, err);
  h->cg_bprev = (double*)dev_alloc(h, vb, err);
  for (int k = 0; k < 5; ++k) h->cg_vec32[k] = (float*)dev_alloc(h, vb / 2, err);
  int dev = 0, ncu = 0;
  if (err == hipSuccess) err = hipGetDevice(&dev);
  if (err == hipSuccess) err = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (err == hipSuccess) {
    h->n_cu = ncu;
    // two 512-thread workgroups per CU; every workgroup of the next kernel
    // re-reduces this many partials, so more would cost L2 traffic
    int g = 2 * ncu;
    const int64_t want = std::max<int64_t>(8, (NF + 63) / 64);
    if (g > want) g = (int)want;
    if (g >= 8) g -= g % 8;
    h->cg_grid = std::max(g, 1);
  }
  h->cg_part = (double*)dev_alloc(h, sizeof(double) * kCgSlots * (size_t)std::max(h->cg_grid, 1), err);
  h->cg_ctrl = (CgCtrl*)dev_alloc(h, sizeof(CgCtrl), err);
  // the solver's convergence report: a pinned, device-mapped host record
  // (host metadata of the handle, also with a caller workspace)
  if (err == hipSuccess && !h->ws_dry)
    err = hipHostMalloc((void**)&h->cg_report_host, sizeof(CgReport),
                        hipHostMallocMapped | hipHostMallocCoherent);
  if (err == hipSuccess && !h->ws_dry) {
    std::memset(h->cg_report_host, 0, sizeof(CgReport));
    err = hipHostGetDevicePointer((void**)&h->cg_report_dev, h->cg_report_host, 0);
  }
  if (err == hipSuccess && !h->ws_dry)
    err = hipEventCreateWithFlags(&h->rb_event, hipEventDisableTiming);
  h->scratch = (StepScratch*)dev_alloc(h, sizeof(StepScratch), err);
  h->offsets = (int32_t*)dev_alloc(h, sizeof(int32_t) * (size_t)(M.n_emit + 1), err);
  h->counts = (int32_t*)dev_alloc(h, sizeof(int32_t) * (size_t)(M.n_emit + 1), err);
  h->solve_stats = (pic_solve_stats*)dev_alloc(h, sizeof(pic_solve_stats), err);
  h->locate_count = (int32_t*)dev_alloc(h, sizeof(int32_t), err);
  // fine walk seeds, located on the device with the exact canonical scan
  for (int k = 0; k < 3; ++k) {
    M.fnb[k] = kFineSeed * M.nb[k];
    M.finv[k] = (double)kFineSeed * M.binv[k];
  }
  M.jump_len2 = (0.25 * edge) * (0.25 * edge);
  // |lambda_k - lambda*_k| <= lam_c max_j |m_kj| |d|_1 (see lam_test)
  M.lam_c = (4.01 + 1.01 * kappa) * 1.1102230246251565e-16;
  M.fseed = (int32_t*)dev_alloc(
      h, sizeof(int32_t) * (size_t)M.fnb[0] * M.fnb[1] * M.fnb[2], err);
  if (err == hipSuccess && !h->ws_dry)
    err = launch_seed_build(M, std::max(8, h->n_cu * 8), nullptr);
  if (err == hipSuccess && !h->ws_dry) err = hipDeviceSynchronize();
  h->grid_push = std::max(8, h->n_cu * 8);
  h->grid_inj = std::max(8, h->n_cu * 2);
  h->grid_fb = 64;
  // One workgroup per resident slot: a push grid that fills the chip in a
  // single round has no tail of late workgroups (measured on the production
  // tip: 3 resident per CU, 91 us per push against 100 us for 8 per CU and
  // 107 us for 4), and fewer injecting workgroups queue behind it.
  for (int f32 = 0; f32 < 2; ++f32) {
    const int per_cu = std::max(1, particle_blocks_per_cu(f32));
    int g = std::min(h->grid_push, std::max(8, h->n_cu * per_cu));
    h->step_push[f32] = g >= 8 ? g - g % 8 : g;
  }
  h->step_inj = std::min(h->grid_inj, std::max(8, (h->n_cu / 2) - (h->n_cu / 2) % 8));
  h->acc_rows = (int64_t*)dev_alloc(
      h, sizeof(int64_t) * 16 * (size_t)(h->grid_push + h->grid_inj + h->grid_fb), err);
  if (err == hipErrorOutOfMemory && h->ws_base) {
    msg = "mesh_create_in: the workspace is smaller than mesh_workspace_bytes";
    return PIC_E_ARG;
  }
  if (err != hipSuccess) {
    msg = std::string("mesh_create: ") + hipGetErrorString(err);
    return PIC_E_DEVICE;
  }
  h->h_e_tet = e_tet;
  h->h_e_nodes = e_nodes;
  h->h_e_area = e_area;
  h->info.n_nodes = N;
  h->info.n_tets = T;
  h->info.n_free = NF;
  h->info.nnz = M.nnz;
  h->info.nnz_field = M.nnz_field;
  h->info.n_emit = M.n_emit;
  return PIC_OK;
}

void free_mesh(pic_mesh* h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  if (h->cg_report_host) (void)hipHostFree(h->cg_report_host);
  h->cg_report_host = nullptr;
  if (h->rb_event) (void)hipEventDestroy(h->rb_event);
  h->rb_event = nullptr;
}

}  // namespace fp
