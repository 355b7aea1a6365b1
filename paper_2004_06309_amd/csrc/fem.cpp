// Finite-element discretisation of (Delta + k^2) u = b (eqs. eqh and eq1):
// Lagrange P1/P2 on tetrahedra, A = -K + M_{k^2} + i B_k, Dirichlet top face
// (z = min z) and first-order absorbing faces elsewhere (exp(-i omega t), so
// d_n u = i k u).  Element matrices use the closed forms of the integrals of
// products of barycentric coordinates, int_T l_p l_q = |T| (1 + d_pq) / 20,
// int_T l_p = |T| / 4, which make every entry exact.
#include <omp.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace helm {

namespace {

// local edges of a tet in P2 order
constexpr int kEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
// local edges of a face (sorted vertices f0 < f1 < f2)
constexpr int kFaceEdge[3][2] = {{0, 1}, {0, 2}, {1, 2}};
// faces of a tet: the vertices opposite to vertex 0..3
constexpr int kTetFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

inline double d3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Barycentric gradients g[4][3] and signed det of [x1-x0, x2-x0, x3-x0].
double tet_gradients(const double* X, double g[4][3]) {
  double J[3][3];
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) J[d][c] = X[3 * (c + 1) + d] - X[d];
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  if (det == 0) return 0;
  // inverse via cofactors: rows of J^{-1} are grad lambda_1..3
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) g[k + 1][d] = inv[k][d];
  for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
  return det;
}

// Element stiffness/mass for unit coefficients.
void element_p1(double vol, const double G[4][4], double* K, double* M) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      K[a * 4 + b] = vol * G[a][b];
      M[a * 4 + b] = vol * (a == b ? 2.0 : 1.0) / 20.0;
    }
}

void element_p2(double vol, const double G[4][4], double* K, double* M) {
  auto dl = [](int p, int q) { return p == q ? 1.0 : 0.0; };
  // stiffness: grad phi_vi = (4 l_i - 1) grad l_i, grad phi_ab = 4 (l_a grad l_b + l_b grad l_a)
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) K[i * 10 + j] = vol * G[i][j] * (i == j ? 0.6 : -0.2);
    for (int e = 0; e < 6; ++e) {
      int a = kEdge[e][0], b = kEdge[e][1];
      auto c = [&](int p) { return p == i ? 3.0 / 20.0 : -1.0 / 20.0; };
      double v = 4.0 * vol * (G[i][b] * c(a) + G[i][a] * c(b));
      K[i * 10 + 4 + e] = v;
      K[(4 + e) * 10 + i] = v;
    }
  }
  for (int e = 0; e < 6; ++e)
    for (int f = 0; f < 6; ++f) {
      int a = kEdge[e][0], b = kEdge[e][1], c = kEdge[f][0], d = kEdge[f][1];
      K[(4 + e) * 10 + 4 + f] = 16.0 * vol / 20.0 *
                                (G[b][d] * (1 + dl(a, c)) + G[b][c] * (1 + dl(a, d)) +
                                 G[a][d] * (1 + dl(b, c)) + G[a][c] * (1 + dl(b, d)));
    }
  // mass: |T|/420 x {vv: 6 | 1, ve: -4 (vertex on edge) | -6, ee: 32 | 16 (shared vertex) | 8}
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) M[i * 10 + j] = vol / 420.0 * (i == j ? 6.0 : 1.0);
    for (int e = 0; e < 6; ++e) {
      bool on = kEdge[e][0] == i || kEdge[e][1] == i;
      double v = vol / 420.0 * (on ? -4.0 : -6.0);
      M[i * 10 + 4 + e] = v;
      M[(4 + e) * 10 + i] = v;
    }
  }
  for (int e = 0; e < 6; ++e)
    for (int f = 0; f < 6; ++f) {
      int shared = (kEdge[e][0] == kEdge[f][0]) + (kEdge[e][0] == kEdge[f][1]) + (kEdge[e][1] == kEdge[f][0]) +
                   (kEdge[e][1] == kEdge[f][1]);
      double v = e == f ? 32.0 : (shared ? 16.0 : 8.0);
      M[(4 + e) * 10 + 4 + f] = vol / 420.0 * v;
    }
}

struct FaceKey {
  int64_t v[3];
  int64_t tet;
  bool operator<(const FaceKey& o) const {
    if (v[0] != o.v[0]) return v[0] < o.v[0];
    if (v[1] != o.v[1]) return v[1] < o.v[1];
    if (v[2] != o.v[2]) return v[2] < o.v[2];
    return tet < o.tet;
  }
  bool same(const FaceKey& o) const { return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2]; }
};

}  // namespace

void face_matrix(int order, double area, double* B) {
  if (order == 1) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) B[a * 3 + b] = area * (a == b ? 2.0 : 1.0) / 12.0;
    return;
  }
  // |F|/180 x {vv: 6 | -1, ve: 0 (vertex on edge) | -4, ee: 32 | 16}
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) B[i * 6 + j] = area / 180.0 * (i == j ? 6.0 : -1.0);
    for (int e = 0; e < 3; ++e) {
      bool on = kFaceEdge[e][0] == i || kFaceEdge[e][1] == i;
      double v = on ? 0.0 : -4.0 * area / 180.0;
      B[i * 6 + 3 + e] = v;
      B[(3 + e) * 6 + i] = v;
    }
  }
  for (int e = 0; e < 3; ++e)
    for (int f = 0; f < 3; ++f) B[(3 + e) * 6 + 3 + f] = area / 180.0 * (e == f ? 32.0 : 16.0);
}

void basis_values(int order, const double* lam, double* phi) {
  if (order == 1) {
    for (int i = 0; i < 4; ++i) phi[i] = lam[i];
    return;
  }
  for (int i = 0; i < 4; ++i) phi[i] = lam[i] * (2.0 * lam[i] - 1.0);
  for (int e = 0; e < 6; ++e) phi[4 + e] = 4.0 * lam[kEdge[e][0]] * lam[kEdge[e][1]];
}

int64_t Discretization::edge_id(int64_t a, int64_t b) const {
  int64_t lo = std::min(a, b), hi = std::max(a, b);
  // edges sorted lexicographically: binary search
  int64_t l = 0, r = ne;
  while (l < r) {
    int64_t m = (l + r) / 2;
    const int64_t* e = &edges[2 * m];
    if (e[0] < lo || (e[0] == lo && e[1] < hi))
      l = m + 1;
    else
      r = m;
  }
  if (l >= ne || edges[2 * l] != lo || edges[2 * l + 1] != hi) fail(HELM_EINVAL, "edge not found");
  return nv + l;
}

void Discretization::face_dofs(const int64_t* f, int64_t* out) const {
  out[0] = f[0];
  out[1] = f[1];
  out[2] = f[2];
  if (order == 2)
    for (int e = 0; e < 3; ++e) out[3 + e] = edge_id(f[kFaceEdge[e][0]], f[kFaceEdge[e][1]]);
}

double Discretization::face_area(const int64_t* f) const {
  const double *a = &xyz[3 * f[0]], *b = &xyz[3 * f[1]], *c = &xyz[3 * f[2]];
  double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  double w[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  return 0.5 * std::sqrt(d3(w, w));
}

void Discretization::dof_coord(int64_t d, double* x) const {
  if (d < nv) {
    for (int k = 0; k < 3; ++k) x[k] = xyz[3 * d + k];
  } else {
    const int64_t* e = &edges[2 * (d - nv)];
    for (int k = 0; k < 3; ++k) x[k] = 0.5 * (xyz[3 * e[0] + k] + xyz[3 * e[1] + k]);
  }
}

void build_discretization(Discretization& D, const helm_mesh& mesh, const double* c_tet, double omega) {
  if (mesh.order != 1 && mesh.order != 2) fail(HELM_EINVAL, "order must be 1 or 2");
  if (mesh.n_nodes <= 0 || mesh.n_tets <= 0 || !mesh.xyz || !mesh.tets) fail(HELM_EINVAL, "empty mesh");
  D = Discretization();
  D.order = mesh.order;
  D.nloc = mesh.order == 1 ? 4 : 10;
  D.nfloc = mesh.order == 1 ? 3 : 6;
  D.nv = mesh.n_nodes;
  D.nt = mesh.n_tets;
  D.omega = omega;
  D.xyz.assign(mesh.xyz, mesh.xyz + 3 * D.nv);
  D.tets.assign(mesh.tets, mesh.tets + 4 * D.nt);
  const int64_t nt = D.nt, nv = D.nv;
  for (int64_t i = 0; i < 4 * nt; ++i)
    if (D.tets[i] < 0 || D.tets[i] >= nv) fail(HELM_EINVAL, "tet vertex index out of range");
  D.ztop = D.xyz[2];
  for (int64_t v = 0; v < nv; ++v) D.ztop = std::min(D.ztop, D.xyz[3 * v + 2]);

  // geometry, orientation, element matrices
  const int nl = D.nloc;
  D.vol.resize(nt);
  D.Ke.resize((size_t)nt * nl * nl);
  D.Me.resize((size_t)nt * nl * nl);
  D.k.resize(nt);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t t = 0; t < nt; ++t) {
    int64_t* tv = &D.tets[4 * t];
    double X[12];
    for (int a = 0; a < 4; ++a)
      for (int d = 0; d < 3; ++d) X[3 * a + d] = D.xyz[3 * tv[a] + d];
    double g[4][3];
    double det = tet_gradients(X, g);
    double hmax = 0;
    for (int e = 0; e < 6; ++e) {
      double s = 0;
      for (int d = 0; d < 3; ++d) {
        double q = X[3 * kEdge[e][0] + d] - X[3 * kEdge[e][1] + d];
        s += q * q;
      }
      hmax = std::max(hmax, s);
    }
    if (!(std::fabs(det) > 1e-12 * hmax * std::sqrt(hmax))) {
      ++bad;
      continue;
    }
    if (det < 0) {  // re-orient: swap vertices 2 and 3
      std::swap(tv[2], tv[3]);
      std::swap(g[2][0], g[3][0]);
      std::swap(g[2][1], g[3][1]);
      std::swap(g[2][2], g[3][2]);
      det = -det;
    }
    double vol = det / 6.0;
    D.vol[t] = vol;
    double G[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) G[a][b] = d3(g[a], g[b]);
    if (D.order == 1)
      element_p1(vol, G, &D.Ke[(size_t)t * 16], &D.Me[(size_t)t * 16]);
    else
      element_p2(vol, G, &D.Ke[(size_t)t * 100], &D.Me[(size_t)t * 100]);
    cplx c(c_tet[2 * t], c_tet[2 * t + 1]);
    D.k[t] = omega / c;
  }
  if (bad) fail(HELM_EINVAL, std::to_string(bad) + " degenerate tet(s)");
  for (int64_t t = 0; t < nt; ++t)
    if (c_tet[2 * t] == 0 && c_tet[2 * t + 1] == 0) fail(HELM_EINVAL, "zero velocity");

  // edges (P2): sorted unique (min, max) pairs
  if (D.order == 2) {
    std::vector<std::pair<int64_t, int64_t>> all((size_t)nt * 6);
    for (int64_t t = 0; t < nt; ++t)
      for (int e = 0; e < 6; ++e) {
        int64_t a = D.tets[4 * t + kEdge[e][0]], b = D.tets[4 * t + kEdge[e][1]];
        all[6 * t + e] = {std::min(a, b), std::max(a, b)};
      }
    std::vector<std::pair<int64_t, int64_t>> u = all;
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    D.ne = (int64_t)u.size();
    D.edges.resize(2 * D.ne);
    for (int64_t i = 0; i < D.ne; ++i) {
      D.edges[2 * i] = u[i].first;
      D.edges[2 * i + 1] = u[i].second;
    }
    D.tet_dofs.resize((size_t)nt * 10);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
      for (int a = 0; a < 4; ++a) D.tet_dofs[10 * t + a] = D.tets[4 * t + a];
      for (int e = 0; e < 6; ++e) {
        auto it = std::lower_bound(u.begin(), u.end(), all[6 * t + e]);
        D.tet_dofs[10 * t + 4 + e] = nv + (it - u.begin());
      }
    }
  } else {
    D.ne = 0;
    D.tet_dofs = D.tets;
  }
  D.n = D.nv + D.ne;

  // boundary faces
  std::vector<FaceKey> fk((size_t)nt * 4);
  for (int64_t t = 0; t < nt; ++t)
    for (int f = 0; f < 4; ++f) {
      FaceKey& k = fk[4 * t + f];
      for (int q = 0; q < 3; ++q) k.v[q] = D.tets[4 * t + kTetFace[f][q]];
      std::sort(k.v, k.v + 3);
      k.tet = t;
    }
  std::sort(fk.begin(), fk.end());
  for (size_t i = 0; i < fk.size();) {
    size_t j = i + 1;
    while (j < fk.size() && fk[j].same(fk[i])) ++j;
    if (j - i > 2) fail(HELM_EINVAL, "face shared by more than two tets");
    if (j - i == 1) {
      for (int q = 0; q < 3; ++q) D.bface.push_back(fk[i].v[q]);
      D.bowner.push_back(fk[i].tet);
      bool top = true;
      for (int q = 0; q < 3; ++q) top = top && D.xyz[3 * fk[i].v[q] + 2] == D.ztop;
      D.bdir.push_back(top ? 1 : 0);
    }
    i = j;
  }
  D.dir_mask.assign(D.n, 0);
  const int64_t nb = (int64_t)D.bowner.size();
  for (int64_t f = 0; f < nb; ++f)
    if (D.bdir[f]) {
      int64_t fd[6];
      D.face_dofs(&D.bface[3 * f], fd);
      for (int q = 0; q < D.nfloc; ++q) D.dir_mask[fd[q]] = 1;
    }

  // global matrix: all tets, absorbing faces, all dofs
  std::vector<int64_t> all_tets(nt);
  std::iota(all_tets.begin(), all_tets.end(), 0);
  std::vector<ImpFace> faces;
  for (int64_t f = 0; f < nb; ++f)
    if (!D.bdir[f]) faces.push_back({{D.bface[3 * f], D.bface[3 * f + 1], D.bface[3 * f + 2]}, D.bowner[f]});
  std::vector<int64_t> all_dofs(D.n);
  std::iota(all_dofs.begin(), all_dofs.end(), 0);
  assemble_local(D, all_tets, faces, all_dofs, D.A);
}

void assemble_local(const Discretization& D, const std::vector<int64_t>& tet_list,
                    const std::vector<ImpFace>& faces, const std::vector<int64_t>& dofs, Csr& out) {
  const int nl = D.nloc, nfl = D.nfloc;
  const int64_t nloc_dofs = (int64_t)dofs.size();
  const bool identity_map = nloc_dofs == D.n;
  auto lid = [&](int64_t g) -> int64_t {
    if (identity_map) return g;
    auto it = std::lower_bound(dofs.begin(), dofs.end(), g);
    if (it == dofs.end() || *it != g) return -1;
    return it - dofs.begin();
  };
  const int64_t ntl = (int64_t)tet_list.size(), nfc = (int64_t)faces.size();
  // local dofs of every listed tet and face
  std::vector<int32_t> tl((size_t)ntl * nl);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ntl; ++i)
    for (int a = 0; a < nl; ++a) {
      int64_t l = lid(D.tet_dofs[(size_t)tet_list[i] * nl + a]);
      tl[(size_t)i * nl + a] = (int32_t)l;
    }
  for (int64_t i = 0; i < ntl * nl; ++i)
    if (tl[i] < 0) fail(HELM_EINVAL, "tet dof outside the local dof list");
  std::vector<int32_t> fl((size_t)nfc * nfl);
  std::vector<double> fB((size_t)nfc * nfl * nfl);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nfc; ++i) {
    int64_t fd[6];
    D.face_dofs(faces[i].v, fd);
    for (int a = 0; a < nfl; ++a) fl[(size_t)i * nfl + a] = (int32_t)lid(fd[a]);
    face_matrix(D.order, D.face_area(faces[i].v), &fB[(size_t)i * nfl * nfl]);
  }
  // row -> (tet, local index) and row -> (face, local index), in list order
  auto invert = [&](const std::vector<int32_t>& ent, int per, std::vector<int64_t>& ptr, std::vector<int64_t>& idx) {
    ptr.assign(nloc_dofs + 1, 0);
    for (size_t e = 0; e < ent.size(); ++e)
      if (ent[e] >= 0) ptr[ent[e] + 1]++;
    for (int64_t r = 0; r < nloc_dofs; ++r) ptr[r + 1] += ptr[r];
    idx.resize(ptr[nloc_dofs]);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t e = 0; e < ent.size(); ++e)
      if (ent[e] >= 0) idx[fill[ent[e]]++] = (int64_t)e;  // e = item * per + a
    (void)per;
  };
  std::vector<int64_t> rt_ptr, rt_idx, rf_ptr, rf_idx;
  invert(tl, nl, rt_ptr, rt_idx);
  invert(fl, nfl, rf_ptr, rf_idx);
  // pattern
  out = Csr();
  out.n = out.m = nloc_dofs;
  out.ptr.assign(nloc_dofs + 1, 0);
  std::vector<std::vector<int32_t>> rowcols(nloc_dofs);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < nloc_dofs; ++r) {
    std::vector<int32_t>& c = rowcols[r];
    if (D.dir_mask[dofs[r]]) {
      c.push_back((int32_t)r);
      continue;
    }
    for (int64_t p = rt_ptr[r]; p < rt_ptr[r + 1]; ++p) {
      int64_t item = rt_idx[p] / nl;
      for (int b = 0; b < nl; ++b) {
        int32_t cc = tl[item * nl + b];
        if (!D.dir_mask[dofs[cc]]) c.push_back(cc);
      }
    }
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
  }
  for (int64_t r = 0; r < nloc_dofs; ++r) out.ptr[r + 1] = out.ptr[r] + (int64_t)rowcols[r].size();
  out.col.resize(out.ptr[nloc_dofs]);
  out.val.assign(out.ptr[nloc_dofs], cplx(0, 0));
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < nloc_dofs; ++r) {
    std::vector<int32_t>& c = rowcols[r];
    std::copy(c.begin(), c.end(), out.col.begin() + out.ptr[r]);
    cplx* v = &out.val[out.ptr[r]];
    auto pos = [&](int32_t cc) { return std::lower_bound(c.begin(), c.end(), cc) - c.begin(); };
    if (D.dir_mask[dofs[r]]) {
      v[0] = 1.0;
    } else {
      for (int64_t p = rt_ptr[r]; p < rt_ptr[r + 1]; ++p) {
        int64_t item = rt_idx[p] / nl;
        int a = (int)(rt_idx[p] % nl);
        int64_t t = tet_list[item];
        cplx k2 = D.k[t] * D.k[t];
        const double* K = &D.Ke[(size_t)t * nl * nl + a * nl];
        const double* M = &D.Me[(size_t)t * nl * nl + a * nl];
        for (int b = 0; b < nl; ++b) {
          int32_t cc = tl[item * nl + b];
          if (D.dir_mask[dofs[cc]]) continue;
          v[pos(cc)] += -K[b] + k2 * M[b];
        }
      }
      for (int64_t p = rf_ptr[r]; p < rf_ptr[r + 1]; ++p) {
        int64_t item = rf_idx[p] / nfl;
        int a = (int)(rf_idx[p] % nfl);
        cplx ik = cplx(0, 1) * D.k[faces[item].owner];
        const double* B = &fB[(size_t)item * nfl * nfl + a * nfl];
        for (int b = 0; b < nfl; ++b) {
          int32_t cc = fl[item * nfl + b];
          if (cc < 0 || D.dir_mask[dofs[cc]]) continue;
          auto q = pos(cc);
          if (q >= (int64_t)c.size() || c[q] != cc) continue;  // face dof outside the tet pattern
          v[q] += ik * B[b];
        }
      }
    }
    std::vector<int32_t>().swap(c);
  }
}

int64_t locate_point(const std::vector<double>& xyz, const std::vector<int64_t>& tets, const double* p,
                     double* lam, const std::vector<int64_t>* candidates) {
  // first tet (in list order) whose barycentric coordinates are all >= -1e-10
  const int64_t nt = candidates ? (int64_t)candidates->size() : (int64_t)tets.size() / 4;
  for (int64_t i = 0; i < nt; ++i) {
    int64_t t = candidates ? (*candidates)[i] : i;
    double X[12];
    for (int a = 0; a < 4; ++a)
      for (int d = 0; d < 3; ++d) X[3 * a + d] = xyz[3 * tets[4 * t + a] + d];
    double g[4][3];
    if (tet_gradients(X, g) == 0) continue;
    double l[4];
    for (int a = 1; a < 4; ++a)
      l[a] = g[a][0] * (p[0] - X[0]) + g[a][1] * (p[1] - X[1]) + g[a][2] * (p[2] - X[2]);
    l[0] = 1.0 - l[1] - l[2] - l[3];
    if (l[0] >= -1e-10 && l[1] >= -1e-10 && l[2] >= -1e-10 && l[3] >= -1e-10) {
      for (int a = 0; a < 4; ++a) lam[a] = l[a];
      return t;
    }
  }
  return -1;
}

}  // namespace helm
