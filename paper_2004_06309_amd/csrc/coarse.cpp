// Coarse space of the two-level preconditioner (eq. 2lvl): Z (n x n_c) maps
// the P1 space of a coarse mesh into the fine space, Z[j, l] = phi^H_l(x_j)
// at the position x_j of fine dof j; E = Z^T A Z with the plain transpose.
// Coarse nodes on the Dirichlet top face are not unknowns, fine Dirichlet rows
// of Z are zero and barycentric values below 1e-12 in magnitude are dropped.
#include <omp.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace helm {

namespace {

// Uniform grid of buckets over the coarse mesh; bucket -> overlapping tets.
struct Locator {
  const std::vector<double>& xyz;
  const std::vector<int64_t>& tets;
  double lo[3], w[3];
  int nb;
  std::vector<int64_t> ptr, idx;

  Locator(const std::vector<double>& x, const std::vector<int64_t>& t) : xyz(x), tets(t) {
    const int64_t nt = (int64_t)t.size() / 4, nv = (int64_t)x.size() / 3;
    double hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = 1e300;
      hi[d] = -1e300;
    }
    for (int64_t v = 0; v < nv; ++v)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], x[3 * v + d]);
        hi[d] = std::max(hi[d], x[3 * v + d]);
      }
    nb = std::max(1, (int)std::cbrt((double)nt / 4.0));
    for (int d = 0; d < 3; ++d) w[d] = (hi[d] - lo[d]) / nb + 1e-300;
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (int64_t q = 0; q < nt; ++q) {
      int b0[3], b1[3];
      for (int d = 0; d < 3; ++d) {
        double mn = 1e300, mx = -1e300;
        for (int a = 0; a < 4; ++a) {
          double c = x[3 * t[4 * q + a] + d];
          mn = std::min(mn, c);
          mx = std::max(mx, c);
        }
        b0[d] = clampb((int)std::floor((mn - lo[d]) / w[d] - 1e-9));
        b1[d] = clampb((int)std::floor((mx - lo[d]) / w[d] + 1e-9));
      }
      for (int i = b0[0]; i <= b1[0]; ++i)
        for (int j = b0[1]; j <= b1[1]; ++j)
          for (int k = b0[2]; k <= b1[2]; ++k) pairs.push_back({i + (int64_t)nb * (j + (int64_t)nb * k), q});
    }
    std::sort(pairs.begin(), pairs.end());
    int64_t nbk = (int64_t)nb * nb * nb;
    ptr.assign(nbk + 1, 0);
    idx.resize(pairs.size());
    for (size_t p = 0; p < pairs.size(); ++p) {
      ptr[pairs[p].first + 1]++;
      idx[p] = pairs[p].second;
    }
    for (int64_t b = 0; b < nbk; ++b) ptr[b + 1] += ptr[b];
  }
  int clampb(int v) const { return std::min(std::max(v, 0), nb - 1); }

  int64_t locate(const double* p, double* lam) const {
    int b[3];
    for (int d = 0; d < 3; ++d) b[d] = clampb((int)std::floor((p[d] - lo[d]) / w[d]));
    int64_t key = b[0] + (int64_t)nb * (b[1] + (int64_t)nb * b[2]);
    std::vector<int64_t> cand(idx.begin() + ptr[key], idx.begin() + ptr[key + 1]);
    return locate_point(xyz, tets, p, lam, &cand);
  }
};

}  // namespace

// Builds Z (rows = fine dofs, columns = free coarse nodes in input order) and
// the coordinates of the coarse unknowns.
void coarse_interpolation(const Discretization& D, const helm_mesh& cm, CsrReal& Z, std::vector<double>& ccoords) {
  if (cm.n_nodes <= 0 || cm.n_tets <= 0 || !cm.xyz || !cm.tets) fail(HELM_EINVAL, "empty coarse mesh");
  std::vector<double> cx(cm.xyz, cm.xyz + 3 * cm.n_nodes);
  std::vector<int64_t> ct(cm.tets, cm.tets + 4 * cm.n_tets);
  for (int64_t i = 0; i < 4 * cm.n_tets; ++i)
    if (ct[i] < 0 || ct[i] >= cm.n_nodes) fail(HELM_EINVAL, "coarse tet vertex out of range");
  double ztop = cx[2];
  for (int64_t v = 0; v < cm.n_nodes; ++v) ztop = std::min(ztop, cx[3 * v + 2]);
  std::vector<int32_t> col_of(cm.n_nodes, -1);
  int32_t nc = 0;
  for (int64_t v = 0; v < cm.n_nodes; ++v)
    if (cx[3 * v + 2] != ztop) col_of[v] = nc++;
  ccoords.resize(3 * (size_t)nc);
  for (int64_t v = 0; v < cm.n_nodes; ++v)
    if (col_of[v] >= 0)
      for (int d = 0; d < 3; ++d) ccoords[3 * col_of[v] + d] = cx[3 * v + d];
  Locator loc(cx, ct);
  const int64_t n = D.n;
  std::vector<int32_t> rc((size_t)n * 4, -1);
  std::vector<double> rv((size_t)n * 4, 0.0);
  int missing = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : missing)
  for (int64_t j = 0; j < n; ++j) {
    if (D.dir_mask[j]) continue;
    double p[3], lam[4];
    D.dof_coord(j, p);
    int64_t t = loc.locate(p, lam);
    if (t < 0) {
      ++missing;
      continue;
    }
    for (int a = 0; a < 4; ++a) {
      if (std::fabs(lam[a]) < 1e-12) continue;
      int32_t c = col_of[ct[4 * t + a]];
      if (c < 0) continue;
      rc[4 * j + a] = c;
      rv[4 * j + a] = lam[a];
    }
  }
  if (missing) fail(HELM_EINVAL, std::to_string(missing) + " fine dofs outside the coarse mesh");
  Z = CsrReal();
  Z.n = n;
  Z.m = nc;
  Z.ptr.assign(n + 1, 0);
  for (int64_t j = 0; j < n; ++j) {
    std::pair<int32_t, double> e[4];
    int ne = 0;
    for (int a = 0; a < 4; ++a)
      if (rc[4 * j + a] >= 0) e[ne++] = {rc[4 * j + a], rv[4 * j + a]};
    std::sort(e, e + ne);
    for (int a = 0; a < ne; ++a) {
      Z.col.push_back(e[a].first);
      Z.val.push_back(e[a].second);
    }
    Z.ptr[j + 1] = (int64_t)Z.col.size();
  }
}

void transpose_real(const CsrReal& A, CsrReal& T) {
  T = CsrReal();
  T.n = A.m;
  T.m = A.n;
  T.ptr.assign(T.n + 1, 0);
  for (int64_t p = 0; p < (int64_t)A.col.size(); ++p) T.ptr[A.col[p] + 1]++;
  for (int64_t i = 0; i < T.n; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.col.size());
  T.val.resize(A.col.size());
  std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int64_t q = fill[A.col[p]]++;
      T.col[q] = (int32_t)i;
      T.val[q] = A.val[p];
    }
}

// E = Z^T A Z (n_c x n_c complex CSR, ascending columns).
void galerkin(const Csr& A, const CsrReal& Z, const CsrReal& ZT, Csr& E) {
  const int64_t nc = Z.m;
  E = Csr();
  E.n = E.m = nc;
  std::vector<std::vector<int32_t>> ec(nc);
  std::vector<std::vector<cplx>> ev(nc);
#pragma omp parallel
  {
    std::vector<cplx> acc(nc, cplx(0, 0));
    std::vector<int32_t> mark(nc, -1), list;
#pragma omp for schedule(dynamic, 64)
    for (int64_t l = 0; l < nc; ++l) {
      list.clear();
      for (int64_t p = ZT.ptr[l]; p < ZT.ptr[l + 1]; ++p) {
        int64_t j = ZT.col[p];
        double zl = ZT.val[p];
        for (int64_t q = A.ptr[j]; q < A.ptr[j + 1]; ++q) {
          int64_t k = A.col[q];
          cplx a = zl * A.val[q];
          for (int64_t s = Z.ptr[k]; s < Z.ptr[k + 1]; ++s) {
            int32_t c = Z.col[s];
            if (mark[c] != (int32_t)l) {
              mark[c] = (int32_t)l;
              acc[c] = 0;
              list.push_back(c);
            }
            acc[c] += a * Z.val[s];
          }
        }
      }
      std::sort(list.begin(), list.end());
      ec[l] = list;
      ev[l].resize(list.size());
      for (size_t i = 0; i < list.size(); ++i) ev[l][i] = acc[list[i]];
    }
  }
  E.ptr.assign(nc + 1, 0);
  for (int64_t l = 0; l < nc; ++l) E.ptr[l + 1] = E.ptr[l] + (int64_t)ec[l].size();
  E.col.resize(E.ptr[nc]);
  E.val.resize(E.ptr[nc]);
  for (int64_t l = 0; l < nc; ++l) {
    std::copy(ec[l].begin(), ec[l].end(), E.col.begin() + E.ptr[l]);
    std::copy(ev[l].begin(), ev[l].end(), E.val.begin() + E.ptr[l]);
  }
}

}  // namespace helm
