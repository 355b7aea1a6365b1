// Overlapping decomposition for the one-level ORAS preconditioner (eq. oras):
// subdomains Gamma_i grown from a non-overlapping tet partition by layers of
// vertex-adjacent tets, Boolean restrictions R_i (sorted global dof lists),
// partition-of-unity weights D_i, and local Helmholtz matrices A_i carrying the
// first-order impedance condition on their artificial interface faces.
//
// Partition of unity: l(j) is the first overlap layer whose tets contain dof
// j, chi_i(j) = max(0, 1 - l(j)/overlap) (1 when overlap = 0), and
// D_i(j) = chi_i(j) / sum_k chi_k(j).  D_i vanishes on the artificial
// interface, where l(j) = overlap.
#include <omp.h>

#include <algorithm>
#include <numeric>

#include "internal.hpp"

namespace helm {

namespace {
constexpr int kTetFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

struct FK {
  int64_t v[3];
  int64_t tet;
  bool operator<(const FK& o) const {
    if (v[0] != o.v[0]) return v[0] < o.v[0];
    if (v[1] != o.v[1]) return v[1] < o.v[1];
    return v[2] < o.v[2];
  }
  bool same(const FK& o) const { return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2]; }
};
}  // namespace

void build_subdomains(const Discretization& D, const int32_t* part, int32_t n_sub, int32_t overlap,
                      std::vector<SubdomainHost>& subs) {
  const int64_t nt = D.nt, nv = D.nv, n = D.n;
  const int nl = D.nloc;
  if (n_sub <= 0) fail(HELM_EINVAL, "n_sub must be positive");
  if (overlap < 0) fail(HELM_EINVAL, "overlap must be >= 0");
  for (int64_t t = 0; t < nt; ++t)
    if (part[t] < 0 || part[t] >= n_sub) fail(HELM_EINVAL, "tet_part entry out of range");
  // vertex -> tets
  std::vector<int64_t> v2t_ptr(nv + 1, 0), v2t(4 * nt);
  for (int64_t i = 0; i < 4 * nt; ++i) v2t_ptr[D.tets[i] + 1]++;
  for (int64_t v = 0; v < nv; ++v) v2t_ptr[v + 1] += v2t_ptr[v];
  {
    std::vector<int64_t> fill(v2t_ptr.begin(), v2t_ptr.end() - 1);
    for (int64_t i = 0; i < 4 * nt; ++i) v2t[fill[D.tets[i]]++] = i / 4;
  }
  // tets of each part
  std::vector<std::vector<int64_t>> part_tets(n_sub);
  for (int64_t t = 0; t < nt; ++t) part_tets[part[t]].push_back(t);
  for (int32_t i = 0; i < n_sub; ++i)
    if (part_tets[i].empty()) fail(HELM_EINVAL, "empty subdomain " + std::to_string(i));
  // sorted global boundary faces for the artificial/physical test
  const int64_t nb = (int64_t)D.bowner.size();
  std::vector<FK> bfk(nb);
  for (int64_t f = 0; f < nb; ++f) {
    for (int q = 0; q < 3; ++q) bfk[f].v[q] = D.bface[3 * f + q];
    bfk[f].tet = f;  // index of the boundary face
  }
  std::sort(bfk.begin(), bfk.end());

  subs.assign(n_sub, SubdomainHost());
#pragma omp parallel
  {
    std::vector<int32_t> layer(nt, -1);
    std::vector<int32_t> lev(n, -1);
    std::vector<uint8_t> vmark(nv, 0);
#pragma omp for schedule(dynamic, 1)
    for (int32_t i = 0; i < n_sub; ++i) {
      SubdomainHost& S = subs[i];
      std::vector<int64_t> cur = part_tets[i];
      for (int64_t t : cur) layer[t] = 0;
      for (int32_t l = 1; l <= overlap; ++l) {
        std::vector<int64_t> verts;
        for (int64_t t : cur)
          for (int a = 0; a < 4; ++a) {
            int64_t v = D.tets[4 * t + a];
            if (!vmark[v]) {
              vmark[v] = 1;
              verts.push_back(v);
            }
          }
        for (int64_t v : verts) {
          vmark[v] = 0;
          for (int64_t p = v2t_ptr[v]; p < v2t_ptr[v + 1]; ++p) {
            int64_t t = v2t[p];
            if (layer[t] < 0) {
              layer[t] = l;
              cur.push_back(t);
            }
          }
        }
      }
      std::sort(cur.begin(), cur.end());
      S.tets = cur;
      // dofs and their first layer
      std::vector<int64_t> dl;
      for (int64_t t : cur)
        for (int a = 0; a < nl; ++a) {
          int64_t d = D.tet_dofs[(size_t)t * nl + a];
          if (lev[d] < 0) {
            lev[d] = layer[t];
            dl.push_back(d);
          } else {
            lev[d] = std::min(lev[d], layer[t]);
          }
        }
      std::sort(dl.begin(), dl.end());
      S.dofs = dl;
      S.level.resize(dl.size());
      S.chi.resize(dl.size());
      S.coords.resize(3 * dl.size());
      for (size_t k = 0; k < dl.size(); ++k) {
        S.level[k] = lev[dl[k]];
        S.chi[k] = overlap == 0 ? 1.0 : std::max(0.0, 1.0 - (double)S.level[k] / overlap);
        D.dof_coord(dl[k], &S.coords[3 * k]);
        lev[dl[k]] = -1;
      }
      // faces of Gamma_i met once: physical boundary or artificial interface
      std::vector<FK> fk(4 * cur.size());
      for (size_t q = 0; q < cur.size(); ++q)
        for (int f = 0; f < 4; ++f) {
          FK& k = fk[4 * q + f];
          for (int c = 0; c < 3; ++c) k.v[c] = D.tets[4 * cur[q] + kTetFace[f][c]];
          std::sort(k.v, k.v + 3);
          k.tet = cur[q];
        }
      std::sort(fk.begin(), fk.end());
      std::vector<ImpFace> imp;
      for (size_t a = 0; a < fk.size();) {
        size_t b = a + 1;
        while (b < fk.size() && fk[b].same(fk[a])) ++b;
        if (b - a == 1) {
          auto it = std::lower_bound(bfk.begin(), bfk.end(), fk[a]);
          bool on_boundary = it != bfk.end() && it->same(fk[a]);
          bool dirichlet = on_boundary && D.bdir[it->tet];
          if (!dirichlet) imp.push_back({{fk[a].v[0], fk[a].v[1], fk[a].v[2]}, fk[a].tet});
        }
        a = b;
      }
      for (int64_t t : cur) layer[t] = -1;
      assemble_local(D, S.tets, imp, S.dofs, S.A);
    }
  }
  // partition of unity
  std::vector<double> chi_sum(n, 0.0);
  for (auto& S : subs)
    for (size_t k = 0; k < S.dofs.size(); ++k) chi_sum[S.dofs[k]] += S.chi[k];
  for (auto& S : subs) {
    S.D.resize(S.dofs.size());
    for (size_t k = 0; k < S.dofs.size(); ++k) S.D[k] = S.chi[k] / chi_sum[S.dofs[k]];
  }
}

}  // namespace helm
