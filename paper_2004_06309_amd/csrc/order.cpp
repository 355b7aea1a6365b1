// Fill-reducing ordering and symbolic analysis of the local direct solvers.
//
// Geometric nested dissection: a node set is split by a plane normal to its
// longest extent; among the coordinate planes next to the median the one with
// the smallest vertex separator wins (nodes on the plane, plus nodes on one
// side still adjacent to the other side).  For Lagrange P2 nodes on a
// structured mesh a plane of element vertices is an exact separator.  Parts
// are ordered before their separator; small parts become dense leaves.
//
// Each leaf and each separator is one supernode: a contiguous column range C_s
// whose frontal matrix has rows C_s + R_s, where R_s collects the original
// couplings of C_s to later columns and the rows of the children's
// contribution blocks.  The parent of s is the supernode owning min(R_s),
// which makes R_c a subset of C_p + R_p (the multifrontal assembly tree).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.hpp"

namespace helm {

void tiles_fwd(int32_t w, int32_t r, int32_t tile_rows, std::vector<TileShape>& out) {
  // forward panel [L11^{-1}; L21 L11^{-1}] : (w + r) rows x w columns,
  // the diagonal-block rows only need the columns up to the tile's last row
  out.clear();
  int32_t m = w + r;
  for (int32_t r0 = 0; r0 < m; r0 += tile_rows) {
    int32_t nr = std::min(tile_rows, m - r0);
    int32_t nc = std::min(w, r0 + nr);
    out.push_back({r0, nr, 0, nc});
  }
}

void tiles_bwd(int32_t w, int32_t r, int32_t tile_rows, std::vector<TileShape>& out) {
  // backward panel [U11^{-1} | -U11^{-1} U12] : w rows x (w + r) columns,
  // a tile starting at row r0 only needs the columns from r0 on
  out.clear();
  for (int32_t r0 = 0; r0 < w; r0 += tile_rows) {
    int32_t nr = std::min(tile_rows, w - r0);
    out.push_back({r0, nr, r0, w + r - r0});
  }
}

namespace {

struct ND {
  const std::vector<int64_t>& ptr;
  const std::vector<int32_t>& adj;
  const std::vector<double>& xyz;
  int leaf;
  std::vector<int8_t> side;          // per node: -1 outside, 0 left, 1 right, 2 separator
  std::vector<int32_t> order;        // new -> old
  std::vector<std::pair<int32_t, int32_t>> blocks;  // (c0, w) in emission order

  ND(const std::vector<int64_t>& p, const std::vector<int32_t>& a, const std::vector<double>& x, int lf, int64_t n)
      : ptr(p), adj(a), xyz(x), leaf(lf), side(n, -1) {}

  void emit(const std::vector<int32_t>& nodes) {
    if (nodes.empty()) return;
    blocks.push_back({(int32_t)order.size(), (int32_t)nodes.size()});
    order.insert(order.end(), nodes.begin(), nodes.end());
  }

  // separator for the split at coordinate value v along axis; returns size
  // (and fills L/R/S when commit is true)
  int64_t try_split(const std::vector<int32_t>& nodes, int axis, double v, bool commit, std::vector<int32_t>* L,
                    std::vector<int32_t>* R, std::vector<int32_t>* S, int64_t* nl, int64_t* nr) {
    for (int32_t u : nodes) {
      double c = xyz[3 * u + axis];
      side[u] = c < v ? 0 : (c > v ? 1 : 2);
    }
    // left nodes adjacent to right nodes join the separator
    std::vector<int32_t> extra;
    for (int32_t u : nodes)
      if (side[u] == 0)
        for (int64_t p = ptr[u]; p < ptr[u + 1]; ++p)
          if (side[adj[p]] == 1) {
            extra.push_back(u);
            break;
          }
    for (int32_t u : extra) side[u] = 2;
    int64_t cl = 0, cr = 0, cs = 0;
    for (int32_t u : nodes) {
      if (side[u] == 0) ++cl;
      else if (side[u] == 1) ++cr;
      else ++cs;
    }
    *nl = cl;
    *nr = cr;
    if (commit) {
      for (int32_t u : nodes) (side[u] == 0 ? L : side[u] == 1 ? R : S)->push_back(u);
    }
    for (int32_t u : nodes) side[u] = -1;
    return cs;
  }

  void run(std::vector<int32_t> nodes) {
    if ((int64_t)nodes.size() <= leaf) {
      emit(nodes);
      return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t u : nodes)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], xyz[3 * u + d]);
        hi[d] = std::max(hi[d], xyz[3 * u + d]);
      }
    int axes[3] = {0, 1, 2};
    std::sort(axes, axes + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    for (int ai = 0; ai < 3; ++ai) {
      int axis = axes[ai];
      if (!(hi[axis] > lo[axis])) break;
      std::vector<double> vals(nodes.size());
      for (size_t i = 0; i < nodes.size(); ++i) vals[i] = xyz[3 * nodes[i] + axis];
      std::vector<double> sorted = vals;
      std::sort(sorted.begin(), sorted.end());
      std::vector<double> uniq = sorted;
      uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
      double med = sorted[sorted.size() / 2];
      int64_t mi = std::lower_bound(uniq.begin(), uniq.end(), med) - uniq.begin();
      double best_cost = 1e300, best_v = 0;
      bool found = false;
      const int64_t nn = (int64_t)nodes.size();
      for (int64_t q = std::max<int64_t>(0, mi - 3); q <= std::min<int64_t>((int64_t)uniq.size() - 1, mi + 3); ++q) {
        int64_t nl, nr;
        int64_t cs = try_split(nodes, axis, uniq[q], false, nullptr, nullptr, nullptr, &nl, &nr);
        if (nl == 0 || nr == 0) continue;
        double bal = (double)std::min(nl, nr) / (double)nn;
        if (bal < 0.2) continue;
        double cost = (double)cs * (1.0 + 0.5 * std::fabs(0.5 - (double)nl / (nl + nr)));
        if (cost < best_cost) {
          best_cost = cost;
          best_v = uniq[q];
          found = true;
        }
      }
      if (!found) continue;
      std::vector<int32_t> L, R, S;
      int64_t nl, nr;
      try_split(nodes, axis, best_v, true, &L, &R, &S, &nl, &nr);
      if ((int64_t)S.size() >= nn / 2) continue;  // not a useful split
      std::vector<int32_t>().swap(nodes);
      run(std::move(L));
      run(std::move(R));
      emit(S);
      return;
    }
    emit(nodes);  // no useful split: dense leaf
  }
};

}  // namespace

void nested_dissection(const Csr& A, const std::vector<double>& coords, int leaf, Symbolic& S, int tile_rows) {
  const int64_t n = A.n;
  if (leaf <= 0) leaf = 64;
  // symmetric adjacency without the diagonal
  std::vector<int64_t> ptr(n + 1, 0);
  std::vector<int32_t> adj;
  {
    std::vector<std::vector<int32_t>> nb(n);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        int32_t j = A.col[p];
        if (j == i) continue;
        nb[i].push_back(j);
        nb[j].push_back((int32_t)i);
      }
    for (int64_t i = 0; i < n; ++i) {
      std::sort(nb[i].begin(), nb[i].end());
      nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
      ptr[i + 1] = ptr[i] + (int64_t)nb[i].size();
    }
    adj.resize(ptr[n]);
    for (int64_t i = 0; i < n; ++i) std::copy(nb[i].begin(), nb[i].end(), adj.begin() + ptr[i]);
  }
  ND nd(ptr, adj, coords, leaf, n);
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  nd.run(std::move(all));

  S = Symbolic();
  S.n = n;
  if (tile_rows != 16 && tile_rows != 32 && tile_rows != 64) fail(HELM_EINVAL, "tile rows must be 16, 32 or 64");
  S.tile_rows = tile_rows;
  S.perm = nd.order;
  S.iperm.assign(n, -1);
  for (int64_t k = 0; k < n; ++k) S.iperm[S.perm[k]] = (int32_t)k;
  const int32_t nsn = (int32_t)nd.blocks.size();
  S.nsn = nsn;
  S.sn_c0.resize(nsn);
  S.sn_w.resize(nsn);
  std::vector<int32_t> sn_of(n);
  for (int32_t s = 0; s < nsn; ++s) {
    S.sn_c0[s] = nd.blocks[s].first;
    S.sn_w[s] = nd.blocks[s].second;
    for (int32_t k = 0; k < S.sn_w[s]; ++k) sn_of[S.sn_c0[s] + k] = s;
  }
  // row structures, parents
  S.sn_parent.assign(nsn, -1);
  S.sn_rptr.assign(nsn + 1, 0);
  std::vector<std::vector<int32_t>> children(nsn);
  std::vector<std::vector<int32_t>> R(nsn);
  for (int32_t s = 0; s < nsn; ++s) {
    int32_t c0 = S.sn_c0[s], c1 = c0 + S.sn_w[s];
    std::vector<int32_t>& r = R[s];
    for (int32_t j = c0; j < c1; ++j) {
      int32_t old = S.perm[j];
      for (int64_t p = ptr[old]; p < ptr[old + 1]; ++p) {
        int32_t nj = S.iperm[adj[p]];
        if (nj >= c1) r.push_back(nj);
      }
    }
    for (int32_t c : children[s])
      for (int32_t x : R[c])
        if (x >= c1) r.push_back(x);
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    if (!r.empty()) {
      int32_t p = sn_of[r[0]];
      S.sn_parent[s] = p;
      children[p].push_back(s);
    }
    S.sn_rptr[s + 1] = S.sn_rptr[s] + (int64_t)r.size();
  }
  S.rows.resize(S.sn_rptr[nsn]);
  for (int32_t s = 0; s < nsn; ++s) std::copy(R[s].begin(), R[s].end(), S.rows.begin() + S.sn_rptr[s]);
  // levels: height (leaves first) for the forward solve, depth for the backward
  S.height.assign(nsn, 0);
  for (int32_t s = 0; s < nsn; ++s)
    if (S.sn_parent[s] >= 0) S.height[S.sn_parent[s]] = std::max(S.height[S.sn_parent[s]], S.height[s] + 1);
  S.depth.assign(nsn, 0);
  for (int32_t s = nsn - 1; s >= 0; --s)
    if (S.sn_parent[s] >= 0) S.depth[s] = S.depth[S.sn_parent[s]] + 1;
  // panel sizes and flops
  S.sn_fwd_off.resize(nsn + 1);
  S.sn_bwd_off.resize(nsn + 1);
  std::vector<TileShape> ts;
  int64_t fo = 0, bo = 0;
  double fl = 0;
  for (int32_t s = 0; s < nsn; ++s) {
    int32_t w = S.sn_w[s], r = (int32_t)(S.sn_rptr[s + 1] - S.sn_rptr[s]);
    S.sn_fwd_off[s] = fo;
    S.sn_bwd_off[s] = bo;
    tiles_fwd(w, r, S.tile_rows, ts);
    for (auto& t : ts) fo += (int64_t)t.nrows * t.ncols;
    tiles_bwd(w, r, S.tile_rows, ts);
    for (auto& t : ts) bo += (int64_t)t.nrows * t.ncols;
    double W = w, Rr = r, M = w + r;
    // partial LU of the front + explicit inverses, complex multiply-adds
    fl += W * W * W / 3.0 + W * W * Rr + W * Rr * Rr + W * W * (Rr + W / 3.0) + W * W * (Rr + W / 3.0);
    S.max_front = std::max(S.max_front, (int32_t)M);
  }
  S.sn_fwd_off[nsn] = fo;
  S.sn_bwd_off[nsn] = bo;
  S.fwd_entries = fo;
  S.bwd_entries = bo;
  S.flops = 8.0 * fl;
}

}  // namespace helm
