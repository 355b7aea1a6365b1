// Preconditioner setup (host analysis + factorisation, device upload), the
// device applications of A, M1^{-1} (eq. oras) and M^{-1} (eq. 2lvl), and the
// right-preconditioned restarted GMRES driver (stop at ||b - A x|| <= tol ||b||,
// Section "Numerical experiments").
//
// GMRES keeps the preconditioned vectors z_j = M^{-1} v_j (flexible storage,
// x = x0 + Z_m y), orthogonalises with classical Gram-Schmidt applied twice
// (CGS2, Hermitian inner product) and solves the small least-squares problem
// on the host in double precision with complex Givens rotations
//   r = sqrt(|a|^2 + |b|^2), c = |a| / r, s = (a / |a|) conj(b) / r.
// The only host/device transfer per iteration is the new Hessenberg column.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <numeric>

#include "ctx.hpp"

namespace helm {

Ctx::~Ctx() {
  if (hev) (void)hipEventDestroy(hev);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  for (int k = 0; k < kMaxBatches; ++k) {
    if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
    if (sb[k]) (void)hipStreamDestroy(sb[k]);
  }
  if (h_host) (void)hipHostFree(h_host);
  if (bh_host) (void)hipHostFree(bh_host);
  if (nh_host) (void)hipHostFree(nh_host);
  free_bg_graphs();
  if (bg_host) (void)hipHostFree(bg_host);
  if (bg_hstat) (void)hipHostFree(bg_hstat);
  for (auto& e : bg_ev)
    if (e) (void)hipEventDestroy(e);
  if (bg_stream) (void)hipStreamDestroy(bg_stream);
}

// Work spaces of the solvers: their sizes follow n, the restart, the coarse
// order and the batches, so they are dropped whenever those can change.
void Ctx::free_solve_work() {
  gm_m = 0;
  gm_n = 0;
  for (auto* v : {&V, &Zk, &w, &partial, &hcol, &htmp, &nrm, &ydev, &coef_w, &coef_v, &npart, &nval}) v->reset();
  blk_m = blk_cap = blk_bases = 0;
  blk_n = 0;
  blk_timed = false;
  for (int r = 0; r < dev::kMaxBlock; ++r) {
    bV[r].reset();
    bZ[r].reset();
    bw[r].reset();
  }
  for (auto* v : {&bhcol, &bhtmp, &bpartial, &by, &bX, &bZb, &bW, &bq, &bt, &bcvec, &bcoef_w, &bcoef_v}) v->reset();
  for (auto* v : {&t, &q, &cvec}) v->reset();
  free_bg_graphs();
  bg_m = 0;
  bg_n = 0;
  for (auto* v : {&bgV, &bgZ, &bgW, &bgX, &bgB, &bgpart, &bgH, &bgC}) v->reset();
  bgstat.reset();
}

void Ctx::free_precond() {
  precond_ready = false;
  free_solve_work();
  subs.clear();
  sym.clear();
  two_level = false;
  Z = CsrReal();
  ZT = CsrReal();
  E = Csr();
  Esym = Symbolic();
  stats = helm_precond_stats{};
  for (auto& b : fine) b.reset();
  nbatch = 1;
  xall.reset();
  xall_b.reset();
  xall_b_S = 0;
  coarse.reset();
  pro_ptr.reset();
  pro_idx.reset();
  pro_w.reset();
  Zp_ptr.reset();
  Zp_col.reset();
  Zp_val.reset();
  AZ_ptr.reset();
  AZ_col.reset();
  AZ_val.reset();
  ZT_ptr.reset();
  ZT_col.reset();
  ZT_val.reset();
}

dev::Batch BatchDev::view() const {
  dev::Batch b;
  b.tf = tf.p;
  b.tb = tb.p;
  b.kf = kf.p;
  b.kb = kb.p;
  b.snj = snj.p;
  b.c64 = c64;
  b.goff_f = goff_f.p;
  b.sn_c0 = c0.p;
  b.sn_w = w.p;
  b.sn_uoff = uoff.p;
  b.sn_frow0 = frow0.p;
  b.sn_roff = roff.p;
  b.rows = rows.p;
  b.bidx = bidx.p;
  b.fcon_ptr = fcon_ptr.p;
  b.fcon_idx = fcon_idx.p;
  b.fcon2 = reinterpret_cast<const int2*>(fcon2.p);
  b.pf = pf.p;
  b.pb = pb.p;
  b.ubuf = ubuf.p;
  b.y = y.p;
  b.x = xout();
  return b;
}

void Profiler::begin(hipStream_t s) {
  if (used + 2 > pool.size()) {
    size_t old = pool.size();
    pool.resize(std::max<size_t>(64, 2 * pool.size()));
    for (size_t i = old; i < pool.size(); ++i) HELM_HIP(hipEventCreate(&pool[i]));
  }
  HELM_HIP(hipEventRecord(pool[used], s));
}

void Profiler::end(int kid, double bytes, hipStream_t s) {
  HELM_HIP(hipEventRecord(pool[used + 1], s));
  pending.push_back({kid, bytes});
  used += 2;
}

void Profiler::harvest() {
  for (size_t k = 0; k < pending.size(); ++k) {
    float ms = 0;
    HELM_HIP(hipEventSynchronize(pool[2 * k + 1]));
    HELM_HIP(hipEventElapsedTime(&ms, pool[2 * k], pool[2 * k + 1]));
    helm_kernel_profile& a = acc[pending[k].first];
    a.launches += 1;
    a.milliseconds += ms;
    a.bytes += pending[k].second;
  }
  pending.clear();
  used = 0;
}

void Profiler::reset() {
  pending.clear();
  used = 0;
  for (auto& a : acc) a = helm_kernel_profile{};
}

Profiler::~Profiler() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

// Solve layout of a batch of analysed and factored matrices: positions,
// per-supernode data, input gather (with the pivot order folded in), routing
// of children's update vectors to the parents' front rows, and the tiles of
// every forward (by height) and backward (by depth) level.  in_idx[i][l] is
// the index in the solve's input vector of row l (original order) of matrix i.
// Supernodes this close to the root of their tree (depth 0: the root
// separator) are solved with four waves per tile.
constexpr int32_t kTopDepth = 0;

void layout_batch(const std::vector<const Symbolic*>& Ss, const std::vector<const std::vector<int64_t>*>& in_idx,
                  const std::vector<NumericOut>& num, int64_t sn_jobs_min, bool c64, BatchHost& B) {
  const int nm = (int)Ss.size();
  B = BatchHost();
  // waves per tile from the tile's bytes per row: a complex64 column is
  // half a complex128 one, so a wave takes twice the columns
  auto wpt_of = [c64](int32_t ncols) { return dev::waves_per_tile(c64 ? (ncols + 1) / 2 : ncols); };
  std::vector<int64_t> pos0(nm + 1, 0), sn0(nm + 1, 0), pf0(nm + 1, 0), pb0(nm + 1, 0), u0(nm + 1, 0),
      fr0(nm + 1, 0);
  int32_t maxlev_f = 0, maxlev_b = 0;
  for (int i = 0; i < nm; ++i) {
    const Symbolic& S = *Ss[i];
    pos0[i + 1] = pos0[i] + S.n;
    sn0[i + 1] = sn0[i] + S.nsn;
    pf0[i + 1] = pf0[i] + S.fwd_entries;
    pb0[i + 1] = pb0[i] + S.bwd_entries;
    u0[i + 1] = u0[i] + (int64_t)S.rows.size();
    int64_t fr = 0;
    for (int32_t s = 0; s < S.nsn; ++s) fr += S.sn_w[s] + (S.sn_rptr[s + 1] - S.sn_rptr[s]);
    fr0[i + 1] = fr0[i] + fr;
    for (int32_t s = 0; s < S.nsn; ++s) {
      maxlev_f = std::max(maxlev_f, S.height[s]);
      maxlev_b = std::max(maxlev_b, S.depth[s]);
    }
    B.max_front = std::max(B.max_front, S.max_front);
    B.flops += S.flops;
  }
  if (pos0[nm] >= (int64_t)INT32_MAX || u0[nm] >= (int64_t)INT32_MAX || fr0[nm] >= (int64_t)INT32_MAX)
    fail(HELM_EINVAL, "batch too large for 32-bit solve indices");
  B.npos = pos0[nm];
  B.nf = pf0[nm];
  B.nb = pb0[nm];
  B.nu = u0[nm];
  const int64_t nsn = sn0[nm];
  B.c0.resize(nsn);
  B.w.resize(nsn);
  B.uoff.resize(nsn);
  B.frow0.resize(nsn);
  B.roff.resize(nsn);
  B.rows.resize(B.nu);
  B.bidx.assign(B.npos, 0);
  std::vector<std::vector<dev::Tile>> lf(maxlev_f + 1), lb(maxlev_b + 1);
  std::vector<char> sn_narrow(nsn, 0), sn_top(nsn, 0);
  std::vector<int32_t> fcon_cnt(fr0[nm] + 1, 0);
  std::vector<std::vector<std::pair<int64_t, int32_t>>> fcon_m(nm);
  std::vector<TileShape> ts;
  for (int i = 0; i < nm; ++i) {
    const Symbolic& S = *Ss[i];
    const std::vector<int32_t>& piv = num[i].piv;
    std::vector<int32_t> kinv(S.n);
    std::vector<int64_t> frl(S.nsn);
    int64_t fr = 0;
    for (int32_t s = 0; s < S.nsn; ++s) {
      const int64_t g = sn0[i] + s;
      const int32_t c0 = S.sn_c0[s], w = S.sn_w[s];
      const int32_t r = (int32_t)(S.sn_rptr[s + 1] - S.sn_rptr[s]);
      B.c0[g] = (int32_t)(pos0[i] + c0);
      B.w[g] = w;
      B.uoff[g] = (int32_t)(u0[i] + S.sn_rptr[s]);
      B.roff[g] = u0[i] + S.sn_rptr[s];
      frl[s] = fr;
      B.frow0[g] = (int32_t)(fr0[i] + fr);
      fr += w + r;
      for (int32_t a = 0; a < r; ++a) B.rows[u0[i] + S.sn_rptr[s] + a] = (int32_t)(pos0[i] + S.rows[S.sn_rptr[s] + a]);
      for (int32_t k = 0; k < w; ++k) {
        const int32_t rho = piv[c0 + k];  // new-order row eliminated at pivot position k
        kinv[rho] = k;
        B.bidx[pos0[i] + c0 + k] = (int32_t)(*in_idx[i])[S.perm[rho]];
      }
      sn_narrow[g] = sn_jobs_min >= 0 && w <= 64 && S.tile_rows == 64;
      sn_top[g] = S.depth[s] <= kTopDepth;
      tiles_fwd(w, r, S.tile_rows, ts);
      int64_t off = pf0[i] + S.sn_fwd_off[s];
      for (auto& t : ts) {
        lf[S.height[s]].push_back({off, (int32_t)g, t.row0, t.nrows, t.col0, t.ncols, B.c0[g], w, B.frow0[g]});
        off += (int64_t)t.nrows * t.ncols;
      }
      tiles_bwd(w, r, S.tile_rows, ts);
      off = pb0[i] + S.sn_bwd_off[s];
      for (auto& t : ts) {
        lb[S.depth[s]].push_back({off, (int32_t)g, t.row0, t.nrows, t.col0, t.ncols, B.c0[g], w, (int32_t)B.roff[g]});
        off += (int64_t)t.nrows * t.ncols;
      }
    }
    // children's updates routed to the parent's front rows
    auto& fl = fcon_m[i];
    for (int32_t c = 0; c < S.nsn; ++c) {
      const int32_t p = S.sn_parent[c];
      if (p < 0) continue;
      const int32_t pc0 = S.sn_c0[p], pw = S.sn_w[p];
      const int32_t* Rp = S.rows.data() + S.sn_rptr[p];
      const int32_t rp = (int32_t)(S.sn_rptr[p + 1] - S.sn_rptr[p]);
      for (int64_t a = S.sn_rptr[c]; a < S.sn_rptr[c + 1]; ++a) {
        const int32_t row = S.rows[a];
        int64_t f;
        if (row >= pc0 && row < pc0 + pw) {
          f = kinv[row];
        } else {
          const int32_t* it = std::lower_bound(Rp, Rp + rp, row);
          if (it == Rp + rp || *it != row) fail(HELM_EINVAL, "internal: child row missing from parent front");
          f = pw + (it - Rp);
        }
        fl.push_back({fr0[i] + frl[p] + f, (int32_t)(u0[i] + a)});
      }
    }
    std::stable_sort(fl.begin(), fl.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                       return x.first < y.first;
                     });
    for (auto& e : fl) fcon_cnt[e.first + 1]++;
  }
  B.fcon_ptr.resize(fr0[nm] + 1);
  B.fcon_ptr[0] = 0;
  for (int64_t f = 0; f < fr0[nm]; ++f) B.fcon_ptr[f + 1] = B.fcon_ptr[f] + fcon_cnt[f + 1];
  B.fcon_idx.resize(B.fcon_ptr[fr0[nm]]);
  {
    std::vector<int32_t> fill(B.fcon_ptr.begin(), B.fcon_ptr.end() - 1);
    for (int i = 0; i < nm; ++i)
      for (auto& e : fcon_m[i]) B.fcon_idx[fill[e.first]++] = e.second;
  }
  // the same lists as index pairs (one load for the common rows)
  B.fcon2.assign(2 * (size_t)std::max<int64_t>(fr0[nm], 1), -1);
  for (int64_t f = 0; f < fr0[nm]; ++f) {
    const int32_t e0 = B.fcon_ptr[f], cnt = B.fcon_ptr[f + 1] - e0;
    if (cnt > 2) {
      B.fcon2[2 * f] = -2 - e0;
      B.fcon2[2 * f + 1] = 0;
    } else {
      if (cnt >= 1) B.fcon2[2 * f] = B.fcon_idx[e0];
      if (cnt == 2) B.fcon2[2 * f + 1] = B.fcon_idx[e0 + 1];
    }
  }
  // algorithmic bytes per level: every panel entry once, plus the vector
  // entries each supernode gathers and writes
  auto r_of = [&](int64_t s) { return (s + 1 < nsn ? B.roff[s + 1] : B.nu) - B.roff[s]; };
  auto level_bytes = [&](const std::vector<dev::Tile>& T, bool fwd, double& panel) {
    double by = 0;
    int32_t last = -1;
    panel = 0;
    for (const auto& t : T) {
      by += 16.0 * t.nrows * t.ncols;
      panel += 16.0 * t.nrows * t.ncols;
      const int32_t s = t.sn;
      if (s == last) continue;
      last = s;
      const double w = B.w[s], r = (double)r_of(s);
      if (fwd) {
        const double nfc = B.fcon_ptr[B.frow0[s] + (int64_t)(w + r)] - B.fcon_ptr[B.frow0[s]];
        by += 16.0 * (w + nfc + w + r);
      } else {
        by += 16.0 * (w + r + w);
      }
    }
    return by;
  };
  // workgroup tasks: tiles grouped by width class, 4 / wpt tiles per group.
  // Forward tiles of narrow supernodes close their level, grouped by
  // supernode (largest first) in row order, and also form one-wave jobs.
  auto sn_entries = [&](int32_t s) { return (int64_t)(B.w[s] + r_of(s)) * B.w[s]; };
  // the top separators of every tree form levels of few tiles: each of
  // their tiles gets a whole workgroup (four waves over its columns) so the
  // level still spreads over the device
  auto wpt_tile = [&](const dev::Tile& t) { return sn_top[t.sn] ? 4 : wpt_of(t.ncols); };
  B.snj_lev.assign(1, 0);
  auto make_tasks = [&](std::vector<std::vector<dev::Tile>>& levels, bool fwd, std::vector<dev::Tile>& tiles,
                        std::vector<dev::Task>& tasks, std::vector<int64_t>& lev, std::vector<double>& bytes,
                        std::vector<double>& pbytes) {
    lev.assign(1, 0);
    for (auto& l : levels) {
      // one-wave jobs only where a level has enough narrow supernodes to
      // fill the device with waves (fewer, longer waves lose to tiles)
      int64_t nnar = 0;
      for (size_t u = 0; u < l.size(); ++u)
        if (fwd && sn_narrow[l[u].sn] && (u == 0 || l[u - 1].sn != l[u].sn)) ++nnar;
      const bool use_sn = nnar > 0 && nnar >= sn_jobs_min;
      auto narrow = [&](const dev::Tile& t) { return use_sn && sn_narrow[t.sn]; };
      double pb = 0;
      bytes.push_back(level_bytes(l, fwd, pb));
      pbytes.push_back(pb);
      // widest class first, larger tiles first: the level's tail holds the
      // shortest workgroups
      std::stable_sort(l.begin(), l.end(), [&](const dev::Tile& a, const dev::Tile& b) {
        const bool na = narrow(a), nb = narrow(b);
        if (na != nb) return nb;
        if (na) {
          const int64_t ea = sn_entries(a.sn), eb = sn_entries(b.sn);
          if (ea != eb) return ea > eb;
          if (a.sn != b.sn) return a.sn < b.sn;
          return a.row0 < b.row0;
        }
        const int wa = wpt_tile(a), wb = wpt_tile(b);
        if (wa != wb) return wa > wb;
        return (int64_t)a.nrows * a.ncols > (int64_t)b.nrows * b.ncols;
      });
      size_t q = 0;
      int64_t ktile = -1;
      while (q < l.size()) {
        if (ktile < 0 && narrow(l[q])) ktile = (int64_t)tasks.size() - lev.back();
        const int wpt = wpt_tile(l[q]);
        const int per = 4 / wpt;
        size_t e = q;
        while (e < l.size() && (int)(e - q) < per && wpt_tile(l[e]) == wpt &&
               narrow(l[e]) == narrow(l[q]))
          ++e;
        tasks.push_back({(int32_t)(tiles.size() + q), (int16_t)(e - q), (int16_t)wpt});
        q = e;
      }
      if (fwd) {
        B.ktile_f.push_back(ktile < 0 ? (int64_t)tasks.size() - lev.back() : ktile);
        for (size_t u = 0; u < l.size(); ++u) {
          const dev::Tile& t = l[u];
          if (!narrow(t) || (u > 0 && l[u - 1].sn == t.sn)) continue;
          const int32_t sn = t.sn;
          B.snj.push_back({t.off, (int32_t)(B.w[sn] + r_of(sn)), B.w[sn], B.c0[sn], B.frow0[sn], B.uoff[sn],
                           (int32_t)(tiles.size() + u)});
        }
        B.snj_lev.push_back((int64_t)B.snj.size());
      }
      tiles.insert(tiles.end(), l.begin(), l.end());
      lev.push_back((int64_t)tasks.size());
    }
  };
  // supernodes of every forward level and their offsets in the level's
  // staging block
  B.goff_f.assign(nsn, 0);
  auto stage_levels = [&](const std::vector<std::vector<dev::Tile>>& levels, std::vector<int32_t>& gsn,
                          std::vector<int64_t>& glev, std::vector<int64_t>& goff, std::vector<int32_t>& gy) {
    glev.assign(1, 0);
    gy.clear();
    for (const auto& l : levels) {
      int64_t cols = 0, widest = 1;
      int32_t last = -1;
      for (const auto& t : l) {
        if (t.sn == last) continue;
        last = t.sn;
        gsn.push_back(t.sn);
        goff[t.sn] = cols;
        const int64_t c = B.w[t.sn];
        cols += c;
        widest = std::max(widest, c);
      }
      glev.push_back((int64_t)gsn.size());
      // a few workgroups per supernode, so the wide blocks of the upper
      // levels are gathered in parallel without launching idle workgroups
      gy.push_back((int32_t)std::min<int64_t>(4, (widest * dev::kMaxBlock + 255) / 256));
      B.stage_cols = std::max(B.stage_cols, cols);
    }
  };
  stage_levels(lf, B.gsn_f, B.gsn_lev_f, B.goff_f, B.gy_f);
  make_tasks(lf, true, B.tf, B.kf, B.lev_f, B.bytes_f, B.pbytes_f);
  make_tasks(lb, false, B.tb, B.kb, B.lev_b, B.bytes_b, B.pbytes_b);
  // LDS input buffer of every level: each slot of a task with wpt < 4 holds
  // its whole tile; a single-tile task takes up to kLevelChunkMax per pass
  auto chunks = [&](const std::vector<dev::Task>& K, const std::vector<dev::Tile>& T, const std::vector<int64_t>& lev,
                    std::vector<int32_t>& out) {
    out.clear();
    for (size_t l = 0; l + 1 < lev.size(); ++l) {
      int64_t c = 64;
      for (int64_t q = lev[l]; q < lev[l + 1]; ++q) {
        int64_t wide = 0;
        for (int u = 0; u < K[q].ntile; ++u) wide = std::max<int64_t>(wide, T[K[q].tile0 + u].ncols);
        // a task of one or two waves per tile streams each tile in one pass
        if (K[q].wpt < 4 && (4 / K[q].wpt) * wide > dev::kLevelChunkMax)
          fail(HELM_EINVAL, "internal: a level tile is wider than its LDS input slot");
        c = std::max<int64_t>(c, K[q].wpt == 4 ? std::min<int64_t>(wide, dev::kLevelChunkMax) : (4 / K[q].wpt) * wide);
      }
      out.push_back((int32_t)std::min<int64_t>((c + 63) / 64 * 64, dev::kLevelChunkMax));
    }
  };
  chunks(B.kf, B.tf, B.lev_f, B.chunk_f);
  chunks(B.kb, B.tb, B.lev_b, B.chunk_b);
  // tasks are sorted widest class first, so a level's narrow tiles (one
  // wave per tile) are its last ones
  auto wide = [&](const std::vector<dev::Task>& K, const std::vector<int64_t>& lev, int wmin,
                  std::vector<int64_t>& out) {
    out.clear();
    for (size_t l = 0; l + 1 < lev.size(); ++l) {
      int64_t nw = 0;
      for (int64_t q = lev[l]; q < lev[l + 1]; ++q)
        if (K[q].wpt >= wmin) nw += K[q].ntile;
      out.push_back(nw);
    }
  };
  wide(B.kf, B.lev_f, 2, B.nwide_f);
  wide(B.kb, B.lev_b, 2, B.nwide_b);
  wide(B.kf, B.lev_f, 4, B.nwide4_f);
  wide(B.kb, B.lev_b, 4, B.nwide4_b);
}

namespace {

// Panel arrays of a batch (factorisation order: matrix after matrix) and
// the device pointers of each matrix's first forward / backward entry.
void alloc_panels(const std::vector<const Symbolic*>& Ss, dev::FactorPrecision prec, BatchDev& Dv,
                  std::vector<void*>& pf, std::vector<void*>& pb) {
  const size_t esz = prec != dev::FactorPrecision::kC128 ? sizeof(std::complex<float>) : sizeof(cplx);
  int64_t nf = 0, nb = 0;
  for (const Symbolic* S : Ss) nf += S->fwd_entries, nb += S->bwd_entries;
  Dv.pf.alloc(esz * (size_t)nf);
  Dv.pb.alloc(esz * (size_t)nb);
  nf = nb = 0;
  for (const Symbolic* S : Ss) {
    pf.push_back(Dv.pf.p + esz * nf);
    pb.push_back(Dv.pb.p + esz * nb);
    nf += S->fwd_entries;
    nb += S->bwd_entries;
  }
}

// Factors a batch on the device into its panels; without a device only the
// layout is built (pivots taken as the identity).  With pre, the device panels were allocated by
// alloc_panels and factorised already, pre holding the pivots.
void build_batch(const std::vector<const Csr*>& As, const std::vector<const Symbolic*>& Ss,
                 const std::vector<const std::vector<int64_t>*>& in_idx, int device, bool numeric,
                 dev::FactorPrecision prec, int32_t split_min, int64_t sn_jobs_min, BatchHost& B,
                 BatchDev& Dv, int32_t& n_perturbed, double& seconds, const std::vector<NumericOut>* pre = nullptr,
                 double* scratch_bytes = nullptr) {
  const int nm = (int)As.size();
  const bool c64 = prec != dev::FactorPrecision::kC128;
  const size_t esz = c64 ? sizeof(std::complex<float>) : sizeof(cplx);
  Dv.c64 = c64 ? 1 : 0;
  std::vector<NumericOut> num(nm);
  const auto t0 = std::chrono::steady_clock::now();
  if (pre) {
    num = *pre;
  } else if (numeric) {
    std::vector<void*> pf, pb;
    alloc_panels(Ss, prec, Dv, pf, pb);
    double sb = 0;
    factor_batch_device(As, Ss, prec, split_min, pf, pb, num, n_perturbed, sb);
    if (scratch_bytes) *scratch_bytes = sb;
  } else {
    // no device: only the layout is built (identity pivots)
    n_perturbed = 0;
    for (int i = 0; i < nm; ++i) {
      num[i].piv.resize(Ss[i]->n);
      std::iota(num[i].piv.begin(), num[i].piv.end(), 0);
    }
  }
  seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // one-wave supernode jobs for complex128 panels (with complex64 panels
  // the narrow tiles stream faster through the tile kernel)
  layout_batch(Ss, in_idx, num, c64 ? -1 : sn_jobs_min, c64, B);
  if (!numeric) return;
  // Panels move from factorisation order (per matrix, per supernode) to
  // solve order: each level's tiles contiguous, in the order its workgroups
  // take them, so a level streams one region of HBM front to back.
  auto relayout = [&](DVec<unsigned char>& P, std::vector<dev::Tile>& T) {
    if (T.empty()) return;
    const int64_t wpe = (int64_t)(esz / 8);  // 8-byte words per entry
    std::vector<int64_t> from(T.size()), to(T.size()), words(T.size());
    int64_t pos = 0;
    for (size_t i = 0; i < T.size(); ++i) {
      const int64_t len = (int64_t)T[i].nrows * T[i].ncols;
      from[i] = T[i].off * wpe;
      to[i] = pos * wpe;
      words[i] = len * wpe;
      T[i].off = pos;
      pos += len;
    }
    bool inside = (size_t)pos * esz == P.n;
    for (size_t i = 0; i < T.size() && inside; ++i) inside = from[i] >= 0 && (size_t)(from[i] + words[i]) * 8 <= P.n;
    if (!inside) fail(HELM_EINVAL, "internal: solve tiles do not cover the panel array");
    DVec<unsigned char> Q;
    Q.alloc(P.n);
    DVec<int64_t> f, t, w;
    f.upload(from);
    t.upload(to);
    w.upload(words);
    dev::copy_tiles(P.p, Q.p, f.p, t.p, w.p, (int64_t)T.size(), nullptr);
    HELM_HIP(hipDeviceSynchronize());
    std::swap(P.p, Q.p);
    std::swap(P.n, Q.n);
  };
  relayout(Dv.pf, B.tf);
  relayout(Dv.pb, B.tb);
  for (auto& j : B.snj) j.off = B.tf[j.tile].off;
  Dv.npos = B.npos;
  Dv.lev_f = B.lev_f;
  Dv.lev_b = B.lev_b;
  Dv.chunk_f = B.chunk_f;
  Dv.chunk_b = B.chunk_b;
  Dv.nwide_f = B.nwide_f;
  Dv.snj.upload(B.snj);
  Dv.snj_lev = B.snj_lev;
  Dv.ktile_f = B.ktile_f;
  Dv.nwide_b = B.nwide_b;
  Dv.nwide4_f = B.nwide4_f;
  Dv.nwide4_b = B.nwide4_b;
  Dv.nw16_f = B.nwide_f;
  Dv.nw16_b = B.nwide_b;
  Dv.blk_tuned = false;
  Dv.gy_f = B.gy_f;
  Dv.bytes_f = B.bytes_f;
  Dv.bytes_b = B.bytes_b;
  Dv.pbytes_f = B.pbytes_f;
  Dv.pbytes_b = B.pbytes_b;
  auto tile_ranges = [](const std::vector<dev::Task>& K, const std::vector<int64_t>& lev) {
    std::vector<int64_t> r(1, 0);
    for (size_t l = 0; l + 1 < lev.size(); ++l)
      r.push_back(lev[l + 1] > lev[l] ? K[lev[l + 1] - 1].tile0 + K[lev[l + 1] - 1].ntile : r.back());
    return r;
  };
  Dv.tiles_f = tile_ranges(B.kf, B.lev_f);
  Dv.tiles_b = tile_ranges(B.kb, B.lev_b);
  Dv.gsn_f.upload(B.gsn_f);
  Dv.goff_f.upload(B.goff_f);
  Dv.gsn_lev_f = B.gsn_lev_f;
  Dv.stage_cols = B.stage_cols;
  Dv.tf.upload(B.tf);
  Dv.tb.upload(B.tb);
  Dv.kf.upload(B.kf);
  Dv.kb.upload(B.kb);
  Dv.c0.upload(B.c0);
  Dv.w.upload(B.w);
  Dv.uoff.upload(B.uoff);
  Dv.frow0.upload(B.frow0);
  Dv.roff.upload(B.roff);
  Dv.rows.upload(B.rows);
  Dv.bidx.upload(B.bidx);
  Dv.fcon_ptr.upload(B.fcon_ptr);
  Dv.fcon_idx.upload(B.fcon_idx);
  Dv.fcon2.upload(B.fcon2);
  Dv.ubuf.alloc(2 * std::max<int64_t>(B.nu, 1));
  Dv.y.alloc(2 * std::max<int64_t>(B.npos, 1));
  Dv.x.alloc(2 * std::max<int64_t>(B.npos, 1));
}

// Forward then backward level sweeps; with profiling on, every level launch
// of the fine batch is timed (the coarse batch is timed as a whole).
// Coarse-batch solve (forward and backward sweeps) through a view whose
// work vectors may lie outside the batch (no profiling).
// The cooperative coarse solve; false (the launch refused, its error
// cleared) when the device cannot co-schedule its grid at this moment, for
// instance while another process holds workgroups: the caller then takes the
// per-level launches, whose result agreed with it at setup.
bool coop_solve(const BatchDev& b, const dev::Batch& v, const double* in, hipStream_t s) {
  if (dev::batch_solve_coop(v, in, b.ranges, b.coop, s) == hipSuccess) return true;
  (void)hipGetLastError();
  return false;
}

void batch_solve_view(const BatchDev& b, const dev::Batch& v, const double* in, hipStream_t s) {
  if (b.coop > 0 && coop_solve(b, v, in, s)) return;
  for (size_t l = 0; l + 1 < b.lev_f.size(); ++l) {
    dev::fwd_level(v, b.lev_f[l], b.ktile_f[l], in, b.chunk_f[l], true, s);
    dev::fwd_sn(v, b.snj_lev[l], b.snj_lev[l + 1] - b.snj_lev[l], in, s);
  }
  for (size_t l = 0; l + 1 < b.lev_b.size(); ++l) dev::bwd_level(v, b.lev_b[l], b.lev_b[l + 1] - b.lev_b[l], b.chunk_b[l], true, s);
}

void batch_solve(const BatchDev& b, const double* in, hipStream_t s, Profiler* prof, bool fine) {
  dev::Batch v = b.view();
  if (!fine && b.coop > 0 && coop_solve(b, v, in, s)) return;
  const bool each = prof && prof->on && fine;
  for (size_t l = 0; l + 1 < b.lev_f.size(); ++l) {
    if (each) prof->begin(s);
    dev::fwd_level(v, b.lev_f[l], b.ktile_f[l], in, b.chunk_f[l], !fine, s);
    dev::fwd_sn(v, b.snj_lev[l], b.snj_lev[l + 1] - b.snj_lev[l], in, s);
    if (each) prof->end(HELM_K_TRSV_FWD, b.bytes_f[l], s);
  }
  for (size_t l = 0; l + 1 < b.lev_b.size(); ++l) {
    if (each) prof->begin(s);
    dev::bwd_level(v, b.lev_b[l], b.lev_b[l + 1] - b.lev_b[l], b.chunk_b[l], !fine, s);
    if (each) prof->end(HELM_K_TRSV_BWD, b.bytes_b[l], s);
  }
}

double sum(const std::vector<double>& v) { return std::accumulate(v.begin(), v.end(), 0.0); }

}  // namespace

namespace {

// Times launch(G) for every candidate (one warm-up, then three timed runs on
// the null stream) and returns the fastest G: the SpMV tile shape is tuned
// on the device for the matrix at hand.
template <class F>
int pick_lanes_per_row(const std::vector<int>& cands, F&& launch) {
  hipEvent_t e0, e1;
  HELM_HIP(hipEventCreate(&e0));
  HELM_HIP(hipEventCreate(&e1));
  int best = cands[0];
  float best_ms = 1e30f;
  for (int G : cands) {
    launch(G);
    HELM_HIP(hipEventRecord(e0, nullptr));
    for (int r = 0; r < 3; ++r) launch(G);
    HELM_HIP(hipEventRecord(e1, nullptr));
    HELM_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HELM_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = G;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

}  // namespace

namespace {

// Average time (ms) of launch() over three runs on the null stream, after one
// warm-up run.
template <class F>
float time_launch(F&& launch) {
  hipEvent_t e0, e1;
  HELM_HIP(hipEventCreate(&e0));
  HELM_HIP(hipEventCreate(&e1));
  launch();
  HELM_HIP(hipEventRecord(e0, nullptr));
  for (int r = 0; r < 3; ++r) launch();
  HELM_HIP(hipEventRecord(e1, nullptr));
  HELM_HIP(hipEventSynchronize(e1));
  float ms = 0;
  HELM_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / 3;
}

// Spreads the low 21 bits of v to every third bit.
uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// Rows in Morton (Z-curve) order of their dof positions: rows handled close
// together in time then share the cache lines of x they gather.
std::vector<int32_t> morton_rows(const Discretization& D) {
  const int64_t n = D.n;
  std::vector<double> xyz(3 * n);
  for (int64_t v = 0; v < D.nv; ++v)
    for (int d = 0; d < 3; ++d) xyz[3 * v + d] = D.xyz[3 * v + d];
  for (int64_t e = 0; e < n - D.nv; ++e)
    for (int d = 0; d < 3; ++d)
      xyz[3 * (D.nv + e) + d] = 0.5 * (D.xyz[3 * D.edges[2 * e] + d] + D.xyz[3 * D.edges[2 * e + 1] + d]);
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = 1e300;
    hi[d] = -1e300;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[3 * i + d]);
      hi[d] = std::max(hi[d], xyz[3 * i + d]);
    }
  // one scale for all axes keeps the curve's cells cubic
  double ext = 0;
  for (int d = 0; d < 3; ++d) ext = std::max(ext, hi[d] - lo[d]);
  const double sc = ext > 0 ? 2097151.0 / ext : 0.0;
  std::vector<std::pair<uint64_t, int32_t>> key(n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = 0;
    for (int d = 0; d < 3; ++d) k |= spread3((uint64_t)((xyz[3 * i + d] - lo[d]) * sc)) << d;
    key[i] = {k, (int32_t)i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = key[i].second;
  return order;
}

// Sliced-ELL copy of A: rows taken in `order`, sorted by length (longest
// first) inside windows of 1024, so a 64-row slice holds rows of similar
// length that were close in `order`.
void build_sell(Ctx& c, const std::vector<int32_t>& order) {
  const Csr& A = c.D.A;
  const int64_t n = A.n;
  const int64_t ns = (n + 63) / 64;
  std::vector<int32_t> perm(ns * 64, 0);
  for (int64_t w0 = 0; w0 < n; w0 += 1024) {
    const int64_t w1 = std::min<int64_t>(n, w0 + 1024);
    std::vector<int32_t> r(order.begin() + w0, order.begin() + w1);
    std::stable_sort(r.begin(), r.end(), [&](int32_t a, int32_t b) {
      return A.ptr[a + 1] - A.ptr[a] > A.ptr[b + 1] - A.ptr[b];
    });
    std::copy(r.begin(), r.end(), perm.begin() + w0);
  }
  std::vector<int64_t> soff(ns + 1, 0);
  std::vector<int32_t> swidth(ns, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int32_t wd = 0;
    for (int64_t q = s * 64; q < std::min<int64_t>(n, s * 64 + 64); ++q)
      wd = std::max<int32_t>(wd, (int32_t)(A.ptr[perm[q] + 1] - A.ptr[perm[q]]));
    swidth[s] = wd;
    soff[s + 1] = soff[s] + 64 * (int64_t)wd;
  }
  std::vector<int32_t> scol(soff[ns], 0);
  std::vector<cplx> sval(soff[ns], cplx(0, 0));
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < ns; ++s)
    for (int64_t q = s * 64; q < std::min<int64_t>(n, s * 64 + 64); ++q) {
      const int64_t row = perm[q], lane = q - s * 64;
      for (int64_t j = 0; j < swidth[s]; ++j) {
        const int64_t p = A.ptr[row] + j;
        const bool real = p < A.ptr[row + 1];
        scol[soff[s] + j * 64 + lane] = real ? A.col[p] : (int32_t)row;
        sval[soff[s] + j * 64 + lane] = real ? A.val[p] : cplx(0, 0);
      }
    }
  c.sell_nslices = ns;
  c.sell_off.upload(soff);
  c.sell_width.upload(swidth);
  c.sell_perm.upload(perm);
  c.sell_col.upload(scol);
  c.sell_val.upload(reinterpret_cast<const double*>(sval.data()), 2 * sval.size());
}

}  // namespace

void upload_matrix(Ctx& c) {
  const Csr& A = c.D.A;
  const int64_t n = A.n;
  c.A_ptr.upload(A.ptr);
  c.A_col.upload(A.col);
  c.A_val.upload(reinterpret_cast<const double*>(A.val.data()), 2 * A.val.size());
  {
    std::vector<int64_t> sp(n + 1, 0);
    std::vector<int32_t> sc;
    std::vector<double> sv;
    sc.reserve(A.nnz());
    sv.reserve(A.nnz());
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        sc.push_back(A.col[p]);
        sv.push_back(A.val[p].real());
      }
      for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
        if (A.val[p].imag() != 0.0) {
          sc.push_back((int32_t)((uint32_t)A.col[p] | 0x80000000u));
          sv.push_back(A.val[p].imag());
        }
      sp[i + 1] = (int64_t)sc.size();
    }
    c.S_ptr.upload(sp);
    c.S_col.upload(sc);
    c.S_val.upload(sv);
    c.S_nnz = (int64_t)sc.size();
  }
  build_sell(c, morton_rows(c.D));
  {
    std::vector<int64_t> xr(9);
    c.A_xrows = dev::xcd_ranges(n, A.ptr.data(), xr.data());
    c.A_xr.upload(xr);
  }
  DVec<double> x, y;
  x.alloc(2 * n);
  y.alloc(2 * n);
  HELM_HIP(hipMemset(x.p, 0, sizeof(double) * 2 * n));
  // every storage and lane count is timed; the fastest is the default
  float best = 1e30f, best_csr = 1e30f, best_x = 1e30f, best_s = 1e30f;
  for (int G : dev::kSpmvCfgs) {
    const float tsp = time_launch([&] {
      dev::spmv_split(n, c.S_ptr.p, c.S_col.p, c.S_val.p, x.p, nullptr, y.p, G, nullptr);
    });
    if (tsp < best_s) {
      best_s = tsp;
      c.g_S = G;
    }
    const float t = time_launch([&] {
      dev::spmv(n, c.A_ptr.p, c.A_col.p, c.A_val.p, nullptr, 0, x.p, nullptr, y.p, G, nullptr);
    });
    if (t < best_csr) {
      best_csr = t;
      c.g_A = G;
    }
    const float tx = time_launch([&] {
      dev::spmv(n, c.A_ptr.p, c.A_col.p, c.A_val.p, c.A_xr.p, c.A_xrows, x.p, nullptr, y.p, G, nullptr);
    });
    if (tx < best_x) {
      best_x = tx;
      c.g_X = G;
    }
  }
  const float ts = time_launch([&] {
    dev::sell_spmv(n, c.sell_nslices, c.sell_off.p, c.sell_width.p, c.sell_perm.p, c.sell_col.p, c.sell_val.p, x.p,
                   nullptr, y.p, nullptr);
  });
  c.spmv_auto = 1;
  best = best_csr;
  if (best_x < best) {
    best = best_x;
    c.spmv_auto = 3;
  }
  if (ts < best) {
    best = ts;
    c.spmv_auto = 2;
  }
  if (best_s < best) c.spmv_auto = 4;
  c.spmv_kind = c.spmv_auto;
  HELM_HIP(hipDeviceSynchronize());
}

namespace {

void spmv_A(Ctx& c, const double* x, const double* b, double* y, hipStream_t s) {
  if (c.spmv_kind == 2)
    dev::sell_spmv(c.D.n, c.sell_nslices, c.sell_off.p, c.sell_width.p, c.sell_perm.p, c.sell_col.p, c.sell_val.p, x,
                   b, y, s);
  else if (c.spmv_kind == 3)
    dev::spmv(c.D.n, c.A_ptr.p, c.A_col.p, c.A_val.p, c.A_xr.p, c.A_xrows, x, b, y, c.g_X, s);
  else if (c.spmv_kind == 4)
    dev::spmv_split(c.D.n, c.S_ptr.p, c.S_col.p, c.S_val.p, x, b, y, c.g_S, s);
  else
    dev::spmv(c.D.n, c.A_ptr.p, c.A_col.p, c.A_val.p, nullptr, 0, x, b, y, c.g_A, s);
}

}  // namespace

// The coarse solve is a chain of small levels whose launch gaps dominate its
// time.  When the device supports it, one cooperative launch with a grid-wide
// barrier per level is timed against per-level launches at a few grid sizes,
// and the fastest is kept.
void choose_coarse_launch(Ctx& c, int mode) {
  BatchDev& b = c.coarse;
  b.coop = 0;
  if (mode == 1) return;
  const int nf = (int)b.lev_f.size() - 1, nb = (int)b.lev_b.size() - 1;
  int attr = 0;
  const bool fits = !b.c64 && nf >= 1 && nb >= 1 && nf <= dev::kMaxLevels && nb <= dev::kMaxLevels;
  const bool coop_ok = hipDeviceGetAttribute(&attr, hipDeviceAttributeCooperativeLaunch, c.device) == hipSuccess &&
                       attr && fits;
  const int gmax = coop_ok ? dev::coop_grid() : 0;
  if (gmax <= 0) {
    if (mode == 2) fail(HELM_EINVAL, "the cooperative coarse solve is not available for this matrix or device");
    return;
  }
  b.ranges.nf = nf;
  b.ranges.nb = nb;
  for (int l = 0; l <= nf; ++l) b.ranges.f[l] = b.lev_f[l];
  for (int l = 0; l <= nb; ++l) b.ranges.b[l] = b.lev_b[l];
  // both launch forms must give the same solution: compare them on a fixed
  // right-hand side before the cooperative one may be used
  const int64_t nc = c.E.n;
  std::vector<double> in(2 * nc), x1(2 * nc), x2(2 * nc);
  for (int64_t i = 0; i < 2 * nc; ++i) in[i] = std::sin(0.37 * (double)i + 0.1);
  HELM_HIP(hipMemcpy(c.cvec.p, in.data(), sizeof(double) * 2 * nc, hipMemcpyHostToDevice));
  batch_solve(b, c.cvec.p, nullptr, nullptr, false);
  HELM_HIP(hipMemcpy(x1.data(), b.xout(), sizeof(double) * 2 * nc, hipMemcpyDeviceToHost));
  b.coop = gmax;
  const bool launched = coop_solve(b, b.view(), c.cvec.p, nullptr);
  b.coop = 0;
  if (!launched) {
    if (mode == 2) fail(HELM_EDEVICE, "the cooperative coarse solve could not be launched");
    return;  // keep the per-level launches
  }
  HELM_HIP(hipMemcpy(x2.data(), b.xout(), sizeof(double) * 2 * nc, hipMemcpyDeviceToHost));
  double dmax = 0, xmax = 0;
  for (int64_t i = 0; i < 2 * nc; ++i) {
    dmax = std::max(dmax, std::abs(x1[i] - x2[i]));
    xmax = std::max(xmax, std::abs(x1[i]));
  }
  if (!(dmax <= 1e-13 * xmax)) {
    if (mode == 2) fail(HELM_EDEVICE, "the cooperative coarse solve disagrees with the per-level launches");
    return;  // keep the per-level launches
  }
  std::vector<int> cands;
  if (mode == 0) cands.push_back(0);
  for (int g : {256, 512, 1024})
    if (g < gmax) cands.push_back(g);
  cands.push_back(gmax);
  b.coop = pick_lanes_per_row(cands, [&](int g) {
    b.coop = g;
    batch_solve(b, c.cvec.p, nullptr, nullptr, false);
  });
}

void precond_setup(Ctx& c, const int32_t* tet_part, int32_t n_sub, int32_t overlap, const helm_mesh* coarse,
                   const helm_precond_opts* opts) {
  auto t0 = std::chrono::steady_clock::now();
  c.free_precond();
  const bool on_device = c.device >= 0;
  const int leaf = opts && opts->leaf_size > 0 ? opts->leaf_size : 48;
  c.n_sub = n_sub;
  c.overlap = overlap;
  build_subdomains(c.D, tet_part, n_sub, overlap, c.subs);
  c.sym.resize(n_sub);
  const int trows = opts && opts->tile_rows > 0 ? opts->tile_rows : 64;
  const int ctrows = opts && opts->coarse_tile_rows > 0 ? opts->coarse_tile_rows : 16;
  if (trows != 16 && trows != 32 && trows != 64) fail(HELM_EINVAL, "tile_rows must be 16, 32 or 64");
  if (ctrows != 16 && ctrows != 32 && ctrows != 64) fail(HELM_EINVAL, "coarse_tile_rows must be 16, 32 or 64");
  const int64_t snmin = !opts || opts->sn_jobs_min == 0 ? 6144 : (opts->sn_jobs_min < 0 ? -1 : opts->sn_jobs_min);
  const int cmode = opts ? opts->coarse_launch : 0;
  if (cmode < 0 || cmode > 2) fail(HELM_EINVAL, "coarse_launch must be 0, 1 or 2");
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t i = 0; i < n_sub; ++i) nested_dissection(c.subs[i].A, c.subs[i].coords, leaf, c.sym[i], trows);
  helm_precond_stats& st = c.stats;
  st.n_sub = n_sub;
  for (auto& S : c.subs) st.n_local_total += (int64_t)S.dofs.size();
  // fine batch
  std::vector<const Csr*> As;
  std::vector<const Symbolic*> Ss;
  std::vector<const std::vector<int64_t>*> in;
  for (int32_t i = 0; i < n_sub; ++i) {
    As.push_back(&c.subs[i].A);
    Ss.push_back(&c.sym[i]);
    in.push_back(&c.subs[i].dofs);
  }
  int32_t npert = 0;
  const int32_t c64mode = opts ? opts->factor_c64 : 0;
  if (c64mode < 0 || c64mode > 2) fail(HELM_EINVAL, "factor_c64 must be 0, 1 or 2");
  const bool c64 = c64mode != 0;
  const int32_t split_opt = opts ? opts->split_front_rows : 0;
  if (split_opt < -1) fail(HELM_EINVAL, "split_front_rows must be -1, 0 or positive");
  const int32_t split_min = split_opt == 0 ? dev::kSplitFrontMin : split_opt;
  const dev::FactorPrecision prec = !c64           ? dev::FactorPrecision::kC128
                                    : c64mode == 1 ? dev::FactorPrecision::kC64
                                                   : dev::FactorPrecision::kC128RoundedC64;
  double fsec = 0, csec = 0;
  // nb consecutive batches of about equal panel entries (their level sweeps
  // overlap on nb streams): batch k ends at the first subdomain count whose
  // running total reaches k / nb of all entries
  const int32_t want = !opts || opts->batches == 0 ? 2 : opts->batches;
  if (want < 1 || want > kMaxBatches) fail(HELM_EINVAL, "batches must be 0 .. 4");
  const int32_t nb = on_device ? std::min(want, n_sub) : 1;
  std::vector<int32_t> bnd(nb + 1, 0);
  bnd[nb] = n_sub;
  {
    double tot = 0, run = 0;
    for (auto& S : c.sym) tot += (double)(S.fwd_entries + S.bwd_entries);
    int32_t i = 0;
    for (int32_t k = 1; k < nb; ++k) {
      while (i < n_sub && run < tot * k / nb) run += (double)(c.sym[i].fwd_entries + c.sym[i].bwd_entries), ++i;
      bnd[k] = std::min(std::max(i, bnd[k - 1] + 1), n_sub - (nb - k));
    }
  }
  auto part = [&](auto& v, int32_t a, int32_t b) {
    return std::vector<typename std::decay_t<decltype(v)>::value_type>(v.begin() + a, v.begin() + b);
  };
  // concurrent batches fill the device together: each takes one-wave jobs
  // at 1 / nb of the threshold
  const int64_t snb = nb > 1 && snmin > 0 ? std::max<int64_t>(1, snmin / nb) : snmin;
  c.nbatch = nb;
  st.factor_entries = 0;
  int64_t npos_all = 0;
  // on the device all subdomains are factorised together (every level's
  // fronts of every batch in the same launches), each into its batch's
  // panel arrays
  std::vector<NumericOut> num_all;
  if (on_device) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<void*> pf, pb;
    for (int32_t k = 0; k < nb; ++k) {
      c.fine[k].pf.reset();
      c.fine[k].pb.reset();
      alloc_panels(part(Ss, bnd[k], bnd[k + 1]), prec, c.fine[k], pf, pb);
    }
    num_all.resize(n_sub);
    double sb = 0;
    factor_batch_device(As, Ss, prec, split_min, pf, pb, num_all, npert, sb);
    st.factor_scratch_bytes = std::max(st.factor_scratch_bytes, sb);
    fsec += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  for (int32_t k = 0; k < nb; ++k) {
    BatchHost fb;
    int32_t np = 0;
    double fs = 0;
    std::vector<NumericOut> pre;
    if (!num_all.empty()) pre.assign(num_all.begin() + bnd[k], num_all.begin() + bnd[k + 1]);
    build_batch(part(As, bnd[k], bnd[k + 1]), part(Ss, bnd[k], bnd[k + 1]), part(in, bnd[k], bnd[k + 1]), c.device,
                on_device, prec, split_min, snb, fb, c.fine[k], np, fs, num_all.empty() ? nullptr : &pre);
    npert += np;
    fsec += fs;
    st.factor_entries += fb.nf + fb.nb;
    st.levels_fwd = std::max(st.levels_fwd, (int32_t)fb.lev_f.size() - 1);
    st.levels_bwd = std::max(st.levels_bwd, (int32_t)fb.lev_b.size() - 1);
    st.max_front = std::max(st.max_front, fb.max_front);
    st.factor_flops += fb.flops;
    npos_all += fb.npos;
  }
  if (nb > 1) {
    // one output vector in subdomain order, as the prolongation map expects
    c.xall.alloc(2 * (size_t)npos_all);
    int64_t o = 0;
    for (int32_t k = 0; k < nb; ++k) {
      c.fine[k].xo = c.xall.p + 2 * o;
      o += c.fine[k].npos;
      c.fine[k].x.reset();
    }
    if (!c.ev_fork) HELM_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
    for (int32_t k = 1; k < nb; ++k) {
      if (!c.sb[k]) HELM_HIP(hipStreamCreateWithFlags(&c.sb[k], hipStreamNonBlocking));
      if (!c.ev_join[k]) HELM_HIP(hipEventCreateWithFlags(&c.ev_join[k], hipEventDisableTiming));
    }
  }
  st.factor_c64 = prec == dev::FactorPrecision::kC64 ? 1 : prec == dev::FactorPrecision::kC128RoundedC64 ? 2 : 0;
  st.batches = nb;
  for (auto& S : c.sym) st.n_supernodes += S.nsn;
  // prolongation map: global dof -> positions with D > 0, in subdomain order
  {
    const int64_t n = c.D.n;
    std::vector<int64_t> ptr(n + 1, 0);
    for (auto& S : c.subs)
      for (size_t k = 0; k < S.dofs.size(); ++k)
        if (S.D[k] > 0) ptr[S.dofs[k] + 1]++;
    for (int64_t g = 0; g < n; ++g) ptr[g + 1] += ptr[g];
    std::vector<int32_t> idx(ptr[n]);
    std::vector<double> wt(ptr[n]);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    int64_t pos0 = 0;
    for (int32_t i = 0; i < n_sub; ++i) {
      const SubdomainHost& S = c.subs[i];
      for (size_t k = 0; k < S.dofs.size(); ++k)
        if (S.D[k] > 0) {
          int64_t q = fill[S.dofs[k]]++;
          idx[q] = (int32_t)(pos0 + c.sym[i].iperm[k]);
          wt[q] = S.D[k];
        }
      pos0 += (int64_t)S.dofs.size();
    }
    if (on_device) {
      c.pro_ptr.upload(ptr);
      c.pro_idx.upload(idx);
      c.pro_w.upload(wt);
    }
  }
  // coarse level
  if (coarse) {
    std::vector<double> ccoords;
    coarse_interpolation(c.D, *coarse, c.Z, ccoords);
    transpose_real(c.Z, c.ZT);
    galerkin(c.D.A, c.Z, c.ZT, c.E);
    const int cleaf = opts && opts->coarse_leaf_size > 0 ? opts->coarse_leaf_size : 256;
    nested_dissection(c.E, ccoords, cleaf, c.Esym, ctrows);
    std::vector<int64_t> ident(c.E.n);
    std::iota(ident.begin(), ident.end(), 0);
    BatchHost cb;
    int32_t np2 = 0;
    double csb = 0;
    build_batch({&c.E}, {&c.Esym}, {&ident}, c.device, on_device, dev::FactorPrecision::kC128, split_min, snmin, cb,
                c.coarse, np2, csec, nullptr, &csb);
    st.factor_scratch_bytes = std::max(st.factor_scratch_bytes, csb);
    npert += np2;
    c.two_level = true;
    st.n_coarse = (int32_t)c.E.n;
    st.coarse_entries = cb.nf + cb.nb;
    if (on_device) {
      // Z with columns renumbered to the coarse solve's output positions
      CsrReal Zp = c.Z;
      for (auto& col : Zp.col) col = c.Esym.iperm[col];
      for (int64_t i = 0; i < Zp.n; ++i) {
        std::vector<std::pair<int32_t, double>> e;
        for (int64_t p = Zp.ptr[i]; p < Zp.ptr[i + 1]; ++p) e.push_back({Zp.col[p], Zp.val[p]});
        std::sort(e.begin(), e.end());
        for (size_t q = 0; q < e.size(); ++q) {
          Zp.col[Zp.ptr[i] + q] = e[q].first;
          Zp.val[Zp.ptr[i] + q] = e[q].second;
        }
      }
      c.Zp_ptr.upload(Zp.ptr);
      c.Zp_col.upload(Zp.col);
      c.Zp_val.upload(Zp.val);
      {
        // (A Z)_ik = sum_j A_ij Z_jk, row by row; real parts, then the
        // nonzero imaginary parts flagged in the column index
        const Csr& A = c.D.A;
        const int64_t n = A.n, nc = c.E.n, blk = 4096, nblk = (n + blk - 1) / blk;
        std::vector<std::vector<int64_t>> bp(nblk);
        std::vector<std::vector<int32_t>> bc(nblk);
        std::vector<std::vector<double>> bv(nblk);
#pragma omp parallel
        {
          std::vector<cplx> acc(nc);
          std::vector<char> seen(nc, 0);
          std::vector<int32_t> touched;
#pragma omp for schedule(dynamic, 1)
          for (int64_t b = 0; b < nblk; ++b) {
            for (int64_t i = b * blk; i < std::min(n, (b + 1) * blk); ++i) {
              touched.clear();
              for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int64_t j = A.col[p];
                for (int64_t q = Zp.ptr[j]; q < Zp.ptr[j + 1]; ++q) {
                  const int32_t k = Zp.col[q];
                  if (!seen[k]) {
                    seen[k] = 1;
                    acc[k] = cplx(0, 0);
                    touched.push_back(k);
                  }
                  acc[k] += A.val[p] * Zp.val[q];
                }
              }
              std::sort(touched.begin(), touched.end());
              for (int32_t k : touched) {
                bc[b].push_back(k);
                bv[b].push_back(acc[k].real());
              }
              for (int32_t k : touched)
                if (acc[k].imag() != 0.0) {
                  bc[b].push_back((int32_t)((uint32_t)k | 0x80000000u));
                  bv[b].push_back(acc[k].imag());
                }
              for (int32_t k : touched) seen[k] = 0;
              bp[b].push_back((int64_t)bc[b].size());
            }
          }
        }
        std::vector<int64_t> ap(1, 0);
        std::vector<int32_t> acol;
        std::vector<double> aval;
        for (int64_t b = 0; b < nblk; ++b) {
          const int64_t base = (int64_t)acol.size();
          for (int64_t e : bp[b]) ap.push_back(base + e);
          acol.insert(acol.end(), bc[b].begin(), bc[b].end());
          aval.insert(aval.end(), bv[b].begin(), bv[b].end());
        }
        c.AZ_ptr.upload(ap);
        c.AZ_col.upload(acol);
        c.AZ_val.upload(aval);
      }
      c.ZT_ptr.upload(c.ZT.ptr);
      c.ZT_col.upload(c.ZT.col);
      c.ZT_val.upload(c.ZT.val);
      c.cvec.alloc(2 * c.E.n);
      DVec<double> x, y;
      x.alloc(2 * c.D.n);
      y.alloc(2 * c.D.n);
      HELM_HIP(hipMemset(x.p, 0, sizeof(double) * 2 * c.D.n));
      c.g_ZT = pick_lanes_per_row({4, 8, 16, 32, 64}, [&](int G) {
        dev::spmv_real(c.ZT.n, c.ZT_ptr.p, c.ZT_col.p, c.ZT_val.p, x.p, y.p, G, nullptr);
      });
      c.g_Zp = pick_lanes_per_row({4, 8}, [&](int G) {
        dev::spmv_real(c.D.n, c.Zp_ptr.p, c.Zp_col.p, c.Zp_val.p, x.p, y.p, G, nullptr);
      });
      DVec<double> x2;
      x2.alloc(2 * c.D.n);
      c.g_AZ = pick_lanes_per_row({1, 2, 4, 8}, [&](int G) {
        dev::coarse_update(c.D.n, c.Zp_ptr.p, c.Zp_col.p, c.Zp_val.p, c.AZ_ptr.p, c.AZ_col.p, c.AZ_val.p, x.p, x.p,
                           y.p, x2.p, G, nullptr);
      });
      choose_coarse_launch(c, cmode);
      st.coarse_grid = c.coarse.coop;
    }
  }
  if (on_device) {
    c.t.alloc(2 * c.D.n);
    c.q.alloc(2 * c.D.n);
    HELM_HIP(hipDeviceSynchronize());
  }
  st.n_perturbed = npert;
  if (npert > 0 && !(opts && opts->perturb_pivots))
    fail(HELM_ESINGULAR, std::to_string(npert) +
                             " zero or tiny pivots (|pivot| <= 1000 eps max|a_ij|) in the local or coarse factors;"
                             " helm_precond_opts.perturb_pivots replaces them instead");
  st.factor_seconds = fsec + csec;
  st.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  c.precond_ready = true;
}

double spmv_bytes(const Ctx& c, bool residual) {
  const double n = (double)c.D.n, nnz = (double)c.D.A.nnz();
  const double entries = c.spmv_kind == 4 ? 12.0 * (double)c.S_nnz : 20.0 * nnz;
  return entries + 8.0 * (n + 1) + 16.0 * n * (residual ? 3 : 2);
}

void apply_A(Ctx& c, const double* x, double* y, hipStream_t s) {
  const bool p = c.prof.on;
  if (p) c.prof.begin(s);
  spmv_A(c, x, nullptr, y, s);
  if (p) c.prof.end(HELM_K_SPMV, spmv_bytes(c, false), s);
}

// Bytes of the work vectors of one coarse correction (Z^T r, and the coarse
// batch's forward result, backward result and update vectors), each region
// 256-byte aligned.
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }
size_t coarse_scratch_bytes(const Ctx& c) {
  const size_t nc = (size_t)c.E.n, np = (size_t)std::max<int64_t>(c.coarse.npos, 1);
  const size_t nu = std::max<size_t>(c.coarse.ubuf.n / 2, 1);
  return align256(16 * nc) + 2 * align256(16 * np) + align256(16 * nu);
}

// q = Z E^{-1} Z^T r with the work vectors in `scratch` (device memory of at
// least coarse_scratch_bytes): the same kernels as apply_coarse, no
// allocation, no timing events.
void apply_coarse_scratch(Ctx& c, const double* r, double* q, hipStream_t s, void* scratch) {
  const size_t nc = (size_t)c.E.n, np = (size_t)std::max<int64_t>(c.coarse.npos, 1);
  unsigned char* base = static_cast<unsigned char*>(scratch);
  double* cv = reinterpret_cast<double*>(base);
  base += align256(16 * nc);
  double* y = reinterpret_cast<double*>(base);
  base += align256(16 * np);
  double* x = reinterpret_cast<double*>(base);
  base += align256(16 * np);
  double* ub = reinterpret_cast<double*>(base);
  dev::spmv_real(c.ZT.n, c.ZT_ptr.p, c.ZT_col.p, c.ZT_val.p, r, cv, c.g_ZT, s);
  dev::Batch v = c.coarse.view();
  v.y = y;
  v.x = x;
  v.ubuf = ub;
  batch_solve_view(c.coarse, v, cv, s);
  dev::spmv_real(c.D.n, c.Zp_ptr.p, c.Zp_col.p, c.Zp_val.p, x, q, c.g_Zp, s);
}

void apply_coarse(Ctx& c, const double* r, double* q, hipStream_t s) {
  const bool p = c.prof.on;
  if (p) c.prof.begin(s);
  dev::spmv_real(c.ZT.n, c.ZT_ptr.p, c.ZT_col.p, c.ZT_val.p, r, c.cvec.p, c.g_ZT, s);
  batch_solve(c.coarse, c.cvec.p, s, &c.prof, false);
  dev::spmv_real(c.D.n, c.Zp_ptr.p, c.Zp_col.p, c.Zp_val.p, c.coarse.x.p, q, c.g_Zp, s);
  if (p) {
    const double zb = 2.0 * (12.0 * (double)c.Z.col.size() + 8.0 * c.D.n) + 16.0 * (c.D.n + c.E.n);
    c.prof.end(HELM_K_COARSE, zb + sum(c.coarse.bytes_f) + sum(c.coarse.bytes_b), s);
  }
}

// Runs f(batch, stream) for every subdomain batch: batches 1.. on their own
// streams, forked from and joined back to s, batch 0 on s; one after the
// other on s while kernels are timed launch by launch.
template <class F>
void for_batches(Ctx& c, hipStream_t s, F&& f) {
  if (c.nbatch == 1 || c.prof.on) {
    for (int k = 0; k < c.nbatch; ++k) f(c.fine[k], s);
    return;
  }
  HELM_HIP(hipEventRecord(c.ev_fork, s));
  for (int k = 1; k < c.nbatch; ++k) {
    HELM_HIP(hipStreamWaitEvent(c.sb[k], c.ev_fork, 0));
    f(c.fine[k], c.sb[k]);
  }
  f(c.fine[0], s);
  for (int k = 1; k < c.nbatch; ++k) {
    HELM_HIP(hipEventRecord(c.ev_join[k], c.sb[k]));
    HELM_HIP(hipStreamWaitEvent(s, c.ev_join[k], 0));
  }
}

void apply_oras(Ctx& c, const double* r, double* z, const double* q, hipStream_t s) {
  Profiler* prof = c.prof.on ? &c.prof : nullptr;
  for_batches(c, s, [&](BatchDev& b, hipStream_t sk) { batch_solve(b, r, sk, prof, true); });
  const bool p = c.prof.on;
  if (p) c.prof.begin(s);
  dev::prolong(c.D.n, c.pro_ptr.p, c.pro_idx.p, c.pro_w.p, c.fine[0].xout(), q, z, s);
  if (p) c.prof.end(HELM_K_PROLONG, 12.0 * c.pro_w.n + 28.0 * c.pro_w.n + 16.0 * c.D.n * (q ? 2 : 1) + 8.0 * c.D.n, s);
}

// Two-level M^{-1} in two stages: the coarse part (q = Z E^{-1} Z^T r,
// t = r - A q; nothing for one level) and the subdomain part (z = sum R_i^T
// D_i A_i^{-1} R_i t + q).  The first stage only writes the work vectors q
// and t, so a solver may enqueue it ahead of a decision it has not taken yet.
void precond_stage1(Ctx& c, const double* r, hipStream_t s) {
  if (!c.two_level) return;
  // q = Z E^{-1} Z^T r and t = r - A q = r - (A Z) E^{-1} Z^T r
  const bool p = c.prof.on;
  if (p) c.prof.begin(s);
  dev::spmv_real(c.ZT.n, c.ZT_ptr.p, c.ZT_col.p, c.ZT_val.p, r, c.cvec.p, c.g_ZT, s);
  batch_solve(c.coarse, c.cvec.p, s, &c.prof, false);
  dev::coarse_update(c.D.n, c.Zp_ptr.p, c.Zp_col.p, c.Zp_val.p, c.AZ_ptr.p, c.AZ_col.p, c.AZ_val.p, c.coarse.x.p, r,
                     c.q.p, c.t.p, c.g_AZ, s);
  if (p) {
    const double zb = 12.0 * (double)c.Z.col.size() + 8.0 * c.E.n + 16.0 * (c.D.n + c.E.n);
    const double ub = 12.0 * (double)(c.Z.col.size() + c.AZ_col.n) + 16.0 * (double)c.D.n + 48.0 * c.D.n;
    c.prof.end(HELM_K_COARSE, zb + ub + sum(c.coarse.bytes_f) + sum(c.coarse.bytes_b), s);
  }
}
void precond_stage2(Ctx& c, const double* r, double* z, hipStream_t s) {
  if (!c.two_level)
    apply_oras(c, r, z, nullptr, s);
  else
    apply_oras(c, c.t.p, z, c.q.p, s);
}

void apply_precond(Ctx& c, const double* r, double* z, hipStream_t s) {
  precond_stage1(c, r, s);
  precond_stage2(c, r, z, s);
}

namespace {

void ensure_norm(Ctx& c) {
  const int nblk = dev::gs_blocks(c.D.n);
  if (c.npart.n < 2 * (size_t)nblk) c.npart.alloc(2 * (size_t)nblk);
  if (!c.nval.p) c.nval.alloc(2);
  if (!c.nh_host) HELM_HIP(hipHostMalloc((void**)&c.nh_host, 2 * sizeof(double), hipHostMallocDefault));
}

double device_norm(Ctx& c, const double* v, hipStream_t s) {
  ensure_norm(c);
  const int nblk = dev::gs_blocks(c.D.n);
  dev::norm2(c.D.n, v, c.npart.p, nblk, c.nval.p, s);
  HELM_HIP(hipMemcpyAsync(c.nh_host, c.nval.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HELM_HIP(hipStreamSynchronize(s));
  return c.nh_host[0];
}

void ensure_gmres(Ctx& c, int m) {
  if (c.gm_m == m && c.gm_n == c.D.n && c.V.p) return;
  const int64_t n = c.D.n;
  c.V.alloc(2 * (size_t)n * (m + 1));
  c.Zk.alloc(2 * (size_t)n * m);
  c.w.alloc(2 * (size_t)n);
  const int nblk = std::max(dev::gs_blocks(n), dev::gs_tiles(n));
  c.partial.alloc(2 * (size_t)nblk * (2 * m + 4));
  c.hcol.alloc(2 * (size_t)(2 * m + 4));
  c.htmp.alloc(2 * (size_t)(2 * m + 4));
  c.coef_w.alloc(2 * (size_t)(m + 2));
  c.coef_v.alloc(2 * (size_t)(m + 2));
  c.nrm.alloc(2);
  c.ydev.alloc(2 * (size_t)(m + 1));
  if (c.h_host) (void)hipHostFree(c.h_host);
  c.h_host = nullptr;
  HELM_HIP(hipHostMalloc((void**)&c.h_host, 2 * sizeof(double) * (2 * m + 4), hipHostMallocDefault));
  if (!c.hev) HELM_HIP(hipEventCreateWithFlags(&c.hev, hipEventDisableTiming));
  c.gm_m = m;
  c.gm_n = n;
}

}  // namespace

namespace {

// One right-hand side at a time.
// Givens step on column jj of H (rotations 0..jj-1 applied, new rotation
// jj, residual vector g updated).
void givens_step(cplx* h, int jj, std::vector<double>& cs, std::vector<cplx>& sn, std::vector<cplx>& g) {
  for (int i = 0; i < jj; ++i) {
    const cplx a = h[i], bb = h[i + 1];
    h[i] = cs[i] * a + sn[i] * bb;
    h[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
  }
  const cplx a = h[jj], bb = h[jj + 1];
  if (a == cplx(0, 0)) {
    cs[jj] = 0;
    sn[jj] = 1;
  } else {
    const double r = std::sqrt(std::norm(a) + std::norm(bb));
    cs[jj] = std::abs(a) / r;
    sn[jj] = (a / std::abs(a)) * std::conj(bb) / r;
  }
  h[jj] = cs[jj] * a + sn[jj] * bb;
  h[jj + 1] = 0;
  g[jj + 1] = -std::conj(sn[jj]) * g[jj];
  g[jj] = cs[jj] * g[jj];
}

dev::PtrSet pset(double* p) {
  dev::PtrSet q{};
  q.p[0] = p;
  return q;
}
dev::PtrSetC csetc(const double* p) {
  dev::PtrSetC q{};
  q.p[0] = p;
  return q;
}

// Pass A of delayed CGS2 over the first ncol columns of V (the last one
// orthogonalised once so far) and c.w, then the pass-B coefficients (c.coef_w,
// c.coef_v) and the host-bound data in c.hcol: [V_{<j}^H w, h_j, |w| slot,
// s (j entries), alpha] with j = ncol - 1.
void dual_pass_a(Ctx& c, int ncol, hipStream_t s) {
  const int64_t n = c.D.n;
  dev::gs_dual(false, 1, n, csetc(c.V.p), pset(c.V.p), n, ncol, csetc(c.coef_w.p), csetc(c.coef_v.p), pset(c.w.p),
               pset(c.partial.p), s);
  dev::gs_final(1, csetc(c.partial.p), dev::gs_tiles(n), 2 * ncol, pset(c.htmp.p), dev::PtrSet{}, 0, s);
  dev::dcgs2_coef(1, csetc(c.htmp.p), ncol, pset(c.coef_w.p), pset(c.coef_v.p), pset(c.hcol.p), s);
}

// Column j of H (unrotated) finished with the second-pass data of v_{j+1}:
// v_{j+1} (once orthogonalised) = alpha v_{j+1} (final) + sum_k s_k v_k, so
// h_{k,j} += h_{j+1,j} s_k (k <= j) and h_{j+1,j} *= alpha.  s holds j + 1
// interleaved complex values.
void finish_column(cplx* h, int j, const double* sv, double alpha) {
  for (int k = 0; k <= j; ++k) h[k] += h[j + 1] * cplx(sv[2 * k], sv[2 * k + 1]);
  h[j + 1] *= alpha;
}

int solve_single(Ctx& c, int32_t nrhs, const double* B, double tol, int m, int maxit, bool x0, bool dcgs2,
                 double* U, hipStream_t s, helm_solve_info* info) {
  ensure_gmres(c, m);
  const int64_t n = c.D.n;
  double* V = c.V.p;
  double* Zk = c.Zk.p;
  std::vector<cplx> H((size_t)(m + 1) * m), g(m + 1), sn(m), hc(m + 1);
  std::vector<double> cs(m);
  std::vector<cplx> y(m);
  int status = HELM_OK;
  for (int32_t j = 0; j < nrhs; ++j) {
    auto t0 = std::chrono::steady_clock::now();
    const double* b = B + 2 * (size_t)n * j;
    double* x = U + 2 * (size_t)n * j;
    helm_solve_info inf{};
    const double bnorm = device_norm(c, b, s);
    if (!std::isfinite(bnorm)) fail(HELM_ENUMERIC, "non-finite right-hand side");
    if (bnorm == 0) {
      dev::fill_zero(2 * n, x, s);
      HELM_HIP(hipStreamSynchronize(s));
      inf.converged = 1;
      if (info) info[j] = inf;
      continue;
    }
    if (!x0) dev::fill_zero(2 * n, x, s);
    int its = 0;
    bool conv = false;
    double rel = 0;
    while (true) {
      spmv_A(c, x, b, V, s);  // r = b - A x
      const double beta = device_norm(c, V, s);
      if (!std::isfinite(beta)) fail(HELM_ENUMERIC, "non-finite residual");
      rel = beta / bnorm;
      if (beta <= tol * bnorm) {
        conv = true;
        break;
      }
      if (its >= maxit) break;
      dev::scale(n, V, 1.0 / beta, V, s);
      std::fill(g.begin(), g.end(), cplx(0, 0));
      g[0] = beta;
      int k = 0;
      precond_stage1(c, V, s);
      for (int jj = 0; jj < m; ++jj) {
        double* vj = V + 2 * (size_t)n * jj;
        double* zj = Zk + 2 * (size_t)n * jj;
        precond_stage2(c, vj, zj, s);
        apply_A(c, zj, c.w.p, s);
        const bool prof = c.prof.on;
        if (prof) c.prof.begin(s);
        const int nt = dev::gs_tiles(n);
        dev::PtrSetC Vs{}, ps{};
        dev::PtrSet ws{}, pw{}, nrm{}, vn{};
        Vs.p[0] = V;
        ps.p[0] = c.partial.p;
        ws.p[0] = c.w.p;
        pw.p[0] = c.partial.p;
        nrm.p[0] = c.hcol.p + 2 * (jj + 1);
        vn.p[0] = V + 2 * (size_t)n * (jj + 1);
        int nout;  // complex entries of hcol the host reads
        if (dcgs2) {
          // pass A: V^H w and V^H v_j | coefficients | pass B: v_j finished,
          // w orthogonalised, |w|^2
          dual_pass_a(c, jj + 1, s);
          dev::gs_dual(true, 1, n, Vs, pset(V), n, jj + 1, csetc(c.coef_w.p), csetc(c.coef_v.p), ws, pw, s);
          dev::norm_final(1, ps, nt, nrm, s);
          nout = 2 * jj + 3;
        } else {
          // CGS2: dots | update + dots | update + norm, each one pass over V
          dev::PtrSetC hs{};
          dev::PtrSet hts{}, hcs{};
          hs.p[0] = c.htmp.p;
          hts.p[0] = c.htmp.p;
          hcs.p[0] = c.hcol.p;
          dev::gs_pass(0, 1, n, Vs, n, jj + 1, hs, ws, pw, s);
          dev::gs_final(1, ps, nt, jj + 1, hts, hcs, 0, s);
          dev::gs_pass(1, 1, n, Vs, n, jj + 1, hs, ws, pw, s);
          dev::gs_final(1, ps, nt, jj + 1, hts, hcs, 1, s);
          dev::gs_pass(2, 1, n, Vs, n, jj + 1, hs, ws, pw, s);
          dev::norm_final(1, ps, nt, nrm, s);
          nout = jj + 2;
        }
        dev::scale_by_inv_set(1, n, csetc(c.w.p), csetc(nrm.p[0]), vn, s);
        if (prof)
          c.prof.end(HELM_K_GS, 16.0 * n * (dcgs2 ? 2.0 * (jj + 1) + 6.0 : 3.0 * (jj + 1) + 7.0), s);
        HELM_HIP(hipMemcpyAsync(c.h_host, c.hcol.p, 2 * sizeof(double) * nout, hipMemcpyDeviceToHost, s));
        HELM_HIP(hipEventRecord(c.hev, s));
        // the next step's coarse stage runs while the host updates the
        // least-squares problem (wasted only when this step ends the cycle)
        if (jj + 1 < m && its + 1 < maxit) precond_stage1(c, V + 2 * (size_t)n * (jj + 1), s);
        HELM_HIP(hipEventSynchronize(c.hev));
        ++its;
        for (int i = 0; i < 2 * nout; ++i)
          if (!std::isfinite(c.h_host[i])) fail(HELM_ENUMERIC, "non-finite Hessenberg entry");
        auto hget = [&](int i) { return cplx(c.h_host[2 * i], c.h_host[2 * i + 1]); };
        cplx* h = H.data() + (size_t)(m + 1) * jj;
        for (int i = 0; i <= jj + 1; ++i) h[i] = hget(i);
        const double hn = h[jj + 1].real();
        if (!dcgs2) {
          givens_step(h, jj, cs, sn, g);
          k = jj + 1;
          if (std::abs(g[jj + 1]) <= tol * bnorm || its >= maxit || hn == 0) break;
          continue;
        }
        // delayed CGS2: v_j's second pass finishes column j - 1 of H
        if (jj >= 1) finish_column(H.data() + (size_t)(m + 1) * (jj - 1), jj - 1, &c.h_host[2 * (jj + 2)], c.h_host[2 * (2 * jj + 2)]);
        if (jj >= 1) givens_step(H.data() + (size_t)(m + 1) * (jj - 1), jj - 1, cs, sn, g);
        // residual estimate from column j as it stands (its last correction,
        // below the orthogonality error of v_{j+1}, comes with the next step)
        double est;
        {
          for (int i = 0; i <= jj + 1; ++i) hc[i] = h[i];
          for (int i = 0; i < jj; ++i) {
            const cplx a = hc[i], bb = hc[i + 1];
            hc[i] = cs[i] * a + sn[i] * bb;
            hc[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
          }
          const double r = std::sqrt(std::norm(hc[jj]) + std::norm(hc[jj + 1]));
          est = hc[jj] == cplx(0, 0) ? std::abs(g[jj]) : std::abs(hc[jj + 1]) / r * std::abs(g[jj]);
        }
        if (est <= tol * bnorm || jj + 1 == m || its >= maxit || hn == 0) {
          if (hn > 0) {
            // finish column j with the dots of v_{j+1}
            dual_pass_a(c, jj + 2, s);
            HELM_HIP(hipMemcpyAsync(c.h_host, c.hcol.p, 2 * sizeof(double) * (2 * jj + 5), hipMemcpyDeviceToHost, s));
            HELM_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < 2 * (2 * jj + 5); ++i)
              if (!std::isfinite(c.h_host[i])) fail(HELM_ENUMERIC, "non-finite Hessenberg entry");
            finish_column(h, jj, &c.h_host[2 * (jj + 3)], c.h_host[2 * (2 * jj + 4)]);
          }
          givens_step(h, jj, cs, sn, g);
          k = jj + 1;
          break;
        }
      }
      // back substitution R y = g
      for (int i = k - 1; i >= 0; --i) {
        cplx acc = g[i];
        for (int l = i + 1; l < k; ++l) acc -= H[(size_t)(m + 1) * l + i] * y[l];
        y[i] = acc / H[(size_t)(m + 1) * i + i];
      }
      HELM_HIP(hipMemcpyAsync(c.ydev.p, y.data(), sizeof(cplx) * k, hipMemcpyHostToDevice, s));
      dev::gemv_acc(n, Zk, n, k, c.ydev.p, x, s);
      HELM_HIP(hipStreamSynchronize(s));  // y is reused by the next cycle
      if (c.prof.on) c.prof.harvest();
    }
    HELM_HIP(hipStreamSynchronize(s));
    if (c.prof.on) c.prof.harvest();
    inf.iterations = its;
    inf.converged = conv ? 1 : 0;
    inf.relres = rel;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) info[j] = inf;
    if (!conv) status = HELM_ENOCONV;
  }
  return status;
}


void ensure_batch_block(BatchDev& b, int S) {
  if (b.blk_S >= S) return;
  const size_t nu = std::max<size_t>(b.ubuf.n / 2, 1), np = std::max<int64_t>(b.npos, 1);
  b.ubuf_b.alloc(2 * nu * S);
  b.y_b.alloc(2 * np * S);
  b.x_b.alloc(2 * np * S);
  if (S == dev::kMaxBlock) b.stage.alloc(sizeof(double) * 2 * dev::kMaxBlock * std::max<int64_t>(b.stage_cols, 1));
  b.blk_S = S;
}

// Complex entries per right-hand side in the block Hessenberg, reduction
// and host buffers (delayed CGS2 reads up to 2 m + 3 of them per step).
size_t blk_ld(int m) { return 2 * (size_t)m + 4; }

}  // namespace

// Krylov bases (V: m + 1 columns, Z_m: m columns, a work vector) of the
// first `count` right-hand sides of a block or server slots.
size_t basis_bytes(int64_t n, int m) { return sizeof(double) * 2 * (size_t)n * (2 * (size_t)m + 2); }

void ensure_bases(Ctx& c, int m, int count) {
  const int64_t n = c.D.n;
  if (c.blk_m != m || c.blk_n != n) {
    for (int r = 0; r < dev::kMaxBlock; ++r) {
      c.bV[r].reset();
      c.bZ[r].reset();
      c.bw[r].reset();
    }
    c.blk_bases = 0;
    c.blk_cap = 0;  // the per-width buffers depend on m too
    c.blk_m = m;
    c.blk_n = n;
  }
  for (int r = c.blk_bases; r < count; ++r) {
    c.bV[r].alloc(2 * (size_t)n * (m + 1));
    c.bZ[r].alloc(2 * (size_t)n * m);
    c.bw[r].alloc(2 * (size_t)n);
    c.blk_bases = r + 1;
  }
}

// Device bytes of the buffers of a block S columns wide (apart from the
// Krylov bases): interleaved block vectors, the subdomain and coarse batch
// work vectors, the staging block of the 16-column level solves, the
// Gram-Schmidt reductions.
size_t width_bytes(const Ctx& c, int m, int S) {
  const size_t n = (size_t)c.D.n;
  size_t e = 5 * n * S;  // bX, bZb, bW, bq, bt (complex entries)
  if (c.two_level) e += (size_t)c.E.n * S;
  auto batch = [&](const BatchDev& b) {
    size_t v = (std::max<size_t>(b.ubuf.n / 2, 1) + 2 * std::max<int64_t>(b.npos, 1)) * S;
    if (S == dev::kMaxBlock) v += dev::kMaxBlock * std::max<int64_t>(b.stage_cols, 1);
    return v;
  };
  int64_t npos_all = 0;
  for (int k = 0; k < c.nbatch; ++k) {
    e += batch(c.fine[k]);
    npos_all += c.fine[k].npos;
  }
  if (c.nbatch > 1) e += (size_t)npos_all * S;
  if (c.two_level) e += batch(c.coarse);
  e += (size_t)dev::kMaxBlock * ((2 + dev::gs_tiles(c.D.n)) * blk_ld(m) + 2 * (m + 2)) + (m + 1);
  return 16 * e;
}

// Buffers of blocks up to S columns wide (bases are separate, ensure_bases).
// 16-column level solves of a fine batch: the tiles a level gives four
// waves each (the others one wave each) are a prefix of the level's tiles.
// The candidates -- the four- and two-wave classes (the default), the
// four-wave class alone, no tile, every tile -- are timed once per level on
// the first 16-column use (three launches each after one untimed) and the
// fastest is kept.  The timed sweeps read whatever the work vectors hold;
// every solve runs its sweeps afresh.  HELM_BLOCK_SPLIT = 0..3 in the
// environment takes candidate 0..3 on every level without timing.
void tune_block_levels(BatchDev& b, const double* in) {
  const dev::Batch v = b.view();
  const char* force = std::getenv("HELM_BLOCK_SPLIT");
  const int forced = force && force[0] >= '0' && force[0] <= '3' && !force[1] ? force[0] - '0' : -1;
  auto pick = [forced](std::initializer_list<int64_t> cand, const std::function<void(int64_t)>& run) {
    if (forced >= 0) return *(cand.begin() + forced);
    std::vector<int64_t> cs;
    for (int64_t x : cand)
      if (std::find(cs.begin(), cs.end(), x) == cs.end()) cs.push_back(x);
    int64_t best = cs[0];
    float tb = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
      const float t = time_launch([&] { run(cs[i]); });
      if (i == 0 || t < tb) {
        tb = t;
        best = cs[i];
      }
    }
    return best;
  };
  for (size_t l = 0; l + 1 < b.tiles_f.size(); ++l) {
    const int64_t t0 = b.tiles_f[l], nt = b.tiles_f[l + 1] - t0;
    b.nw16_f[l] = pick({b.nwide_f[l], b.nwide4_f[l], 0, nt}, [&](int64_t nw) {
      dev::fwd_level_mfma(v, b.gsn_f.p + b.gsn_lev_f[l], b.gsn_lev_f[l + 1] - b.gsn_lev_f[l], b.gy_f[l], t0, nt, nw,
                          in, b.y_b.p, b.ubuf_b.p, b.stage.p, false, nullptr);
    });
  }
  for (size_t l = 0; l + 1 < b.tiles_b.size(); ++l) {
    const int64_t t0 = b.tiles_b[l], nt = b.tiles_b[l + 1] - t0;
    b.nw16_b[l] = pick({b.nwide_b[l], b.nwide4_b[l], 0, nt}, [&](int64_t nw) {
      dev::bwd_level_mfma(v, t0, nt, nw, b.y_b.p, b.xout_b(), false, nullptr);
    });
  }
  b.blk_tuned = true;
}

void ensure_width(Ctx& c, int m, int S) {
  const int64_t n = c.D.n;
  if (c.blk_m != m || c.blk_n != n) ensure_bases(c, m, 0);
  if (c.blk_cap < S) {
    c.free_bg_graphs();  // captured block steps point into these buffers
    c.bhcol.alloc(2 * (size_t)dev::kMaxBlock * blk_ld(m));
    c.bhtmp.alloc(2 * (size_t)dev::kMaxBlock * blk_ld(m));
    c.bpartial.alloc(2 * (size_t)dev::kMaxBlock * dev::gs_tiles(n) * blk_ld(m));
    c.bcoef_w.alloc(2 * (size_t)dev::kMaxBlock * (m + 2));
    c.bcoef_v.alloc(2 * (size_t)dev::kMaxBlock * (m + 2));
    c.by.alloc(2 * (size_t)(m + 1));
    c.bX.alloc(2 * (size_t)n * S);
    c.bZb.alloc(2 * (size_t)n * S);
    c.bW.alloc(2 * (size_t)n * S);
    c.bq.alloc(2 * (size_t)n * S);
    c.bt.alloc(2 * (size_t)n * S);
    if (c.two_level) c.bcvec.alloc(2 * (size_t)c.E.n * S);
    if (c.bh_host) (void)hipHostFree(c.bh_host);
    c.bh_host = nullptr;
    HELM_HIP(hipHostMalloc((void**)&c.bh_host, 2 * sizeof(double) * dev::kMaxBlock * blk_ld(m), hipHostMallocDefault));
    const bool first = c.blk_cap == 0 && !c.blk_timed;
    c.blk_cap = S;
    if (first) {
      // order of the multi-vector SpMV: plain or over XCD row ranges, the faster
      HELM_HIP(hipMemset(c.bX.p, 0, sizeof(double) * 2 * n * S));
      const float td = time_launch([&] {
        dev::csr_spmv_block(n, c.A_ptr.p, c.A_col.p, c.A_val.p, nullptr, 0, S, c.bX.p, nullptr, c.bW.p, nullptr);
      });
      const float tx = time_launch([&] {
        dev::csr_spmv_block(n, c.A_ptr.p, c.A_col.p, c.A_val.p, c.A_xr.p, c.A_xrows, S, c.bX.p, nullptr, c.bW.p,
                            nullptr);
      });
      c.blk_xcd = tx < td;
      c.blk_timed = true;
    }
  }
  int64_t npos_all = 0;
  bool grows = c.nbatch > 1 && c.xall_b_S < S;
  for (int k = 0; k < c.nbatch; ++k) grows = grows || c.fine[k].blk_S < S;
  if (c.two_level) grows = grows || c.coarse.blk_S < S;
  if (grows) c.free_bg_graphs();
  for (int k = 0; k < c.nbatch; ++k) {
    ensure_batch_block(c.fine[k], S);
    npos_all += c.fine[k].npos;
  }
  if (c.nbatch > 1 && c.xall_b_S < S) {
    c.xall_b.alloc(2 * (size_t)npos_all * S);
    c.xall_b_S = S;
  }
  if (c.two_level) ensure_batch_block(c.coarse, S);
  if (S == dev::kMaxBlock) {
    // bX holds n x kMaxBlock entries: any input serves the timed sweeps
    if (c.nbatch > 1) {
      size_t o = 0;
      for (int k = 0; k < c.nbatch; ++k) {
        c.fine[k].xo_b = c.xall_b.p + 2 * o * S;
        o += (size_t)c.fine[k].npos;
      }
    }
    for (int k = 0; k < c.nbatch; ++k)
      if (!c.fine[k].blk_tuned) tune_block_levels(c.fine[k], c.bX.p);
  }
}

namespace {

void ensure_block(Ctx& c, int m, int S, int bases) {
  ensure_bases(c, m, bases);
  ensure_width(c, m, S);
}

// Forward then backward sweeps of a batch for S interleaved right-hand sides.
void batch_solve_block(BatchDev& b, int S, const double* in, hipStream_t s, Profiler* prof, bool fine) {
  dev::Batch v = b.view();
  const bool each = prof && prof->on && fine;
  const bool mfma = S == dev::kMaxBlock;
  for (size_t l = 0; l + 1 < b.tiles_f.size(); ++l) {
    if (each) prof->begin(s);
    if (mfma)
      dev::fwd_level_mfma(v, b.gsn_f.p + b.gsn_lev_f[l], b.gsn_lev_f[l + 1] - b.gsn_lev_f[l], b.gy_f[l], b.tiles_f[l],
                          b.tiles_f[l + 1] - b.tiles_f[l], b.nw16_f[l], in, b.y_b.p, b.ubuf_b.p, b.stage.p, !fine,
                          s);
    else
      dev::fwd_level_block(v, b.tiles_f[l], b.tiles_f[l + 1] - b.tiles_f[l], S, in, b.y_b.p, b.ubuf_b.p, !fine, s);
    if (each) prof->end(HELM_K_TRSV_FWD, b.pbytes_f[l] + S * (b.bytes_f[l] - b.pbytes_f[l]), s);
  }
  for (size_t l = 0; l + 1 < b.tiles_b.size(); ++l) {
    if (each) prof->begin(s);
    if (mfma)
      dev::bwd_level_mfma(v, b.tiles_b[l], b.tiles_b[l + 1] - b.tiles_b[l], b.nw16_b[l], b.y_b.p, b.xout_b(), !fine,
                          s);
    else
      dev::bwd_level_block(v, b.tiles_b[l], b.tiles_b[l + 1] - b.tiles_b[l], S, b.y_b.p, b.xout_b(), !fine, s);
    if (each) prof->end(HELM_K_TRSV_BWD, b.pbytes_b[l] + S * (b.bytes_b[l] - b.pbytes_b[l]), s);
  }
}

void spmv_block(Ctx& c, int S, const double* x, const double* b, double* y, hipStream_t s) {
  if (c.blk_force == 3 || (c.blk_force == 0 && c.blk_xcd))
    dev::csr_spmv_block(c.D.n, c.A_ptr.p, c.A_col.p, c.A_val.p, c.A_xr.p, c.A_xrows, S, x, b, y, s);
  else
    dev::csr_spmv_block(c.D.n, c.A_ptr.p, c.A_col.p, c.A_val.p, nullptr, 0, S, x, b, y, s);
}

// Z = M^{-1} X for S interleaved vectors (eq. 2lvl, or eq. oras one-level).
// Local solves of all subdomain batches for S interleaved right-hand sides:
// concurrent on their streams, or one after the other while kernels are timed.
void fine_solve_block(Ctx& c, int S, const double* in, hipStream_t s) {
  Profiler* prof = c.prof.on ? &c.prof : nullptr;
  for_batches(c, s, [&](BatchDev& b, hipStream_t sk) { batch_solve_block(b, S, in, sk, prof, true); });
}

void apply_precond_block(Ctx& c, int S, const double* X, double* Z, hipStream_t s) {
  if (c.nbatch > 1) {
    // every batch's interleaved outputs follow those of the batches before it
    size_t o = 0;
    for (int k = 0; k < c.nbatch; ++k) {
      c.fine[k].xo_b = c.xall_b.p + 2 * o * S;
      o += (size_t)c.fine[k].npos;
    }
  }
  const int64_t n = c.D.n;
  const bool p = c.prof.on;
  if (c.two_level) {
    if (p) c.prof.begin(s);
    dev::spmv_real_block(c.ZT.n, c.ZT_ptr.p, c.ZT_col.p, c.ZT_val.p, S, X, c.bcvec.p, s);
    batch_solve_block(c.coarse, S, c.bcvec.p, s, &c.prof, false);
    // q = Z x_c, t = x - (A Z) x_c
    dev::coarse_update_block(n, c.Zp_ptr.p, c.Zp_col.p, c.Zp_val.p, c.AZ_ptr.p, c.AZ_col.p, c.AZ_val.p, S,
                             c.coarse.x_b.p, X, c.bq.p, c.bt.p, s);
    if (p) c.prof.end(HELM_K_COARSE, 0.0, s);
    fine_solve_block(c, S, c.bt.p, s);
  } else {
    fine_solve_block(c, S, X, s);
  }
  if (p) c.prof.begin(s);
  dev::prolong_block(n, c.pro_ptr.p, c.pro_idx.p, c.pro_w.p, S, c.fine[0].xout_b(), c.two_level ? c.bq.p : nullptr, Z,
                     s);
  if (p) c.prof.end(HELM_K_PROLONG, 0.0, s);
}

// Pseudo-block GMRES: nb <= kMaxBlock right-hand sides, each with its own
// Krylov space, Hessenberg matrix, Givens rotations and stopping test; every
// Arnoldi step applies M^{-1} and A to all active vectors at once (one pass
// over the factor panels and over A for the whole block).
int solve_block(Ctx& c, int nb, const double* const* Bp, double* const* Up, double tol, int m, int maxit, bool x0,
                bool dcgs2, hipStream_t s, helm_solve_info* info) {
  int S = 2;
  while (S < nb) S *= 2;
  ensure_block(c, m, S, nb);
  const int64_t n = c.D.n;
  const size_t n2 = 2 * (size_t)n;
  const int nt = dev::gs_tiles(n);
  struct St {
    double bnorm = 0, rel = 0;
    int its = 0, k = 0;
    bool conv = false, finished = false, incycle = false, done = false;
    std::vector<cplx> H, g, sn, y;
    std::vector<double> cs;
    std::chrono::steady_clock::time_point t0;
    double secs = 0;
  };
  std::vector<St> st(nb);
  for (int r = 0; r < nb; ++r) {
    St& q = st[r];
    q.t0 = std::chrono::steady_clock::now();
    q.H.assign((size_t)(m + 1) * m, 0);
    q.g.assign(m + 1, 0);
    q.sn.assign(m, 0);
    q.y.assign(m, 0);
    q.cs.assign(m, 0);
    q.bnorm = device_norm(c, Bp[r], s);
    if (!std::isfinite(q.bnorm)) fail(HELM_ENUMERIC, "non-finite right-hand side");
    if (q.bnorm == 0 || !x0) dev::fill_zero(n2, Up[r], s);
    if (q.bnorm == 0) q.conv = q.finished = true;
  }
  while (true) {
    bool any = false;
    for (int r = 0; r < nb; ++r) {
      St& q = st[r];
      if (q.finished) continue;
      double* v0 = c.bV[r].p;
      spmv_A(c, Up[r], Bp[r], v0, s);  // r = b - A x
      const double beta = device_norm(c, v0, s);
      if (!std::isfinite(beta)) fail(HELM_ENUMERIC, "non-finite residual");
      q.rel = beta / q.bnorm;
      if (beta <= tol * q.bnorm) {
        q.conv = q.finished = true;
        continue;
      }
      if (q.its >= maxit) {
        q.finished = true;
        continue;
      }
      dev::scale(n, v0, 1.0 / beta, v0, s);
      std::fill(q.g.begin(), q.g.end(), cplx(0, 0));
      q.g[0] = beta;
      q.incycle = true;
      q.done = false;
      q.k = 0;
      any = true;
    }
    if (!any) break;
    for (int jj = 0; jj < m; ++jj) {
      std::vector<int> act;
      for (int r = 0; r < nb; ++r)
        if (st[r].incycle && !st[r].done) act.push_back(r);
      if (act.empty()) break;
      const int na = (int)act.size();
      dev::PtrSetC src{};
      dev::PtrSet dz{}, dw{};
      for (int q = 0; q < na; ++q) {
        src.p[q] = c.bV[act[q]].p + n2 * jj;
        dz.p[q] = c.bZ[act[q]].p + n2 * jj;
        dw.p[q] = c.bw[act[q]].p;
      }
      dev::pack(n, S, src, c.bX.p, s);
      apply_precond_block(c, S, c.bX.p, c.bZb.p, s);
      dev::unpack(n, S, c.bZb.p, dz, s);
      const bool prof = c.prof.on;
      if (prof) c.prof.begin(s);
      spmv_block(c, S, c.bZb.p, nullptr, c.bW.p, s);
      if (prof) c.prof.end(HELM_K_SPMV, 0.0, s);
      dev::unpack(n, S, c.bW.p, dw, s);
      // Gram-Schmidt over the active right-hand sides (slot q holds act[q])
      if (prof) c.prof.begin(s);
      const size_t ld = blk_ld(m);
      dev::PtrSetC Vs{}, hs{}, ps{}, wc{}, nc{}, cwc{}, cvc{};
      dev::PtrSet Vw{}, ws{}, hts{}, hcs{}, pw{}, nrm{}, vn{}, cwp{}, cvp{};
      for (int q = 0; q < na; ++q) {
        const int r = act[q];
        Vs.p[q] = c.bV[r].p;
        Vw.p[q] = c.bV[r].p;
        hs.p[q] = c.bhtmp.p + 2 * (size_t)q * ld;
        hts.p[q] = c.bhtmp.p + 2 * (size_t)q * ld;
        hcs.p[q] = c.bhcol.p + 2 * (size_t)q * ld;
        ps.p[q] = c.bpartial.p + 2 * (size_t)q * nt * ld;
        pw.p[q] = c.bpartial.p + 2 * (size_t)q * nt * ld;
        ws.p[q] = c.bw[r].p;
        wc.p[q] = c.bw[r].p;
        nrm.p[q] = hcs.p[q] + 2 * (jj + 1);
        nc.p[q] = nrm.p[q];
        vn.p[q] = c.bV[r].p + n2 * (jj + 1);
        cwp.p[q] = c.bcoef_w.p + 2 * (size_t)q * (m + 2);
        cvp.p[q] = c.bcoef_v.p + 2 * (size_t)q * (m + 2);
        cwc.p[q] = cwp.p[q];
        cvc.p[q] = cvp.p[q];
      }
      int nout;
      if (dcgs2) {
        // delayed CGS2: dual dots | coefficients | v_j finished, w orthogonalised
        dev::gs_dual(false, na, n, Vs, Vw, n, jj + 1, cwc, cvc, ws, pw, s);
        dev::gs_final(na, ps, nt, 2 * (jj + 1), hts, dev::PtrSet{}, 0, s);
        dev::dcgs2_coef(na, hs, jj + 1, cwp, cvp, hcs, s);
        dev::gs_dual(true, na, n, Vs, Vw, n, jj + 1, cwc, cvc, ws, pw, s);
        dev::norm_final(na, ps, nt, nrm, s);
        nout = 2 * jj + 3;
      } else {
        dev::gs_pass(0, na, n, Vs, n, jj + 1, hs, ws, pw, s);
        dev::gs_final(na, ps, nt, jj + 1, hts, hcs, 0, s);
        dev::gs_pass(1, na, n, Vs, n, jj + 1, hs, ws, pw, s);
        dev::gs_final(na, ps, nt, jj + 1, hts, hcs, 1, s);
        dev::gs_pass(2, na, n, Vs, n, jj + 1, hs, ws, pw, s);
        dev::norm_final(na, ps, nt, nrm, s);
        nout = jj + 2;
      }
      dev::scale_by_inv_set(na, n, wc, nc, vn, s);
      if (prof)
        c.prof.end(HELM_K_GS, na * 16.0 * n * (dcgs2 ? 2.0 * (jj + 1) + 6.0 : 3.0 * (jj + 1) + 7.0), s);
      HELM_HIP(hipMemcpyAsync(c.bh_host, c.bhcol.p, 2 * sizeof(double) * na * ld, hipMemcpyDeviceToHost, s));
      HELM_HIP(hipStreamSynchronize(s));
      if (c.prof.on) c.prof.harvest();
      std::vector<int> ending;  // slots whose cycle ends at this step (delayed CGS2)
      for (int q = 0; q < na; ++q) {
        St& u = st[act[q]];
        const double* hh = c.bh_host + 2 * (size_t)q * ld;
        for (int i = 0; i < 2 * nout; ++i)
          if (!std::isfinite(hh[i])) fail(HELM_ENUMERIC, "non-finite Hessenberg entry");
        cplx* h = u.H.data() + (size_t)(m + 1) * jj;
        for (int i = 0; i <= jj + 1; ++i) h[i] = cplx(hh[2 * i], hh[2 * i + 1]);
        const double hn = h[jj + 1].real();
        ++u.its;
        u.k = jj + 1;
        if (!dcgs2) {
          givens_step(h, jj, u.cs, u.sn, u.g);
          if (std::abs(u.g[jj + 1]) <= tol * u.bnorm || u.its >= maxit || hn == 0) u.done = true;
          continue;
        }
        if (jj >= 1) {
          cplx* hp = u.H.data() + (size_t)(m + 1) * (jj - 1);
          finish_column(hp, jj - 1, hh + 2 * (jj + 2), hh[2 * (2 * jj + 2)]);
          givens_step(hp, jj - 1, u.cs, u.sn, u.g);
        }
        std::vector<cplx> hc(h, h + jj + 2);
        for (int i = 0; i < jj; ++i) {
          const cplx a = hc[i], bb = hc[i + 1];
          hc[i] = u.cs[i] * a + u.sn[i] * bb;
          hc[i + 1] = -std::conj(u.sn[i]) * a + u.cs[i] * bb;
        }
        const double rr = std::sqrt(std::norm(hc[jj]) + std::norm(hc[jj + 1]));
        const double est = hc[jj] == cplx(0, 0) ? std::abs(u.g[jj]) : std::abs(hc[jj + 1]) / rr * std::abs(u.g[jj]);
        if (est <= tol * u.bnorm || u.its >= maxit || hn == 0 || jj + 1 == m) {
          u.done = true;
          if (hn > 0)
            ending.push_back(q);
          else
            givens_step(h, jj, u.cs, u.sn, u.g);
        }
      }
      if (!ending.empty()) {
        // finish column j of the slots that stop here with the dots of v_{j+1}
        const int ne = (int)ending.size();
        dev::PtrSetC Ve{}, pe{}, he{}, cwe{}, cve{};
        dev::PtrSet Vwe{}, we{}, pwe{}, hte{}, hce{}, cwpe{}, cvpe{};
        for (int e = 0; e < ne; ++e) {
          const int q = ending[e];
          Ve.p[e] = Vs.p[q];
          Vwe.p[e] = Vw.p[q];
          we.p[e] = ws.p[q];
          pwe.p[e] = pw.p[q];
          pe.p[e] = ps.p[q];
          hte.p[e] = hts.p[q];
          he.p[e] = hs.p[q];
          hce.p[e] = hcs.p[q];
          cwpe.p[e] = cwp.p[q];
          cvpe.p[e] = cvp.p[q];
          cwe.p[e] = cwc.p[q];
          cve.p[e] = cvc.p[q];
        }
        dev::gs_dual(false, ne, n, Ve, Vwe, n, jj + 2, cwe, cve, we, pwe, s);
        dev::gs_final(ne, pe, nt, 2 * (jj + 2), hte, dev::PtrSet{}, 0, s);
        dev::dcgs2_coef(ne, he, jj + 2, cwpe, cvpe, hce, s);
        HELM_HIP(hipMemcpyAsync(c.bh_host, c.bhcol.p, 2 * sizeof(double) * na * ld, hipMemcpyDeviceToHost, s));
        HELM_HIP(hipStreamSynchronize(s));
        for (int e = 0; e < ne; ++e) {
          const int q = ending[e];
          St& u = st[act[q]];
          const double* hh = c.bh_host + 2 * (size_t)q * ld;
          for (int i = 0; i < 2 * (2 * jj + 5); ++i)
            if (!std::isfinite(hh[i])) fail(HELM_ENUMERIC, "non-finite Hessenberg entry");
          cplx* h = u.H.data() + (size_t)(m + 1) * jj;
          finish_column(h, jj, hh + 2 * (jj + 3), hh[2 * (2 * jj + 4)]);
          givens_step(h, jj, u.cs, u.sn, u.g);
        }
      }
    }
    // cycle end: x += Z_k y for every right-hand side of the cycle
    for (int r = 0; r < nb; ++r) {
      St& u = st[r];
      if (!u.incycle) continue;
      const int k = u.k;
      for (int i = k - 1; i >= 0; --i) {
        cplx acc = u.g[i];
        for (int l = i + 1; l < k; ++l) acc -= u.H[(size_t)(m + 1) * l + i] * u.y[l];
        u.y[i] = acc / u.H[(size_t)(m + 1) * i + i];
      }
      HELM_HIP(hipMemcpyAsync(c.by.p, u.y.data(), sizeof(cplx) * k, hipMemcpyHostToDevice, s));
      dev::gemv_acc(n, c.bZ[r].p, n, k, c.by.p, Up[r], s);
      HELM_HIP(hipStreamSynchronize(s));
      u.incycle = false;
    }
  }
  HELM_HIP(hipStreamSynchronize(s));
  if (c.prof.on) c.prof.harvest();
  int status = HELM_OK;
  const double total = std::chrono::duration<double>(std::chrono::steady_clock::now() - st[0].t0).count();
  for (int r = 0; r < nb; ++r) {
    if (info) {
      info[r].iterations = st[r].its;
      info[r].converged = st[r].conv ? 1 : 0;
      info[r].relres = st[r].rel;
      info[r].seconds = total;
    }
    if (!st[r].conv) status = HELM_ENOCONV;
  }
  return status;
}

// ---- block GMRES ---------------------------------------------------------
//
// One block Krylov space for up to 16 right-hand sides (right-preconditioned
// flexible block GMRES): the block residual R_0 = V_0 beta, each step
// Z_j = M^{-1} V_j, W = A Z_j, block CGS2 against V_0..V_j (two passes of
// tall-skinny MFMA contractions), CholQR2 of W into V_{j+1} R_{j+1}; the
// block Hessenberg matrix is reduced by Householder reflections on the host
// (FP64) and every right-hand side's residual estimate is read off the
// rotated right-hand side.  At a restart the columns whose true residual
// reached the tolerance leave the block.  All device work of a step runs on
// the solve stream with one copy to the host at its end, so a step can be
// replayed from a captured graph.

}  // namespace

void Ctx::free_bg_graphs() {
  for (auto& g : bg_graph)
    if (g) (void)hipGraphExecDestroy(g);
  bg_graph.clear();
  bg_graph_s = 0;
}

namespace {

constexpr size_t kBlk = 2 * 16 * (size_t)16;  // doubles of a 16 x 16 complex block
constexpr int64_t kGramWgsMax = 1 << 30;

struct BgLayout {
  // offsets (doubles) into bgH
  size_t htot, htmp, r1, r2, g0, g1, g2, t1, t2, total;
};
BgLayout bg_layout(int m) {
  BgLayout L{};
  size_t o = 0;
  L.htot = o;
  o += (size_t)(m + 1) * kBlk;
  L.htmp = o;
  o += (size_t)(m + 1) * kBlk;
  for (size_t* f : {&L.r1, &L.r2, &L.g0, &L.g1, &L.g2, &L.t1, &L.t2}) {
    *f = o;
    o += kBlk;
  }
  L.total = o;
  return L;
}

// 16 x 16 blocks of the partial-sum buffer: bgs_dots writes at most
// max(nb + 2, 16) blocks per workgroup, bgs_mul one per workgroup
size_t bg_part_blocks(int64_t n, int m) {
  return std::max<size_t>((size_t)dev::bgs_wgs(n) * std::max(m + 2, 16), (size_t)dev::bgs_mul_wgs(n));
}

size_t bg_bytes(int64_t n, int m) {
  const size_t blk = 2 * 16 * (size_t)n;  // doubles of an n x 16 block
  const size_t part = bg_part_blocks(n, m) * kBlk;
  return sizeof(double) * ((size_t)(2 * m + 1) * blk + 3 * blk + part + bg_layout(m).total + (size_t)m * kBlk);
}

void ensure_bg(Ctx& c, int m) {
  const int64_t n = c.D.n;
  ensure_width(c, c.blk_m > 0 ? c.blk_m : m, dev::kMaxBlock);
  if (c.bg_m == m && c.bg_n == n && c.bgV.p) return;
  c.free_bg_graphs();
  const size_t blk = 2 * 16 * (size_t)n;
  c.bgV.alloc(blk * (m + 1));
  c.bgZ.alloc(blk * m);
  c.bgW.alloc(blk);
  c.bgX.alloc(blk);
  c.bgB.alloc(blk);
  c.bgpart.alloc(bg_part_blocks(n, m) * kBlk);
  c.bgH.alloc(bg_layout(m).total);
  c.bgC.alloc((size_t)m * kBlk);
  c.bgstat.alloc(2);
  if (c.bg_host) (void)hipHostFree(c.bg_host);
  c.bg_host = nullptr;
  HELM_HIP(hipHostMalloc((void**)&c.bg_host, sizeof(double) * ((size_t)(m + 1) * kBlk + 2 * kBlk), hipHostMallocDefault));
  if (!c.bg_hstat) HELM_HIP(hipHostMalloc((void**)&c.bg_hstat, 2 * sizeof(int), hipHostMallocDefault));
  c.bg_m = m;
  c.bg_n = n;
}

// Column norms of an n x 16 block from its Gram matrix (host copy).
std::vector<double> gram_diag(const double* G, int sa) {
  std::vector<double> d(sa);
  for (int q = 0; q < sa; ++q) d[q] = std::sqrt(std::max(0.0, G[2 * (q * 17)]));
  return d;
}

// Y = Y Q with the Gram partials of the result reduced into G (device).
void gram_of(Ctx& c, const double* Y, double* G, hipStream_t s) {
  const int64_t n = c.D.n;
  dev::bgs_mul(n, nullptr, 0, 0, nullptr, 1.0, Y, const_cast<double*>(Y), c.bgpart.p, s);
  dev::bgs_reduce(c.bgpart.p, dev::bgs_mul_wgs(n), 1, G, nullptr, false, s);
}

// Device work of block Arnoldi step j (sa active columns): Z_j = M^{-1} V_j,
// W = A Z_j, two CGS passes against V_0..V_j (coefficients summed into
// htot), CholQR2 of W into V_{j+1} (R1, R2, status), then the copy of the
// block column and the factors to bg_host.  Enqueued on s only.
void bg_step_device(Ctx& c, int j, int sa, hipStream_t s) {
  const int64_t n = c.D.n;
  const size_t blk = 2 * 16 * (size_t)n;
  const BgLayout L = bg_layout(c.bg_m);
  double* H = c.bgH.p;
  const double* Vj = c.bgV.p + blk * j;
  double* Zj = c.bgZ.p + blk * j;
  double* W = c.bgW.p;
  apply_precond_block(c, dev::kMaxBlock, Vj, Zj, s);
  spmv_block(c, dev::kMaxBlock, Zj, nullptr, W, s);
  const bool prof = c.prof.on;
  if (prof) c.prof.begin(s);
  const int nb = j + 1, mwg = dev::bgs_mul_wgs(n);
  // pass 1: V^H W and W^H W (the scale breakdowns are measured against)
  int prows = dev::bgs_dots(n, c.bgV.p, blk, nb, true, W, c.bgpart.p, s);
  dev::bgs_reduce(c.bgpart.p, prows, nb + 1, H + L.htmp, nullptr, false, s);
  dev::copy((int64_t)nb * kBlk, H + L.htmp, H + L.htot, s);
  dev::copy(kBlk, H + L.htmp + nb * kBlk, H + L.g0, s);
  dev::bgs_mul(n, c.bgV.p, blk, nb, H + L.htmp, -1.0, W, W, nullptr, s);
  // pass 2
  prows = dev::bgs_dots(n, c.bgV.p, blk, nb, false, W, c.bgpart.p, s);
  dev::bgs_reduce(c.bgpart.p, prows, nb, H + L.htmp, H + L.htot, true, s);
  dev::bgs_mul(n, c.bgV.p, blk, nb, H + L.htmp, -1.0, W, W, c.bgpart.p, s);
  dev::bgs_reduce(c.bgpart.p, mwg, 1, H + L.g1, nullptr, false, s);
  // CholQR2: W = V_{j+1} R2 R1
  double* Vn = c.bgV.p + blk * (j + 1);
  dev::chol16(H + L.g1, sa, H + L.g0, 1e-24, H + L.r1, H + L.t1, c.bgstat.p, s);
  dev::bgs_mul(n, W, 0, 1, H + L.t1, 1.0, nullptr, Vn, c.bgpart.p, s);
  dev::bgs_reduce(c.bgpart.p, mwg, 1, H + L.g2, nullptr, false, s);
  dev::chol16(H + L.g2, sa, nullptr, 1e-12, H + L.r2, H + L.t2, c.bgstat.p + 1, s);
  dev::bgs_mul(n, Vn, 0, 1, H + L.t2, 1.0, nullptr, Vn, nullptr, s);
  if (prof) c.prof.end(HELM_K_GS, 16.0 * 16.0 * (double)n * (4.0 * nb + 12.0), s);
  HELM_HIP(hipMemcpyAsync(c.bg_host, H + L.htot, sizeof(double) * nb * kBlk, hipMemcpyDeviceToHost, s));
  HELM_HIP(hipMemcpyAsync(c.bg_host + (size_t)(c.bg_m + 1) * kBlk, H + L.r1, sizeof(double) * 2 * kBlk,
                          hipMemcpyDeviceToHost, s));
  HELM_HIP(hipMemcpyAsync(c.bg_hstat, c.bgstat.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
}

// Step j from its captured graph (captured on first use for sa columns), on
// the library's graph stream, ordered after the caller's earlier work on s
// and before its later work.
void bg_step(Ctx& c, int j, int sa, bool graphs, hipStream_t s) {
  if (!graphs || c.prof.on) {
    bg_step_device(c, j, sa, s);
    return;
  }
  if (!c.bg_stream) HELM_HIP(hipStreamCreateWithFlags(&c.bg_stream, hipStreamNonBlocking));
  for (auto& e : c.bg_ev)
    if (!e) HELM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  if (c.bg_graph_s != sa || (int)c.bg_graph.size() != c.bg_m) {
    c.free_bg_graphs();
    c.bg_graph.assign(c.bg_m, nullptr);
    c.bg_graph_s = sa;
  }
  hipStream_t g = c.bg_stream;
  HELM_HIP(hipEventRecord(c.bg_ev[0], s));
  HELM_HIP(hipStreamWaitEvent(g, c.bg_ev[0], 0));
  if (!c.bg_graph[j]) {
    hipGraph_t gr = nullptr;
    HELM_HIP(hipStreamBeginCapture(g, hipStreamCaptureModeRelaxed));
    try {
      bg_step_device(c, j, sa, g);
    } catch (...) {
      (void)hipStreamEndCapture(g, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
      throw;
    }
    HELM_HIP(hipStreamEndCapture(g, &gr));
    hipGraphExec_t e = nullptr;
    const hipError_t err = hipGraphInstantiate(&e, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HELM_HIP(err);
    c.bg_graph[j] = e;
  }
  HELM_HIP(hipGraphLaunch(c.bg_graph[j], g));
  HELM_HIP(hipEventRecord(c.bg_ev[1], g));
  HELM_HIP(hipStreamWaitEvent(s, c.bg_ev[1], 0));
}

// Householder reflector (LAPACK zlarfg convention): H^H (alpha; x) = (beta; 0)
// with H = I - tau v v^H, v(0) = 1.  x is overwritten by v(1:).
void house(cplx& alpha, cplx* x, int len, cplx& tau) {
  double xn = 0;
  for (int i = 0; i < len; ++i) xn += std::norm(x[i]);
  xn = std::sqrt(xn);
  if (xn == 0 && alpha.imag() == 0) {
    tau = 0;
    return;
  }
  double beta = -std::copysign(std::sqrt(std::norm(alpha) + xn * xn), alpha.real());
  tau = (beta - alpha) / beta;
  const cplx sc = 1.0 / (alpha - beta);
  for (int i = 0; i < len; ++i) x[i] *= sc;
  alpha = beta;
}

// y <- H^H y = y - conj(tau) v (v^H y) on rows [k, k + len]
void apply_house(const cplx* v, cplx tau, cplx* y, int len) {
  if (tau == cplx(0, 0)) return;
  cplx d = y[0];
  for (int i = 1; i <= len; ++i) d += std::conj(v[i - 1]) * y[i];
  d *= std::conj(tau);
  y[0] -= d;
  for (int i = 1; i <= len; ++i) y[i] -= d * v[i - 1];
}

int solve_bgmres(Ctx& c, int nrhs, const double* const* Bp, double* const* Up, double tol, int m, int maxit, bool x0,
                 bool graphs, hipStream_t s, helm_solve_info* info, bool& fallback) {
  fallback = false;
  ensure_bg(c, m);
  const int64_t n = c.D.n;
  const size_t blk = 2 * 16 * (size_t)n;
  const BgLayout L = bg_layout(m);
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> bnorm(nrhs), rel(nrhs, 0);
  std::vector<int> its(nrhs, 0), conv(nrhs, 0), act;
  for (int r = 0; r < nrhs; ++r) {
    bnorm[r] = device_norm(c, Bp[r], s);
    if (!std::isfinite(bnorm[r])) fail(HELM_ENUMERIC, "non-finite right-hand side");
    if (bnorm[r] == 0 || !x0) dev::fill_zero(2 * n, Up[r], s);
    if (bnorm[r] == 0)
      conv[r] = 1;
    else
      act.push_back(r);
  }
  std::vector<double> hG(kBlk);
  // Householder data of a cycle: columns of the rotated block Hessenberg
  // matrix (ld rows), reflector vectors and factors, rotated right-hand sides
  std::vector<cplx> Hh, V, tau, G, Y;
  bool pack_needed = true;
  while (!act.empty()) {
    const int sa = (int)act.size();
    if (pack_needed) {
      dev::PtrSetC bs{}, us{};
      for (int q = 0; q < sa; ++q) {
        bs.p[q] = Bp[act[q]];
        us.p[q] = Up[act[q]];
      }
      dev::pack(n, 16, bs, c.bgB.p, s);
      dev::pack(n, 16, us, c.bgX.p, s);
      pack_needed = false;
    }
    // true block residual R = B - A X into V_0, its Gram matrix
    spmv_block(c, 16, c.bgX.p, c.bgB.p, c.bgV.p, s);
    gram_of(c, c.bgV.p, c.bgH.p + L.g0, s);
    HELM_HIP(hipMemcpyAsync(hG.data(), c.bgH.p + L.g0, sizeof(double) * kBlk, hipMemcpyDeviceToHost, s));
    HELM_HIP(hipStreamSynchronize(s));
    const std::vector<double> rn = gram_diag(hG.data(), sa);
    std::vector<int> keep;
    bool changed = false;
    for (int q = 0; q < sa; ++q) {
      const int r = act[q];
      if (!std::isfinite(rn[q])) fail(HELM_ENUMERIC, "non-finite residual");
      rel[r] = rn[q] / bnorm[r];
      if (rn[q] <= tol * bnorm[r]) {
        conv[r] = 1;
        changed = true;
      } else if (its[r] >= maxit) {
        changed = true;
      } else {
        keep.push_back(r);
      }
    }
    if (changed) {
      // finished columns leave the block: write every column back, repack
      dev::PtrSet us{};
      for (int q = 0; q < sa; ++q) us.p[q] = Up[act[q]];
      dev::unpack(n, 16, c.bgX.p, us, s);
      act = keep;
      pack_needed = true;
      continue;
    }
    // R_0 = V_0 beta (CholQR2)
    double* H = c.bgH.p;
    dev::chol16(H + L.g0, sa, H + L.g0, 1e-28, H + L.r1, H + L.t1, c.bgstat.p, s);
    dev::bgs_mul(n, c.bgV.p, 0, 1, H + L.t1, 1.0, nullptr, c.bgV.p, c.bgpart.p, s);
    dev::bgs_reduce(c.bgpart.p, dev::bgs_mul_wgs(n), 1, H + L.g2, nullptr, false, s);
    dev::chol16(H + L.g2, sa, nullptr, 1e-12, H + L.r2, H + L.t2, c.bgstat.p + 1, s);
    dev::bgs_mul(n, c.bgV.p, 0, 1, H + L.t2, 1.0, nullptr, c.bgV.p, nullptr, s);
    HELM_HIP(hipMemcpyAsync(c.bg_host + (size_t)(m + 1) * kBlk, H + L.r1, sizeof(double) * 2 * kBlk,
                            hipMemcpyDeviceToHost, s));
    HELM_HIP(hipMemcpyAsync(c.bg_hstat, c.bgstat.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HELM_HIP(hipStreamSynchronize(s));
    if (c.bg_hstat[0] || c.bg_hstat[1]) {
      // the residuals are (numerically) linearly dependent: hand the
      // remaining columns, with their current iterates, to pseudo-block GMRES
      dev::PtrSet us{};
      for (int q = 0; q < sa; ++q) us.p[q] = Up[act[q]];
      dev::unpack(n, 16, c.bgX.p, us, s);
      HELM_HIP(hipStreamSynchronize(s));
      fallback = true;
      std::vector<const double*> b2;
      std::vector<double*> u2;
      for (int r : act) {
        b2.push_back(Bp[r]);
        u2.push_back(Up[r]);
      }
      std::vector<helm_solve_info> inf2(act.size());
      const int st = solve_block(c, (int)act.size(), b2.data(), u2.data(), tol, m, std::max(1, maxit - its[act[0]]),
                                 true, true, s, inf2.data());
      for (size_t q = 0; q < act.size(); ++q) {
        its[act[q]] += inf2[q].iterations;
        conv[act[q]] = inf2[q].converged;
        rel[act[q]] = inf2[q].relres;
      }
      (void)st;
      act.clear();
      break;
    }
    // beta = R2 R1 (upper s x s); G = [beta; 0]
    const int ld = (m + 1) * sa;
    auto hostblk = [&](size_t off, int a, int col) {
      const double* p = c.bg_host + off + 2 * (size_t)(a * 16 + col);
      return cplx(p[0], p[1]);
    };
    const size_t offR1 = (size_t)(m + 1) * kBlk, offR2 = offR1 + kBlk;
    auto rprod = [&](int a, int col) {  // (R2 R1)[a][col]
      cplx v = 0;
      for (int k = 0; k < sa; ++k) v += hostblk(offR2, a, k) * hostblk(offR1, k, col);
      return v;
    };
    G.assign((size_t)ld * sa, 0);
    for (int a = 0; a < sa; ++a)
      for (int q = 0; q < sa; ++q) G[(size_t)q * ld + a] = rprod(a, q);
    Hh.assign((size_t)ld * m * sa, 0);
    V.assign((size_t)m * sa * sa, 0);
    tau.assign((size_t)m * sa, 0);
    int k = 0;
    for (int j = 0; j < m; ++j) {
      bg_step(c, j, sa, graphs, s);
      HELM_HIP(hipStreamSynchronize(s));
      if (c.prof.on) c.prof.harvest();
      for (size_t i = 0; i < (size_t)(j + 1) * kBlk + 2 * kBlk; ++i) {
        const size_t at = i < (size_t)(j + 1) * kBlk ? i : offR1 + (i - (size_t)(j + 1) * kBlk);
        if (!std::isfinite(c.bg_host[at])) fail(HELM_ENUMERIC, "non-finite block Hessenberg entry");
      }
      const bool brk = c.bg_hstat[0] != 0 || c.bg_hstat[1] != 0;
      // block column j: H̄[jb s + a][j s + q] = htot_jb[a][q]; R_{j+1} below
      for (int q = 0; q < sa; ++q) {
        const int jc = j * sa + q;
        cplx* col = Hh.data() + (size_t)jc * ld;
        for (int jb = 0; jb <= j; ++jb)
          for (int a = 0; a < sa; ++a) col[jb * sa + a] = hostblk((size_t)jb * kBlk, a, q);
        for (int a = 0; a < sa; ++a) col[(j + 1) * sa + a] = brk ? cplx(0, 0) : rprod(a, q);
        // earlier reflectors, then this column's
        for (int pc = 0; pc < jc; ++pc) apply_house(V.data() + (size_t)pc * sa, tau[pc], col + pc, sa);
        cplx alpha = col[jc];
        cplx* x = col + jc + 1;
        for (int i = 0; i < sa; ++i) V[(size_t)jc * sa + i] = x[i];
        house(alpha, V.data() + (size_t)jc * sa, sa, tau[jc]);
        col[jc] = alpha;
        for (int i = 0; i < sa; ++i) x[i] = 0;
        for (int g = 0; g < sa; ++g) apply_house(V.data() + (size_t)jc * sa, tau[jc], G.data() + (size_t)g * ld + jc, sa);
      }
      for (int r : act) ++its[r];
      k = j + 1;
      bool all = true;
      for (int q = 0; q < sa; ++q) {
        double e = 0;
        for (int a = 0; a < sa; ++a) e += std::norm(G[(size_t)q * ld + (j + 1) * sa + a]);
        if (std::sqrt(e) > tol * bnorm[act[q]]) all = false;
      }
      if (brk || all || its[act[0]] >= maxit) break;
    }
    // Y = Rtri^{-1} G(0 : k sa) and X += sum_j Z_j Y_j
    const int kk = k * sa;
    Y.assign((size_t)kk * sa, 0);
    for (int q = 0; q < sa; ++q)
      for (int i = kk - 1; i >= 0; --i) {
        cplx acc = G[(size_t)q * ld + i];
        for (int l = i + 1; l < kk; ++l) acc -= Hh[(size_t)l * ld + i] * Y[(size_t)q * kk + l];
        Y[(size_t)q * kk + i] = acc / Hh[(size_t)i * ld + i];
      }
    std::vector<double> Cb((size_t)k * kBlk, 0.0);
    for (int jb = 0; jb < k; ++jb)
      for (int a = 0; a < sa; ++a)
        for (int q = 0; q < sa; ++q) {
          const cplx v = Y[(size_t)q * kk + jb * sa + a];
          Cb[(size_t)jb * kBlk + 2 * (a * 16 + q)] = v.real();
          Cb[(size_t)jb * kBlk + 2 * (a * 16 + q) + 1] = v.imag();
        }
    HELM_HIP(hipMemcpyAsync(c.bgC.p, Cb.data(), sizeof(double) * Cb.size(), hipMemcpyHostToDevice, s));
    dev::bgs_mul(n, c.bgZ.p, blk, k, c.bgC.p, 1.0, c.bgX.p, c.bgX.p, nullptr, s);
    HELM_HIP(hipStreamSynchronize(s));  // Cb is reused
  }
  HELM_HIP(hipStreamSynchronize(s));
  if (c.prof.on) c.prof.harvest();
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int status = HELM_OK;
  for (int r = 0; r < nrhs; ++r) {
    if (info) {
      info[r].iterations = its[r];
      info[r].converged = conv[r];
      info[r].relres = rel[r];
      info[r].seconds = secs;
    }
    if (!conv[r]) status = HELM_ENOCONV;
  }
  return status;
}

}  // namespace

int solve(Ctx& c, int32_t nrhs, const double* B, double tol, const helm_solve_opts* opts, double* U, hipStream_t s,
          helm_solve_info* info) {
  const int m = opts && opts->restart > 0 ? opts->restart : 50;
  const int maxit = opts && opts->maxit > 0 ? opts->maxit : 1000;
  const bool x0 = opts && (opts->flags & HELM_SOLVE_X0);
  const bool dcgs2 = !(opts && (opts->flags & HELM_SOLVE_CGS2));
  const int block = opts && opts->block > 0 ? std::min(opts->block, dev::kMaxBlock) : 1;
  if (m > 50) fail(HELM_EINVAL, "restart must be <= 50");
  if (!(tol > 0)) fail(HELM_EINVAL, "tol must be positive");
  if (block <= 1 || nrhs <= 1) return solve_single(c, nrhs, B, tol, m, maxit, x0, dcgs2, U, s, info);
  const int64_t n = c.D.n;
  const bool bgm = opts && (opts->flags & HELM_SOLVE_BLOCK_GMRES);
  const bool graphs = opts && (opts->flags & HELM_SOLVE_GRAPHS);
  int status = HELM_OK;
  for (int32_t j0 = 0; j0 < nrhs; j0 += block) {
    const int nb = std::min<int>(block, nrhs - j0);
    std::vector<const double*> Bp(nb);
    std::vector<double*> Up(nb);
    for (int r = 0; r < nb; ++r) {
      Bp[r] = B + 2 * (size_t)n * (j0 + r);
      Up[r] = U + 2 * (size_t)n * (j0 + r);
    }
    int st;
    if (nb == 1) {
      st = solve_single(c, 1, Bp[0], tol, m, maxit, x0, dcgs2, Up[0], s, info ? info + j0 : nullptr);
    } else if (bgm) {
      bool fb = false;
      st = solve_bgmres(c, nb, Bp.data(), Up.data(), tol, m, maxit, x0, graphs, s, info ? info + j0 : nullptr, fb);
      c.bg_fallbacks += fb ? 1 : 0;
    } else {
      st = solve_block(c, nb, Bp.data(), Up.data(), tol, m, maxit, x0, dcgs2, s, info ? info + j0 : nullptr);
    }
    if (st != HELM_OK) status = st;
  }
  return status;
}

// ---- continuous-batching server -------------------------------------------
//
// Requests (one right-hand side each) wait in a FIFO queue and are admitted
// into free slots of a pseudo-block GMRES whenever a slot frees up, not only
// between batches: every slot runs its own restart cycles (its own Krylov
// dimension, Hessenberg matrix, rotations and stopping test), and each
// Arnoldi step applies M^{-1} and A to all active slots in one pass over the
// panels and over A.  Gram-Schmidt runs once per group of slots at the same
// Krylov dimension.  A step is split into launch (kernels and the Hessenberg
// copy enqueued on the server's stream) and finish (wait, least squares,
// cycle ends, completions, admissions), so several servers on different
// streams overlap on the device.

Server::Server(Ctx& ctx, const helm_server_opts* o, hipStream_t st) : c(ctx), s(st) {
  m = o && o->restart > 0 ? o->restart : 50;
  maxit = o && o->maxit > 0 ? o->maxit : 1000;
  tol = o && o->tol > 0 ? o->tol : 1e-6;
  dcgs2 = !(o && (o->flags & HELM_SOLVE_CGS2));
  if (m > 50) fail(HELM_EINVAL, "restart must be <= 50");
  int want = o && o->slots > 0 ? o->slots : dev::kMaxBlock;
  if (want > dev::kMaxBlock) fail(HELM_EINVAL, "at most 16 slots");
  // admission by memory: a slot's Krylov basis and the block width it needs
  // are allocated when a request is admitted into it, within the budget
  size_t free_b = 0, total_b = 0;
  HELM_HIP(hipMemGetInfo(&free_b, &total_b));
  // memory the context already holds for this restart (slots opened by an
  // earlier server) counts towards the budget, not against the free memory
  budget = o && o->mem_bytes > 0 ? o->mem_bytes : held() + 0.75 * (double)free_b;
  slots_n = want;
  slot.resize(slots_n);
  for (auto& q : slot) {
    q.H.assign((size_t)(m + 1) * m, 0);
    q.g.assign(m + 1, 0);
    q.sn.assign(m, 0);
    q.cs.assign(m, 0);
    q.y.assign(m, 0);
  }
  if (!open_slot(0)) fail(HELM_ENOMEM, "no device memory for a server slot within the budget");
  HELM_HIP(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
}

static int pow2_width(int k) {
  int S = 2;
  while (S < k) S *= 2;
  return S;
}

double Server::bytes_for(int bases, int width) const {
  return (double)bases * (double)basis_bytes(c.D.n, m) + (double)width_bytes(c, m, width);
}

double Server::held() const { return c.blk_m == m ? bytes_for(c.blk_bases, c.blk_cap) : 0.0; }

// Makes slot q usable: its Krylov basis (and those of the slots below it)
// and the block width q + 1 needs, if the budget allows them.
bool Server::open_slot(int q) {
  const int bases = std::max(c.blk_m == m ? c.blk_bases : 0, q + 1);
  const int width = std::max(c.blk_m == m ? c.blk_cap : 0, pow2_width(q + 1));
  if (bytes_for(bases, width) > budget) return false;
  try {
    ensure_bases(c, m, bases);
    ensure_width(c, m, width);
  } catch (const Error& e) {
    if (e.code != HELM_ENOMEM || active() == 0) throw;
    return false;  // the device is full: wait for a slot that holds memory
  }
  return true;
}

Server::~Server() { (void)hipEventDestroy(done_ev); }

void Server::submit(const double* b, double* u, int64_t tag) {
  if (!live.insert(tag).second) fail(HELM_EINVAL, "tag " + std::to_string(tag) + " is already queued or in flight");
  queue.push_back({b, u, tag, std::chrono::steady_clock::now()});
}

void Server::emit(std::vector<helm_server_event>& out, const helm_server_event& e) {
  live.erase(e.tag);
  out.push_back(e);
}

// Starts (or restarts) a cycle of slot q from its current iterate: r = b - A x.
// Returns false when the request is finished (converged, maxit, or error).
bool Server::start_cycle(int q, std::vector<helm_server_event>& out) {
  Slot& z = slot[q];
  const int64_t n = c.D.n;
  double* v0 = c.bV[q].p;
  spmv_A(c, z.u, z.b, v0, s);
  const double beta = device_norm(c, v0, s);
  z.rel = beta / z.bnorm;
  int status = HELM_OK;
  if (!std::isfinite(beta)) status = HELM_ENUMERIC;
  else if (beta <= tol * z.bnorm) z.conv = true;
  if (status != HELM_OK || z.conv || z.its >= maxit) {
    helm_server_event e{};
    e.tag = z.tag;
    e.iterations = z.its;
    e.converged = z.conv ? 1 : 0;
    e.status = status != HELM_OK ? status : (z.conv ? HELM_OK : HELM_ENOCONV);
    e.relres = z.rel;
    e.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - z.t0).count();
    emit(out, e);
    z.busy = false;
    return false;
  }
  dev::scale(n, v0, 1.0 / beta, v0, s);
  std::fill(z.g.begin(), z.g.end(), cplx(0, 0));
  z.g[0] = beta;
  z.jj = 0;
  return true;
}

void Server::admit(std::vector<helm_server_event>& out) {
  const int64_t n = c.D.n;
  for (int q = 0; q < slots_n && !queue.empty(); ++q) {
    if (slot[q].busy) continue;
    // slots open lowest first, so a higher one needs at least as much memory
    if (q >= c.blk_bases && !open_slot(q)) break;
    Request r = queue.front();
    queue.pop_front();
    Slot& z = slot[q];
    z.b = r.b;
    z.u = r.u;
    z.tag = r.tag;
    z.t0 = r.t0;
    z.its = 0;
    z.conv = false;
    z.busy = true;
    dev::fill_zero(2 * n, z.u, s);
    z.bnorm = device_norm(c, z.b, s);
    if (!std::isfinite(z.bnorm) || z.bnorm == 0) {
      helm_server_event e{};
      e.tag = z.tag;
      e.converged = z.bnorm == 0 ? 1 : 0;
      e.status = z.bnorm == 0 ? HELM_OK : HELM_ENUMERIC;
      e.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - z.t0).count();
      emit(out, e);
      z.busy = false;
      --q;  // the slot is free again
      continue;
    }
    start_cycle(q, out);
  }
}

int Server::launch() {
  const int64_t n = c.D.n;
  const size_t n2 = 2 * (size_t)n;
  act.clear();
  for (int q = 0; q < slots_n; ++q)
    if (slot[q].busy) act.push_back(q);
  if (act.empty()) return 0;
  // block width: slot q is column q, so the smallest power of two above the
  // highest busy slot (free slots in between are zero columns)
  int S = 2;
  while (S < act.back() + 1) S *= 2;
  dev::PtrSetC src{};
  dev::PtrSet dz{}, dw{};
  for (int q : act) {
    src.p[q] = c.bV[q].p + n2 * slot[q].jj;
    dz.p[q] = c.bZ[q].p + n2 * slot[q].jj;
    dw.p[q] = c.bw[q].p;
  }
  // slots map to their own columns of the block (inactive ones are zero)
  dev::pack(n, S, src, c.bX.p, s);
  apply_precond_block(c, S, c.bX.p, c.bZb.p, s);
  dev::unpack(n, S, c.bZb.p, dz, s);
  spmv_block(c, S, c.bZb.p, nullptr, c.bW.p, s);
  dev::unpack(n, S, c.bW.p, dw, s);
  // Gram-Schmidt, one call per group of slots at the same Krylov dimension
  const int nt = dev::gs_tiles(n);
  std::vector<int> done(act.size(), 0);
  for (size_t a = 0; a < act.size(); ++a) {
    if (done[a]) continue;
    const int jj = slot[act[a]].jj;
    dev::PtrSetC Vs{}, hs{}, ps{}, wc{}, nc{}, cwc{}, cvc{};
    dev::PtrSet Vw{}, ws{}, hts{}, hcs{}, pw{}, nrm{}, vn{}, cwp{}, cvp{};
    int na = 0;
    for (size_t b2 = a; b2 < act.size(); ++b2) {
      const int q = act[b2];
      if (done[b2] || slot[q].jj != jj) continue;
      done[b2] = 1;
      Vs.p[na] = c.bV[q].p;
      Vw.p[na] = c.bV[q].p;
      cwp.p[na] = c.bcoef_w.p + 2 * (size_t)q * (m + 2);
      cvp.p[na] = c.bcoef_v.p + 2 * (size_t)q * (m + 2);
      cwc.p[na] = cwp.p[na];
      cvc.p[na] = cvp.p[na];
      hs.p[na] = c.bhtmp.p + 2 * (size_t)q * blk_ld(m);
      hts.p[na] = c.bhtmp.p + 2 * (size_t)q * blk_ld(m);
      hcs.p[na] = c.bhcol.p + 2 * (size_t)q * blk_ld(m);
      ps.p[na] = c.bpartial.p + 2 * (size_t)q * nt * blk_ld(m);
      pw.p[na] = c.bpartial.p + 2 * (size_t)q * nt * blk_ld(m);
      ws.p[na] = c.bw[q].p;
      wc.p[na] = c.bw[q].p;
      nrm.p[na] = hcs.p[na] + 2 * (jj + 1);
      nc.p[na] = nrm.p[na];
      vn.p[na] = c.bV[q].p + n2 * (jj + 1);
      ++na;
    }
    if (dcgs2) {
      dev::gs_dual(false, na, n, Vs, Vw, n, jj + 1, cwc, cvc, ws, pw, s);
      dev::gs_final(na, ps, nt, 2 * (jj + 1), hts, dev::PtrSet{}, 0, s);
      dev::dcgs2_coef(na, hs, jj + 1, cwp, cvp, hcs, s);
      dev::gs_dual(true, na, n, Vs, Vw, n, jj + 1, cwc, cvc, ws, pw, s);
    } else {
      dev::gs_pass(0, na, n, Vs, n, jj + 1, hs, ws, pw, s);
      dev::gs_final(na, ps, nt, jj + 1, hts, hcs, 0, s);
      dev::gs_pass(1, na, n, Vs, n, jj + 1, hs, ws, pw, s);
      dev::gs_final(na, ps, nt, jj + 1, hts, hcs, 1, s);
      dev::gs_pass(2, na, n, Vs, n, jj + 1, hs, ws, pw, s);
    }
    dev::norm_final(na, ps, nt, nrm, s);
    dev::scale_by_inv_set(na, n, wc, nc, vn, s);
  }
  HELM_HIP(hipMemcpyAsync(c.bh_host, c.bhcol.p, 2 * sizeof(double) * slots_n * blk_ld(m), hipMemcpyDeviceToHost, s));
  HELM_HIP(hipEventRecord(done_ev, s));
  inflight = true;
  return (int)act.size();
}

void Server::finish(std::vector<helm_server_event>& out) {
  const int64_t n = c.D.n;
  if (inflight) {
    HELM_HIP(hipEventSynchronize(done_ev));
    inflight = false;
    std::vector<int> ending, close;  // slots finishing their column j / ending their cycle
    for (int q : act) {
      Slot& z = slot[q];
      const int jj = z.jj;
      const double* hh = c.bh_host + 2 * (size_t)q * blk_ld(m);
      const int nout = dcgs2 ? 2 * jj + 3 : jj + 2;
      bool bad = false;
      for (int i = 0; i < 2 * nout; ++i) bad = bad || !std::isfinite(hh[i]);
      ++z.its;
      if (bad) {
        helm_server_event e{};
        e.tag = z.tag;
        e.iterations = z.its;
        e.status = HELM_ENUMERIC;
        e.relres = z.rel;
        e.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - z.t0).count();
        emit(out, e);
        z.busy = false;
        continue;
      }
      cplx* h = z.H.data() + (size_t)(m + 1) * jj;
      for (int i = 0; i <= jj + 1; ++i) h[i] = cplx(hh[2 * i], hh[2 * i + 1]);
      const double hn = h[jj + 1].real();
      bool end;
      if (!dcgs2) {
        givens_step(h, jj, z.cs, z.sn, z.g);
        end = std::abs(z.g[jj + 1]) <= tol * z.bnorm || z.its >= maxit || hn == 0 || jj + 1 == m;
      } else {
        // v_j's second pass finishes column j - 1; column j is estimated
        // as it stands and finished at the cycle's end
        if (jj >= 1) {
          cplx* hp = z.H.data() + (size_t)(m + 1) * (jj - 1);
          finish_column(hp, jj - 1, hh + 2 * (jj + 2), hh[2 * (2 * jj + 2)]);
          givens_step(hp, jj - 1, z.cs, z.sn, z.g);
        }
        std::vector<cplx> hc(h, h + jj + 2);
        for (int i = 0; i < jj; ++i) {
          const cplx a = hc[i], bb = hc[i + 1];
          hc[i] = z.cs[i] * a + z.sn[i] * bb;
          hc[i + 1] = -std::conj(z.sn[i]) * a + z.cs[i] * bb;
        }
        const double rr = std::sqrt(std::norm(hc[jj]) + std::norm(hc[jj + 1]));
        const double est = hc[jj] == cplx(0, 0) ? std::abs(z.g[jj]) : std::abs(hc[jj + 1]) / rr * std::abs(z.g[jj]);
        end = est <= tol * z.bnorm || z.its >= maxit || hn == 0 || jj + 1 == m;
        if (end && hn > 0) {
          ending.push_back(q);
          continue;
        }
        if (end) givens_step(h, jj, z.cs, z.sn, z.g);
      }
      if (!end) {
        z.jj = jj + 1;
        continue;
      }
      close.push_back(q);
    }
    // delayed CGS2: the slots that stop here finish column j with the dots
    // of v_{j+1}, one call per group at the same Krylov dimension
    const int nt = dev::gs_tiles(n);
    std::vector<int> grouped(ending.size(), 0);
    for (size_t a = 0; a < ending.size(); ++a) {
      if (grouped[a]) continue;
      const int jj = slot[ending[a]].jj;
      dev::PtrSetC Vs{}, ps{}, hs{}, cwc{}, cvc{};
      dev::PtrSet Vw{}, ws{}, pw{}, hts{}, hcs{}, cwp{}, cvp{};
      int na = 0;
      for (size_t b2 = a; b2 < ending.size(); ++b2) {
        const int q = ending[b2];
        if (grouped[b2] || slot[q].jj != jj) continue;
        grouped[b2] = 1;
        Vs.p[na] = c.bV[q].p;
        Vw.p[na] = c.bV[q].p;
        ws.p[na] = c.bw[q].p;
        ps.p[na] = c.bpartial.p + 2 * (size_t)q * nt * blk_ld(m);
        pw.p[na] = c.bpartial.p + 2 * (size_t)q * nt * blk_ld(m);
        hs.p[na] = c.bhtmp.p + 2 * (size_t)q * blk_ld(m);
        hts.p[na] = c.bhtmp.p + 2 * (size_t)q * blk_ld(m);
        hcs.p[na] = c.bhcol.p + 2 * (size_t)q * blk_ld(m);
        cwp.p[na] = c.bcoef_w.p + 2 * (size_t)q * (m + 2);
        cvp.p[na] = c.bcoef_v.p + 2 * (size_t)q * (m + 2);
        cwc.p[na] = cwp.p[na];
        cvc.p[na] = cvp.p[na];
        ++na;
      }
      dev::gs_dual(false, na, n, Vs, Vw, n, jj + 2, cwc, cvc, ws, pw, s);
      dev::gs_final(na, ps, nt, 2 * (jj + 2), hts, dev::PtrSet{}, 0, s);
      dev::dcgs2_coef(na, hs, jj + 2, cwp, cvp, hcs, s);
    }
    if (!ending.empty()) {
      HELM_HIP(hipMemcpyAsync(c.bh_host, c.bhcol.p, 2 * sizeof(double) * slots_n * blk_ld(m), hipMemcpyDeviceToHost,
                              s));
      HELM_HIP(hipStreamSynchronize(s));
    }
    for (int q : ending) {
      Slot& z = slot[q];
      const int jj = z.jj;
      const double* hh = c.bh_host + 2 * (size_t)q * blk_ld(m);
      bool bad = false;
      for (int i = 0; i < 2 * (2 * jj + 5); ++i) bad = bad || !std::isfinite(hh[i]);
      if (bad) {
        helm_server_event e{};
        e.tag = z.tag;
        e.iterations = z.its;
        e.status = HELM_ENUMERIC;
        e.relres = z.rel;
        e.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - z.t0).count();
        emit(out, e);
        z.busy = false;
        continue;
      }
      cplx* h = z.H.data() + (size_t)(m + 1) * jj;
      finish_column(h, jj, hh + 2 * (jj + 3), hh[2 * (2 * jj + 4)]);
      givens_step(h, jj, z.cs, z.sn, z.g);
      close.push_back(q);
    }
    for (int q : close) {
      // cycle end: x += Z_k y, then the true residual decides
      Slot& z = slot[q];
      const int k = z.jj + 1;
      for (int i = k - 1; i >= 0; --i) {
        cplx acc = z.g[i];
        for (int l = i + 1; l < k; ++l) acc -= z.H[(size_t)(m + 1) * l + i] * z.y[l];
        z.y[i] = acc / z.H[(size_t)(m + 1) * i + i];
      }
      HELM_HIP(hipMemcpyAsync(c.by.p, z.y.data(), sizeof(cplx) * k, hipMemcpyHostToDevice, s));
      dev::gemv_acc(n, c.bZ[q].p, n, k, c.by.p, z.u, s);
      HELM_HIP(hipStreamSynchronize(s));
      start_cycle(q, out);
    }
  }
  admit(out);
}

}  // namespace helm
