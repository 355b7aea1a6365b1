// Host side of the device factorisation (device_factor.hip): the scatter
// lists of the original entries, the extend-add maps, the per-level front
// jobs and their workspace; the pivots come back for the solve layout.
#include <omp.h>

#include <algorithm>
#include <limits>
#include <map>
#include <numeric>
#include <set>

#include "ctx.hpp"

namespace helm {

namespace {

// Front scatter list of one matrix: for every supernode, the front positions
// (row + col * m) and value indices of its original entries (those with
// min(row, col) among its columns, in the symbolic ordering).
void scatter_lists(const Csr& A, const Symbolic& S, int64_t val0, std::vector<int64_t>& sn_ptr,
                   std::vector<int32_t>& pos, std::vector<int32_t>& val) {
  const int64_t n = A.n;
  std::vector<int64_t> tptr(n + 1, 0);
  for (int64_t p = 0; p < A.nnz(); ++p) tptr[A.col[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  std::vector<int32_t> trow(A.nnz());
  std::vector<int64_t> tidx(A.nnz());
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        const int64_t q = fill[A.col[p]]++;
        trow[q] = (int32_t)i;
        tidx[q] = p;
      }
  }
  std::vector<int32_t> fpos(n, -1);
  sn_ptr.assign(S.nsn + 1, 0);
  pos.clear();
  val.clear();
  for (int32_t s = 0; s < S.nsn; ++s) {
    const int32_t c0 = S.sn_c0[s], w = S.sn_w[s], c1 = c0 + w;
    const int32_t* R = S.rows.data() + S.sn_rptr[s];
    const int32_t r = (int32_t)(S.sn_rptr[s + 1] - S.sn_rptr[s]);
    const int64_t m = w + r;
    for (int32_t k = 0; k < w; ++k) fpos[c0 + k] = k;
    for (int32_t a = 0; a < r; ++a) fpos[R[a]] = w + a;
    for (int32_t j = c0; j < c1; ++j) {
      const int32_t old = S.perm[j];
      for (int64_t p = A.ptr[old]; p < A.ptr[old + 1]; ++p) {
        const int32_t nc = S.iperm[A.col[p]];
        if (nc < c0) continue;
        if (fpos[nc] < 0) fail(HELM_EINVAL, "internal: entry outside its front");
        pos.push_back((int32_t)(fpos[j] + (int64_t)fpos[nc] * m));
        val.push_back((int32_t)(val0 + p));
      }
      for (int64_t p = tptr[old]; p < tptr[old + 1]; ++p) {
        const int32_t nr = S.iperm[trow[p]];
        if (nr < c1) continue;
        if (fpos[nr] < 0) fail(HELM_EINVAL, "internal: entry outside its front");
        pos.push_back((int32_t)(fpos[nr] + (int64_t)fpos[j] * m));
        val.push_back((int32_t)(val0 + tidx[p]));
      }
    }
    for (int32_t k = 0; k < w; ++k) fpos[c0 + k] = -1;
    for (int32_t a = 0; a < r; ++a) fpos[R[a]] = -1;
    sn_ptr[s + 1] = (int64_t)pos.size();
  }
}

// ep[a] for a child's rows a: the position of that row in its parent's front.
void extend_add_map(const Symbolic& S, int32_t* ep) {
  std::vector<int32_t> fpos(S.n, -1);
  std::vector<std::vector<int32_t>> children(S.nsn);
  for (int32_t s = 0; s < S.nsn; ++s)
    if (S.sn_parent[s] >= 0) children[S.sn_parent[s]].push_back(s);
  for (int32_t p = 0; p < S.nsn; ++p) {
    const int32_t c0 = S.sn_c0[p], w = S.sn_w[p];
    const int32_t* R = S.rows.data() + S.sn_rptr[p];
    const int32_t r = (int32_t)(S.sn_rptr[p + 1] - S.sn_rptr[p]);
    for (int32_t k = 0; k < w; ++k) fpos[c0 + k] = k;
    for (int32_t a = 0; a < r; ++a) fpos[R[a]] = w + a;
    for (int32_t c : children[p])
      for (int64_t a = S.sn_rptr[c]; a < S.sn_rptr[c + 1]; ++a) {
        if (fpos[S.rows[a]] < 0) fail(HELM_EINVAL, "internal: child row missing from parent front");
        ep[a] = fpos[S.rows[a]];
        // sorted row lists map to increasing front positions (the split
        // assembly relies on it)
        if (a > S.sn_rptr[c] && ep[a] <= ep[a - 1]) fail(HELM_EINVAL, "internal: unsorted child rows");
      }
    for (int32_t k = 0; k < w; ++k) fpos[c0 + k] = -1;
    for (int32_t a = 0; a < r; ++a) fpos[R[a]] = -1;
  }
}

}  // namespace

void factor_batch_device(const std::vector<const Csr*>& As, const std::vector<const Symbolic*>& Ss,
                         dev::FactorPrecision prec, int32_t split_min, const std::vector<void*>& pf,
                         const std::vector<void*>& pb, std::vector<NumericOut>& num, int32_t& n_perturbed,
                         double& scratch_bytes) {
  const int nm = (int)As.size();
  std::vector<int64_t> pos0(nm + 1, 0), sn0(nm + 1, 0), rows0(nm + 1, 0), nnz0(nm + 1, 0);
  for (int i = 0; i < nm; ++i) {
    pos0[i + 1] = pos0[i] + Ss[i]->n;
    sn0[i + 1] = sn0[i] + Ss[i]->nsn;
    rows0[i + 1] = rows0[i] + (int64_t)Ss[i]->rows.size();
    nnz0[i + 1] = nnz0[i] + As[i]->nnz();
  }
  if (nnz0[nm] >= (int64_t)INT32_MAX) fail(HELM_EINVAL, "batch too large for 32-bit value indices");
  std::vector<double> anorm(nm, 0.0);
  std::vector<std::vector<int64_t>> sptr(nm);
  std::vector<std::vector<int32_t>> spos(nm), sval(nm);
  std::vector<int32_t> ep(std::max<int64_t>(rows0[nm], 1));
  std::string errmsg;
  int errcode = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nm; ++i) {
    try {
      for (const cplx& v : As[i]->val) anorm[i] = std::max(anorm[i], std::abs(v));
      scatter_lists(*As[i], *Ss[i], nnz0[i], sptr[i], spos[i], sval[i]);
      extend_add_map(*Ss[i], ep.data() + rows0[i]);
    } catch (const Error& e) {
#pragma omp critical
      {
        if (!errcode) {
          errcode = e.code;
          errmsg = e.what();
        }
      }
    }
  }
  if (errcode) fail(errcode, errmsg);
  for (int i = 0; i < nm; ++i)
    if (!(anorm[i] > 0)) fail(HELM_ESINGULAR, "zero local matrix");

  // device inputs: values, scatter lists, extend-add map
  std::vector<int64_t> asm0(nm + 1, 0);
  for (int i = 0; i < nm; ++i) asm0[i + 1] = asm0[i] + (int64_t)spos[i].size();
  DVec<double> aval;
  DVec<int32_t> asm_pos, asm_val, ep_d;
  {
    std::vector<cplx> v(nnz0[nm]);
    std::vector<int32_t> pa(asm0[nm]), va(asm0[nm]);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nm; ++i) {
      std::copy(As[i]->val.begin(), As[i]->val.end(), v.begin() + nnz0[i]);
      std::copy(spos[i].begin(), spos[i].end(), pa.begin() + asm0[i]);
      std::copy(sval[i].begin(), sval[i].end(), va.begin() + asm0[i]);
    }
    aval.upload(reinterpret_cast<const double*>(v.data()), 2 * v.size());
    asm_pos.upload(pa);
    asm_val.upload(va);
    ep_d.upload(ep);
  }

  // Schur complement offsets, children lists, levels.  A supernode's Schur
  // complement (r x r) is live from its own level (its height in the
  // elimination tree) until its parent's level has assembled it; offsets
  // come from a best-fit arena run level by level (a level's new
  // complements are placed before the ones it consumes are released), so
  // the buffer holds the largest set live at once instead of all of them.
  const int64_t nsn = sn0[nm];
  int32_t H = 0;
  for (int i = 0; i < nm; ++i)
    for (int32_t s = 0; s < Ss[i]->nsn; ++s) H = std::max(H, Ss[i]->height[s]);
  std::vector<std::vector<std::pair<int, int32_t>>> levels(H + 1);
  std::vector<std::vector<int64_t>> release(H + 1);  // complements consumed by each level
  for (int i = 0; i < nm; ++i) {
    const Symbolic& S = *Ss[i];
    for (int32_t s = 0; s < S.nsn; ++s) {
      levels[S.height[s]].push_back({i, s});
      if (S.sn_parent[s] >= 0) release[S.height[S.sn_parent[s]]].push_back(sn0[i] + s);
    }
  }
  auto rsz = [&](int i, int32_t s) { return Ss[i]->sn_rptr[s + 1] - Ss[i]->sn_rptr[s]; };
  std::vector<int64_t> uoff(nsn, 0), usz(nsn, 0);
  int64_t upd_entries = 0;
  {
    // free holes below the top, indexed by offset (to merge neighbours) and
    // by size (best fit, lowest offset among equals)
    std::map<int64_t, int64_t> by_off;
    std::set<std::pair<int64_t, int64_t>> by_size;
    auto add_hole = [&](int64_t o, int64_t n) {
      by_off[o] = n;
      by_size.insert({n, o});
    };
    auto drop_hole = [&](std::map<int64_t, int64_t>::iterator it) {
      by_size.erase({it->second, it->first});
      return by_off.erase(it);
    };
    int64_t top = 0;
    for (int32_t l = 0; l <= H; ++l) {
      for (auto& e : levels[l]) {
        const int64_t g = sn0[e.first] + e.second, r = rsz(e.first, e.second), n = r * r;
        usz[g] = n;
        if (n == 0) continue;
        auto fit = by_size.lower_bound({n, std::numeric_limits<int64_t>::min()});
        if (fit != by_size.end()) {
          const int64_t o = fit->second, rest = fit->first - n;
          drop_hole(by_off.find(o));
          uoff[g] = o;
          if (rest > 0) add_hole(o + n, rest);
        } else {
          uoff[g] = top;
          top += n;
        }
      }
      upd_entries = std::max(upd_entries, top);
      for (int64_t g : release[l]) {
        if (usz[g] == 0) continue;
        int64_t o = uoff[g], n = usz[g];
        auto nx = by_off.lower_bound(o);
        if (nx != by_off.end() && nx->first == o + n) {
          n += nx->second;
          nx = drop_hole(nx);
        }
        if (nx != by_off.begin()) {
          auto pv = std::prev(nx);
          if (pv->first + pv->second == o) {
            o = pv->first;
            n += pv->second;
            drop_hole(pv);
          }
        }
        if (o + n == top)
          top = o;
        else
          add_hole(o, n);
      }
    }
  }
  std::vector<dev::FrontChild> kids;
  std::vector<int32_t> kid0(nsn + 1, 0);
  for (int i = 0; i < nm; ++i) {
    const Symbolic& S = *Ss[i];
    std::vector<std::vector<int32_t>> ch(S.nsn);
    for (int32_t s = 0; s < S.nsn; ++s)
      if (S.sn_parent[s] >= 0) ch[S.sn_parent[s]].push_back(s);
    for (int32_t s = 0; s < S.nsn; ++s) {
      kid0[sn0[i] + s] = (int32_t)kids.size();
      for (int32_t c : ch[s]) kids.push_back({uoff[sn0[i] + c], rows0[i] + S.sn_rptr[c], (int32_t)rsz(i, c), 0});
    }
  }
  kid0[nsn] = (int32_t)kids.size();
  DVec<dev::FrontChild> kids_d;
  kids_d.upload(kids);
  // workspace and Schur complements in the working precision: complex64
  // entries take one double each, complex128 entries two
  const size_t wpe = prec == dev::FactorPrecision::kC64 ? 1 : 2;
  DVec<double> upd;
  upd.alloc(wpe * std::max<int64_t>(upd_entries, 1));

  // jobs, level by level, in chunks whose workspace fits the budget
  auto job_ws = [&](int i, int32_t s) {
    const Symbolic& S = *Ss[i];
    const int64_t w = S.sn_w[s], m = w + (S.sn_rptr[s + 1] - S.sn_rptr[s]);
    return m * m + 2 * m * w;
  };
  int64_t biggest = 1, level_max = 1;
  for (auto& L : levels) {
    int64_t t = 0;
    for (auto& e : L) {
      biggest = std::max(biggest, job_ws(e.first, e.second));
      t += job_ws(e.first, e.second);
    }
    level_max = std::max(level_max, t);
  }
  const int64_t budget = std::max(biggest, std::min<int64_t>(level_max, (int64_t)1 << 30));  // complex entries
  std::vector<dev::FrontJob> jobs;
  std::vector<std::pair<int64_t, int64_t>> launches;  // [first job, end)
  for (auto& L : levels) {
    std::stable_sort(L.begin(), L.end(), [&](const std::pair<int, int32_t>& a, const std::pair<int, int32_t>& b) {
      return job_ws(a.first, a.second) > job_ws(b.first, b.second);
    });
    int64_t used = 0, first = (int64_t)jobs.size();
    for (auto& e : L) {
      const int i = e.first;
      const int32_t s = e.second;
      const Symbolic& S = *Ss[i];
      const int64_t need = job_ws(i, s);
      if (used + need > budget && (int64_t)jobs.size() > first) {
        launches.push_back({first, (int64_t)jobs.size()});
        first = (int64_t)jobs.size();
        used = 0;
      }
      const int32_t w = S.sn_w[s], m = w + (int32_t)(S.sn_rptr[s + 1] - S.sn_rptr[s]);
      dev::FrontJob J{};
      J.F = used;
      J.X = used + (int64_t)m * m;
      J.Y = J.X + (int64_t)m * w;
      J.upd = uoff[sn0[i] + s];
      J.pf = pf[i];
      J.pb = pb[i];
      J.pfo = S.sn_fwd_off[s];
      J.pbo = S.sn_bwd_off[s];
      J.asm0 = asm0[i] + sptr[i][s];
      J.asm1 = asm0[i] + sptr[i][s + 1];
      J.m = m;
      J.w = w;
      J.c0 = S.sn_c0[s];
      J.piv0 = (int32_t)(pos0[i] + S.sn_c0[s]);
      J.kid0 = kid0[sn0[i] + s];
      J.kid1 = kid0[sn0[i] + s + 1];
      J.anorm = anorm[i];
      jobs.push_back(J);
      used += need;
    }
    if ((int64_t)jobs.size() > first) launches.push_back({first, (int64_t)jobs.size()});
  }
  for (int i = 0; i < nm; ++i)
    if (Ss[i]->tile_rows != Ss[0]->tile_rows) fail(HELM_EINVAL, "internal: mixed tile heights in a batch");
  // within each launch, the fronts of at least split_min rows first: they
  // take the several-workgroups form (split_min < 0: none)
  std::vector<int64_t> nsplit(launches.size(), 0);
  std::vector<int32_t> mmax(launches.size(), 0), wmax(launches.size(), 0);
  for (size_t q = 0; q < launches.size(); ++q) {
    auto first = jobs.begin() + launches[q].first, last = jobs.begin() + launches[q].second;
    auto mid = std::stable_partition(first, last,
                                     [&](const dev::FrontJob& J) { return split_min >= 0 && J.m >= split_min; });
    nsplit[q] = mid - first;
    for (auto it = first; it != mid; ++it) {
      mmax[q] = std::max(mmax[q], it->m);
      wmax[q] = std::max(wmax[q], it->w);
    }
  }
  DVec<dev::FrontJob> jobs_d;
  jobs_d.upload(jobs);
  DVec<double> ws;
  ws.alloc(wpe * (size_t)budget);
  scratch_bytes = 0;
  DVec<int32_t> piv_d, swp_d, npert_d;
  piv_d.alloc(std::max<int64_t>(pos0[nm], 1));
  swp_d.alloc(std::max<int64_t>(pos0[nm], 1));
  npert_d.alloc(std::max<size_t>(jobs.size(), 1));
  scratch_bytes = 8.0 * (double)(ws.n + upd.n + aval.n) + 4.0 * (double)(asm_pos.n + asm_val.n + ep_d.n + piv_d.n +
                                                                        swp_d.n + npert_d.n) +
                  (double)sizeof(dev::FrontChild) * kids_d.n + (double)sizeof(dev::FrontJob) * jobs_d.n;
  for (size_t q = 0; q < launches.size(); ++q) {
    const int64_t f = launches[q].first, ns = nsplit[q], nj = launches[q].second - f;
    dev::factor_fronts_split(jobs_d.p + f, (int)ns, mmax[q], wmax[q], ws.p, upd.p, asm_pos.p, asm_val.p, aval.p,
                             kids_d.p, ep_d.p, piv_d.p, swp_d.p, npert_d.p + f, prec, Ss[0]->tile_rows, nullptr);
    dev::factor_fronts(jobs_d.p + f + ns, (int)(nj - ns), ws.p, upd.p, asm_pos.p, asm_val.p, aval.p, kids_d.p,
                       ep_d.p, piv_d.p, npert_d.p + f + ns, prec, Ss[0]->tile_rows, nullptr);
  }
  HELM_HIP(hipGetLastError());
  HELM_HIP(hipDeviceSynchronize());
  std::vector<int32_t> piv(pos0[nm]), np(jobs.size());
  if (!piv.empty()) HELM_HIP(hipMemcpy(piv.data(), piv_d.p, sizeof(int32_t) * piv.size(), hipMemcpyDeviceToHost));
  if (!np.empty()) HELM_HIP(hipMemcpy(np.data(), npert_d.p, sizeof(int32_t) * np.size(), hipMemcpyDeviceToHost));
  n_perturbed = std::accumulate(np.begin(), np.end(), 0);
  for (int i = 0; i < nm; ++i) {
    num[i].piv.assign(piv.begin() + pos0[i], piv.begin() + pos0[i + 1]);
    num[i].n_perturbed = 0;
  }
}

}  // namespace helm
