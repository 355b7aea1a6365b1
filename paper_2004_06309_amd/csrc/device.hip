// HIP kernels of the per-iteration path (gfx950, 64-wide wavefronts).
//
//  - fwd_level / bwd_level: one level of the batched supernodal forward and
//    backward solves of all subdomains at once (local solves of eq. oras).
//    One workgroup (4 waves) per tile of <= 64 panel rows; each lane owns a
//    row, the four waves split the input columns, the input vector (gathered
//    through index lists, restriction fused in) sits in LDS, and the panel is
//    streamed column by column (64 rows x 16 B = 1 KiB coalesced per wave).
//  - spmv / spmv_real: CSR products, a group of lanes per row.
//  - prolong: partition-of-unity weighted sum of the local solutions.
//  - Gram-Schmidt reductions: per-block partial sums reduced in a fixed order
//    (no atomics), so every result is bitwise repeatable.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "device.hpp"

namespace helm {
namespace dev {

namespace {

constexpr int kWG = 256;
constexpr int kChunk = kLevelChunkMax;  // input columns staged in LDS per pass (at most)

__device__ __forceinline__ void cfma(double& ar, double& ai, double2 a, double2 v) {
  ar = fma(a.x, v.x, ar);
  ar = fma(-a.y, v.y, ar);
  ai = fma(a.x, v.y, ai);
  ai = fma(a.y, v.x, ai);
}

__device__ __forceinline__ double2 widen(double2 a) { return a; }
__device__ __forceinline__ double2 widen(float2 a) { return make_double2((double)a.x, (double)a.y); }

// Panels are streamed once per sweep: non-temporal loads keep them from
// evicting the reused vectors from the caches.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldp(const double2* p) {
  const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ldp(const float2* p) {
  const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2*>(p));
  return make_float2(v.x, v.y);
}

// Streams columns k0, k0 + ks, ... (< k1) of a tile (column-major, ld = nr)
// against vin, eight independent loads in flight per lane.
template <class PT>
__device__ __forceinline__ void tile_dot(const PT* __restrict__ p, int nr, const double2* vin, int k0, int k1, int ks,
                                        double& ar, double& ai) {
  int k = k0;
  double br = 0, bi = 0;
  for (; k + 7 * ks < k1; k += 8 * ks) {
    PT a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = ldp(p + (int64_t)(k + u * ks) * nr);
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      cfma(ar, ai, widen(a[u]), vin[k + u * ks]);
      cfma(br, bi, widen(a[u + 1]), vin[k + (u + 1) * ks]);
    }
  }
  for (; k < k1; k += ks) cfma(ar, ai, widen(ldp(p + (int64_t)k * nr)), vin[k]);
  ar += br;
  ai += bi;
}

// Calls f(i) for the child-update entries routed to front row fr, in list
// order: rows with at most two read them from their index pair (one load),
// longer lists from fcon_ptr / fcon_idx.
template <class F>
__device__ __forceinline__ void for_children(const Batch& b, int fr, F&& f) {
  const int2 c = b.fcon2[fr];
  if (c.x >= 0) {
    f(c.x);
    if (c.y >= 0) f(c.y);
  } else if (c.x < -1) {
    for (int e = -2 - c.x; e < b.fcon_ptr[fr + 1]; ++e) f(b.fcon_idx[e]);
  }
}

// Lanes per tile row group: a tile with few rows spreads its columns over
// 64 / R lane groups of R = nrows lanes (the last 64 mod R lanes idle).
__device__ __forceinline__ int row_group(int nrows) { return nrows <= 32 ? max(nrows, 1) : 64; }

// Work split of a workgroup (4 waves) over the tiles of its task.
struct Split {
  int my;      // tile slot of this wave
  int part;    // this wave's share of the tile's columns
  int wpt;     // waves per tile
  int region;  // LDS entries per tile slot
  bool has;    // the slot holds a tile
};

__device__ __forceinline__ Split split_of(const Task& task, int chunk) {
  Split sp;
  // the wave index is the same on all lanes: scalar, so the wave's tile
  // descriptor is a scalar load
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  sp.wpt = task.wpt;
  sp.my = wv / sp.wpt;
  sp.part = wv % sp.wpt;
  sp.region = chunk / (4 / sp.wpt);
  sp.has = sp.my < task.ntile;
  return sp;
}

// One workgroup task of a forward level (vin: chunk LDS entries, at least
// 4 / wpt times the widest tile of a task with wpt < 4; red: 4 x 64 LDS
// entries).
template <class PT>
__device__ __forceinline__ void fwd_task(const Task& task, const Batch& b, const double2* __restrict__ bin,
                                         double2* vin, double2 (*red)[64], int chunk) {
  const Split sp = split_of(task, chunk);
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Tile t{};
  if (sp.has) t = b.tf[task.tile0 + sp.my];
  const int s = t.sn, c0 = t.c0, w = t.w, frow0 = t.aux;
  double2* vt = vin + sp.my * sp.region;
  const int R = row_group(t.nrows), G = 64 / R, grp = lane / R, row_l = lane % R;
  const PT* __restrict__ P = reinterpret_cast<const PT*>(b.pf) + t.off + row_l;
  const double2* __restrict__ ub = reinterpret_cast<const double2*>(b.ubuf);
  // the children's updates to this lane's output row (rows past the pivot
  // block) are fetched before the panel, off the critical path
  const bool out = sp.has && sp.part == 0 && lane < t.nrows;
  const int row = t.row0 + lane;
  double er = 0, ei = 0;
  int uo = 0;
  if (out && row >= w) {
    uo = b.sn_uoff[s] + row - w;
    for_children(b, frow0 + row, [&](int i) {
      const double2 u = ub[i];
      er += u.x;
      ei += u.y;
    });
  }
  double ar = 0, ai = 0;
  // all waves of a workgroup run the same number of passes: one, unless the
  // workgroup holds a single wide tile
  const int npass = sp.wpt == 4 ? (t.ncols + chunk - 1) / chunk : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int cb = pass * sp.region;
    const int cn = sp.has ? min(sp.region, t.ncols - cb) : 0;
    for (int k = sp.part * 64 + lane; k < cn; k += 64 * sp.wpt) {
      const int kk = cb + k;
      double2 v = bin[b.bidx[c0 + kk]];
      for_children(b, frow0 + kk, [&](int i) {
        const double2 u = ub[i];
        v.x -= u.x;
        v.y -= u.y;
      });
      vt[k] = v;
    }
    __syncthreads();
    if (sp.has && row_l < t.nrows && grp < G) {
      const int per = (cn + sp.wpt - 1) / sp.wpt;
      const int k0 = sp.part * per, k1 = min(cn, k0 + per);
      tile_dot(P + (int64_t)cb * t.nrows, t.nrows, vt, k0 + grp, k1, G, ar, ai);
    }
    __syncthreads();
  }
  red[wv][lane] = make_double2(ar, ai);
  __syncthreads();
  if (out) {
    double rr = 0, ii = 0;
    for (int q = 0; q < sp.wpt; ++q)
      for (int g = lane; g < G * R; g += R) {
        rr += red[wv + q][g].x;
        ii += red[wv + q][g].y;
      }
    if (row < w)
      reinterpret_cast<double2*>(b.y)[c0 + row] = make_double2(rr, ii);
    else
      reinterpret_cast<double2*>(b.ubuf)[uo] = make_double2(rr + er, ii + ei);
  }
}

template <class PT>
__device__ __forceinline__ void bwd_task(const Task& task, const Batch& b, double2* vin, double2 (*red)[64],
                                         int chunk) {
  const Split sp = split_of(task, chunk);
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Tile t{};
  if (sp.has) t = b.tb[task.tile0 + sp.my];
  const int c0 = t.c0, w = t.w;
  const int64_t roff = t.aux;
  double2* vt = vin + sp.my * sp.region;
  const int R = row_group(t.nrows), G = 64 / R, grp = lane / R, row_l = lane % R;
  const PT* __restrict__ P = reinterpret_cast<const PT*>(b.pb) + t.off + row_l;
  const double2* __restrict__ yv = reinterpret_cast<const double2*>(b.y);
  const double2* xv = reinterpret_cast<const double2*>(b.x);
  double ar = 0, ai = 0;
  const int npass = sp.wpt == 4 ? (t.ncols + chunk - 1) / chunk : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int cb = pass * sp.region;
    const int cn = sp.has ? min(sp.region, t.ncols - cb) : 0;
    for (int k = sp.part * 64 + lane; k < cn; k += 64 * sp.wpt) {
      const int c = t.col0 + cb + k;
      vt[k] = c < w ? yv[c0 + c] : xv[b.rows[roff + (c - w)]];
    }
    __syncthreads();
    if (sp.has && row_l < t.nrows && grp < G) {
      const int per = (cn + sp.wpt - 1) / sp.wpt;
      const int k0 = sp.part * per, k1 = min(cn, k0 + per);
      tile_dot(P + (int64_t)cb * t.nrows, t.nrows, vt, k0 + grp, k1, G, ar, ai);
    }
    __syncthreads();
  }
  red[wv][lane] = make_double2(ar, ai);
  __syncthreads();
  if (sp.has && sp.part == 0 && lane < t.nrows) {
    double rr = 0, ii = 0;
    for (int q = 0; q < sp.wpt; ++q)
      for (int g = lane; g < G * R; g += R) {
        rr += red[wv + q][g].x;
        ii += red[wv + q][g].y;
      }
    reinterpret_cast<double2*>(b.x)[c0 + t.row0 + lane] = make_double2(rr, ii);
  }
}

// The input-column buffer is dynamic LDS sized per level (chunk entries), so
// levels of narrow tiles keep more workgroups resident per CU.
// The grid holds at most as many workgroups as fit on the device at once;
// each sweeps tasks blockIdx.x, blockIdx.x + gridDim.x, ... (widest first),
// so a level costs no workgroup launches beyond the first wave of them.
template <class PT, int kCoarse>
__global__ __launch_bounds__(kWG) void fwd_level_kernel(const Task* __restrict__ tasks, int ntasks, Batch b,
                                                        const double2* __restrict__ bin, int chunk) {
  extern __shared__ double2 vin[];
  __shared__ double2 red[4][64];
  for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
    fwd_task<PT>(tasks[t], b, bin, vin, red, chunk);
    __syncthreads();  // red and vin are rewritten by the next task
  }
}

template <class PT, int kCoarse>
__global__ __launch_bounds__(kWG) void bwd_level_kernel(const Task* __restrict__ tasks, int ntasks, Batch b,
                                                        int chunk) {
  extern __shared__ double2 vin[];
  __shared__ double2 red[4][64];
  for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
    bwd_task<PT>(tasks[t], b, vin, red, chunk);
    __syncthreads();
  }
}

// Forward solve of narrow supernodes (w <= 64), one wave per supernode.
// Lane k holds gathered input k; lane l owns row l of every 64-row tile, and
// the wave streams up to four tiles side by side (column k of each), so a
// supernode's whole panel is one stream of loads after a single gather.
__device__ __forceinline__ double bcast(double x, int k) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, k);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// acc[q] += tile q (rows lane, columns 0..w-1) * v, NQ tiles at P + 64 q w
// (tile q has rows[q] rows, tiles q >= nq are skipped), 8 loads in flight
// per lane.  Lanes past a tile's last row re-read that row: their sums are
// never stored, and every load stays inside the tile.
template <class PT, int NQ>
__device__ __forceinline__ void sn_stream(const PT* __restrict__ P, int w, int nq, const int* rows, double2 v,
                                          double2* acc) {
  constexpr int KU = 8 / NQ;
  const int lane = threadIdx.x & 63;
  const PT* base[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) base[q] = P + (int64_t)q * 64 * w + min(lane, max(rows[q], 1) - 1);
  for (int k = 0; k < w; k += KU) {
    PT a[KU][NQ];
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        PT z{};
        a[u][q] = (k + u < w && q < nq) ? ldp(base[q] + (int64_t)(k + u) * rows[q]) : z;
      }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (k + u >= w) break;
      const double2 x = make_double2(bcast(v.x, k + u), bcast(v.y, k + u));
#pragma unroll
      for (int q = 0; q < NQ; ++q) cfma(acc[q].x, acc[q].y, widen(a[u][q]), x);
    }
  }
}

template <class PT>
__global__ __launch_bounds__(kWG) void fwd_sn_kernel(const SnJob* __restrict__ jobs, int njobs, Batch b,
                                                     const double2* __restrict__ bin) {
  const int lane = threadIdx.x & 63;
  const double2* __restrict__ ub = reinterpret_cast<const double2*>(b.ubuf);
  // the job index is wave-uniform, so the job lives in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int j = blockIdx.x * 4 + wave; j < njobs; j += gridDim.x * 4) {
    const SnJob jb = jobs[j];
    const int m = jb.m, w = jb.w;
    // inputs: restricted right-hand side minus the children's updates
    double2 v = make_double2(0.0, 0.0);
    if (lane < w) {
      v = bin[b.bidx[jb.c0 + lane]];
      for_children(b, jb.frow0 + lane, [&](int i) {
        const double2 u = ub[i];
        v.x -= u.x;
        v.y -= u.y;
      });
    }
    const PT* __restrict__ P = reinterpret_cast<const PT*>(b.pf) + jb.off;
    for (int q0 = 0; q0 * 64 < m; q0 += 4) {
      const int nq = min(4, (m - q0 * 64 + 63) / 64);
      int rows[4];
      double2 acc[4];
      // rows past the pivot block start from the children's updates
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rows[q] = q < nq ? min(64, m - (q0 + q) * 64) : 0;
        acc[q] = make_double2(0.0, 0.0);
        const int row = (q0 + q) * 64 + lane;
        if (q < nq && lane < rows[q] && row >= w)
          for_children(b, jb.frow0 + row, [&](int i) {
            const double2 u = ub[i];
            acc[q].x += u.x;
            acc[q].y += u.y;
          });
      }
      const PT* Pq = P + (int64_t)q0 * 64 * w;
      if (nq == 1)
        sn_stream<PT, 1>(Pq, w, nq, rows, v, acc);
      else if (nq == 2)
        sn_stream<PT, 2>(Pq, w, nq, rows, v, acc);
      else
        sn_stream<PT, 4>(Pq, w, nq, rows, v, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = (q0 + q) * 64 + lane;
        if (q < nq && lane < rows[q]) {
          if (row < w)
            reinterpret_cast<double2*>(b.y)[jb.c0 + row] = acc[q];
          else
            reinterpret_cast<double2*>(b.ubuf)[jb.uoff + row - w] = acc[q];
        }
      }
    }
  }
}

// Whole forward + backward solve of a small batch (the coarse matrix) in one
// cooperative launch: the workgroups sweep each level's tasks and meet at a
// grid-wide barrier before the next level, instead of one launch per level.
__global__ __launch_bounds__(kWG) void batch_solve_coop_kernel(Batch b, const double2* __restrict__ bin,
                                                               LevelRanges lv) {
  __shared__ double2 vin[kChunk];
  __shared__ double2 red[4][64];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int l = 0; l < lv.nf; ++l) {
    for (int64_t t = lv.f[l] + blockIdx.x; t < lv.f[l + 1]; t += gridDim.x) {
      fwd_task<double2>(b.kf[t], b, bin, vin, red, kChunk);
      __syncthreads();
    }
    grid.sync();
  }
  for (int l = 0; l < lv.nb; ++l) {
    for (int64_t t = lv.b[l] + blockIdx.x; t < lv.b[l + 1]; t += gridDim.x) {
      bwd_task<double2>(b.kb[t], b, vin, red, kChunk);
      __syncthreads();
    }
    grid.sync();
  }
}

// XCD-aware workgroup order for grids that are a multiple of 8: workgroups
// are dealt round-robin to the 8 XCDs, so workgroup b takes block
// (b % 8) * per + b / 8 and every XCD sweeps a contiguous eighth of the
// blocks, keeping the x entries that block gathers in its own L2.
__device__ __forceinline__ int64_t xcd_block() {
  const unsigned per = gridDim.x / 8;
  return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// One row of a CSR matrix per G lanes; each lane takes U entries per pass
// (entries base + u G + lane), loading all U columns, then all U values and
// x entries before the multiply-adds, so a wave keeps U gathers in flight
// instead of one dependent col -> x chain per entry.  With kXcd, workgroup b
// runs on XCD b % 8 (workgroups are dealt round-robin) and takes the
// (b / 8)-th block of that XCD's row range [xr[b % 8], xr[b % 8 + 1]).
// Entries are complex (VT = double2), or real parts and imaginary parts
// stored as separate real entries (VT = double): an imaginary entry carries
// bit 31 in its column index and multiplies i x[col].  A of the Helmholtz
// problem is complex only on the absorbing boundary, so the split storage
// moves 12 B per entry instead of 20 B.
template <class VT>
__device__ __forceinline__ void spmv_fma(double& ar, double& ai, int c, VT v, const double2* __restrict__ x);
template <>
__device__ __forceinline__ void spmv_fma<double2>(double& ar, double& ai, int c, double2 v,
                                                  const double2* __restrict__ x) {
  cfma(ar, ai, v, x[c]);
}
template <>
__device__ __forceinline__ void spmv_fma<double>(double& ar, double& ai, int c, double v,
                                                 const double2* __restrict__ x) {
  const double2 xv = x[c & 0x7fffffff];
  const bool im = c < 0;  // i x = (-x.y, x.x)
  ar = fma(v, im ? -xv.y : xv.x, ar);
  ai = fma(v, im ? xv.x : xv.y, ai);
}

template <int G, int U, bool kXcd, class VT>
__global__ __launch_bounds__(kWG) void spmv_kernel(int64_t n, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                   const int64_t* __restrict__ xr, const double2* __restrict__ x,
                                                   const double2* __restrict__ bvec, double2* __restrict__ y) {
  int64_t row, end = n;
  if (kXcd) {
    row = xr[blockIdx.x & 7] + ((int64_t)(blockIdx.x >> 3) * kWG + threadIdx.x) / G;
    end = xr[(blockIdx.x & 7) + 1];
  } else {
    row = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G;
  }
  const int l = threadIdx.x % G;
  double ar = 0, ai = 0;
  if (row < end) {
    const int64_t p1 = ptr[row + 1];
    for (int64_t base = ptr[row] + l; base < p1; base += G * U) {
      int c[U];
      VT v[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ok[u] = base + u * G < p1;
        c[u] = ok[u] ? col[base + u * G] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = ok[u] ? val[base + u * G] : VT{};
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) spmv_fma<VT>(ar, ai, c[u], v[u], x);
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    ar += __shfl_xor(ar, o, G);
    ai += __shfl_xor(ai, o, G);
  }
  if (row < end && l == 0) {
    if (bvec) {
      double2 bb = bvec[row];
      y[row] = make_double2(bb.x - ar, bb.y - ai);
    } else {
      y[row] = make_double2(ar, ai);
    }
  }
}

// Sliced ELL (slices of 64 rows = one wavefront): slice s holds rows
// perm[64 s .. 64 s + 63], padded to the slice's longest row, stored
// column-major inside the slice so each lane owns a row and every load of a
// wave is one contiguous 1 KiB (values) / 256 B (columns) line.
__global__ __launch_bounds__(kWG) void sell_kernel(int64_t n, int64_t nslices, const int64_t* __restrict__ soff,
                                                   const int32_t* __restrict__ swidth,
                                                   const int32_t* __restrict__ perm, const int32_t* __restrict__ col,
                                                   const double2* __restrict__ val, const double2* __restrict__ x,
                                                   const double2* __restrict__ bvec, double2* __restrict__ y) {
  // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so
  // workgroup b works on block (b % 8) * per + b / 8 and every XCD sweeps a
  // contiguous eighth of the rows (their x entries stay in its own L2)
  const unsigned per = gridDim.x / 8;
  const int64_t vb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t s = vb * (kWG / 64) + (threadIdx.x >> 6);
  if (s >= nslices) return;
  const int lane = threadIdx.x & 63;
  const int64_t slot = s * 64 + lane;
  const int64_t off = soff[s] + lane;
  const int wdt = swidth[s];
  double ar = 0, ai = 0, br = 0, bi = 0;
  int j = 0;
  for (; j + 4 <= wdt; j += 4) {
    const int c0 = col[off + (int64_t)(j + 0) * 64], c1 = col[off + (int64_t)(j + 1) * 64];
    const int c2 = col[off + (int64_t)(j + 2) * 64], c3 = col[off + (int64_t)(j + 3) * 64];
    const double2 v0 = val[off + (int64_t)(j + 0) * 64], v1 = val[off + (int64_t)(j + 1) * 64];
    const double2 v2 = val[off + (int64_t)(j + 2) * 64], v3 = val[off + (int64_t)(j + 3) * 64];
    cfma(ar, ai, v0, x[c0]);
    cfma(br, bi, v1, x[c1]);
    cfma(ar, ai, v2, x[c2]);
    cfma(br, bi, v3, x[c3]);
  }
  for (; j < wdt; ++j) cfma(ar, ai, val[off + (int64_t)j * 64], x[col[off + (int64_t)j * 64]]);
  ar += br;
  ai += bi;
  if (slot >= n) return;
  const int row = perm[slot];
  if (bvec) {
    const double2 bb = bvec[row];
    y[row] = make_double2(bb.x - ar, bb.y - ai);
  } else {
    y[row] = make_double2(ar, ai);
  }
}

template <int G>
__global__ __launch_bounds__(kWG) void spmv_real_kernel(int64_t n, const int64_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t row = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G;
  const int l = threadIdx.x % G;
  double ar = 0, ai = 0;
  if (row < n) {
    const int64_t p1 = ptr[row + 1];
    for (int64_t p = ptr[row] + l; p < p1; p += G) {
      double a = val[p];
      double2 v = x[col[p]];
      ar = fma(a, v.x, ar);
      ai = fma(a, v.y, ai);
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    ar += __shfl_xor(ar, o, G);
    ai += __shfl_xor(ai, o, G);
  }
  if (row < n && l == 0) y[row] = make_double2(ar, ai);
}

// Both fine-grid products of the coarse solution cx, row by row (G lanes
// per row): q = Z cx (real Z) and t = r - (A Z) cx, A Z in split storage
// (real entries; bit 31 of the column marks an imaginary part).
template <int G>
__global__ __launch_bounds__(kWG) void coarse_update_kernel(int64_t n, const int64_t* __restrict__ zptr,
                                                            const int32_t* __restrict__ zcol,
                                                            const double* __restrict__ zval,
                                                            const int64_t* __restrict__ aptr,
                                                            const int32_t* __restrict__ acol,
                                                            const double* __restrict__ aval,
                                                            const double2* __restrict__ cx,
                                                            const double2* __restrict__ r, double2* __restrict__ q,
                                                            double2* __restrict__ t) {
  const int64_t row = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G;
  const int l = threadIdx.x % G;
  double qr = 0, qi = 0, ar = 0, ai = 0;
  if (row < n) {
    const int64_t z1 = zptr[row + 1], a1 = aptr[row + 1];
    for (int64_t p = zptr[row] + l; p < z1; p += G) {
      const double z = zval[p];
      const double2 v = cx[zcol[p]];
      qr = fma(z, v.x, qr);
      qi = fma(z, v.y, qi);
    }
    for (int64_t p = aptr[row] + l; p < a1; p += G) spmv_fma<double>(ar, ai, acol[p], aval[p], cx);
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    qr += __shfl_xor(qr, o, G);
    qi += __shfl_xor(qi, o, G);
    ar += __shfl_xor(ar, o, G);
    ai += __shfl_xor(ai, o, G);
  }
  if (row < n && l == 0) {
    q[row] = make_double2(qr, qi);
    const double2 rr = r[row];
    t[row] = make_double2(rr.x - ar, rr.y - ai);
  }
}

__global__ __launch_bounds__(kWG) void prolong_kernel(int64_t n, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ idx, const double* __restrict__ w,
                                                      const double2* __restrict__ xl, const double2* __restrict__ q,
                                                      double2* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (g >= n) return;
  double ar = 0, ai = 0;
  if (q) {
    ar = q[g].x;
    ai = q[g].y;
  }
  for (int64_t p = ptr[g]; p < ptr[g + 1]; ++p) {
    double2 v = xl[idx[p]];
    double c = w[p];
    ar = fma(c, v.x, ar);
    ai = fma(c, v.y, ai);
  }
  z[g] = make_double2(ar, ai);
}

// ---- Gram-Schmidt ----------------------------------------------------------

__global__ __launch_bounds__(kWG) void gs_dots_final_kernel(PtrSetC parts, int nblk, int ncol, PtrSet hs_, PtrSet haccs,
                                                            int accumulate) {
  __shared__ double2 sm[kWG];
  const double2* __restrict__ partial = reinterpret_cast<const double2*>(parts.p[blockIdx.y]);
  double2* __restrict__ h = reinterpret_cast<double2*>(hs_.p[blockIdx.y]);
  double2* __restrict__ hacc = reinterpret_cast<double2*>(haccs.p[blockIdx.y]);
  const int k = blockIdx.x, tid = threadIdx.x;
  double ar = 0, ai = 0;
  for (int b = tid; b < nblk; b += kWG) {
    double2 v = partial[(int64_t)b * ncol + k];
    ar += v.x;
    ai += v.y;
  }
  sm[tid] = make_double2(ar, ai);
  __syncthreads();
  for (int st = kWG / 2; st > 0; st >>= 1) {
    if (tid < st) {
      sm[tid].x += sm[tid + st].x;
      sm[tid].y += sm[tid + st].y;
    }
    __syncthreads();
  }
  if (tid == 0) {
    h[k] = sm[0];
    if (hacc) {
      if (accumulate)
        hacc[k] = make_double2(hacc[k].x + sm[0].x, hacc[k].y + sm[0].y);
      else
        hacc[k] = sm[0];
    }
  }
}

// One CGS2 pass over a 64-row tile of V (all ncol columns staged in LDS,
// padded to avoid bank conflicts):
//   kUpdate: w -= V h                (h: device, ncol entries)
//   kDots:   partial[blk*ncol + k] = sum_rows conj(V[i,k]) w[i]
//   kNorm:   partial[blk] = sum_rows |w[i]|^2   (real, stored in .x)
constexpr int kGsRows = 64;
constexpr int kGsMaxCols = 64;

template <bool kUpdate, bool kDots, bool kNorm>
__global__ __launch_bounds__(kWG) void gs_pass_kernel(int64_t n, PtrSetC Vs, int64_t ld, int ncol, PtrSetC hs_,
                                                      PtrSet ws, PtrSet parts) {
  // right-hand side blockIdx.y
  const double2* __restrict__ V = reinterpret_cast<const double2*>(Vs.p[blockIdx.y]);
  const double2* __restrict__ h = reinterpret_cast<const double2*>(hs_.p[blockIdx.y]);
  double2* __restrict__ w = reinterpret_cast<double2*>(ws.p[blockIdx.y]);
  double2* __restrict__ partial = reinterpret_cast<double2*>(parts.p[blockIdx.y]);
  // dynamic LDS: tile[ncol][kGsRows + 1], then h, the new w, and the
  // per-wave partial sums of the update and of the dots
  extern __shared__ double2 lds[];
  double2 (*tile)[kGsRows + 1] = reinterpret_cast<double2 (*)[kGsRows + 1]>(lds);
  double2* hs = lds + (size_t)ncol * (kGsRows + 1);
  double2* wn = hs + kGsMaxCols;
  double2* ured = wn + kGsRows;         // [4][kGsRows]
  double2* dred = ured + 4 * kGsRows;   // [4][kGsMaxCols]
  double* red = reinterpret_cast<double*>(dred + 4 * kGsMaxCols);
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (kUpdate && tid < ncol) hs[tid] = h[tid];
  double dr = 0, di = 0;  // dots: column `lane`, rows [16 wv, 16 wv + 16) of every tile
  double nrm = 0;         // norm: row `tid` of every tile
  const int64_t ntiles = (n + kGsRows - 1) / kGsRows;
  // Software pipeline: wave q holds columns q, q + 4, ... of the next tile
  // (and wave 0 the next tile's w) in registers; they are loaded right after
  // the current tile is staged, so the loads overlap its arithmetic.
  constexpr int kU = kGsMaxCols / 4;
  double2 a[kU];
  double2 wnext = make_double2(0.0, 0.0);
  auto load_next = [&](int64_t tb) {
    const int64_t i = tb * kGsRows + lane;
    const bool valid = tb < ntiles && i < n;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = wv + 4 * u;
      a[u] = (k < ncol && valid) ? V[(int64_t)k * ld + i] : make_double2(0.0, 0.0);
    }
    if (tid < kGsRows) wnext = valid ? w[i] : make_double2(0.0, 0.0);
  };
  load_next(blockIdx.x);
  for (int64_t tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
    const int64_t i = tb * kGsRows + lane;
    const bool valid = i < n;
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (wv + 4 * u < ncol) tile[wv + 4 * u][lane] = a[u];
    const double2 wcur = wnext;
    __syncthreads();
    load_next(tb + gridDim.x);
    if (kUpdate) {
      // wave q sums the columns k = q mod 4 of row `lane`
      double ur = 0, ui = 0;
      for (int k = wv; k < ncol; k += 4) cfma(ur, ui, tile[k][lane], hs[k]);
      ured[wv * kGsRows + lane] = make_double2(ur, ui);
      __syncthreads();
    }
    if (tid < kGsRows) {
      double2 wi = wcur;
      if (kUpdate) {
        for (int q = 0; q < 4; ++q) {
          wi.x -= ured[q * kGsRows + tid].x;
          wi.y -= ured[q * kGsRows + tid].y;
        }
        if (valid) w[i] = wi;
      }
      wn[tid] = wi;
      if (kNorm) nrm = fma(wi.x, wi.x, fma(wi.y, wi.y, nrm));
    }
    __syncthreads();
    if (kDots && lane < ncol) {
      for (int r = wv * 16; r < wv * 16 + 16; ++r) {
        const double2 v = tile[lane][r], x = wn[r];
        dr = fma(v.x, x.x, dr);
        dr = fma(v.y, x.y, dr);
        di = fma(v.x, x.y, di);
        di = fma(-v.y, x.x, di);
      }
    }
    __syncthreads();  // the next tile overwrites tile and wn
  }
  if (kDots) {
    if (lane < ncol) dred[wv * kGsMaxCols + lane] = make_double2(dr, di);
    __syncthreads();
    if (tid < ncol) {
      double ar = 0, ai = 0;
      for (int q = 0; q < 4; ++q) {
        ar += dred[q * kGsMaxCols + tid].x;
        ai += dred[q * kGsMaxCols + tid].y;
      }
      partial[(int64_t)blockIdx.x * ncol + tid] = make_double2(ar, ai);
    }
  }
  if (kNorm) {
    if (tid < kGsRows) red[tid] = nrm;
    __syncthreads();
    if (tid == 0) {
      double sum = 0;
      for (int r = 0; r < kGsRows; ++r) sum += red[r];
      partial[blockIdx.x] = make_double2(sum, 0.0);
    }
  }
}

// Delayed CGS2 (two passes over V per Arnoldi step instead of three): the
// last column v_j of V (ncol = j + 1 columns) was orthogonalised once when it
// was made; its second pass is folded into the next step.
// Pass A: partial dots V^H w (ncol entries) and V^H v_j (ncol more, the last
// being |v_j|^2) of every 64-row tile, staged through LDS so lane k of each
// wave sums column k over a quarter of the tile's rows;
// partial[blk * 2 ncol + k] and partial[blk * 2 ncol + ncol + k].
template <int kU>  // columns per wave (ncol <= 4 kU): fewer prefetch registers for short bases
__global__ __launch_bounds__(kWG) void gs_dots_kernel(int64_t n, PtrSetC Vs, int64_t ld, int ncol, PtrSet ws,
                                                      PtrSet parts) {
  const double2* __restrict__ V = reinterpret_cast<const double2*>(Vs.p[blockIdx.y]);
  const double2* __restrict__ w = reinterpret_cast<const double2*>(ws.p[blockIdx.y]);
  double2* __restrict__ partial = reinterpret_cast<double2*>(parts.p[blockIdx.y]);
  extern __shared__ double2 lds[];
  double2 (*tile)[kGsRows + 1] = reinterpret_cast<double2 (*)[kGsRows + 1]>(lds);
  double2* wn = lds + (size_t)ncol * (kGsRows + 1);
  double2* dred = wn + kGsRows;           // [4][kGsMaxCols]
  double2* ered = dred + 4 * kGsMaxCols;  // [4][kGsMaxCols]
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6), j = ncol - 1;
  double dr = 0, di = 0, er = 0, ei = 0;  // dots of column `lane` with w and with v_j
  const int64_t ntiles = (n + kGsRows - 1) / kGsRows;
  double2 a[kU];
  double2 wnext = make_double2(0.0, 0.0);
  auto load_next = [&](int64_t tb) {
    const int64_t i = tb * kGsRows + lane;
    const bool valid = tb < ntiles && i < n;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = wv + 4 * u;
      a[u] = (k < ncol && valid) ? V[(int64_t)k * ld + i] : make_double2(0.0, 0.0);
    }
    if (tid < kGsRows) wnext = valid ? w[i] : make_double2(0.0, 0.0);
  };
  load_next(blockIdx.x);
  for (int64_t tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (wv + 4 * u < ncol) tile[wv + 4 * u][lane] = a[u];
    if (tid < kGsRows) wn[tid] = wnext;
    __syncthreads();
    load_next(tb + gridDim.x);
    if (lane < ncol) {
      for (int r = wv * 16; r < wv * 16 + 16; ++r) {
        const double2 v = tile[lane][r], x = wn[r], y = tile[j][r];
        dr = fma(v.x, x.x, dr);
        dr = fma(v.y, x.y, dr);
        di = fma(v.x, x.y, di);
        di = fma(-v.y, x.x, di);
        er = fma(v.x, y.x, er);
        er = fma(v.y, y.y, er);
        ei = fma(v.x, y.y, ei);
        ei = fma(-v.y, y.x, ei);
      }
    }
    __syncthreads();  // the next tile overwrites tile and wn
  }
  if (lane < ncol) {
    dred[wv * kGsMaxCols + lane] = make_double2(dr, di);
    ered[wv * kGsMaxCols + lane] = make_double2(er, ei);
  }
  __syncthreads();
  if (tid < ncol) {
    double ar = 0, ai = 0, br = 0, bi = 0;
    for (int q = 0; q < 4; ++q) {
      ar += dred[q * kGsMaxCols + tid].x;
      ai += dred[q * kGsMaxCols + tid].y;
      br += ered[q * kGsMaxCols + tid].x;
      bi += ered[q * kGsMaxCols + tid].y;
    }
    partial[(int64_t)blockIdx.x * 2 * ncol + tid] = make_double2(ar, ai);
    partial[(int64_t)blockIdx.x * 2 * ncol + ncol + tid] = make_double2(br, bi);
  }
}

// Pass B of delayed CGS2 with one row per thread (no staging: every row
// needs all ncol columns, and the coefficients are shared by all rows):
// v_j <- (v_j - V_{<j} cv) * cv[j].x, w <- w - V_{<j} cw - v_j(old) cw[j],
// partial squared norms of the new w in partial[blockIdx.x].x.
__global__ __launch_bounds__(kWG) void gs_update_rows_kernel(int64_t n, PtrSetC Vs, PtrSet Vw, int64_t ld, int ncol,
                                                             PtrSetC cws, PtrSetC cvs, PtrSet ws, PtrSet parts) {
  const double2* __restrict__ V = reinterpret_cast<const double2*>(Vs.p[blockIdx.y]);
  double2* __restrict__ vw = reinterpret_cast<double2*>(Vw.p[blockIdx.y]);
  double2* __restrict__ w = reinterpret_cast<double2*>(ws.p[blockIdx.y]);
  double2* __restrict__ partial = reinterpret_cast<double2*>(parts.p[blockIdx.y]);
  __shared__ double2 cw[kGsMaxCols], cv[kGsMaxCols];
  __shared__ double red[kWG / 64];
  const int tid = threadIdx.x, j = ncol - 1;
  if (tid < ncol) {
    cw[tid] = reinterpret_cast<const double2*>(cws.p[blockIdx.y])[tid];
    cv[tid] = reinterpret_cast<const double2*>(cvs.p[blockIdx.y])[tid];
  }
  __syncthreads();
  double nrm = 0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + tid; i < n; i += (int64_t)gridDim.x * kWG) {
    double ur = 0, ui = 0, vr = 0, vi = 0;
    int k = 0;
    for (; k + 8 <= j; k += 8) {
      double2 a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = V[(int64_t)(k + u) * ld + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        cfma(ur, ui, a[u], cw[k + u]);
        cfma(vr, vi, a[u], cv[k + u]);
      }
    }
    for (; k < j; ++k) {
      const double2 a = V[(int64_t)k * ld + i];
      cfma(ur, ui, a, cw[k]);
      cfma(vr, vi, a, cv[k]);
    }
    const double2 vo = V[(int64_t)j * ld + i];
    double2 wi = w[i];
    const double2 dj = cw[j];
    const double ia = cv[j].x;
    wi.x -= ur + (vo.x * dj.x - vo.y * dj.y);
    wi.y -= ui + (vo.x * dj.y + vo.y * dj.x);
    w[i] = wi;
    vw[(int64_t)j * ld + i] = make_double2((vo.x - vr) * ia, (vo.y - vi) * ia);
    nrm = fma(wi.x, wi.x, fma(wi.y, wi.y, nrm));
  }
  for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = nrm;
  __syncthreads();
  if (tid == 0) {
    double sum = 0;
    for (int q = 0; q < kWG / 64; ++q) sum += red[q];
    partial[blockIdx.x] = make_double2(sum, 0.0);
  }
}

// Coefficients of pass B from the reduced dots of pass A (dots[0, ncol): t =
// V^H w, dots[ncol, 2 ncol): g = V^H v_j): s = g_{<j}, a = sqrt(g_j - |s|^2),
// h_j = (t_j - s^H t_{<j}) / a; cw_k = t_k - s_k h_j / a (k < j),
// cw_j = h_j / a; cv_k = s_k, cv_j = 1 / a.  out (host-bound) gets
// [t_0 .. t_{j-1}, h_j, (slot for |w|), s_0 .. s_{j-1}, a].  ncol <= 64.
__global__ __launch_bounds__(64) void dcgs2_coef_kernel(PtrSetC dots_, int ncol, PtrSet cws, PtrSet cvs,
                                                         PtrSet outs) {
  const double2* __restrict__ t = reinterpret_cast<const double2*>(dots_.p[blockIdx.y]);
  const double2* __restrict__ g = t + ncol;
  double2* __restrict__ cw = reinterpret_cast<double2*>(cws.p[blockIdx.y]);
  double2* __restrict__ cv = reinterpret_cast<double2*>(cvs.p[blockIdx.y]);
  double2* __restrict__ out = reinterpret_cast<double2*>(outs.p[blockIdx.y]);
  const int j = ncol - 1, k = threadIdx.x;  // one wave, lane k < j owns column k
  const double2 gk = k < j ? g[k] : make_double2(0.0, 0.0);
  const double2 tk = k < j ? t[k] : make_double2(0.0, 0.0);
  double ss = gk.x * gk.x + gk.y * gk.y;
  double str = gk.x * tk.x + gk.y * tk.y;  // conj(s_k) t_k
  double sti = gk.x * tk.y - gk.y * tk.x;
  for (int o = 32; o > 0; o >>= 1) {
    ss += __shfl_xor(ss, o, 64);
    str += __shfl_xor(str, o, 64);
    sti += __shfl_xor(sti, o, 64);
  }
  const double2 gj = g[j], tj = t[j];
  double a2 = gj.x - ss;
  if (!(a2 > 0)) a2 = gj.x;  // no usable correction: keep v_j as it is
  const double a = sqrt(a2), ia = 1.0 / a;
  const double hr = (tj.x - str) * ia, hi = (tj.y - sti) * ia;
  if (k < j) {
    // s_k h_j / a
    const double pr = (gk.x * hr - gk.y * hi) * ia, pi = (gk.x * hi + gk.y * hr) * ia;
    cw[k] = make_double2(tk.x - pr, tk.y - pi);
    cv[k] = gk;
    out[k] = tk;
    out[j + 2 + k] = gk;
  } else if (k == j) {
    cw[j] = make_double2(hr * ia, hi * ia);
    cv[j] = make_double2(ia, 0.0);
    out[j] = make_double2(hr, hi);
    out[2 * j + 2] = make_double2(a, 0.0);
  }
}

__global__ __launch_bounds__(kWG) void norm_final2_kernel(PtrSetC parts, int nblk, PtrSet outs) {
  __shared__ double sm[kWG];
  const double2* __restrict__ partial = reinterpret_cast<const double2*>(parts.p[blockIdx.y]);
  double2* __restrict__ out = reinterpret_cast<double2*>(outs.p[blockIdx.y]);
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += kWG) s += partial[b].x;
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = kWG / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = make_double2(sqrt(sm[0]), 0.0);
}

__global__ __launch_bounds__(kWG) void norm_partial_kernel(int64_t n, const double2* __restrict__ w,
                                                           double* __restrict__ partial) {
  __shared__ double sm[kWG];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
    double2 v = w[i];
    s = fma(v.x, v.x, s);
    s = fma(v.y, v.y, s);
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = kWG / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kWG) void norm_final_kernel(const double* __restrict__ partial, int nblk,
                                                         double2* __restrict__ out) {
  __shared__ double sm[kWG];
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += kWG) s += partial[b];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = kWG / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = make_double2(sqrt(sm[0]), 0.0);
}

__global__ __launch_bounds__(kWG) void scale_by_inv_kernel(int64_t n, PtrSetC ws, PtrSetC nrms, PtrSet vs) {
  const double2* __restrict__ w = reinterpret_cast<const double2*>(ws.p[blockIdx.y]);
  const double2* __restrict__ nrm = reinterpret_cast<const double2*>(nrms.p[blockIdx.y]);
  double2* __restrict__ v = reinterpret_cast<double2*>(vs.p[blockIdx.y]);
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const double d = nrm[0].x;
  const double inv = d != 0.0 ? 1.0 / d : 0.0;
  const double2 a = w[i];
  v[i] = make_double2(a.x * inv, a.y * inv);
}

__global__ __launch_bounds__(kWG) void scale_kernel(int64_t n, const double2* __restrict__ w, double alpha,
                                                    double2* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const double2 a = w[i];
  v[i] = make_double2(a.x * alpha, a.y * alpha);
}

__global__ __launch_bounds__(kWG) void gemv_acc_kernel(int64_t n, const double2* __restrict__ Z, int64_t ld, int k,
                                                       const double2* __restrict__ y, double2* __restrict__ x) {
  __shared__ double2 ys[1024];
  for (int j = threadIdx.x; j < k; j += kWG) ys[j] = y[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  double ar = 0, ai = 0;
  for (int j = 0; j < k; ++j) cfma(ar, ai, Z[(int64_t)j * ld + i], ys[j]);
  double2 xi = x[i];
  x[i] = make_double2(xi.x + ar, xi.y + ai);
}

__global__ __launch_bounds__(kWG) void fill_zero_kernel(int64_t n, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ __launch_bounds__(kWG) void copy_kernel(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) b[i] = a[i];
}

inline unsigned blocks_for(int64_t n, int per = kWG) { return (unsigned)((n + per - 1) / per); }
// Same, rounded up to a multiple of 8 (grids of kernels that use xcd_block).
inline unsigned blocks8_for(int64_t n) { return (blocks_for(n) + 7) / 8 * 8; }

__global__ __launch_bounds__(kWG) void copy_tiles_kernel(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                         const int64_t* __restrict__ from,
                                                         const int64_t* __restrict__ to,
                                                         const int64_t* __restrict__ words, int64_t ntiles) {
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t* a = src + from[t];
    uint64_t* d = dst + to[t];
    const int64_t n = words[t];
    for (int64_t i = threadIdx.x; i < n; i += kWG) d[i] = a[i];
  }
}

}  // namespace

int waves_per_tile(int ncols) { return ncols <= 96 ? 1 : (ncols <= 384 ? 2 : 4); }

void copy_tiles(const void* src, void* dst, const int64_t* from, const int64_t* to, const int64_t* words,
                int64_t ntiles, hipStream_t s) {
  if (ntiles <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ntiles, 1 << 20);
  copy_tiles_kernel<<<grid, kWG, 0, s>>>(reinterpret_cast<const uint64_t*>(src), reinterpret_cast<uint64_t*>(dst),
                                         from, to, words, ntiles);
}

// Workgroups of a level kernel resident on the current device at once
// (cached per kernel, LDS size and device).
static int resident_grid(const void* fn, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1 << 30;
  const auto key = std::make_tuple(fn, lds, dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int ncu = 0, per = 0;
  int g = 1 << 30;  // unknown: one workgroup per task
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kWG, lds) == hipSuccess && per > 0 && ncu > 0)
    g = per * ncu;
  cache.emplace(key, g);
  return g;
}

template <class K, class... A>
static void level_go(K kernel, int64_t ntasks, size_t lds, hipStream_t s, A... args) {
  const int64_t g = std::min<int64_t>(ntasks, resident_grid(reinterpret_cast<const void*>(kernel), lds));
  kernel<<<(unsigned)g, kWG, lds, s>>>(args...);
}

void fwd_level(const Batch& b, int64_t task0, int64_t ntasks, const double* bin, int chunk, bool coarse,
               hipStream_t s) {
  if (ntasks <= 0) return;
  const Task* k = b.kf + task0;
  const int nt = (int)ntasks;
  const double2* in = reinterpret_cast<const double2*>(bin);
  const size_t lds = sizeof(double2) * (size_t)chunk;
  if (coarse)
    level_go(fwd_level_kernel<double2, 1>, ntasks, lds, s, k, nt, b, in, chunk);
  else if (b.c64)
    level_go(fwd_level_kernel<float2, 0>, ntasks, lds, s, k, nt, b, in, chunk);
  else
    level_go(fwd_level_kernel<double2, 0>, ntasks, lds, s, k, nt, b, in, chunk);
}

void fwd_sn(const Batch& b, int64_t job0, int64_t njobs, const double* bin, hipStream_t s) {
  if (njobs <= 0) return;
  const SnJob* j = b.snj + job0;
  const int nj = (int)njobs;
  const double2* in = reinterpret_cast<const double2*>(bin);
  const int64_t wgs = (njobs + 3) / 4;
  if (b.c64)
    level_go(fwd_sn_kernel<float2>, wgs, 0, s, j, nj, b, in);
  else
    level_go(fwd_sn_kernel<double2>, wgs, 0, s, j, nj, b, in);
}

void bwd_level(const Batch& b, int64_t task0, int64_t ntasks, int chunk, bool coarse, hipStream_t s) {
  if (ntasks <= 0) return;
  const Task* k = b.kb + task0;
  const int nt = (int)ntasks;
  const size_t lds = sizeof(double2) * (size_t)chunk;
  if (coarse)
    level_go(bwd_level_kernel<double2, 1>, ntasks, lds, s, k, nt, b, chunk);
  else if (b.c64)
    level_go(bwd_level_kernel<float2, 0>, ntasks, lds, s, k, nt, b, chunk);
  else
    level_go(bwd_level_kernel<double2, 0>, ntasks, lds, s, k, nt, b, chunk);
}

int coop_grid() {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_solve_coop_kernel, kWG, 0) != hipSuccess) return 0;
  return per * ncu;
}

hipError_t batch_solve_coop(const Batch& b, const double* bin, const LevelRanges& lv, int grid, hipStream_t s) {
  Batch bb = b;
  const double2* in = reinterpret_cast<const double2*>(bin);
  LevelRanges l = lv;
  void* args[] = {&bb, &in, &l};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batch_solve_coop_kernel), dim3(grid), dim3(kWG),
                                    args, 0, s);
}

template <int G, int U, bool R, class VT>
void spmv_go(int64_t n, const int64_t* ptr, const int32_t* col, const VT* v2, const int64_t* xr, int64_t xrows,
             const double2* x2, const double2* b2, double2* y2, hipStream_t s) {
  // with R, 8 x the block count of the longest XCD range, else one block per kWG / G rows
  const unsigned grid = R ? 8 * blocks_for(xrows * G) : blocks_for(n * G);
  spmv_kernel<G, U, R, VT><<<grid, kWG, 0, s>>>(n, ptr, col, v2, xr, x2, b2, y2);
}

template <bool R, class VT>
void spmv_launch(int64_t n, const int64_t* ptr, const int32_t* col, const VT* v2, const int64_t* xr,
                 int64_t xrows, const double2* x2, const double2* b2, double2* y2, int cfg, hipStream_t s) {
  switch (cfg) {
    case spmv_cfg(4, 4): spmv_go<4, 4, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(4, 8): spmv_go<4, 8, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(8, 1): spmv_go<8, 1, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(8, 2): spmv_go<8, 2, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(8, 4): spmv_go<8, 4, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(16, 1): spmv_go<16, 1, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(16, 2): spmv_go<16, 2, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    case spmv_cfg(32, 1): spmv_go<32, 1, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
    default: spmv_go<4, 1, R, VT>(n, ptr, col, v2, xr, xrows, x2, b2, y2, s); break;
  }
}

int64_t xcd_ranges(int64_t n, const int64_t* ptr, int64_t xr[9]) {
  xr[0] = 0;
  int64_t r = 0, longest = 0;
  for (int k = 1; k < 8; ++k) {
    const int64_t target = (ptr[n] * k) / 8;
    while (r < n && ptr[r] < target) ++r;
    xr[k] = r;
  }
  xr[8] = n;
  for (int k = 0; k < 8; ++k) longest = std::max<int64_t>(longest, xr[k + 1] - xr[k]);
  return longest;
}

void spmv(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const int64_t* xr, int64_t xrows,
          const double* x, const double* b, double* y, int cfg, hipStream_t s) {
  if (n <= 0) return;
  auto v2 = reinterpret_cast<const double2*>(val);
  auto x2 = reinterpret_cast<const double2*>(x);
  auto b2 = reinterpret_cast<const double2*>(b);
  auto y2 = reinterpret_cast<double2*>(y);
  if (xr)
    spmv_launch<true, double2>(n, ptr, col, v2, xr, xrows, x2, b2, y2, cfg, s);
  else
    spmv_launch<false, double2>(n, ptr, col, v2, nullptr, 0, x2, b2, y2, cfg, s);
}

void spmv_split(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const double* x,
                const double* b, double* y, int cfg, hipStream_t s) {
  if (n <= 0) return;
  spmv_launch<false, double>(n, ptr, col, val, nullptr, 0, reinterpret_cast<const double2*>(x),
                             reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(y), cfg, s);
}

void sell_spmv(int64_t n, int64_t nslices, const int64_t* soff, const int32_t* swidth, const int32_t* perm,
               const int32_t* col, const double* val, const double* x, const double* b, double* y, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)((nslices + 3) / 4);
  sell_kernel<<<(nb + 7) / 8 * 8, kWG, 0, s>>>(
      n, nslices, soff, swidth, perm, col, reinterpret_cast<const double2*>(val), reinterpret_cast<const double2*>(x),
      reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(y));
}

void spmv_real(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const double* x, double* y,
               int G, hipStream_t s) {
  if (n <= 0) return;
  auto x2 = reinterpret_cast<const double2*>(x);
  auto y2 = reinterpret_cast<double2*>(y);
  switch (G) {
    case 8: spmv_real_kernel<8><<<blocks_for(n * 8), kWG, 0, s>>>(n, ptr, col, val, x2, y2); break;
    case 16: spmv_real_kernel<16><<<blocks_for(n * 16), kWG, 0, s>>>(n, ptr, col, val, x2, y2); break;
    case 32: spmv_real_kernel<32><<<blocks_for(n * 32), kWG, 0, s>>>(n, ptr, col, val, x2, y2); break;
    case 64: spmv_real_kernel<64><<<blocks_for(n * 64), kWG, 0, s>>>(n, ptr, col, val, x2, y2); break;
    default: spmv_real_kernel<4><<<blocks_for(n * 4), kWG, 0, s>>>(n, ptr, col, val, x2, y2); break;
  }
}

void coarse_update(int64_t n, const int64_t* zptr, const int32_t* zcol, const double* zval, const int64_t* aptr,
                   const int32_t* acol, const double* aval, const double* cx, const double* r, double* q, double* t,
                   int G, hipStream_t s) {
  if (n <= 0) return;
  auto c2 = reinterpret_cast<const double2*>(cx);
  auto r2 = reinterpret_cast<const double2*>(r);
  auto q2 = reinterpret_cast<double2*>(q);
  auto t2 = reinterpret_cast<double2*>(t);
  if (G == 8)
    coarse_update_kernel<8><<<blocks_for(n * 8), kWG, 0, s>>>(n, zptr, zcol, zval, aptr, acol, aval, c2, r2, q2, t2);
  else if (G == 2)
    coarse_update_kernel<2><<<blocks_for(n * 2), kWG, 0, s>>>(n, zptr, zcol, zval, aptr, acol, aval, c2, r2, q2, t2);
  else if (G == 1)
    coarse_update_kernel<1><<<blocks_for(n), kWG, 0, s>>>(n, zptr, zcol, zval, aptr, acol, aval, c2, r2, q2, t2);
  else
    coarse_update_kernel<4><<<blocks_for(n * 4), kWG, 0, s>>>(n, zptr, zcol, zval, aptr, acol, aval, c2, r2, q2, t2);
}

void prolong(int64_t n, const int64_t* ptr, const int32_t* idx, const double* w, const double* xl, const double* q,
             double* z, hipStream_t s) {
  if (n <= 0) return;
  prolong_kernel<<<blocks_for(n), kWG, 0, s>>>(n, ptr, idx, w, reinterpret_cast<const double2*>(xl),
                                               reinterpret_cast<const double2*>(q), reinterpret_cast<double2*>(z));
}

int gs_blocks(int64_t n) {
  int64_t b = (n + kWG * 4 - 1) / (kWG * 4);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

void gs_final(int nr, const PtrSetC& partial, int nblk, int ncol, const PtrSet& h, const PtrSet& hacc,
              int accumulate, hipStream_t s) {
  gs_dots_final_kernel<<<dim3((unsigned)ncol, (unsigned)nr), kWG, 0, s>>>(partial, nblk, ncol, h, hacc, accumulate);
}

int gs_tiles(int64_t n) {
  const int64_t t = (n + kGsRows - 1) / kGsRows;
  return (int)(t < 2048 ? t : 2048);  // workgroups; each loops over 64-row tiles
}

void gs_pass(int mode, int nr, int64_t n, const PtrSetC& V, int64_t ld, int ncol, const PtrSetC& h, const PtrSet& w,
             const PtrSet& partial, hipStream_t s) {
  const dim3 grid((unsigned)gs_tiles(n), (unsigned)nr);
  const size_t lds = sizeof(double2) * ((size_t)ncol * (kGsRows + 1) + kGsMaxCols + kGsRows + 4 * kGsRows +
                                        4 * kGsMaxCols) +
                     sizeof(double) * kGsRows;
  if (mode == 0)
    gs_pass_kernel<false, true, false><<<grid, kWG, lds, s>>>(n, V, ld, ncol, h, w, partial);
  else if (mode == 1)
    gs_pass_kernel<true, true, false><<<grid, kWG, lds, s>>>(n, V, ld, ncol, h, w, partial);
  else
    gs_pass_kernel<true, false, true><<<grid, kWG, lds, s>>>(n, V, ld, ncol, h, w, partial);
}

void gs_dual(bool update, int nr, int64_t n, const PtrSetC& V, const PtrSet& Vw, int64_t ld, int ncol,
             const PtrSetC& cw, const PtrSetC& cv, const PtrSet& w, const PtrSet& partial, hipStream_t s) {
  const dim3 grid((unsigned)gs_tiles(n), (unsigned)nr);
  const size_t lds = sizeof(double2) * ((size_t)ncol * (kGsRows + 1) + kGsRows + 8 * kGsMaxCols);
  if (update)
    gs_update_rows_kernel<<<grid, kWG, 0, s>>>(n, V, Vw, ld, ncol, cw, cv, w, partial);
  else if (ncol <= 16)
    gs_dots_kernel<4><<<grid, kWG, lds, s>>>(n, V, ld, ncol, w, partial);
  else if (ncol <= 32)
    gs_dots_kernel<8><<<grid, kWG, lds, s>>>(n, V, ld, ncol, w, partial);
  else
    gs_dots_kernel<kGsMaxCols / 4><<<grid, kWG, lds, s>>>(n, V, ld, ncol, w, partial);
}
void dcgs2_coef(int nr, const PtrSetC& dots, int ncol, const PtrSet& cw, const PtrSet& cv, const PtrSet& out,
                hipStream_t s) {
  dcgs2_coef_kernel<<<dim3(1, (unsigned)nr), 64, 0, s>>>(dots, ncol, cw, cv, out);
}
void norm_final(int nr, const PtrSetC& partial, int nblk, const PtrSet& out, hipStream_t s) {
  norm_final2_kernel<<<dim3(1, (unsigned)nr), kWG, 0, s>>>(partial, nblk, out);
}

void norm2(int64_t n, const double* w, double* partial, int nblk, double* out, hipStream_t s) {
  norm_partial_kernel<<<(unsigned)nblk, kWG, 0, s>>>(n, reinterpret_cast<const double2*>(w), partial);
  norm_final_kernel<<<1, kWG, 0, s>>>(partial, nblk, reinterpret_cast<double2*>(out));
}

void scale_by_inv_set(int nr, int64_t n, const PtrSetC& w, const PtrSetC& nrm, const PtrSet& v, hipStream_t s) {
  if (n <= 0) return;
  scale_by_inv_kernel<<<dim3(blocks_for(n), (unsigned)nr), kWG, 0, s>>>(n, w, nrm, v);
}

void scale(int64_t n, const double* w, double alpha, double* v, hipStream_t s) {
  if (n <= 0) return;
  scale_kernel<<<blocks_for(n), kWG, 0, s>>>(n, reinterpret_cast<const double2*>(w), alpha,
                                             reinterpret_cast<double2*>(v));
}

void gemv_acc(int64_t n, const double* Z, int64_t ld, int k, const double* y, double* x, hipStream_t s) {
  if (n <= 0 || k <= 0) return;
  gemv_acc_kernel<<<blocks_for(n), kWG, 0, s>>>(n, reinterpret_cast<const double2*>(Z), ld, k,
                                                reinterpret_cast<const double2*>(y), reinterpret_cast<double2*>(x));
}

// ---- fixed scratch of the allocation-free entry point ----------------------
//
// One file-scope array per device (each GPU the library runs on holds its own
// copy until the process ends).  In host code `scratch` names a host-side
// stand-in, not the device array: its device address is looked up once per
// device with hipGetSymbolAddress and only that address is ever handed to
// kernels or copies.

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

void fill_zero(int64_t n, double* p, hipStream_t s) {
  if (n <= 0) return;
  fill_zero_kernel<<<blocks_for(n), kWG, 0, s>>>(n, p);
}

void copy(int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  copy_kernel<<<blocks_for(n), kWG, 0, s>>>(n, src, dst);
}

}  // namespace dev
}  // namespace helm
