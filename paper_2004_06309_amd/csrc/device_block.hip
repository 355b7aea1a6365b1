// Multi-right-hand-side kernels (pseudo-block GMRES: S Krylov spaces advanced
// together, the operator and the preconditioner applied to all S vectors in
// one pass over A and over the factor panels).
//
// Block vectors are interleaved: entry (i, r) of an n x S block sits at
// i * S + r, so every gather of a row fetches S contiguous complex values.
// The level kernels stream each panel tile once for all S columns: one
// wavefront per tile, a lane per tile row holding S accumulators.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"

namespace helm {
namespace dev {

namespace {

constexpr int kWG = 256;
constexpr int kBlkLds = 1024;  // complex entries of the staged input block

__device__ __forceinline__ void cfma(double& ar, double& ai, double2 a, double2 v) {
  ar = fma(a.x, v.x, ar);
  ar = fma(-a.y, v.y, ar);
  ai = fma(a.x, v.y, ai);
  ai = fma(a.y, v.x, ai);
}
__device__ __forceinline__ double2 widen(double2 a) { return a; }
__device__ __forceinline__ double2 widen(float2 a) { return make_double2((double)a.x, (double)a.y); }

template <class PT, int S, int kCoarse>
__global__ __launch_bounds__(64) void fwd_block_kernel(const Tile* __restrict__ tiles, Batch b,
                                                       const double2* __restrict__ bin, double2* __restrict__ yb,
                                                       double2* __restrict__ ubb) {
  __shared__ double2 vin[kBlkLds];
  constexpr int CB = kBlkLds / S;
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  const int sn = t.sn, c0 = b.sn_c0[sn], w = b.sn_w[sn], frow0 = b.sn_frow0[sn];
  const PT* __restrict__ P = reinterpret_cast<const PT*>(b.pf) + t.off + lane;
  double ar[S], ai[S];
#pragma unroll
  for (int r = 0; r < S; ++r) ar[r] = ai[r] = 0;
  for (int cb = 0; cb < t.ncols; cb += CB) {
    const int cn = min(CB, t.ncols - cb);
    for (int e = lane; e < cn * S; e += 64) {
      const int k = e / S, r = e % S, kk = cb + k;
      double2 v = bin[(int64_t)b.bidx[c0 + kk] * S + r];
      const int fr = frow0 + kk;
      for (int q = b.fcon_ptr[fr]; q < b.fcon_ptr[fr + 1]; ++q) {
        const double2 u = ubb[(int64_t)b.fcon_idx[q] * S + r];
        v.x -= u.x;
        v.y -= u.y;
      }
      vin[e] = v;
    }
    __syncthreads();
    if (lane < t.nrows) {
      const PT* p = P + (int64_t)cb * t.nrows;
      int k = 0;
      for (; k + 2 <= cn; k += 2) {
        const double2 a0 = widen(p[(int64_t)k * t.nrows]);
        const double2 a1 = widen(p[(int64_t)(k + 1) * t.nrows]);
#pragma unroll
        for (int r = 0; r < S; ++r) {
          cfma(ar[r], ai[r], a0, vin[k * S + r]);
          cfma(ar[r], ai[r], a1, vin[(k + 1) * S + r]);
        }
      }
      for (; k < cn; ++k) {
        const double2 a0 = widen(p[(int64_t)k * t.nrows]);
#pragma unroll
        for (int r = 0; r < S; ++r) cfma(ar[r], ai[r], a0, vin[k * S + r]);
      }
    }
    __syncthreads();
  }
  if (lane < t.nrows) {
    const int row = t.row0 + lane;
    if (row < w) {
#pragma unroll
      for (int r = 0; r < S; ++r) yb[(int64_t)(c0 + row) * S + r] = make_double2(ar[r], ai[r]);
    } else {
      const int fr = frow0 + row;
      for (int q = b.fcon_ptr[fr]; q < b.fcon_ptr[fr + 1]; ++q) {
        const int64_t src = (int64_t)b.fcon_idx[q] * S;
#pragma unroll
        for (int r = 0; r < S; ++r) {
          const double2 u = ubb[src + r];
          ar[r] += u.x;
          ai[r] += u.y;
        }
      }
      const int64_t dst = (int64_t)(b.sn_uoff[sn] + row - w) * S;
#pragma unroll
      for (int r = 0; r < S; ++r) ubb[dst + r] = make_double2(ar[r], ai[r]);
    }
  }
}

template <class PT, int S, int kCoarse>
__global__ __launch_bounds__(64) void bwd_block_kernel(const Tile* __restrict__ tiles, Batch b,
                                                       const double2* __restrict__ yb, double2* __restrict__ xb) {
  __shared__ double2 vin[kBlkLds];
  constexpr int CB = kBlkLds / S;
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  const int sn = t.sn, c0 = b.sn_c0[sn], w = b.sn_w[sn];
  const int64_t roff = b.sn_roff[sn];
  const PT* __restrict__ P = reinterpret_cast<const PT*>(b.pb) + t.off + lane;
  double ar[S], ai[S];
#pragma unroll
  for (int r = 0; r < S; ++r) ar[r] = ai[r] = 0;
  for (int cb = 0; cb < t.ncols; cb += CB) {
    const int cn = min(CB, t.ncols - cb);
    for (int e = lane; e < cn * S; e += 64) {
      const int k = e / S, r = e % S, c = t.col0 + cb + k;
      vin[e] = c < w ? yb[(int64_t)(c0 + c) * S + r] : xb[(int64_t)b.rows[roff + (c - w)] * S + r];
    }
    __syncthreads();
    if (lane < t.nrows) {
      const PT* p = P + (int64_t)cb * t.nrows;
      int k = 0;
      for (; k + 2 <= cn; k += 2) {
        const double2 a0 = widen(p[(int64_t)k * t.nrows]);
        const double2 a1 = widen(p[(int64_t)(k + 1) * t.nrows]);
#pragma unroll
        for (int r = 0; r < S; ++r) {
          cfma(ar[r], ai[r], a0, vin[k * S + r]);
          cfma(ar[r], ai[r], a1, vin[(k + 1) * S + r]);
        }
      }
      for (; k < cn; ++k) {
        const double2 a0 = widen(p[(int64_t)k * t.nrows]);
#pragma unroll
        for (int r = 0; r < S; ++r) cfma(ar[r], ai[r], a0, vin[k * S + r]);
      }
    }
    __syncthreads();
  }
  if (lane < t.nrows) {
    const int64_t dst = (int64_t)(c0 + t.row0 + lane) * S;
#pragma unroll
    for (int r = 0; r < S; ++r) xb[dst + r] = make_double2(ar[r], ai[r]);
  }
}

// ---- MFMA form for 16 right-hand sides --------------------------------------
// A tile (<= 64 rows x ncols) times the 16-column input block is a small
// dense contraction: it runs on v_mfma_{f64,f32}_16x16x4 as four 16-row
// blocks, the complex product split into four real MFMAs
//   Dre += Are Bre - Aim Bim,  Dim += Are Bim + Aim Bre.
// Operand layout of the 16x16x4 MFMA: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register j of lane l is D[row][l % 16] with
// row = 4 (l / 16) + j for FP32 and row = 4 j + l / 16 for FP64 (both
// checked on the device).
// Complex128 panels use FP64 MFMA; complex64 panels use FP32 MFMA with the
// input block rounded to FP32 (FP32 accumulation; the outer flexible GMRES
// stays in FP64).
typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mf;
template <>
struct Mf<double> {
  using V4 = dv4;
  using C2 = double2;
  static __device__ __forceinline__ V4 mma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int j) { return 4 * j + lk; }
};
template <>
struct Mf<float> {
  using V4 = fv4;
  using C2 = float2;
  static __device__ __forceinline__ V4 mma(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int j) { return 4 * lk + j; }
};

// ---- staged MFMA form ------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kWG) void gather_fwd_kernel(const int32_t* __restrict__ sns, Batch b,
                                                         const double2* __restrict__ bin,
                                                         const double2* __restrict__ ubb,
                                                         typename Mf<T>::C2* __restrict__ G) {
  using C2 = typename Mf<T>::C2;
  const int sn = sns[blockIdx.x];
  const int c0 = b.sn_c0[sn], w = b.sn_w[sn], frow0 = b.sn_frow0[sn];
  C2* g = G + b.goff_f[sn] * 16;
  // workgroup blockIdx.y of gridDim.y takes every gridDim.y-th 256 entries;
  // an entry's input index and child-update pair are loaded together, then
  // the input and the (at most two) updates; a row with more children walks
  // its list
  for (int e = blockIdx.y * kWG + threadIdx.x; e < w * 16; e += gridDim.y * kWG) {
    const int k = e >> 4, r = e & 15;
    const int fr = frow0 + k;
    const int bi = b.bidx[c0 + k];
    const int2 c2 = b.fcon2[fr];
    double2 v = bin[(int64_t)bi * 16 + r];
    const double2 u0 = *(c2.x >= 0 ? ubb + (int64_t)c2.x * 16 + r : bin + r);
    const double2 u1 = *(c2.y >= 0 ? ubb + (int64_t)c2.y * 16 + r : bin + r);
    if (c2.x >= 0) {
      v.x -= u0.x;
      v.y -= u0.y;
      if (c2.y >= 0) {
        v.x -= u1.x;
        v.y -= u1.y;
      }
    } else if (c2.x < -1) {
      for (int q = -2 - c2.x; q < b.fcon_ptr[fr + 1]; ++q) {
        const double2 u = ubb[(int64_t)b.fcon_idx[q] * 16 + r];
        v.x -= u.x;
        v.y -= u.y;
      }
    }
    g[e] = C2{(T)v.x, (T)v.y};
  }
}

// Panel loads are streamed once per sweep: non-temporal, so they do not
// evict the staged input blocks and vectors from the caches.
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

// Streams the k-steps k0 = ks0, ks0 + kst, ... < cn (a k-step is four
// columns) of a panel tile P (nr rows, column-major) against the input block
// Bk (16 right-hand sides per column) into the accumulators of the row
// blocks rb < nrb.  The loads of the next k-step are issued before the MFMAs
// of the current one, into the other of two register sets, so no loaded
// register is copied (a copy would make the wave wait for the load just
// issued).  Every load is issued unconditionally, at a clamped address: rows
// past nr read row nr - 1 (rows whose results are never stored), columns
// past cn read column cn - 1 and meet a zero B entry, so the waits the
// compiler places count exactly the other set's loads.
template <class T>
__device__ __forceinline__ void mfma_stream(const typename Mf<T>::C2* __restrict__ P, int nr, int cn,
                                            const typename Mf<T>::C2* __restrict__ Bk, int ks0, int kst,
                                            typename Mf<T>::V4* dre, typename Mf<T>::V4* dim) {
  using C2 = typename Mf<T>::C2;
  if (ks0 >= cn) return;  // uniform: the wave has no k-step
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int nrb = (nr + 15) >> 4;
  int roff[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) roff[rb] = min(16 * rb + lr, nr - 1);
  auto load = [&](int k0, C2& bv, C2 (&a)[4]) {
    const int k = min(k0 + lk, cn - 1);
    bv = Bk[k * 16 + lr];
    const C2* pc = P + (int64_t)k * nr;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) a[rb] = ldp(pc + roff[rb]);
  };
  auto step = [&](int k0, const C2& b, const C2 (&a)[4]) {
    const C2 bv = k0 + lk < cn ? b : C2{0, 0};
    const decltype(bv.y) nby = -bv.y;  // a.y (-b.y) is -(a.y b.y) exactly
    // row blocks past the tile are skipped (uniform branches: nrb is the
    // same on every lane)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      if (rb < nrb) {
        dre[rb] = Mf<T>::mma(a[rb].x, bv.x, dre[rb]);
        dim[rb] = Mf<T>::mma(a[rb].x, bv.y, dim[rb]);
        dre[rb] = Mf<T>::mma(a[rb].y, nby, dre[rb]);
        dim[rb] = Mf<T>::mma(a[rb].y, bv.x, dim[rb]);
      }
    }
  };
  C2 b0, a0[4], b1, a1[4];
  load(ks0, b0, a0);
  // the k-steps go in pairs (an odd count loads a step past cn and skips
  // its MFMAs); the scheduling barriers keep each k-step's loads ahead of
  // the MFMAs of the step before it
  for (int k0 = ks0; k0 < cn; k0 += 2 * kst) {
    load(k0 + kst, b1, a1);
    __builtin_amdgcn_sched_barrier(0);
    step(k0, b0, a0);
    __builtin_amdgcn_sched_barrier(0);
    load(k0 + 2 * kst, b0, a0);
    __builtin_amdgcn_sched_barrier(0);
    if (k0 + kst < cn) step(k0 + kst, b1, a1);  // uniform
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Children's updates routed to front row fr, for right-hand side r: the
// first two entries of the row's list come as one index pair (fcon2), so
// the values are one load away; a row with more than two walks its list.
// uu holds the pair's values, loaded beforehand (a missing entry is not
// used); the sum is taken in list order.
__device__ __forceinline__ void add_children(const Batch& b, int fr, int2 c2, const double2* uu, const double2* ubb,
                                             int r, double& ar, double& ai) {
  if (c2.x >= 0) {
    ar += uu[0].x;
    ai += uu[0].y;
    if (c2.y >= 0) {
      ar += uu[1].x;
      ai += uu[1].y;
    }
  } else if (c2.x < -1) {
    for (int e = -2 - c2.x; e < b.fcon_ptr[fr + 1]; ++e) {
      const double2 u = ubb[(int64_t)b.fcon_idx[e] * 16 + r];
      ar += u.x;
      ai += u.y;
    }
  }
}

// The level kernels' launch bounds keep their register budget at or below
// 256 (at least three waves per SIMD for complex128): with a larger budget
// the compiler may hold MFMA accumulators in AGPRs and move them through
// VGPRs around every MFMA.
template <class T, int kFwd, int kCoarse>
__global__ __launch_bounds__(kWG, sizeof(T) == 4 ? 4 : 3) void level_mfma_kernel(const Tile* __restrict__ tiles, Batch b,
                                                         const typename Mf<T>::C2* __restrict__ G,
                                                         double2* __restrict__ out, double2* __restrict__ ubb) {
  using C2 = typename Mf<T>::C2;
  using V4 = typename Mf<T>::V4;
  // partial sums of the 4 waves, two row blocks at a time: [wave][rb2][j][lane]
  __shared__ C2 red[4][2][4][64];
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sn = t.sn, c0 = b.sn_c0[sn], w = b.sn_w[sn];
  const C2* __restrict__ P = reinterpret_cast<const C2*>(kFwd ? b.pf : b.pb) + t.off;
  const C2* Bk = G + (b.goff_f[sn] + t.col0) * 16;  // the staged forward input block
  V4 dre[4], dim[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) dre[rb] = dim[rb] = V4{0, 0, 0, 0};
  // 4 waves per tile: wave q takes the k-steps q, q + 4, ... of the tile;
  // the partial accumulators are summed through LDS
  mfma_stream<T>(P, t.nrows, t.ncols, Bk, 4 * wv, 16, dre, dim);
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[wv][q][j][lane] = C2{dre[2 * h + q][j], dim[2 * h + q][j]};
    __syncthreads();
    // 512 outputs (32 rows x 16 right-hand sides) of this half, 2 per
    // thread: the update rows' child-update pairs and values are loaded for
    // both outputs before either is stored
    const int frow0 = b.sn_frow0[sn], uoff = b.sn_uoff[sn];
    int2 c2[2];
    double2 uu[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int o = threadIdx.x + i * kWG, rloc = 32 * h + (o >> 4), r = o & 15, row = t.row0 + rloc;
      const bool upd = kFwd && rloc < t.nrows && row >= w;
      const int2 c = b.fcon2[upd ? frow0 + row : 0];
      c2[i] = upd ? c : make_int2(-1, -1);
      uu[i][0] = *(c2[i].x >= 0 ? ubb + (int64_t)c2[i].x * 16 + r : out + r);
      uu[i][1] = *(c2[i].y >= 0 ? ubb + (int64_t)c2[i].y * 16 + r : out + r);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int o = threadIdx.x + i * kWG;
      const int rloc = 32 * h + (o >> 4), r = o & 15;
      if (rloc < t.nrows) {
        const int q = (rloc >> 4) - 2 * h, rr = rloc & 15;
        int l, j;
        if (sizeof(T) == 8) {  // FP64: row = 4 j + l / 16
          j = rr >> 2;
          l = (rr & 3) * 16 + r;
        } else {               // FP32: row = 4 (l / 16) + j
          j = rr & 3;
          l = (rr >> 2) * 16 + r;
        }
        double ar = 0, ai = 0;
#pragma unroll
        for (int wq = 0; wq < 4; ++wq) {
          ar += (double)red[wq][q][j][l].x;
          ai += (double)red[wq][q][j][l].y;
        }
        const int row = t.row0 + rloc;
        if (!kFwd || row < w) {
          out[(int64_t)(c0 + row) * 16 + r] = make_double2(ar, ai);
        } else {
          add_children(b, frow0 + row, c2[i], uu[i], ubb, r, ar, ai);
          ubb[(int64_t)(uoff + row - w) * 16 + r] = make_double2(ar, ai);
        }
      }
    }
    __syncthreads();
  }
}

// Narrow tiles (at most 96 input columns): one wave per tile, all four
// 16-row blocks of the tile in that wave, so there is no cross-wave
// reduction; the accumulators go straight to y / the update vectors (FP64
// accumulator register j of lane l holds row 4 j + l / 16, FP32 row
// 4 (l / 16) + j, right-hand side l % 16).
template <class T, int kFwd, int kCoarse>
__global__ __launch_bounds__(kWG, sizeof(T) == 4 ? 5 : 4) void level_mfma_narrow_kernel(const Tile* __restrict__ tiles, int64_t ntiles,
                                                                Batch b, const typename Mf<T>::C2* __restrict__ G,
                                                                double2* __restrict__ out,
                                                                double2* __restrict__ ubb) {
  using C2 = typename Mf<T>::C2;
  using V4 = typename Mf<T>::V4;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lr = lane & 15, lk = lane >> 4;
  const int64_t ti = (int64_t)blockIdx.x * (kWG / 64) + wv;
  if (ti >= ntiles) return;  // a whole wave; the kernel has no barrier
  const Tile t = tiles[ti];
  const int sn = t.sn, c0 = b.sn_c0[sn], w = b.sn_w[sn];
  const C2* __restrict__ P = reinterpret_cast<const C2*>(kFwd ? b.pf : b.pb) + t.off;
  const C2* Bk = G + (b.goff_f[sn] + t.col0) * 16;  // the staged forward input block
  const int nr = t.nrows, nrb = (nr + 15) >> 4;
  V4 dre[4], dim[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) dre[rb] = dim[rb] = V4{0, 0, 0, 0};
  mfma_stream<T>(P, nr, t.ncols, Bk, 0, 4, dre, dim);
  // per row block, the update rows' child-update pairs, then their values,
  // then the stores (rows without updates read y, any valid address)
  const int frow0 = b.sn_frow0[sn], uoff = b.sn_uoff[sn];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    if (rb >= nrb) break;
    int2 c2[4];
    double2 uu[4][2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rloc = 16 * rb + Mf<T>::row(lk, j), row = t.row0 + rloc;
      const bool upd = kFwd && rloc < nr && row >= w;
      const int2 c = b.fcon2[upd ? frow0 + row : 0];
      c2[j] = upd ? c : make_int2(-1, -1);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uu[j][0] = *(c2[j].x >= 0 ? ubb + (int64_t)c2[j].x * 16 + lr : out + lr);
      uu[j][1] = *(c2[j].y >= 0 ? ubb + (int64_t)c2[j].y * 16 + lr : out + lr);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rloc = 16 * rb + Mf<T>::row(lk, j);
      if (rloc >= nr) continue;
      double ar = (double)dre[rb][j], ai = (double)dim[rb][j];
      const int row = t.row0 + rloc;
      if (!kFwd || row < w) {
        out[(int64_t)(c0 + row) * 16 + lr] = make_double2(ar, ai);
      } else {
        add_children(b, frow0 + row, c2[j], uu[j], ubb, lr, ar, ai);
        ubb[(int64_t)(uoff + row - w) * 16 + lr] = make_double2(ar, ai);
      }
    }
  }
}

// Stages a pass of a tile's input block into G: entries e = base + q stride
// (q < 8) of the cn columns from cb, entry e being column col0 + cb + e / 16
// and right-hand side e % 16.  Forward: the restricted right-hand side,
// gathered through bidx (restriction, nested-dissection permutation and
// pivot order in one index), minus the children's updates routed to the
// column's front row (at most two, read through fcon2; longer lists through
// fcon_idx).  Backward: the forward result for the pivot columns, the
// ancestors' backward results (through the supernode's row list) for the
// others.  All eight entries' index loads are issued first, then all value
// loads, so a pass costs two memory round trips.  The backward loads are
// unconditional (entries past the pass read a valid dummy address and are
// not stored), so no load waits behind a branch.
template <class T, int kFwd>
__device__ __forceinline__ void stage_pass(const Batch& b, const Tile& t, int cb, int cn, int base, int stride,
                                           typename Mf<T>::C2* G, const double2* __restrict__ src,
                                           const double2* aux) {
  using C2 = typename Mf<T>::C2;
  constexpr int kQ = 8;
  if constexpr (!kFwd) {
    int rv[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = base + q * stride;
      const int c = t.col0 + cb + (e >> 4);
      // an ancestor column reads its position from the row list; the
      // others read bidx[0] (any valid address) and ignore it
      const bool up = e < cn * 16 && c >= t.w;
      rv[q] = *(up ? b.rows + t.aux + (c - t.w) : b.bidx);
    }
    double2 v[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = base + q * stride;
      const int c = t.col0 + cb + (e >> 4), r = e & 15;
      const bool in = e < cn * 16;
      v[q] = *(!in ? src + r : (c < t.w ? src + (int64_t)(t.c0 + c) * 16 + r : aux + (int64_t)rv[q] * 16 + r));
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = base + q * stride;
      if (e < cn * 16) G[e] = C2{(T)v[q].x, (T)v[q].y};
    }
  } else {
    int idx[kQ];
    int2 ch[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = base + q * stride;
      const bool in = e < cn * 16;
      const int c = t.col0 + cb + (e >> 4);
      idx[q] = in ? b.bidx[t.c0 + c] : 0;
      ch[q] = in ? b.fcon2[t.aux + c] : make_int2(-1, -1);
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = base + q * stride;
      if (e >= cn * 16) continue;
      const int r = e & 15;
      double2 v = src[(int64_t)idx[q] * 16 + r];
      const int2 c2 = ch[q];
      if (c2.x >= 0) {
        const double2 u0 = aux[(int64_t)c2.x * 16 + r];
        v.x -= u0.x;
        v.y -= u0.y;
        if (c2.y >= 0) {
          const double2 u1 = aux[(int64_t)c2.y * 16 + r];
          v.x -= u1.x;
          v.y -= u1.y;
        }
      } else if (c2.x < -1) {
        const int fr = t.aux + t.col0 + cb + (e >> 4);
        for (int k = -2 - c2.x; k < b.fcon_ptr[fr + 1]; ++k) {
          const double2 u = aux[(int64_t)b.fcon_idx[k] * 16 + r];
          v.x -= u.x;
          v.y -= u.y;
        }
      }
      G[e] = C2{(T)v.x, (T)v.y};
    }
  }
}

constexpr int kCB = 128;  // input columns staged per pass of a wide tile (4 waves)
constexpr int kCBn = 32;  // per pass of a narrow tile (one wave)
// stage_pass stages eight entries per thread
static_assert(kCB * 16 == 8 * kWG && kCBn * 16 == 8 * 64, "a pass is eight entries per thread");

// Output row rloc (of the tile) for right-hand side r: forward pivot rows
// and backward rows go to out; forward update rows add the children's
// updates routed to that front row and go to the supernode's update vector.
template <int kFwd>
__device__ __forceinline__ void put_row(const Batch& b, const Tile& t, int rloc, int r, double ar, double ai,
                                        double2* out, double2* ubb) {
  const int row = t.row0 + rloc;
  if (!kFwd || row < t.w) {
    out[(int64_t)(t.c0 + row) * 16 + r] = make_double2(ar, ai);
  } else {
    const int fr = t.aux + row;
    for (int e = b.fcon_ptr[fr]; e < b.fcon_ptr[fr + 1]; ++e) {
      const double2 u = ubb[(int64_t)b.fcon_idx[e] * 16 + r];
      ar += u.x;
      ai += u.y;
    }
    ubb[(int64_t)(b.sn_uoff[t.sn] + row - t.w) * 16 + r] = make_double2(ar, ai);
  }
}

// One level of the 16-right-hand-side backward sweep, the input gather
// fused in (a backward tile holds all input columns of its rows, so a narrow
// supernode's input is gathered once; the forward sweep keeps the staged
// gather, whose supernodes have several row tiles over the same input): a
// workgroup stages its tile's input block (16 right-hand sides per column)
// in LDS a pass of columns at a time and multiplies the panel tile into it
// on MFMA.  Workgroups [0, nwide) take one wide tile each (its k-steps
// shared by the four waves, wave q taking q, q + 4, ..., partial sums added
// through LDS); the others take four narrow tiles, a wave each.
template <class T, int kFwd, int kCoarse>
__global__ __launch_bounds__(kWG, 3) void level_fused_kernel(const Tile* __restrict__ tiles, int64_t ntiles,
                                                          int64_t nwide, Batch b, const double2* __restrict__ src,
                                                          const double2* aux, double2* out, double2* ubb) {
  using C2 = typename Mf<T>::C2;
  using V4 = typename Mf<T>::V4;
  __shared__ C2 G[kCB * 16];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lr = lane & 15,
            lk = lane >> 4;
  V4 dre[4], dim[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) dre[rb] = dim[rb] = V4{0, 0, 0, 0};
  const C2* __restrict__ panels = reinterpret_cast<const C2*>(kFwd ? b.pf : b.pb);
  if ((int64_t)blockIdx.x < nwide) {
    const Tile t = tiles[blockIdx.x];
    for (int cb = 0; cb < t.ncols; cb += kCB) {
      const int cn = min(kCB, t.ncols - cb);
      stage_pass<T, kFwd>(b, t, cb, cn, threadIdx.x, kWG, G, src, aux);
      __syncthreads();
      mfma_stream<T>(panels + t.off + (int64_t)cb * t.nrows, t.nrows, cn, G, 4 * wv, 16, dre, dim);
      __syncthreads();
    }
    // partial sums of the 4 waves, two row blocks at a time, in the staging
    // buffer: [wave][rb2][j][lane] (4 x 2 x 4 x 64 = kCB x 16 entries)
    C2 (*red)[2][4][64] = reinterpret_cast<C2 (*)[2][4][64]>(G);
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wv][q][j][lane] = C2{dre[2 * h + q][j], dim[2 * h + q][j]};
      __syncthreads();
      // 512 outputs (32 rows x 16 right-hand sides) of this half, 2 per thread
      for (int o = threadIdx.x; o < 512; o += kWG) {
        const int rloc = 32 * h + (o >> 4), r = o & 15;
        if (rloc < t.nrows) {
          const int q = (rloc >> 4) - 2 * h, rr = rloc & 15;
          int l, j;
          if (sizeof(T) == 8) {  // FP64: row = 4 j + l / 16
            j = rr >> 2;
            l = (rr & 3) * 16 + r;
          } else {               // FP32: row = 4 (l / 16) + j
            j = rr & 3;
            l = (rr >> 2) * 16 + r;
          }
          double ar = 0, ai = 0;
#pragma unroll
          for (int wq = 0; wq < 4; ++wq) {
            ar += (double)red[wq][q][j][l].x;
            ai += (double)red[wq][q][j][l].y;
          }
          put_row<kFwd>(b, t, rloc, r, ar, ai, out, ubb);
        }
      }
      __syncthreads();
    }
    return;
  }
  // narrow tiles: a wave each, the staging buffer split into four
  const int64_t g0 = nwide + ((int64_t)blockIdx.x - nwide) * 4;
  const int64_t ti = g0 + wv;
  const bool has = ti < ntiles;
  Tile t{};
  if (has) t = tiles[ti];
  int np = 0;  // passes: the most any tile of the workgroup needs (uniform)
  for (int q = 0; q < 4; ++q)
    if (g0 + q < ntiles) np = max(np, (tiles[g0 + q].ncols + kCBn - 1) / kCBn);
  C2* Gw = G + wv * kCBn * 16;
  const int nr = t.nrows, nrb = (nr + 15) >> 4;
  const C2* __restrict__ P = panels + t.off;
  for (int p = 0; p < np; ++p) {
    const int cb = p * kCBn;
    const int cn = has ? max(0, min(kCBn, t.ncols - cb)) : 0;
    stage_pass<T, kFwd>(b, t, cb, cn, lane, 64, Gw, src, aux);
    __syncthreads();
    mfma_stream<T>(P + (int64_t)cb * nr, nr, cn, Gw, 0, 4, dre, dim);
    __syncthreads();
  }
  if (!has) return;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    if (rb >= nrb) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rloc = 16 * rb + Mf<T>::row(lk, j);
      if (rloc < nr) put_row<kFwd>(b, t, rloc, lr, (double)dre[rb][j], (double)dim[rb][j], out, ubb);
    }
  }
}

// Block SpMV over CSR: S consecutive lanes share a row and take one
// right-hand side each, so every x gather is one contiguous S x 16 B line.
// With kXcd, XCD k sweeps the rows [xr[k], xr[k+1]) (as in the single-vector
// kernel).
template <int S, bool kXcd>
__global__ __launch_bounds__(kWG) void csr_block_kernel(int64_t n, const int64_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double2* __restrict__ val,
                                                        const int64_t* __restrict__ xr,
                                                        const double2* __restrict__ x,
                                                        const double2* __restrict__ bvec, double2* __restrict__ y) {
  int64_t i, end = n;
  int r;
  if (kXcd) {
    const int64_t e0 = (int64_t)(blockIdx.x >> 3) * kWG + threadIdx.x;
    i = xr[blockIdx.x & 7] + e0 / S;
    r = (int)(e0 % S);
    end = xr[(blockIdx.x & 7) + 1];
  } else {
    const int64_t e0 = (int64_t)blockIdx.x * kWG + threadIdx.x;
    i = e0 / S;
    r = (int)(e0 % S);
  }
  if (i >= end) return;
  const int64_t e = i * S + r;
  double ar = 0, ai = 0, br = 0, bi = 0;
  const int64_t p1 = ptr[i + 1];
  int64_t p = ptr[i];
  // eight entries per step: all column loads, then the values and the x
  // gathers, so a lane keeps eight gathers in flight (even entries sum into
  // a, odd ones into b, in the order of the short loop below)
  for (; p + 8 <= p1; p += 8) {
    int c[8];
    double2 v[8], xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = col[p + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = val[p + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = x[(int64_t)c[u] * S + r];
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      cfma(ar, ai, v[u], xv[u]);
      cfma(br, bi, v[u + 1], xv[u + 1]);
    }
  }
  for (; p + 2 <= p1; p += 2) {
    const int c0 = col[p], c1 = col[p + 1];
    const double2 v0 = val[p], v1 = val[p + 1];
    cfma(ar, ai, v0, x[(int64_t)c0 * S + r]);
    cfma(br, bi, v1, x[(int64_t)c1 * S + r]);
  }
  if (p < p1) cfma(ar, ai, val[p], x[(int64_t)col[p] * S + r]);
  ar += br;
  ai += bi;
  if (bvec) {
    const double2 bb = bvec[e];
    y[e] = make_double2(bb.x - ar, bb.y - ai);
  } else {
    y[e] = make_double2(ar, ai);
  }
}

template <int S>
__global__ __launch_bounds__(kWG) void spmv_real_block_kernel(int64_t n, const int64_t* __restrict__ ptr,
                                                              const int32_t* __restrict__ col,
                                                              const double* __restrict__ val,
                                                              const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= n * S) return;
  const int64_t row = e / S;
  const int r = (int)(e % S);
  double ar = 0, ai = 0;
  const int64_t p1 = ptr[row + 1];
  int64_t p = ptr[row];
  // eight entries per step (loads first, then the multiply-adds in order)
  for (; p + 8 <= p1; p += 8) {
    int c[8];
    double a[8];
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = col[p + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = val[p + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[(int64_t)c[u] * S + r];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      ar = fma(a[u], v[u].x, ar);
      ai = fma(a[u], v[u].y, ai);
    }
  }
  for (; p < p1; ++p) {
    const double a = val[p];
    const double2 v = x[(int64_t)col[p] * S + r];
    ar = fma(a, v.x, ar);
    ai = fma(a, v.y, ai);
  }
  y[e] = make_double2(ar, ai);
}

// q = Z cx and t = x - (A Z) cx for S interleaved right-hand sides (A Z in
// split storage: bit 31 of a column marks an imaginary part).
template <int S>
__global__ __launch_bounds__(kWG) void coarse_update_block_kernel(
    int64_t n, const int64_t* __restrict__ zptr, const int32_t* __restrict__ zcol, const double* __restrict__ zval,
    const int64_t* __restrict__ aptr, const int32_t* __restrict__ acol, const double* __restrict__ aval,
    const double2* __restrict__ cx, const double2* __restrict__ x, double2* __restrict__ q, double2* __restrict__ t) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= n * S) return;
  const int64_t row = e / S;
  const int r = (int)(e % S);
  double qr = 0, qi = 0, ar = 0, ai = 0;
  for (int64_t p = zptr[row]; p < zptr[row + 1]; ++p) {
    const double z = zval[p];
    const double2 v = cx[(int64_t)zcol[p] * S + r];
    qr = fma(z, v.x, qr);
    qi = fma(z, v.y, qi);
  }
  auto az = [&](int c, double a, double2 v) {
    const bool im = c < 0;  // i v = (-v.y, v.x)
    ar = fma(a, im ? -v.y : v.x, ar);
    ai = fma(a, im ? v.x : v.y, ai);
  };
  const int64_t p1 = aptr[row + 1];
  int64_t p = aptr[row];
  // four entries of A Z per step (loads first, then the multiply-adds in order)
  for (; p + 4 <= p1; p += 4) {
    int c[4];
    double a[4];
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = acol[p + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = aval[p + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = cx[(int64_t)(c[u] & 0x7fffffff) * S + r];
#pragma unroll
    for (int u = 0; u < 4; ++u) az(c[u], a[u], v[u]);
  }
  for (; p < p1; ++p) {
    const int c = acol[p];
    az(c, aval[p], cx[(int64_t)(c & 0x7fffffff) * S + r]);
  }
  q[e] = make_double2(qr, qi);
  const double2 xx = x[e];
  t[e] = make_double2(xx.x - ar, xx.y - ai);
}

template <int S>
__global__ __launch_bounds__(kWG) void prolong_block_kernel(int64_t n, const int64_t* __restrict__ ptr,
                                                            const int32_t* __restrict__ idx,
                                                            const double* __restrict__ w,
                                                            const double2* __restrict__ xl,
                                                            const double2* __restrict__ q, double2* __restrict__ z) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= n * S) return;
  const int64_t g = e / S;
  const int r = (int)(e % S);
  double ar = 0, ai = 0;
  if (q) {
    ar = q[e].x;
    ai = q[e].y;
  }
  for (int64_t p = ptr[g]; p < ptr[g + 1]; ++p) {
    const double2 v = xl[(int64_t)idx[p] * S + r];
    const double c = w[p];
    ar = fma(c, v.x, ar);
    ai = fma(c, v.y, ai);
  }
  z[e] = make_double2(ar, ai);
}

template <int S>
__global__ __launch_bounds__(kWG) void pack_kernel(int64_t n, PtrSetC src, double2* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= n * S) return;
  const int64_t i = e / S;
  const int r = (int)(e % S);
  const double2* p = reinterpret_cast<const double2*>(src.p[r]);
  dst[e] = p ? p[i] : make_double2(0.0, 0.0);
}

template <int S>
__global__ __launch_bounds__(kWG) void unpack_kernel(int64_t n, const double2* __restrict__ src, PtrSet dst) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= n * S) return;
  const int64_t i = e / S;
  const int r = (int)(e % S);
  double2* p = reinterpret_cast<double2*>(dst.p[r]);
  if (p) p[i] = src[e];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kWG - 1) / kWG); }

// Calls f(std::integral_constant<int, S>) for the supported block widths.
template <class F>
void with_width(int S, F&& f) {
  switch (S) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: break;
  }
}

}  // namespace

void fwd_level_block(const Batch& b, int64_t tile0, int64_t ntiles, int S, const double* bin, double* yb, double* ubb,
                     bool coarse, hipStream_t s) {
  if (ntiles <= 0) return;
  const Tile* t = b.tf + tile0;
  auto in = reinterpret_cast<const double2*>(bin);
  auto y = reinterpret_cast<double2*>(yb);
  auto u = reinterpret_cast<double2*>(ubb);
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    if (coarse)
      fwd_block_kernel<double2, W, 1><<<(unsigned)ntiles, 64, 0, s>>>(t, b, in, y, u);
    else if (b.c64)
      fwd_block_kernel<float2, W, 0><<<(unsigned)ntiles, 64, 0, s>>>(t, b, in, y, u);
    else
      fwd_block_kernel<double2, W, 0><<<(unsigned)ntiles, 64, 0, s>>>(t, b, in, y, u);
  });
}

void bwd_level_block(const Batch& b, int64_t tile0, int64_t ntiles, int S, const double* yb, double* xb, bool coarse,
                     hipStream_t s) {
  if (ntiles <= 0) return;
  const Tile* t = b.tb + tile0;
  auto y = reinterpret_cast<const double2*>(yb);
  auto x = reinterpret_cast<double2*>(xb);
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    if (coarse)
      bwd_block_kernel<double2, W, 1><<<(unsigned)ntiles, 64, 0, s>>>(t, b, y, x);
    else if (b.c64)
      bwd_block_kernel<float2, W, 0><<<(unsigned)ntiles, 64, 0, s>>>(t, b, y, x);
    else
      bwd_block_kernel<double2, W, 0><<<(unsigned)ntiles, 64, 0, s>>>(t, b, y, x);
  });
}

// Tiles [tile0, tile0 + nwide) go to the 4-wave kernel, the rest (narrow,
// at the end of the level) to the one-wave-per-tile kernel.
template <class T, int kFwd, int kCoarse>
void level_mfma_launch(const Batch& b, const Tile* tiles, int64_t ntiles, int64_t nwide,
                       const typename Mf<T>::C2* G, double2* out, double2* u, hipStream_t s) {
  if (nwide > 0) level_mfma_kernel<T, kFwd, kCoarse><<<(unsigned)nwide, kWG, 0, s>>>(tiles, b, G, out, u);
  const int64_t nn = ntiles - nwide;
  if (nn > 0)
    level_mfma_narrow_kernel<T, kFwd, kCoarse><<<(unsigned)((nn + 3) / 4), kWG, 0, s>>>(tiles + nwide, nn, b, G, out,
                                                                                        u);
}

void fwd_level_mfma(const Batch& b, const int32_t* sns, int64_t nsn, int gy, int64_t tile0, int64_t ntiles,
                    int64_t nwide, const double* bin, double* yb, double* ubb, void* stage, bool coarse,
                    hipStream_t s) {
  if (ntiles <= 0) return;
  auto in = reinterpret_cast<const double2*>(bin);
  auto y = reinterpret_cast<double2*>(yb);
  auto u = reinterpret_cast<double2*>(ubb);
  if (b.c64 && !coarse) {
    auto G = reinterpret_cast<float2*>(stage);
    gather_fwd_kernel<float><<<dim3((unsigned)nsn, (unsigned)gy), kWG, 0, s>>>(sns, b, in, u, G);
    level_mfma_launch<float, 1, 0>(b, b.tf + tile0, ntiles, nwide, G, y, u, s);
  } else {
    auto G = reinterpret_cast<double2*>(stage);
    gather_fwd_kernel<double><<<dim3((unsigned)nsn, (unsigned)gy), kWG, 0, s>>>(sns, b, in, u, G);
    if (coarse)
      level_mfma_launch<double, 1, 1>(b, b.tf + tile0, ntiles, nwide, G, y, u, s);
    else
      level_mfma_launch<double, 1, 0>(b, b.tf + tile0, ntiles, nwide, G, y, u, s);
  }
}

// One launch per level: nwide wide tiles (the level's first ones) take a
// workgroup each, the narrow ones four per workgroup.
template <class T, int kCoarse>
void bwd_fused_launch(const Batch& b, const Tile* tiles, int64_t ntiles, int64_t nwide, const double2* y, double2* x,
                      hipStream_t s) {
  const int64_t grid = nwide + (ntiles - nwide + 3) / 4;
  level_fused_kernel<T, 0, kCoarse><<<(unsigned)grid, kWG, 0, s>>>(tiles, ntiles, nwide, b, y, x, x, nullptr);
}

void bwd_level_mfma(const Batch& b, int64_t tile0, int64_t ntiles, int64_t nwide, const double* yb, double* xb,
                    bool coarse, hipStream_t s) {
  if (ntiles <= 0) return;
  auto y = reinterpret_cast<const double2*>(yb);
  auto x = reinterpret_cast<double2*>(xb);
  if (b.c64 && !coarse)
    bwd_fused_launch<float, 0>(b, b.tb + tile0, ntiles, nwide, y, x, s);
  else if (coarse)
    bwd_fused_launch<double, 1>(b, b.tb + tile0, ntiles, nwide, y, x, s);
  else
    bwd_fused_launch<double, 0>(b, b.tb + tile0, ntiles, nwide, y, x, s);
}

void csr_spmv_block(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const int64_t* xr,
                    int64_t xrows, int S, const double* x, const double* b, double* y, hipStream_t s) {
  if (n <= 0) return;
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    auto v2 = reinterpret_cast<const double2*>(val);
    auto x2 = reinterpret_cast<const double2*>(x);
    auto b2 = reinterpret_cast<const double2*>(b);
    auto y2 = reinterpret_cast<double2*>(y);
    if (xr)
      csr_block_kernel<W, true><<<8 * blocks_for(xrows * W), kWG, 0, s>>>(n, ptr, col, v2, xr, x2, b2, y2);
    else
      csr_block_kernel<W, false><<<blocks_for(n * W), kWG, 0, s>>>(n, ptr, col, v2, nullptr, x2, b2, y2);
  });
}

void spmv_real_block(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, int S, const double* x,
                     double* y, hipStream_t s) {
  if (n <= 0) return;
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    spmv_real_block_kernel<W><<<blocks_for(n * W), kWG, 0, s>>>(n, ptr, col, val, reinterpret_cast<const double2*>(x),
                                                                 reinterpret_cast<double2*>(y));
  });
}

void coarse_update_block(int64_t n, const int64_t* zptr, const int32_t* zcol, const double* zval,
                         const int64_t* aptr, const int32_t* acol, const double* aval, int S, const double* cx,
                         const double* x, double* q, double* t, hipStream_t s) {
  if (n <= 0) return;
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    coarse_update_block_kernel<W><<<blocks_for(n * W), kWG, 0, s>>>(
        n, zptr, zcol, zval, aptr, acol, aval, reinterpret_cast<const double2*>(cx),
        reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(q), reinterpret_cast<double2*>(t));
  });
}

void prolong_block(int64_t n, const int64_t* ptr, const int32_t* idx, const double* wt, int S, const double* xl,
                   const double* q, double* z, hipStream_t s) {
  if (n <= 0) return;
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    prolong_block_kernel<W><<<blocks_for(n * W), kWG, 0, s>>>(n, ptr, idx, wt, reinterpret_cast<const double2*>(xl),
                                                               reinterpret_cast<const double2*>(q),
                                                               reinterpret_cast<double2*>(z));
  });
}

void pack(int64_t n, int S, const PtrSetC& src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    pack_kernel<W><<<blocks_for(n * W), kWG, 0, s>>>(n, src, reinterpret_cast<double2*>(dst));
  });
}

void unpack(int64_t n, int S, const double* src, const PtrSet& dst, hipStream_t s) {
  if (n <= 0) return;
  with_width(S, [&](auto w) {
    constexpr int W = decltype(w)::value;
    unpack_kernel<W><<<blocks_for(n * W), kWG, 0, s>>>(n, reinterpret_cast<const double2*>(src), dst);
  });
}

}  // namespace dev
}  // namespace helm
