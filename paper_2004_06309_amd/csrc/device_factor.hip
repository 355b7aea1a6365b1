// Multifrontal numeric LU of a batch of local matrices on the device (the
// local direct solvers of the ORAS preconditioner, eq. oras, and the coarse
// matrix E of eq. 2lvl), level by level of the elimination trees.
//
// One workgroup owns one frontal matrix F (order m = w + r, column-major in a
// level workspace) and does, in order:
//   1. assembly: zero F, scatter the original entries of the supernode's
//      arrowhead, extend-add the children's Schur complements (children in
//      ascending order, so the sums are deterministic);
//   2. blocked right-looking partial LU of the w fully-summed columns, pivot
//      rows searched among the fully-summed rows only (P F11 = L11 U11,
//      L21 = F21 U11^{-1}, U12 = L11^{-1} P F12, F22 - L21 U12 left in place);
//   3. the Schur complement F22 copied out for the parent;
//   4. the explicit-inverse panels of the partitioned-inverse solve:
//        X = [I; L21] L11^{-1}   (m x w, right triangular solve by blocks)
//        Y = U11^{-1} [I | -U12] (w x m, left triangular solve by blocks)
//   5. X and Y written into the solve tiles (complex128 or complex64).
// Every rank-32 update of steps 2 and 4 is a complex GEMM on the 16x16x4
// MFMA (four real MFMAs per complex product); the pivot search, the
// 32-column panel factorisation and the 32 x 32 triangular solves run on the
// vector units.
//
// The whole factorisation runs in one of two working precisions: complex128
// (FP64 MFMA; the panels are stored in complex128, or rounded once to
// complex64), or complex64 (fronts, Schur complements and panels in
// complex64, FP32 MFMA accumulating in FP32; the original entries are
// rounded on assembly).  The complex64 form halves the workspace and runs
// the updates at the FP32 MFMA rate (twice the FP64 one).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "device.hpp"

namespace helm {
namespace dev {

namespace {

constexpr int kFW = 256;  // threads of a front workgroup
constexpr int kNB = 32;   // block size of the partial LU and the panel solves

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

// Working precision R: its complex type, the 16x16x4 MFMA, the accumulator
// layout and the pivot tolerances.
template <class R>
struct Fp;
template <>
struct Fp<double> {
  using C = double2;
  using V4 = dv4;
  static __device__ __forceinline__ C mk(double a, double b) { return make_double2(a, b); }
  static __device__ __forceinline__ V4 mma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of D held in accumulator register j of a lane with l / 16 = hi
  static __device__ __forceinline__ int drow(int hi, int j) { return 4 * j + hi; }
  static constexpr double kTiny = kTinyPivot;
  static constexpr double kEps = DBL_EPSILON;
};
template <>
struct Fp<float> {
  using C = float2;
  using V4 = fv4;
  static __device__ __forceinline__ C mk(double a, double b) { return make_float2((float)a, (float)b); }
  static __device__ __forceinline__ V4 mma(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int hi, int j) { return 4 * hi + j; }
  static constexpr double kTiny = kTinyPivotF32;
  static constexpr double kEps = FLT_EPSILON;
};

template <class C>
__device__ __forceinline__ void csub_mul(C& x, C a, C b) {
  x.x -= a.x * b.x - a.y * b.y;
  x.y -= a.x * b.y + a.y * b.x;
}
// a / d as (a conj(d)) / |d|^2
template <class C>
__device__ __forceinline__ C cdivd(C a, C d) {
  const auto q = d.x * d.x + d.y * d.y;
  C r;
  r.x = (a.x * d.x + a.y * d.y) / q;
  r.y = (a.y * d.x - a.x * d.y) / q;
  return r;
}

// C[M x N] -= A[M x K] B[K x N] (complex, column-major), by the whole
// workgroup: each wave computes (16 RB) x (16 CB) output tiles as RB x CB
// MFMA blocks.  The MFMA computes the transposed block C^T = B^T A^T, so the
// 16 lanes that share an accumulator column hold 16 consecutive rows of C
// (coalesced loads and stores).  The accumulators start from C and the
// products enter negated, so C is read once, before the first product, and
// written once; the operands of the next 4-wide k step are loaded while the
// MFMAs of the current one run.  16x16x4 operand layout: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register j of lane l
// is D[Fp<R>::drow(l / 16, j)][l % 16].
template <class R, int RB = 2, int CB = 2>
__device__ void wg_gemm_sub(int M, int N, int K, const typename Fp<R>::C* A, int64_t lda,
                            const typename Fp<R>::C* B, int64_t ldb, typename Fp<R>::C* C, int64_t ldc) {
  using F = Fp<R>;
  using Cx = typename F::C;
  using V4 = typename F::V4;
  constexpr int TR = 16 * RB, TC = 16 * CB;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lo = lane & 15, hi = lane >> 4;
  const int tm = (M + TR - 1) / TR, tn = (N + TC - 1) / TC;
  for (int t = wv; t < tm * tn; t += kFW / 64) {
    const int r0 = (t % tm) * TR, c0 = (t / tm) * TC;
    V4 dre[CB][RB], dim[CB][RB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = c0 + 16 * cb + F::drow(hi, j), row = r0 + 16 * rb + lo;
          const Cx c = (row < M && col < N) ? C[row + (int64_t)col * ldc] : F::mk(0.0, 0.0);
          dre[cb][rb][j] = c.x;
          dim[cb][rb][j] = c.y;
        }
    Cx av[RB], bv[CB];
    auto load = [&](int k, Cx* a, Cx* b) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int row = r0 + 16 * rb + lo;
        a[rb] = (row < M && k < K) ? A[row + (int64_t)k * lda] : F::mk(0.0, 0.0);
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int col = c0 + 16 * cb + lo;
        b[cb] = (col < N && k < K) ? B[k + (int64_t)col * ldb] : F::mk(0.0, 0.0);
      }
    };
    load(hi, av, bv);
    for (int k0 = 0; k0 < K; k0 += 4) {
      Cx an[RB], bn[CB];
      load(k0 + 4 + hi, an, bn);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          dre[cb][rb] = F::mma(-bv[cb].x, av[rb].x, dre[cb][rb]);
          dre[cb][rb] = F::mma(bv[cb].y, av[rb].y, dre[cb][rb]);
          dim[cb][rb] = F::mma(-bv[cb].x, av[rb].y, dim[cb][rb]);
          dim[cb][rb] = F::mma(-bv[cb].y, av[rb].x, dim[cb][rb]);
        }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) av[rb] = an[rb];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) bv[cb] = bn[cb];
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = c0 + 16 * cb + F::drow(hi, j), row = r0 + 16 * rb + lo;
          if (row < M && col < N) {
            Cx c;
            c.x = dre[cb][rb][j];
            c.y = dim[cb][rb][j];
            C[row + (int64_t)col * ldc] = c;
          }
        }
  }
  __syncthreads();
}

// Triangular solves of many short vectors with the kNB x kNB block T (LDS,
// column-major, identity beyond kb).  The vectors go through LDS 64 at a
// time; the 4 consecutive lanes that share a vector (always in one wave, so
// their LDS accesses stay in program order) split its entries mod 4, and the
// recurrence runs over the block's kNB steps.
constexpr int kChunkV = kFW / 4;  // vectors per LDS chunk

// Columns of G (kb x ncols, ld): L x = b with L unit lower.
template <class C>
__device__ void solve_cols_unit_lower(C* G, int64_t ld, int kb, int ncols, const C* T, C* buf) {
  const int v = threadIdx.x >> 2, q = threadIdx.x & 3;
  for (int c0 = 0; c0 < ncols; c0 += kChunkV) {
    const int nc = min(kChunkV, ncols - c0);
    for (int e = threadIdx.x; e < kNB * kChunkV; e += kFW) {
      const int i = e % kNB, c = e / kNB;
      buf[e] = (i < kb && c < nc) ? G[i + (int64_t)(c0 + c) * ld] : C{0, 0};
    }
    __syncthreads();
    C* x = buf + v * kNB;
    for (int k = 0; k < kNB - 1; ++k) {
      const C xk = x[k];
      for (int i = q; i < kNB; i += 4)
        if (i > k) csub_mul(x[i], T[i + k * kNB], xk);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kNB * kChunkV; e += kFW) {
      const int i = e % kNB, c = e / kNB;
      if (i < kb && c < nc) G[i + (int64_t)(c0 + c) * ld] = buf[e];
    }
    __syncthreads();
  }
}

// Rows of G (nrows x kb, ld): x L = b with L unit lower, last entry first.
template <class C>
__device__ void solve_rows_right_unit_lower(C* G, int64_t ld, int kb, int nrows, const C* T, C* buf) {
  const int v = threadIdx.x >> 2, q = threadIdx.x & 3;
  for (int r0 = 0; r0 < nrows; r0 += kChunkV) {
    const int nr = min(kChunkV, nrows - r0);
    // buf[c + row * kNB]: one row's entries contiguous
    for (int e = threadIdx.x; e < kNB * kChunkV; e += kFW) {
      const int row = e % kChunkV, c = e / kChunkV;
      buf[c + row * kNB] = (c < kb && row < nr) ? G[r0 + row + (int64_t)c * ld] : C{0, 0};
    }
    __syncthreads();
    C* x = buf + v * kNB;
    for (int c2 = kNB - 1; c2 > 0; --c2) {
      const C xc = x[c2];
      for (int c = q; c < kNB; c += 4)
        if (c < c2) csub_mul(x[c], xc, T[c2 + c * kNB]);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kNB * kChunkV; e += kFW) {
      const int row = e % kChunkV, c = e / kChunkV;
      if (c < kb && row < nr) G[r0 + row + (int64_t)c * ld] = buf[c + row * kNB];
    }
    __syncthreads();
  }
}

// Columns of G (kb x ncols, ld): U y = b with U upper (its diagonal
// included), last entry first.
template <class C>
__device__ void solve_cols_upper(C* G, int64_t ld, int kb, int ncols, const C* T, C* buf) {
  const int v = threadIdx.x >> 2, q = threadIdx.x & 3;
  for (int c0 = 0; c0 < ncols; c0 += kChunkV) {
    const int nc = min(kChunkV, ncols - c0);
    for (int e = threadIdx.x; e < kNB * kChunkV; e += kFW) {
      const int i = e % kNB, c = e / kNB;
      buf[e] = (i < kb && c < nc) ? G[i + (int64_t)(c0 + c) * ld] : C{0, 0};
    }
    __syncthreads();
    C* y = buf + v * kNB;
    for (int k = kNB - 1; k >= 0; --k) {
      if (q == (k & 3)) y[k] = cdivd(y[k], T[k + k * kNB]);
      __builtin_amdgcn_wave_barrier();
      const C yk = y[k];
      for (int i = q; i < k; i += 4) csub_mul(y[i], T[i + k * kNB], yk);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kNB * kChunkV; e += kFW) {
      const int i = e % kNB, c = e / kNB;
      if (i < kb && c < nc) G[i + (int64_t)(c0 + c) * ld] = buf[e];
    }
    __syncthreads();
  }
}

// (value, index) maximum over the workgroup of NT threads; ties go to the
// lower index.
template <int NT = kFW>
__device__ void wg_argmax(double& v, int& idx, double* sv, int* si) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[wv] = v;
    si[wv] = idx;
  }
  __syncthreads();
  v = sv[0];
  idx = si[0];
  for (int q = 1; q < NT / 64; ++q)
    if (sv[q] > v || (sv[q] == v && si[q] < idx)) {
      v = sv[q];
      idx = si[q];
    }
  __syncthreads();
}

// Copies the kb x kb diagonal block at F (ld) into T (kNB x kNB), padded
// with the identity beyond kb.
template <class C>
__device__ void load_diag_block(const C* F, int64_t ld, int kb, C* T) {
  for (int e = threadIdx.x; e < kNB * kNB; e += kFW) {
    const int i = e % kNB, j = e / kNB;
    T[e] = (i < kb && j < kb) ? F[i + (int64_t)j * ld] : C{i == j ? 1 : 0, 0};
  }
  __syncthreads();
}

// One front per workgroup, in working precision R; the panels are written
// in complex64 when c64 is set (always so for R = float).
template <class R>
__global__ __launch_bounds__(kFW) void front_kernel(const FrontJob* __restrict__ jobs,
                                                    typename Fp<R>::C* __restrict__ ws,
                                                    typename Fp<R>::C* __restrict__ upd,
                                                    const int32_t* __restrict__ asm_pos,
                                                    const int32_t* __restrict__ asm_val,
                                                    const double2* __restrict__ aval,
                                                    const FrontChild* __restrict__ kids,
                                                    const int32_t* __restrict__ ep, int32_t* __restrict__ piv,
                                                    int32_t* __restrict__ npert, int c64, int tile_rows) {
  using F = Fp<R>;
  using Cx = typename F::C;
  __shared__ Cx T[kNB * kNB];
  __shared__ Cx buf[kNB * kChunkV];
  __shared__ double sv[kFW / 64];
  __shared__ int si[kFW / 64];
  const FrontJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int m = J.m, w = J.w, r = m - w;
  const int64_t mm = (int64_t)m * m;
  void* pf = J.pf;
  void* pb = J.pb;
  Cx* Fm = ws + J.F;

  // 1. assembly
  for (int64_t e = tid; e < mm; e += kFW) Fm[e] = F::mk(0.0, 0.0);
  __syncthreads();
  for (int64_t q = J.asm0 + tid; q < J.asm1; q += kFW) {
    const double2 a = aval[asm_val[q]];
    Fm[asm_pos[q]] = F::mk(a.x, a.y);
  }
  __syncthreads();
  for (int c = J.kid0; c < J.kid1; ++c) {
    const FrontChild K = kids[c];
    const Cx* S = upd + K.upd;
    const int32_t* map = ep + K.ep;
    const int64_t rc2 = (int64_t)K.r * K.r;
    for (int64_t e = tid; e < rc2; e += kFW) {
      const int a = (int)(e % K.r), b = (int)(e / K.r);
      Cx& f = Fm[map[a] + (int64_t)map[b] * m];
      const Cx s = S[e];
      f.x += s.x;
      f.y += s.y;
    }
    __syncthreads();
  }

  // 2. partial LU of the first w columns, pivots among rows [k, w)
  int32_t* perm = piv + J.piv0;
  int n_pert = 0;
  for (int k = tid; k < w; k += kFW) perm[k] = J.c0 + k;
  __syncthreads();
  for (int k0 = 0; k0 < w; k0 += kNB) {
    const int kb = min(kNB, w - k0);
    for (int k = k0; k < k0 + kb; ++k) {
      Cx* colk = Fm + (int64_t)k * m;
      double best = -1.0;
      int p = k;
      for (int i = k + tid; i < w; i += kFW) {
        const double a = hypot((double)colk[i].x, (double)colk[i].y);
        if (a > best) {
          best = a;
          p = i;
        }
      }
      wg_argmax(best, p, sv, si);
      if (p != k) {
        for (int j = tid; j < m; j += kFW) {
          const Cx t = Fm[k + (int64_t)j * m];
          Fm[k + (int64_t)j * m] = Fm[p + (int64_t)j * m];
          Fm[p + (int64_t)j * m] = t;
        }
        if (tid == 0) {
          const int32_t t = perm[k];
          perm[k] = perm[p];
          perm[p] = t;
        }
        __syncthreads();
      }
      if (!(best > F::kTiny * J.anorm)) {
        // zero or tiny pivot column: replaced by a small diagonal (counted;
        // setup then fails unless replacements were asked for)
        if (tid == 0) colk[k] = F::mk(sqrt(F::kEps) * J.anorm, 0.0);
        ++n_pert;
        __syncthreads();
      }
      const Cx d = colk[k];
      for (int i = k + 1 + tid; i < m; i += kFW) {
        const Cx l = cdivd(colk[i], d);
        colk[i] = l;
        for (int j = k + 1; j < k0 + kb; ++j) csub_mul(Fm[i + (int64_t)j * m], l, Fm[k + (int64_t)j * m]);
      }
      __syncthreads();
    }
    const int j0 = k0 + kb;
    if (j0 >= m) continue;
    // U12 rows of this block: unit-lower solve with the block's diagonal
    load_diag_block(Fm + k0 + (int64_t)k0 * m, m, kb, T);
    solve_cols_unit_lower(Fm + k0 + (int64_t)j0 * m, m, kb, m - j0, T, buf);
    wg_gemm_sub<R>(m - j0, m - j0, kb, Fm + j0 + (int64_t)k0 * m, m, Fm + k0 + (int64_t)j0 * m, m,
                   Fm + j0 + (int64_t)j0 * m, m);
  }

  if (tid == 0) npert[blockIdx.x] = n_pert;

  // 3. Schur complement for the parent
  if (r > 0) {
    Cx* S = upd + J.upd;
    const int64_t r2 = (int64_t)r * r;
    for (int64_t e = tid; e < r2; e += kFW) {
      const int a = (int)(e % r), b = (int)(e / r);
      S[e] = Fm[w + a + (int64_t)(w + b) * m];
    }
  }

  // 4a. X = [I; L21] L11^{-1}, block columns from the last to the first
  Cx* X = ws + J.X;
  const int nblk = (w + kNB - 1) / kNB;
  for (int jb = nblk - 1; jb >= 0; --jb) {
    const int j0 = jb * kNB, kb = min(kNB, w - j0), jend = j0 + kb;
    const int64_t cnt = (int64_t)m * kb;
    for (int64_t e = tid; e < cnt; e += kFW) {
      const int i = (int)(e % m), c = j0 + (int)(e / m);
      Cx v;
      if (i < j0)
        v = F::mk(0.0, 0.0);
      else if (i < w)
        v = F::mk(i == c ? 1.0 : 0.0, 0.0);
      else
        v = Fm[i + (int64_t)c * m];
      X[i + (int64_t)c * m] = v;
    }
    __syncthreads();
    if (jend < w)
      wg_gemm_sub<R>(m - j0, kb, w - jend, X + j0 + (int64_t)jend * m, m, Fm + jend + (int64_t)j0 * m, m,
                     X + j0 + (int64_t)j0 * m, m);
    load_diag_block(Fm + j0 + (int64_t)j0 * m, m, kb, T);
    solve_rows_right_unit_lower(X + j0 + (int64_t)j0 * m, m, kb, m - j0, T, buf);
  }

  // 4b. Y = U11^{-1} [I | -U12], block rows from the last to the first
  Cx* Y = ws + J.Y;
  for (int ib = nblk - 1; ib >= 0; --ib) {
    const int i0 = ib * kNB, kb = min(kNB, w - i0), iend = i0 + kb;
    const int64_t cnt = (int64_t)kb * m;
    for (int64_t e = tid; e < cnt; e += kFW) {
      const int q = (int)(e % kb), c = (int)(e / kb), row = i0 + q;
      Cx v;
      if (c < w) {
        v = F::mk(row == c ? 1.0 : 0.0, 0.0);
      } else {
        const Cx u = Fm[row + (int64_t)c * m];
        v.x = -u.x;
        v.y = -u.y;
      }
      Y[row + (int64_t)c * w] = v;
    }
    __syncthreads();
    if (iend < w)
      wg_gemm_sub<R>(kb, m - i0, w - iend, Fm + i0 + (int64_t)iend * m, m, Y + iend + (int64_t)i0 * w, w,
                     Y + i0 + (int64_t)i0 * w, w);
    load_diag_block(Fm + i0 + (int64_t)i0 * m, m, kb, T);
    solve_cols_upper(Y + i0 + (int64_t)i0 * w, w, kb, m - i0, T, buf);
  }

  // 5. solve tiles (column-major inside a tile); diagonal-block entries
  // outside the triangle are stored as zeros
  auto put = [&](void* dst, int64_t at, Cx v) {
    if (c64)
      reinterpret_cast<float2*>(dst)[at] = make_float2((float)v.x, (float)v.y);
    else
      reinterpret_cast<double2*>(dst)[at] = make_double2((double)v.x, (double)v.y);
  };
  int64_t off = J.pfo;
  for (int r0 = 0; r0 < m; r0 += tile_rows) {
    const int nr = min(tile_rows, m - r0), nc = min(w, r0 + nr);
    const int64_t cnt = (int64_t)nr * nc;
    for (int64_t e = tid; e < cnt; e += kFW) {
      const int i = (int)(e % nr), col = (int)(e / nr), row = r0 + i;
      put(pf, off + e, (row < w && col > row) ? F::mk(0.0, 0.0) : X[row + (int64_t)col * m]);
    }
    off += cnt;
  }
  off = J.pbo;
  for (int r0 = 0; r0 < w; r0 += tile_rows) {
    const int nr = min(tile_rows, w - r0), nc = m - r0;
    const int64_t cnt = (int64_t)nr * nc;
    for (int64_t e = tid; e < cnt; e += kFW) {
      const int i = (int)(e % nr), row = r0 + i, col = r0 + (int)(e / nr);
      put(pb, off + e, (col < w && col < row) ? F::mk(0.0, 0.0) : Y[row + (int64_t)col * w]);
    }
    off += cnt;
  }
}

// ---- large fronts: several workgroups per front ---------------------------
// Near the top of the elimination trees a level has a few dozen fronts of a
// thousand rows or more, so one workgroup per front leaves most of the device
// idle for most of the factorisation.  Fronts of at least kSplitFrontMin rows
// are therefore factorised by a sequence of launches, each spreading every
// front over many workgroups:
//   assembly   one workgroup per kStrip-column strip of F;
//   for each kNB-column block of the partial LU:
//     panel    one workgroup per front: pivot search and elimination inside
//              the block's columns (the row interchanges are applied to those
//              columns only, and recorded);
//     update   one workgroup per kStrip-column strip: the block's row
//              interchanges, then, right of the block, the U12 rows and the
//              rank-kNB update of the strip below the block;
//   panels     one workgroup per kStrip-row strip of X = [I; L21] L11^{-1}
//              (its rows are independent right triangular solves; the strip
//              also copies its rows of the Schur complement and writes its
//              forward solve tiles), or per kStrip-column strip of
//              Y = U11^{-1} [I | -U12] (independent columns);
//   Y tiles    one workgroup per backward solve tile.
// Every entry goes through the same operations in the same order as in
// front_kernel, so both forms give the same factors.
constexpr int kStrip = 64;

template <class R>
__global__ __launch_bounds__(kFW) void split_assemble_kernel(
    const FrontJob* __restrict__ jobs, typename Fp<R>::C* __restrict__ ws, const typename Fp<R>::C* __restrict__ upd,
    const int32_t* __restrict__ asm_pos, const int32_t* __restrict__ asm_val, const double2* __restrict__ aval,
    const FrontChild* __restrict__ kids, const int32_t* __restrict__ ep, int32_t* __restrict__ piv,
    int32_t* __restrict__ npert) {
  using F = Fp<R>;
  using Cx = typename F::C;
  const FrontJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x, m = J.m, c0 = blockIdx.y * kStrip;
  if (c0 >= m) return;
  const int c1 = min(m, c0 + kStrip);
  Cx* Fm = ws + J.F;
  if (blockIdx.y == 0) {
    for (int k = tid; k < J.w; k += kFW) piv[J.piv0 + k] = J.c0 + k;
    if (tid == 0) npert[blockIdx.x] = 0;
  }
  Cx* Fs = Fm + (int64_t)c0 * m;
  const int64_t cnt = (int64_t)m * (c1 - c0);
  for (int64_t e = tid; e < cnt; e += kFW) Fs[e] = F::mk(0.0, 0.0);
  __syncthreads();
  for (int64_t q = J.asm0 + tid; q < J.asm1; q += kFW) {
    const int32_t pos = asm_pos[q];
    const int col = pos / m;
    if (col >= c0 && col < c1) {
      const double2 a = aval[asm_val[q]];
      Fm[pos] = F::mk(a.x, a.y);
    }
  }
  __syncthreads();
  for (int c = J.kid0; c < J.kid1; ++c) {
    const FrontChild K = kids[c];
    const Cx* S = upd + K.upd;
    const int32_t* map = ep + K.ep;
    // the child's rows map to increasing front positions: the child columns
    // landing in this strip are one range [b0, b1)
    int lo = 0, hi = K.r;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (map[mid] < c0) lo = mid + 1; else hi = mid;
    }
    const int b0 = lo;
    hi = K.r;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (map[mid] < c1) lo = mid + 1; else hi = mid;
    }
    const int64_t ncnt = (int64_t)(lo - b0) * K.r;
    for (int64_t e = tid; e < ncnt; e += kFW) {
      const int a = (int)(e % K.r), b = b0 + (int)(e / K.r);
      Cx& f = Fm[map[a] + (int64_t)map[b] * m];
      const Cx sv = S[a + (int64_t)b * K.r];
      f.x += sv.x;
      f.y += sv.y;
    }
    __syncthreads();
  }
}

// The panel step runs on kPW threads: its column loops are latency bound.
constexpr int kPW = 1024;

template <class R>
__global__ __launch_bounds__(kPW) void split_panel_kernel(const FrontJob* __restrict__ jobs,
                                                          typename Fp<R>::C* __restrict__ ws,
                                                          int32_t* __restrict__ piv, int32_t* __restrict__ swp,
                                                          int32_t* __restrict__ npert, int k0) {
  using F = Fp<R>;
  using Cx = typename F::C;
  __shared__ double sv[kPW / 64];
  __shared__ int si[kPW / 64];
  const FrontJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x, m = J.m, w = J.w;
  if (k0 >= w) return;
  const int kb = min(kNB, w - k0);
  Cx* Fm = ws + J.F;
  int32_t* perm = piv + J.piv0;
  int32_t* sw = swp + J.piv0;
  int n_pert = 0;
  for (int k = k0; k < k0 + kb; ++k) {
    Cx* colk = Fm + (int64_t)k * m;
    double best = -1.0;
    int p = k;
    for (int i = k + tid; i < w; i += kPW) {
      const double a = hypot((double)colk[i].x, (double)colk[i].y);
      if (a > best) {
        best = a;
        p = i;
      }
    }
    wg_argmax<kPW>(best, p, sv, si);
    if (p != k) {
      if (tid < kb) {
        const int64_t j = k0 + tid;
        const Cx t = Fm[k + j * m];
        Fm[k + j * m] = Fm[p + j * m];
        Fm[p + j * m] = t;
      }
      if (tid == 0) {
        const int32_t t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
    }
    if (tid == 0) sw[k] = p;
    __syncthreads();
    if (!(best > F::kTiny * J.anorm)) {
      if (tid == 0) colk[k] = F::mk(sqrt(F::kEps) * J.anorm, 0.0);
      ++n_pert;
      __syncthreads();
    }
    const Cx d = colk[k];
    for (int i = k + 1 + tid; i < m; i += kPW) {
      const Cx l = cdivd(colk[i], d);
      colk[i] = l;
      for (int j = k + 1; j < k0 + kb; ++j) csub_mul(Fm[i + (int64_t)j * m], l, Fm[k + (int64_t)j * m]);
    }
    __syncthreads();
  }
  if (tid == 0) npert[blockIdx.x] += n_pert;
}

// The row interchanges of pivots [ks, ks + kn) composed into one
// permutation by the first wave (one map entry per lane) and applied to the
// columns [c0, c1) outside [skip0, skip1), 32 columns at a time through buf.
template <class Cx>
__device__ void apply_interchanges(Cx* Fm, int m, const int32_t* sw, int ks, int kn, int c0, int c1, int skip0,
                                   int skip1, Cx* buf) {
  __shared__ int prow[2 * kNB], psrc[2 * kNB];
  __shared__ int nperm;
  const int tid = threadIdx.x;
  if (tid < 64) {
    int key = -1, val = -1, used = 0;
    const int myp = tid < kn ? sw[ks + tid] : 0;  // all the block's pivots in one load
    for (int k = ks; k < ks + kn; ++k) {
      const int p = __shfl(myp, k - ks, 64);
      if (p == k) continue;
      int lk, lp;
      const unsigned long long mk = __ballot(key == k);
      if (mk) {
        lk = __ffsll((long long)mk) - 1;
      } else {
        lk = used++;
        if (tid == lk) key = val = k;
      }
      const unsigned long long mp = __ballot(key == p);
      if (mp) {
        lp = __ffsll((long long)mp) - 1;
      } else {
        lp = used++;
        if (tid == lp) key = val = p;
      }
      const int vk = __shfl(val, lk, 64), vp = __shfl(val, lp, 64);
      if (tid == lk) val = vp;
      if (tid == lp) val = vk;
    }
    if (tid < used) {
      prow[tid] = key;
      psrc[tid] = val;
    }
    if (tid == 0) nperm = used;
  }
  __syncthreads();
  constexpr int kCols = kNB * kChunkV / (2 * kNB);
  const int np = max(nperm, 1);
  for (int cb = c0; cb < c1; cb += kCols) {
    const int cnt = (nperm > 0 ? np : 0) * min(kCols, c1 - cb);
    for (int e = tid; e < cnt; e += kFW) {
      const int col = cb + e / np;
      if (col < skip0 || col >= skip1) buf[e] = Fm[psrc[e % np] + (int64_t)col * m];
    }
    __syncthreads();
    for (int e = tid; e < cnt; e += kFW) {
      const int col = cb + e / np;
      if (col < skip0 || col >= skip1) Fm[prow[e % np] + (int64_t)col * m] = buf[e];
    }
    __syncthreads();
  }
}

template <class R>
__global__ __launch_bounds__(kFW) void split_update_kernel(const FrontJob* __restrict__ jobs,
                                                           typename Fp<R>::C* __restrict__ ws,
                                                           const int32_t* __restrict__ swp, int k0) {
  using F = Fp<R>;
  using Cx = typename F::C;
  __shared__ Cx T[kNB * kNB];
  __shared__ Cx buf[kNB * kChunkV];
  const FrontJob J = jobs[blockIdx.x];
  const int m = J.m, w = J.w;
  if (k0 >= w) return;
  const int c0 = blockIdx.y * kStrip;
  if (c0 >= m) return;
  const int kb = min(kNB, w - k0), j0 = k0 + kb, c1 = min(m, c0 + kStrip);
  Cx* Fm = ws + J.F;
  apply_interchanges(Fm, m, swp + J.piv0, k0, kb, c0, c1, k0, j0, buf);
  if (c1 <= j0) return;
  const int js = max(c0, j0), nc = c1 - js;
  load_diag_block(Fm + k0 + (int64_t)k0 * m, m, kb, T);
  solve_cols_unit_lower(Fm + k0 + (int64_t)js * m, m, kb, nc, T, buf);
  // U12 of the strip is still in buf (one chunk: nc <= kChunkV), zero
  // beyond kb rows and nc columns
  wg_gemm_sub<R>(m - j0, nc, kb, Fm + j0 + (int64_t)k0 * m, m, buf, kNB, Fm + j0 + (int64_t)js * m, m);
}

// Entries of the solve tile starting at row r0 of a panel: forward tiles are
// min(tile_rows, m - r0) x min(w, r0 + nr), backward ones
// min(tile_rows, w - r0) x (m - r0); offset of the tile starting at row r0.
__device__ __forceinline__ int64_t fwd_tile_offset(int m, int w, int tile_rows, int r0) {
  int64_t off = 0;
  for (int t0 = 0; t0 < r0; t0 += tile_rows) {
    const int nr = min(tile_rows, m - t0);
    off += (int64_t)nr * min(w, t0 + nr);
  }
  return off;
}
__device__ __forceinline__ int64_t bwd_tile_offset(int m, int w, int tile_rows, int r0) {
  int64_t off = 0;
  for (int t0 = 0; t0 < r0; t0 += tile_rows) off += (int64_t)min(tile_rows, w - t0) * (m - t0);
  return off;
}

template <class C>
__device__ __forceinline__ void put_entry(void* dst, int64_t at, C v, int c64) {
  if (c64)
    reinterpret_cast<float2*>(dst)[at] = make_float2((float)v.x, (float)v.y);
  else
    reinterpret_cast<double2*>(dst)[at] = make_double2((double)v.x, (double)v.y);
}

// blockIdx.y < sx: row strip of X (and its Schur complement rows and forward
// tiles); otherwise column strip of Y.
template <class R>
__global__ __launch_bounds__(kFW) void split_panels_kernel(const FrontJob* __restrict__ jobs,
                                                           typename Fp<R>::C* __restrict__ ws,
                                                           typename Fp<R>::C* __restrict__ upd, int c64,
                                                           int tile_rows, int sx) {
  using F = Fp<R>;
  using Cx = typename F::C;
  __shared__ Cx T[kNB * kNB];
  __shared__ Cx buf[kNB * kChunkV];
  const FrontJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x, m = J.m, w = J.w, r = m - w;
  const Cx* Fm = ws + J.F;
  const int nblk = (w + kNB - 1) / kNB;
  if ((int)blockIdx.y < sx) {
    const int a0 = blockIdx.y * kStrip;
    if (a0 >= m) return;
    const int h = min(kStrip, m - a0);
    // Schur complement rows of this strip
    if (r > 0 && a0 + h > w) {
      Cx* S = upd + J.upd;
      const int ra = max(a0, w) - w, nra = a0 + h - w - ra;
      const int64_t cnt = (int64_t)nra * r;
      for (int64_t e = tid; e < cnt; e += kFW) {
        const int a = ra + (int)(e % nra), b = (int)(e / nra);
        S[a + (int64_t)b * r] = Fm[w + a + (int64_t)(w + b) * m];
      }
    }
    Cx* X = ws + J.X;
    for (int jb = nblk - 1; jb >= 0; --jb) {
      const int j0 = jb * kNB, kb = min(kNB, w - j0), jend = j0 + kb;
      const int64_t cnt = (int64_t)h * kb;
      for (int64_t e = tid; e < cnt; e += kFW) {
        const int i = a0 + (int)(e % h), c = j0 + (int)(e / h);
        Cx v;
        if (i < j0)
          v = F::mk(0.0, 0.0);
        else if (i < w)
          v = F::mk(i == c ? 1.0 : 0.0, 0.0);
        else
          v = Fm[i + (int64_t)c * m];
        X[i + (int64_t)c * m] = v;
      }
      __syncthreads();
      if (a0 + h <= j0) continue;  // rows above the block: zero
      if (jend < w)
        wg_gemm_sub<R, 1, 2>(h, kb, w - jend, X + a0 + (int64_t)jend * m, m, Fm + jend + (int64_t)j0 * m, m,
                             X + a0 + (int64_t)j0 * m, m);
      load_diag_block(Fm + j0 + (int64_t)j0 * m, m, kb, T);
      solve_rows_right_unit_lower(X + a0 + (int64_t)j0 * m, m, kb, h, T, buf);
    }
    // forward tiles of the strip's rows
    for (int r0 = a0; r0 < a0 + h; r0 += tile_rows) {
      const int nr = min(tile_rows, m - r0), nc = min(w, r0 + nr);
      const int64_t off = J.pfo + fwd_tile_offset(m, w, tile_rows, r0);
      const int64_t cnt = (int64_t)nr * nc;
      for (int64_t e = tid; e < cnt; e += kFW) {
        const int i = (int)(e % nr), col = (int)(e / nr), row = r0 + i;
        put_entry(J.pf, off + e, (row < w && col > row) ? F::mk(0.0, 0.0) : X[row + (int64_t)col * m], c64);
      }
    }
  } else {
    const int cs = (blockIdx.y - sx) * kStrip;
    if (cs >= m) return;
    const int nc = min(kStrip, m - cs);
    Cx* Y = ws + J.Y;
    for (int ib = nblk - 1; ib >= 0; --ib) {
      const int i0 = ib * kNB, kb = min(kNB, w - i0), iend = i0 + kb;
      const int64_t cnt = (int64_t)kb * nc;
      for (int64_t e = tid; e < cnt; e += kFW) {
        const int q = (int)(e % kb), c = cs + (int)(e / kb), row = i0 + q;
        Cx v;
        if (c < w) {
          v = F::mk(row == c ? 1.0 : 0.0, 0.0);
        } else {
          const Cx u = Fm[row + (int64_t)c * m];
          v.x = -u.x;
          v.y = -u.y;
        }
        Y[row + (int64_t)c * w] = v;
      }
      __syncthreads();
      if (cs + nc <= i0) continue;  // columns left of the block: zero
      if (iend < w)
        wg_gemm_sub<R, 2, 1>(kb, nc, w - iend, Fm + i0 + (int64_t)iend * m, m, Y + iend + (int64_t)cs * w, w,
                             Y + i0 + (int64_t)cs * w, w);
      load_diag_block(Fm + i0 + (int64_t)i0 * m, m, kb, T);
      solve_cols_upper(Y + i0 + (int64_t)cs * w, w, kb, nc, T, buf);
    }
  }
}

template <class R>
__global__ __launch_bounds__(kFW) void split_ytiles_kernel(const FrontJob* __restrict__ jobs,
                                                           const typename Fp<R>::C* __restrict__ ws,
                                                           int c64, int tile_rows) {
  using F = Fp<R>;
  using Cx = typename F::C;
  const FrontJob J = jobs[blockIdx.x];
  const int m = J.m, w = J.w, r0 = blockIdx.y * tile_rows;
  if (r0 >= w) return;
  const Cx* Y = ws + J.Y;
  const int nr = min(tile_rows, w - r0), ncol = m - r0;
  const int64_t off = J.pbo + bwd_tile_offset(m, w, tile_rows, r0);
  const int64_t cnt = (int64_t)nr * ncol;
  for (int64_t e = threadIdx.x; e < cnt; e += kFW) {
    const int i = (int)(e % nr), row = r0 + i, col = r0 + (int)(e / nr);
    put_entry(J.pb, off + e, (col < w && col < row) ? F::mk(0.0, 0.0) : Y[row + (int64_t)col * w], c64);
  }
}

template <class R>
void split_launch(const FrontJob* jobs, int njobs, int mmax, int wmax, void* ws, void* upd, const int32_t* asm_pos,
                  const int32_t* asm_val, const double2* aval, const FrontChild* kids, const int32_t* ep,
                  int32_t* piv, int32_t* swp, int32_t* npert, int c64, int tile_rows,
                  hipStream_t s) {
  using Cx = typename Fp<R>::C;
  Cx* W = reinterpret_cast<Cx*>(ws);
  Cx* U = reinterpret_cast<Cx*>(upd);
  const unsigned ns = (unsigned)((mmax + kStrip - 1) / kStrip);
  split_assemble_kernel<R><<<dim3(njobs, ns), kFW, 0, s>>>(jobs, W, U, asm_pos, asm_val, aval, kids, ep, piv, npert);
  for (int k0 = 0; k0 < wmax; k0 += kNB) {
    split_panel_kernel<R><<<njobs, kPW, 0, s>>>(jobs, W, piv, swp, npert, k0);
    split_update_kernel<R><<<dim3(njobs, ns), kFW, 0, s>>>(jobs, W, swp, k0);
  }
  split_panels_kernel<R><<<dim3(njobs, 2 * ns), kFW, 0, s>>>(jobs, W, U, c64, tile_rows, (int)ns);
  split_ytiles_kernel<R><<<dim3(njobs, (unsigned)((wmax + tile_rows - 1) / tile_rows)), kFW, 0, s>>>(jobs, W, c64,
                                                                                                     tile_rows);
}

}  // namespace

void factor_fronts(const FrontJob* jobs, int njobs, void* ws, void* upd, const int32_t* asm_pos,
                   const int32_t* asm_val, const double* aval, const FrontChild* kids, const int32_t* ep,
                   int32_t* piv, int32_t* npert, FactorPrecision prec, int tile_rows,
                   hipStream_t s) {
  if (njobs <= 0) return;
  const double2* a = reinterpret_cast<const double2*>(aval);
  if (prec == FactorPrecision::kC64) {
    front_kernel<float><<<(unsigned)njobs, kFW, 0, s>>>(jobs, reinterpret_cast<float2*>(ws),
                                                        reinterpret_cast<float2*>(upd), asm_pos, asm_val, a, kids, ep,
                                                        piv, npert, 1, tile_rows);
  } else {
    front_kernel<double><<<(unsigned)njobs, kFW, 0, s>>>(
        jobs, reinterpret_cast<double2*>(ws), reinterpret_cast<double2*>(upd), asm_pos, asm_val, a, kids, ep, piv,
        npert, prec == FactorPrecision::kC128RoundedC64 ? 1 : 0, tile_rows);
  }
}

void factor_fronts_split(const FrontJob* jobs, int njobs, int mmax, int wmax, void* ws, void* upd,
                         const int32_t* asm_pos, const int32_t* asm_val, const double* aval, const FrontChild* kids,
                         const int32_t* ep, int32_t* piv, int32_t* swp, int32_t* npert,
                         FactorPrecision prec, int tile_rows, hipStream_t s) {
  if (njobs <= 0) return;
  const double2* a = reinterpret_cast<const double2*>(aval);
  if (prec == FactorPrecision::kC64)
    split_launch<float>(jobs, njobs, mmax, wmax, ws, upd, asm_pos, asm_val, a, kids, ep, piv, swp, npert, 1,
                        tile_rows, s);
  else
    split_launch<double>(jobs, njobs, mmax, wmax, ws, upd, asm_pos, asm_val, a, kids, ep, piv, swp, npert,
                         prec == FactorPrecision::kC128RoundedC64 ? 1 : 0, tile_rows, s);
}

}  // namespace dev
}  // namespace helm
