// Block Gram-Schmidt of block GMRES on MFMA (gfx950).
//
// A block is n x 16 complex, interleaved: entry (i, c) at i * 16 + c, the
// layout of the preconditioner's multi-right-hand-side vectors.  The Krylov
// basis is a sequence of such blocks V_0, V_1, ... (block-major).  The work
// of one block Arnoldi step is a handful of tall-skinny contractions:
//
//   dots:   P_j = V_j^H W            (16 x 16 per basis block, reduction over
//                                     the n rows: per-workgroup partial sums,
//                                     then a fixed-order reduction)
//   mul:    Y = Y0 +- sum_j X_j C_j  (rows times 16 x 16 coefficient blocks;
//                                     optionally the Gram matrix Y^H Y of the
//                                     result in the same pass)
//   chol16: G = L L^H of a 16 x 16 Gram matrix, R = L^H and T = L^{-H}
//
// all on v_mfma_f64_16x16x4f64, the complex products split into four real
// MFMAs.  Operand layout of that instruction: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator register q of lane l is
// D[4 q + l / 16][l % 16].
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace helm {
namespace dev {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dv4 mma(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kWaves = 4;   // waves per workgroup
constexpr int kBPW = 4;     // basis blocks per wave in bgs_dots
constexpr int kJG = kWaves * kBPW;  // basis blocks per dots workgroup (grid y splits the rest)

// Waves per group of kBPW basis blocks in bgs_dots: with fewer than three
// groups (nbt <= 8) the waves of a workgroup split the group's row tiles
// (four or two per group) instead of idling.
__host__ __device__ inline int bgs_wpg(int nbt) {
  const int g = (nbt + kBPW - 1) / kBPW;
  return g == 1 ? kWaves : (g == 2 ? kWaves / 2 : 1);
}

// dots: partial[(p * nbt + jb) * 256 + a * 16 + c] = sum over the rows of
// partial row p of conj(X_jb[row][a]) W[row][c].  With nbt <= 8, block
// group g (blocks 4 g .. 4 g + 3) is taken by bgs_wpg(nbt) waves; wave sub
// of them walks the 16-row tiles blockIdx.x * wpg + sub, stepping by
// gridDim.x * wpg, and writes partial row p = blockIdx.x * wpg + sub (so
// gridDim.x * wpg partial rows in all).  Otherwise grid y cuts the blocks
// into gridDim.y slices of at most 16 consecutive blocks, as equal as
// possible, dealt in turn to the four waves of a workgroup, which walk the
// same tiles (W fetched from HBM once, read from cache by the others).
// X_jb = X + jb * ldx for jb < nb, and block nb (with_w) is W itself (its
// Gram matrix).  All operands of a tile are loaded before its MFMAs, which
// run with the blocks innermost.
__global__ __launch_bounds__(64 * kWaves, 3) void bgs_dots_kernel(int64_t n, const double2* __restrict__ X, int64_t ldx,
                                                                int nb, int with_w, const double2* __restrict__ W,
                                                                double2* __restrict__ partial) {
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nbt = nb + with_w;
  const int wpg = bgs_wpg(nbt), sub = wv % wpg;
  // blocks of this wave: jb = jb0 + q jst, q < njb
  int jb0, jst, njb;
  if (wpg > 1) {
    jb0 = (wv / wpg) * kBPW;
    jst = 1;
    njb = min(kBPW, nbt - jb0);
  } else {
    // gridDim.y slices of consecutive blocks, as equal as possible; the
    // blocks of a slice dealt to its four waves in turn
    const int y = blockIdx.y, ny = gridDim.y;
    const int s0 = (int)((int64_t)nbt * y / ny), s1 = (int)((int64_t)nbt * (y + 1) / ny);
    jb0 = s0 + wv;
    jst = kWaves;
    njb = jb0 < s1 ? (s1 - jb0 + kWaves - 1) / kWaves : 0;
  }
  if (njb <= 0) return;  // whole wave; no barrier in this kernel
  dv4 dre[kBPW], dim[kBPW];
#pragma unroll
  for (int q = 0; q < kBPW; ++q) dre[q] = dim[q] = dv4{0, 0, 0, 0};
  const double2* Xq[kBPW];
#pragma unroll
  for (int q = 0; q < kBPW; ++q) {
    const int jb = jb0 + q * jst;
    Xq[q] = jb < nb ? X + jb * ldx : W;
  }
  const int64_t ntiles = (n + 15) >> 4;
  // lane l takes row 4 t + l / 16 of the tile at k-step t, column l % 16
  const int rk = lane >> 4, col = lane & 15;
  const int64_t prow = (int64_t)blockIdx.x * wpg + sub;
  for (int64_t tile = prow; tile < ntiles; tile += (int64_t)gridDim.x * wpg) {
    const int64_t i0 = tile << 4;
    double2 w[4], v[4][kBPW];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t row = i0 + 4 * t + rk;
      const bool in = row < n;
      w[t] = in ? W[row * 16 + col] : make_double2(0, 0);
#pragma unroll
      for (int q = 0; q < kBPW; ++q) v[t][q] = (q < njb && in) ? Xq[q][row * 16 + col] : make_double2(0, 0);
    }
    // conj(v) w: re = vr wr + vi wi, im = vr wi - vi wr
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int q = 0; q < kBPW; ++q) dre[q] = mma(v[t][q].x, w[t].x, dre[q]);
#pragma unroll
      for (int q = 0; q < kBPW; ++q) dim[q] = mma(v[t][q].x, w[t].y, dim[q]);
#pragma unroll
      for (int q = 0; q < kBPW; ++q) dre[q] = mma(v[t][q].y, w[t].y, dre[q]);
#pragma unroll
      for (int q = 0; q < kBPW; ++q) dim[q] = mma(-v[t][q].y, w[t].x, dim[q]);
    }
  }
  // register r of lane l holds entry (4 r + l / 16, l % 16) of each block
#pragma unroll
  for (int q = 0; q < kBPW; ++q) {
    if (q >= njb) break;
    double2* out = partial + (prow * nbt + jb0 + q * jst) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(4 * r + rk) * 16 + col] = make_double2(dre[q][r], dim[q][r]);
  }
}

// out[jb * 256 + e] = sum_wg partial[(wg * nbt + jb) * 256 + e]; acc (may be
// null) receives the sum too (+= when accumulate).  Sixteen threads per
// output sum the workgroups wg = u mod 16 in order, then the sixteen sums are
// added in a fixed order, so the result is bitwise repeatable.
constexpr int kRedT = 16;
__global__ __launch_bounds__(256) void bgs_reduce_kernel(const double2* __restrict__ partial, int nwg, int nbt,
                                                         double2* __restrict__ out, double2* __restrict__ acc,
                                                         int accumulate) {
  __shared__ double2 part[kRedT][256 / kRedT];
  constexpr int kOut = 256 / kRedT;  // outputs per block
  const int u = threadIdx.x / kOut, o = threadIdx.x % kOut;
  const int64_t e = (int64_t)blockIdx.x * kOut + o;
  const int64_t ne = (int64_t)nbt * 256;
  double sr = 0, si = 0;
  if (e < ne) {
    int wg = u;
    for (; wg + 3 * kRedT < nwg; wg += 4 * kRedT) {
      const double2 p0 = partial[(int64_t)wg * ne + e];
      const double2 p1 = partial[(int64_t)(wg + kRedT) * ne + e];
      const double2 p2 = partial[(int64_t)(wg + 2 * kRedT) * ne + e];
      const double2 p3 = partial[(int64_t)(wg + 3 * kRedT) * ne + e];
      sr += p0.x;
      si += p0.y;
      sr += p1.x;
      si += p1.y;
      sr += p2.x;
      si += p2.y;
      sr += p3.x;
      si += p3.y;
    }
    for (; wg < nwg; wg += kRedT) {
      const double2 p = partial[(int64_t)wg * ne + e];
      sr += p.x;
      si += p.y;
    }
  }
  part[u][o] = make_double2(sr, si);
  __syncthreads();
  if (u != 0 || e >= ne) return;
  sr = 0;
  si = 0;
  for (int k = 0; k < kRedT; ++k) {
    sr += part[k][o].x;
    si += part[k][o].y;
  }
  if (out) out[e] = make_double2(sr, si);
  if (acc) {
    if (accumulate) {
      const double2 a = acc[e];
      acc[e] = make_double2(a.x + sr, a.y + si);
    } else {
      acc[e] = make_double2(sr, si);
    }
  }
}

constexpr int kMulTiles = 2;  // 16-row tiles per wave in bgs_mul

// Y = (Y0 or 0) + sign * sum_{jb < nb} X_jb C_jb over 16-row tiles, C_jb =
// C + 256 jb (16 x 16, entry (a, c) at a * 16 + c); with gram, the
// workgroup's partial sum of Y^H Y goes to gram[blockIdx.x * 256 + ...].
// Y may alias Y0 and X (each wave reads its own rows before it writes them;
// rows past n, never stored, read row n - 1).  The operands of block jb + 1
// are loaded, into the other of two register sets, before the MFMAs of
// block jb; a step past nb meets zero coefficients.
__global__ __launch_bounds__(64 * kWaves, 3) void bgs_mul_kernel(int64_t n, const double2* X, int64_t ldx,
                                                                  int nb, const double2* __restrict__ C, double sign,
                                                                  const double2* Y0, double2* Y,
                                                                  double2* __restrict__ gram) {
  __shared__ double2 red[kWaves][256];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rk = lane >> 4, col = lane & 15;
  const int64_t base = ((int64_t)blockIdx.x * kWaves + wv) * kMulTiles * 16;
  dv4 dre[kMulTiles], dim[kMulTiles];
  // accumulators start from Y0 (all loads issued before the first use):
  // register q of lane l is row 4 q + l / 16
  // (without Y0 the loads read Y, any valid rows, and are replaced by zeros)
  const double2* ysrc = Y0 ? Y0 : Y;
  const double keep = Y0 ? 1.0 : 0.0;
  double2 y[kMulTiles][4];
#pragma unroll
  for (int tt = 0; tt < kMulTiles; ++tt)
#pragma unroll
    for (int q = 0; q < 4; ++q) y[tt][q] = ysrc[min(base + 16 * tt + 4 * q + rk, n - 1) * 16 + col];
#pragma unroll
  for (int tt = 0; tt < kMulTiles; ++tt)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dre[tt][q] = keep != 0.0 ? y[tt][q].x : 0.0;
      dim[tt][q] = keep != 0.0 ? y[tt][q].y : 0.0;
    }
  if (nb > 0) {
    // A operand at k-step t: X_jb[row l % 16][column 4 t + l / 16] (the four
    // lanes of a row read 64 contiguous bytes); B operand: C_jb[4 t + l / 16]
    // [l % 16]
    int64_t arow[kMulTiles];
#pragma unroll
    for (int tt = 0; tt < kMulTiles; ++tt) arow[tt] = min(base + 16 * tt + col, n - 1) * 16 + rk;
    auto load = [&](int jb, double2 (&cb)[4], double2 (&a)[kMulTiles][4]) {
      const int j = min(jb, nb - 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) cb[t] = C[j * 256 + (4 * t + rk) * 16 + col];
      const double2* Xj = X + j * ldx;
#pragma unroll
      for (int tt = 0; tt < kMulTiles; ++tt)
#pragma unroll
        for (int t = 0; t < 4; ++t) a[tt][t] = Xj[arow[tt] + 4 * t];
    };
    auto step = [&](int jb, const double2 (&c)[4], const double2 (&a)[kMulTiles][4]) {
      const bool on = jb < nb;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 cb = on ? c[t] : make_double2(0, 0);
        // (ar + i ai)(cr + i ci), a scaled by sign
#pragma unroll
        for (int tt = 0; tt < kMulTiles; ++tt) dre[tt] = mma(sign * a[tt][t].x, cb.x, dre[tt]);
#pragma unroll
        for (int tt = 0; tt < kMulTiles; ++tt) dim[tt] = mma(sign * a[tt][t].x, cb.y, dim[tt]);
#pragma unroll
        for (int tt = 0; tt < kMulTiles; ++tt) dre[tt] = mma(-sign * a[tt][t].y, cb.y, dre[tt]);
#pragma unroll
        for (int tt = 0; tt < kMulTiles; ++tt) dim[tt] = mma(sign * a[tt][t].y, cb.x, dim[tt]);
      }
    };
    double2 c0[4], a0[kMulTiles][4], c1[4], a1[kMulTiles][4];
    load(0, c0, a0);
    for (int jb = 0; jb < nb; jb += 2) {
      load(jb + 1, c1, a1);
      __builtin_amdgcn_sched_barrier(0);
      step(jb, c0, a0);
      __builtin_amdgcn_sched_barrier(0);
      load(jb + 2, c0, a0);
      __builtin_amdgcn_sched_barrier(0);
      step(jb + 1, c1, a1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  dv4 gre = dv4{0, 0, 0, 0}, gim = dv4{0, 0, 0, 0};
#pragma unroll
  for (int tt = 0; tt < kMulTiles; ++tt) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = base + 16 * tt + 4 * q + rk;
      if (row < n) Y[row * 16 + col] = make_double2(dre[tt][q], dim[tt][q]);
    }
    if (gram) {
      // register q of lane l holds Y[row 4 q + l / 16][l % 16]: the A and B
      // operands of Y^H Y at k-step q (rows past n taken as zeros)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool in = base + 16 * tt + 4 * q + rk < n;
        const double yr = in ? dre[tt][q] : 0.0, yi = in ? dim[tt][q] : 0.0;
        gre = mma(yr, yr, gre);
        gre = mma(yi, yi, gre);
        gim = mma(yr, yi, gim);
        gim = mma(-yi, yr, gim);
      }
    }
  }
  if (gram) {
#pragma unroll
    for (int r = 0; r < 4; ++r) red[wv][(4 * r + rk) * 16 + col] = make_double2(gre[r], gim[r]);
    __syncthreads();
    for (int e = threadIdx.x; e < 256; e += 64 * kWaves) {
      double2 s = red[0][e];
#pragma unroll
      for (int u = 1; u < kWaves; ++u) {
        s.x += red[u][e].x;
        s.y += red[u][e].y;
      }
      gram[(int64_t)blockIdx.x * 256 + e] = s;
    }
  }
}

// Cholesky of the leading s x s part of a Hermitian 16 x 16 matrix G
// (entry (a, c) at a * 16 + c): G = L L^H.  Writes R = L^H and T = L^{-H}
// (16 x 16, zero outside the leading s x s part) and status[0] = 0, or 1 + k
// when pivot k is not above tiny * scale, scale = max_k ref[k * 17] (ref:
// the Gram matrix the columns are measured against; null: 1).  One wave:
// at step k lane i < s computes L[i][k]; the inverse is formed a column per
// lane.
__global__ __launch_bounds__(64) void chol16_kernel(const double2* __restrict__ G, int s, const double2* __restrict__ ref,
                                                    double tiny, double2* __restrict__ R, double2* __restrict__ T,
                                                    int* __restrict__ status) {
  __shared__ double2 L[16][17], Li[16][17];
  __shared__ int st_s;
  const int lane = threadIdx.x;
  for (int e = lane; e < 256; e += 64) {
    L[e / 16][e % 16] = make_double2(0, 0);
    Li[e / 16][e % 16] = make_double2(0, 0);
  }
  double scale = 1.0;
  if (ref) {
    scale = 0;
    for (int k = 0; k < s; ++k) scale = fmax(scale, ref[k * 17].x);
  }
  if (lane == 0) st_s = 0;
  __syncthreads();
  for (int k = 0; k < s; ++k) {
    if (lane == 0) {
      double d = G[k * 17].x;
      for (int j = 0; j < k; ++j) d -= L[k][j].x * L[k][j].x + L[k][j].y * L[k][j].y;
      if (!(d > tiny * scale)) {
        st_s = 1 + k;
        d = 1.0;  // keeps the arithmetic finite; the status marks the failure
      }
      L[k][k] = make_double2(sqrt(d), 0);
    }
    __syncthreads();
    if (st_s) break;
    const int i = lane;
    if (i > k && i < s) {
      // L[i][k] = (G[i][k] - sum_j L[i][j] conj(L[k][j])) / L[k][k]
      double xr = G[i * 16 + k].x, xi = G[i * 16 + k].y;
      for (int j = 0; j < k; ++j) {
        const double2 p = L[i][j], q = L[k][j];
        xr -= p.x * q.x + p.y * q.y;
        xi -= p.y * q.x - p.x * q.y;
      }
      const double lkk = L[k][k].x;
      L[i][k] = make_double2(xr / lkk, xi / lkk);
    }
    __syncthreads();
  }
  const int st = st_s;
  if (!st && lane < s) {
    // column c = lane of L^{-1}: forward substitution
    const int c = lane;
    Li[c][c] = make_double2(1.0 / L[c][c].x, 0);
    for (int i = c + 1; i < s; ++i) {
      double xr = 0, xi = 0;
      for (int j = c; j < i; ++j) {
        const double2 p = L[i][j], q = Li[j][c];
        xr -= p.x * q.x - p.y * q.y;
        xi -= p.x * q.y + p.y * q.x;
      }
      Li[i][c] = make_double2(xr / L[i][i].x, xi / L[i][i].x);
    }
  }
  __syncthreads();
  for (int e = lane; e < 256; e += 64) {
    const int a = e / 16, c = e % 16;
    // R = L^H: R[a][c] = conj(L[c][a]); T = L^{-H}: T[a][c] = conj(Li[c][a])
    R[e] = make_double2(L[c][a].x, -L[c][a].y);
    T[e] = st ? make_double2(0, 0) : make_double2(Li[c][a].x, -Li[c][a].y);
  }
  if (lane == 0) status[0] = st;
}

}  // namespace

int bgs_wgs(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  // two workgroups per CU per group of basis blocks (grid y adds more),
  // each walking at least a few tiles
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles / 4, 512));
}

int bgs_mul_wgs(int64_t n) { return (int)((n + 16 * kMulTiles * kWaves - 1) / (16 * kMulTiles * kWaves)); }

int bgs_dots(int64_t n, const double* X, int64_t ldx, int nb, bool with_w, const double* W, double* partial,
             hipStream_t s) {
  const int nbt = nb + (with_w ? 1 : 0);
  if (nbt <= 0) return 0;
  const int wpg = bgs_wpg(nbt);
  dim3 grid(bgs_wgs(n), wpg > 1 ? 1 : (nbt + kJG - 1) / kJG);
  bgs_dots_kernel<<<grid, 64 * kWaves, 0, s>>>(n, reinterpret_cast<const double2*>(X), ldx / 2, nb, with_w ? 1 : 0,
                                                reinterpret_cast<const double2*>(W),
                                                reinterpret_cast<double2*>(partial));
  return (int)grid.x * wpg;
}

void bgs_reduce(const double* partial, int nwg, int nbt, double* out, double* acc, bool accumulate, hipStream_t s) {
  const int64_t m = (int64_t)nbt * 256;
  bgs_reduce_kernel<<<(int)((m + 15) / 16), 256, 0, s>>>(reinterpret_cast<const double2*>(partial), nwg, nbt,
                                                             reinterpret_cast<double2*>(out),
                                                             reinterpret_cast<double2*>(acc), accumulate ? 1 : 0);
}

void bgs_mul(int64_t n, const double* X, int64_t ldx, int nb, const double* C, double sign, const double* Y0,
             double* Y, double* gram, hipStream_t s) {
  bgs_mul_kernel<<<bgs_mul_wgs(n), 64 * kWaves, 0, s>>>(
      n, reinterpret_cast<const double2*>(X), ldx / 2, nb, reinterpret_cast<const double2*>(C), sign,
      reinterpret_cast<const double2*>(Y0), reinterpret_cast<double2*>(Y), reinterpret_cast<double2*>(gram));
}

void chol16(const double* G, int s_act, const double* ref, double tiny, double* R, double* T, int* status,
            hipStream_t s) {
  chol16_kernel<<<1, 64, 0, s>>>(reinterpret_cast<const double2*>(G), s_act, reinterpret_cast<const double2*>(ref),
                                 tiny, reinterpret_cast<double2*>(R), reinterpret_cast<double2*>(T), status);
}

}  // namespace dev
}  // namespace helm
