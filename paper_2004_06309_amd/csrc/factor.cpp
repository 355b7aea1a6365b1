// Multifrontal numeric LU of a local matrix (the local direct solvers of the
// ORAS preconditioner, eq. oras) and its conversion to the solve layout.
//
// Each supernode s assembles its frontal matrix F (order w + r: its own
// columns, then the rows R_s), adds the children's contribution blocks,
// eliminates its w fully-summed columns with partial pivoting restricted to
// the fully-summed rows (P F11 = L11 U11, L21 = F21 U11^{-1},
// U12 = L11^{-1} P F12) and passes the Schur complement F22 - L21 U12 up.
//
// The triangular solves are then written as dense products with explicit
// inverses ("partitioned inverse" form), so each supernode of the forward and
// backward solves is a single matrix-vector product over its panel:
//   forward  [y_s; u_s] = [L11^{-1}; L21 L11^{-1}] P (b_s - updates)
//   backward x_s = [U11^{-1} | -U11^{-1} U12] [y_s; x(R_s)]
// The panels are stored in tiles of up to 64 rows, column-major inside a tile.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>

#include "device.hpp"
#include "internal.hpp"

namespace helm {

namespace {

// C[M x N] += alpha * A[M x K] * B[K x N]   (column-major, complex)
void gemm_acc(int M, int N, int K, cplx alpha, const cplx* A, int64_t lda, const cplx* B, int64_t ldb, cplx* C,
              int64_t ldc) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  const double* Ad = reinterpret_cast<const double*>(A);
  for (int j = 0; j < N; ++j) {
    double* c = reinterpret_cast<double*>(C + (int64_t)j * ldc);
    int k = 0;
    for (; k + 1 < K; k += 2) {
      cplx b0 = alpha * B[k + (int64_t)j * ldb], b1 = alpha * B[k + 1 + (int64_t)j * ldb];
      const double* a0 = Ad + 2 * (int64_t)k * lda;
      const double* a1 = Ad + 2 * (int64_t)(k + 1) * lda;
      const double b0r = b0.real(), b0i = b0.imag(), b1r = b1.real(), b1i = b1.imag();
      if (b0r == 0 && b0i == 0 && b1r == 0 && b1i == 0) continue;
#pragma omp simd
      for (int i = 0; i < M; ++i) {
        double ar0 = a0[2 * i], ai0 = a0[2 * i + 1], ar1 = a1[2 * i], ai1 = a1[2 * i + 1];
        c[2 * i] += ar0 * b0r - ai0 * b0i + ar1 * b1r - ai1 * b1i;
        c[2 * i + 1] += ar0 * b0i + ai0 * b0r + ar1 * b1i + ai1 * b1r;
      }
    }
    for (; k < K; ++k) {
      cplx b0 = alpha * B[k + (int64_t)j * ldb];
      const double* a0 = Ad + 2 * (int64_t)k * lda;
      const double b0r = b0.real(), b0i = b0.imag();
#pragma omp simd
      for (int i = 0; i < M; ++i) {
        double ar0 = a0[2 * i], ai0 = a0[2 * i + 1];
        c[2 * i] += ar0 * b0r - ai0 * b0i;
        c[2 * i + 1] += ar0 * b0i + ai0 * b0r;
      }
    }
  }
}

inline cplx cdiv(cplx a, cplx b) {
  double d = b.real() * b.real() + b.imag() * b.imag();
  return cplx((a.real() * b.real() + a.imag() * b.imag()) / d, (a.imag() * b.real() - a.real() * b.imag()) / d);
}

// Blocked right-looking partial LU of the first w columns of the m x m front
// F (ld = m); pivot rows are searched among rows [k, w) only.
void partial_lu(cplx* F, int m, int w, int32_t* piv, double anorm, int32_t& n_pert) {
  const int nb = 32;
  for (int k = 0; k < w; ++k) piv[k] = k;
  for (int k0 = 0; k0 < w; k0 += nb) {
    int kb = std::min(nb, w - k0);
    for (int k = k0; k < k0 + kb; ++k) {
      cplx* colk = F + (int64_t)k * m;
      int p = k;
      double best = std::abs(colk[k]);
      for (int i = k + 1; i < w; ++i) {
        double a = std::abs(colk[i]);
        if (a > best) {
          best = a;
          p = i;
        }
      }
      if (p != k) {
        for (int j = 0; j < m; ++j) std::swap(F[k + (int64_t)j * m], F[p + (int64_t)j * m]);
        std::swap(piv[k], piv[p]);
      }
      if (!(best > dev::kTinyPivot * anorm)) {
        if (!(anorm > 0)) fail(HELM_ESINGULAR, "zero pivot in a frontal matrix");
        colk[k] = cplx(std::sqrt(std::numeric_limits<double>::epsilon()) * anorm, 0.0);
        ++n_pert;
      }
      cplx d = colk[k];
      for (int i = k + 1; i < m; ++i) colk[i] = cdiv(colk[i], d);
      // update the remaining columns of the panel
      for (int j = k + 1; j < k0 + kb; ++j) {
        cplx f = F[k + (int64_t)j * m];
        if (f == cplx(0, 0)) continue;
        cplx* cj = F + (int64_t)j * m;
        for (int i = k + 1; i < m; ++i) cj[i] -= colk[i] * f;
      }
    }
    int j0 = k0 + kb;
    if (j0 >= m) continue;
    // U12 rows of this panel: forward substitution with the unit-lower panel
    for (int j = j0; j < m; ++j) {
      cplx* cj = F + (int64_t)j * m;
      for (int k = k0; k < k0 + kb; ++k) {
        cplx f = cj[k];
        if (f == cplx(0, 0)) continue;
        const cplx* ck = F + (int64_t)k * m;
        for (int i = k + 1; i < k0 + kb; ++i) cj[i] -= ck[i] * f;
      }
    }
    // trailing update
    gemm_acc(m - j0, m - j0, kb, cplx(-1, 0), F + j0 + (int64_t)k0 * m, m, F + k0 + (int64_t)j0 * m, m,
             F + j0 + (int64_t)j0 * m, m);
  }
}

}  // namespace

void factor_numeric(const Csr& A, const Symbolic& S, cplx* fwd, cplx* bwd, NumericOut& out) {
  const int64_t n = A.n;
  const int32_t nsn = S.nsn;
  out.piv.assign(n, 0);
  out.n_perturbed = 0;
  // transpose for the column part of the assembly
  std::vector<int64_t> tptr(n + 1, 0);
  for (int64_t p = 0; p < A.nnz(); ++p) tptr[A.col[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  std::vector<int32_t> trow(A.nnz());
  std::vector<cplx> tval(A.nnz());
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        int64_t q = fill[A.col[p]]++;
        trow[q] = (int32_t)i;
        tval[q] = A.val[p];
      }
  }
  double anorm = 0;
  for (int64_t p = 0; p < A.nnz(); ++p) anorm = std::max(anorm, std::abs(A.val[p]));

  std::vector<int32_t> fpos(n, -1);
  std::vector<std::unique_ptr<cplx[]>> cb(nsn);  // contribution blocks awaiting their parent
  std::vector<std::vector<int32_t>> children(nsn);
  for (int32_t s = 0; s < nsn; ++s)
    if (S.sn_parent[s] >= 0) children[S.sn_parent[s]].push_back(s);
  std::vector<TileShape> ts;
  std::vector<cplx> F, Linv, Loff, Uinv, Uoff;
  std::vector<int32_t> piv;

  for (int32_t s = 0; s < nsn; ++s) {
    const int32_t c0 = S.sn_c0[s], w = S.sn_w[s];
    const int32_t c1 = c0 + w;
    const int32_t* R = S.rows.data() + S.sn_rptr[s];
    const int32_t r = (int32_t)(S.sn_rptr[s + 1] - S.sn_rptr[s]);
    const int32_t m = w + r;
    for (int32_t k = 0; k < w; ++k) fpos[c0 + k] = k;
    for (int32_t a = 0; a < r; ++a) fpos[R[a]] = w + a;
    F.assign((size_t)m * m, cplx(0, 0));
    // original entries with min(row, col) in C_s
    for (int32_t j = c0; j < c1; ++j) {
      int32_t old = S.perm[j];
      for (int64_t p = A.ptr[old]; p < A.ptr[old + 1]; ++p) {
        int32_t nc = S.iperm[A.col[p]];
        if (nc >= c0) F[fpos[j] + (int64_t)fpos[nc] * m] += A.val[p];
      }
      for (int64_t p = tptr[old]; p < tptr[old + 1]; ++p) {
        int32_t nr = S.iperm[trow[p]];
        if (nr >= c1) F[fpos[nr] + (int64_t)fpos[j] * m] += tval[p];
      }
    }
    // extend-add the children's contribution blocks
    for (int32_t c : children[s]) {
      const int32_t* Rc = S.rows.data() + S.sn_rptr[c];
      const int32_t rc = (int32_t)(S.sn_rptr[c + 1] - S.sn_rptr[c]);
      const cplx* C = cb[c].get();
      std::vector<int32_t> map(rc);
      for (int32_t a = 0; a < rc; ++a) map[a] = fpos[Rc[a]];
      for (int32_t b = 0; b < rc; ++b) {
        cplx* Fc = F.data() + (int64_t)map[b] * m;
        const cplx* Cc = C + (int64_t)b * rc;
        for (int32_t a = 0; a < rc; ++a) Fc[map[a]] += Cc[a];
      }
      cb[c].reset();
    }
    piv.resize(w);
    partial_lu(F.data(), m, w, piv.data(), anorm, out.n_perturbed);
    for (int32_t k = 0; k < w; ++k) out.piv[c0 + k] = c0 + piv[k];
    if (r > 0) {
      cb[s].reset(new cplx[(size_t)r * r]);
      for (int32_t b = 0; b < r; ++b)
        std::memcpy(cb[s].get() + (int64_t)b * r, F.data() + w + (int64_t)(w + b) * m, sizeof(cplx) * r);
    }
    // explicit inverses of the diagonal factors
    Linv.assign((size_t)w * w, cplx(0, 0));
    for (int32_t j = 0; j < w; ++j) {
      cplx* x = Linv.data() + (int64_t)j * w;
      x[j] = 1.0;
      for (int32_t k = j; k < w; ++k) {
        cplx xk = x[k];
        if (xk == cplx(0, 0)) continue;
        const cplx* lk = F.data() + (int64_t)k * m;
        for (int32_t i = k + 1; i < w; ++i) x[i] -= lk[i] * xk;
      }
    }
    Uinv.assign((size_t)w * w, cplx(0, 0));
    for (int32_t j = 0; j < w; ++j) {
      cplx* x = Uinv.data() + (int64_t)j * w;
      x[j] = 1.0;
      for (int32_t k = j; k >= 0; --k) {
        x[k] = cdiv(x[k], F[k + (int64_t)k * m]);
        cplx xk = x[k];
        if (xk == cplx(0, 0)) continue;
        const cplx* uk = F.data() + (int64_t)k * m;
        for (int32_t i = 0; i < k; ++i) x[i] -= uk[i] * xk;
      }
    }
    // L21 L11^{-1}  (r x w) and -U11^{-1} U12  (w x r)
    Loff.assign((size_t)r * w, cplx(0, 0));
    gemm_acc(r, w, w, cplx(1, 0), F.data() + w, m, Linv.data(), w, Loff.data(), r);
    Uoff.assign((size_t)w * r, cplx(0, 0));
    gemm_acc(w, r, w, cplx(-1, 0), Uinv.data(), w, F.data() + (int64_t)w * m, m, Uoff.data(), w);
    // pack tiles
    cplx* fp = fwd + S.sn_fwd_off[s];
    tiles_fwd(w, r, S.tile_rows, ts);
    for (auto& t : ts) {
      for (int32_t c = 0; c < t.ncols; ++c)
        for (int32_t i = 0; i < t.nrows; ++i) {
          int32_t row = t.row0 + i, col = t.col0 + c;
          cplx v;
          if (row < w)
            v = col <= row ? Linv[row + (int64_t)col * w] : cplx(0, 0);
          else
            v = Loff[(row - w) + (int64_t)col * r];
          fp[(int64_t)c * t.nrows + i] = v;
        }
      fp += (int64_t)t.nrows * t.ncols;
    }
    cplx* bp = bwd + S.sn_bwd_off[s];
    tiles_bwd(w, r, S.tile_rows, ts);
    for (auto& t : ts) {
      for (int32_t c = 0; c < t.ncols; ++c)
        for (int32_t i = 0; i < t.nrows; ++i) {
          int32_t row = t.row0 + i, col = t.col0 + c;
          cplx v;
          if (col < w)
            v = col >= row ? Uinv[row + (int64_t)col * w] : cplx(0, 0);
          else
            v = Uoff[row + (int64_t)(col - w) * w];
          bp[(int64_t)c * t.nrows + i] = v;
        }
      bp += (int64_t)t.nrows * t.ncols;
    }
    for (int32_t k = 0; k < w; ++k) fpos[c0 + k] = -1;
    for (int32_t a = 0; a < r; ++a) fpos[R[a]] = -1;
  }
}

}  // namespace helm
