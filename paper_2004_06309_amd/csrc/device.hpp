// Launchers of the HIP kernels (device.hip).  Complex vectors are interleaved
// (re, im) doubles; every launch is asynchronous on the given stream.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace helm {
namespace dev {

// A pivot is taken as zero when |pivot| <= kTinyPivot max|a_ij| (the
// factorisations replace it by sqrt(eps) max|a_ij| and count it).
constexpr double kTinyPivot = 1000.0 * 2.220446049250313e-16;
// The same test for a factorisation in complex64 arithmetic: 16 FP32 eps
// (a pivot that small carries no correct digit after FP32 elimination).
constexpr double kTinyPivotF32 = 16.0 * 1.1920928955078125e-07;

// Up to kMaxBlock device pointers, one per right-hand side of a block
// (passed by value as a kernel argument; a null entry is a padding column).
constexpr int kMaxBlock = 16;
struct PtrSet {
  double* p[kMaxBlock];
};
struct PtrSetC {
  const double* p[kMaxBlock];
};

// Mirrors helm::TileDesc.
struct Tile {
  int64_t off;
  int32_t sn, row0, nrows, col0, ncols;
  int32_t c0;   // the supernode's first batch position
  int32_t w;    // its pivot columns
  int32_t aux;  // forward: its first front row in fcon_ptr; backward: offset of R_s in rows
};

// A supernode of at most 64 pivot columns whose forward panel is solved by
// one wave: its 64-row tiles lie back to back from off (tile q at
// off + 64 q w, the last one m - 64 q rows), each w columns wide.
struct SnJob {
  int64_t off;
  int32_t m;      // front rows (w + |R_s|)
  int32_t w;      // pivot columns (<= 64)
  int32_t c0;     // first batch position
  int32_t frow0;  // first front row in fcon_ptr
  int32_t uoff;   // offset of its update vector in ubuf
  int32_t tile;   // index of its first tile in the forward tile list
};

// A workgroup's share of a level: ntile consecutive tiles, each handled by
// wpt waves (ntile * wpt <= 4).
struct Task {
  int32_t tile0;
  int16_t ntile;
  int16_t wpt;
};

// Device arrays of one batch of factored matrices (all fine subdomains, or
// the coarse matrix); the panels are the partitioned-inverse tiles written
// by device_factor.hip.
struct Batch {
  const Tile* tf = nullptr;        // forward tiles, grouped by level
  const Tile* tb = nullptr;        // backward tiles, grouped by level
  const Task* kf = nullptr;        // forward workgroup tasks, grouped by level
  const Task* kb = nullptr;        // backward workgroup tasks
  const SnJob* snj = nullptr;      // one-wave forward supernodes, grouped by level
  const int32_t* sn_c0 = nullptr;  // first position of the supernode
  const int32_t* sn_w = nullptr;   // columns
  const int32_t* sn_uoff = nullptr;  // offset of its update vector in ubuf
  const int32_t* sn_frow0 = nullptr; // first front row in the fcon index
  const int64_t* sn_roff = nullptr;  // offset of R_s in rows
  const int32_t* rows = nullptr;   // R lists (batch positions)
  const int32_t* bidx = nullptr;   // pivot position -> input-vector index
  const int32_t* fcon_ptr = nullptr; // front row -> child update entries
  const int32_t* fcon_idx = nullptr;
  const int2* fcon2 = nullptr;     // front row -> first two entries, or (-2 - list start, 0)
  const int32_t* sn_r = nullptr;   // |R_s|
  const int64_t* goff_f = nullptr; // column offset of the supernode's staged block (forward level scratch)
  const void* pf = nullptr;        // forward panels (complex128, or complex64 when c64)
  const void* pb = nullptr;        // backward panels
  int c64 = 0;
  double* ubuf = nullptr;          // update vectors
  double* y = nullptr;             // forward result (pivot order)
  double* x = nullptr;             // backward result (column order)
};

// One level of the forward / backward sweep: tasks [task0, task0 + ntasks).
// coarse selects a separate instantiation so profiles tell the two apart.
// chunk: LDS entries for the level's input columns (level_chunk).
void fwd_level(const Batch& b, int64_t task0, int64_t ntasks, const double* bin, int chunk, bool coarse,
               hipStream_t s);
void bwd_level(const Batch& b, int64_t task0, int64_t ntasks, int chunk, bool coarse, hipStream_t s);
// Forward solve of the one-wave supernodes [job0, job0 + njobs) of a level.
void fwd_sn(const Batch& b, int64_t job0, int64_t njobs, const double* bin, hipStream_t s);
// dst[to[t] + i] = src[from[t] + i] for i < words[t], t < ntiles (8-byte
// words; device pointers): moves panel tiles into their solve order.
void copy_tiles(const void* src, void* dst, const int64_t* from, const int64_t* to, const int64_t* words,
                int64_t ntiles, hipStream_t s);
// Largest LDS input buffer a level solve uses (entries).
constexpr int kLevelChunkMax = 2048;
// One frontal matrix of the device factorisation (offsets in complex
// entries).
struct FrontJob {
  int64_t F, X, Y;     // front (m x m), forward panel X (m x w), backward panel Y (w x m) in the workspace
  int64_t upd;         // Schur complement (r x r) in the update buffer
  void* pf;            // forward / backward panel arrays of the job's matrix
  void* pb;            //   (complex128 or complex64 entries)
  int64_t pfo, pbo;    // first forward / backward tile entry in those arrays
  int64_t asm0, asm1;  // range of the front's original entries in the assembly lists
  int32_t m, w;        // front order, fully-summed columns
  int32_t c0;          // first column of the supernode in its matrix
  int32_t piv0;        // batch position of that column (pivot output)
  int32_t kid0, kid1;  // range of the children in the child list
  double anorm;        // max |a_ij| of the matrix (zero-pivot replacement scale)
};
// A child's Schur complement and the front rows its rows map to.
struct FrontChild {
  int64_t upd;  // offset in the update buffer
  int64_t ep;   // offset of its r front positions in the extend-add map
  int32_t r, pad;
};
// Factors a list of independent fronts (one workgroup each): assembly from
// the scatter lists (F[asm_pos[q]] = aval[asm_val[q]]) and the children,
// partial LU, Schur complement into upd, pivots into piv (batch positions),
// zero-pivot replacements per job into npert, explicit-inverse panels into
// the solve tiles of each job's pf / pb.  ws holds each job's F, X and Y;
// ws and upd hold complex entries of the working precision (complex64 for
// kC64, complex128 otherwise); aval is complex128.
enum class FactorPrecision {
  kC128,            // complex128 arithmetic, complex128 panels
  kC128RoundedC64,  // complex128 arithmetic, panels rounded once to complex64
  kC64,             // complex64 arithmetic (FP32 MFMA), complex64 panels
};
void factor_fronts(const FrontJob* jobs, int njobs, void* ws, void* upd, const int32_t* asm_pos,
                   const int32_t* asm_val, const double* aval, const FrontChild* kids, const int32_t* ep,
                   int32_t* piv, int32_t* npert, FactorPrecision prec, int tile_rows, hipStream_t s);
// The same for fronts factorised by several workgroups each, in a sequence
// of launches (assembly by column strips; per 32-column block a one-
// workgroup panel step and a column-strip update step; the X / Y panels by
// row / column strips; the backward tiles).  mmax / wmax: largest m / w of
// the jobs; swp: one int per pivot position (the row interchanges, batch
// positions as piv).  ep must map every child's rows to increasing front
// positions.  Same results as factor_fronts.
void factor_fronts_split(const FrontJob* jobs, int njobs, int mmax, int wmax, void* ws, void* upd,
                         const int32_t* asm_pos, const int32_t* asm_val, const double* aval, const FrontChild* kids,
                         const int32_t* ep, int32_t* piv, int32_t* swp, int32_t* npert, FactorPrecision prec,
                         int tile_rows, hipStream_t s);
// Fronts of at least this many rows take factor_fronts_split by default.
constexpr int kSplitFrontMin = 256;

// Task ranges of every level of a batch (a kernel argument).
constexpr int kMaxLevels = 40;
struct LevelRanges {
  int nf, nb;
  int64_t f[kMaxLevels + 1], b[kMaxLevels + 1];
};
// Largest co-resident grid of the cooperative batch solve (0 if unknown).
int coop_grid();
// Forward + backward solve of a complex128 batch in one cooperative launch.
hipError_t batch_solve_coop(const Batch& b, const double* bin, const LevelRanges& lv, int grid, hipStream_t s);
// Waves per tile chosen for a tile with ncols input columns.
int waves_per_tile(int ncols);

// Tile shape of the CSR SpMV: G lanes per row, U entries per lane per pass.
constexpr int spmv_cfg(int G, int U) { return G | (U << 8); }
// Shapes the CSR SpMV is built for.
constexpr int kSpmvCfgs[] = {spmv_cfg(4, 1),  spmv_cfg(4, 4),  spmv_cfg(4, 8),  spmv_cfg(8, 1), spmv_cfg(8, 2),
                             spmv_cfg(8, 4),  spmv_cfg(16, 1), spmv_cfg(16, 2), spmv_cfg(32, 1)};
// y = A x, or y = b - A x when b != nullptr (complex CSR) with tile shape
// cfg (one of kSpmvCfgs).  xr (device, 9 entries, or nullptr): row ranges
// [xr[k], xr[k+1]) swept by XCD k; xrows = the longest range.
void spmv(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const int64_t* xr, int64_t xrows,
          const double* x, const double* b, double* y, int cfg, hipStream_t s);
// Same product from the split storage: real CSR entries, where an entry
// with bit 31 set in its column index is an imaginary part (multiplies
// i x[col & 0x7fffffff]).
void spmv_split(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const double* x,
                const double* b, double* y, int cfg, hipStream_t s);
// Row ranges for the 8 XCDs holding equal numbers of CSR entries (host;
// xr[0] = 0, xr[8] = n); returns the longest range.
int64_t xcd_ranges(int64_t n, const int64_t* ptr, int64_t xr[9]);
// Same product from the sliced-ELL copy of A (64-row slices).
void sell_spmv(int64_t n, int64_t nslices, const int64_t* soff, const int32_t* swidth, const int32_t* perm,
               const int32_t* col, const double* val, const double* x, const double* b, double* y, hipStream_t s);
// y = A x with a real CSR matrix and complex vectors; G lanes per row.
void spmv_real(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const double* x, double* y,
               int G, hipStream_t s);
// q = Z cx and t = r - (A Z) cx for a coarse solution cx (complex vectors):
// Z real CSR, A Z in the split storage of spmv_split; G = 1, 2, 4 or 8
// lanes per row.
void coarse_update(int64_t n, const int64_t* zptr, const int32_t* zcol, const double* zval, const int64_t* aptr,
                   const int32_t* acol, const double* aval, const double* cx, const double* r, double* q, double* t,
                   int G, hipStream_t s);
// coarse_update for S interleaved right-hand sides (device_block.hip).
void coarse_update_block(int64_t n, const int64_t* zptr, const int32_t* zcol, const double* zval,
                         const int64_t* aptr, const int32_t* acol, const double* aval, int S, const double* cx,
                         const double* x, double* q, double* t, hipStream_t s);
// z[g] = sum_p w[p] xl[idx[p]] over p in [ptr[g], ptr[g+1]) (+ q[g] if q).
void prolong(int64_t n, const int64_t* ptr, const int32_t* idx, const double* w, const double* xl, const double* q,
             double* z, hipStream_t s);

// Blocks for norm2's partial sums.
int gs_blocks(int64_t n);
// Fused CGS2 pass over 64-row tiles (gs_tiles(n) workgroups per
// right-hand side, ncol <= 64), for nr right-hand sides at once (entry r of
// each pointer set belongs to right-hand side r):
// mode 0: partial dots V^H w; mode 1: w -= V h then partial dots of the new
// w; mode 2: w -= V h then partial squared norms (reduce with norm_final).
int gs_tiles(int64_t n);
void gs_pass(int mode, int nr, int64_t n, const PtrSetC& V, int64_t ld, int ncol, const PtrSetC& h, const PtrSet& w,
             const PtrSet& partial, hipStream_t s);
// h[k] = sum_b partial[b*ncol + k]; hacc[k] = (or +=) h[k], per right-hand side
void gs_final(int nr, const PtrSetC& partial, int nblk, int ncol, const PtrSet& h, const PtrSet& hacc,
              int accumulate, hipStream_t s);
void norm_final(int nr, const PtrSetC& partial, int nblk, const PtrSet& out, hipStream_t s);
// Delayed CGS2 passes over ncol = j + 1 columns of V (see device.hip):
// update = false: partial dots V^H w and V^H v_j (2 ncol per tile, reduce
// with gs_final over 2 ncol); update = true: v_j and w updated with the
// coefficients cw, cv (written to column j through Vw), partial |w|^2.
void gs_dual(bool update, int nr, int64_t n, const PtrSetC& V, const PtrSet& Vw, int64_t ld, int ncol,
             const PtrSetC& cw, const PtrSetC& cv, const PtrSet& w, const PtrSet& partial, hipStream_t s);
// Pass-B coefficients and the host-bound Hessenberg data from the reduced
// pass-A dots (2 ncol entries per right-hand side); one wave per RHS.
void dcgs2_coef(int nr, const PtrSetC& dots, int ncol, const PtrSet& cw, const PtrSet& cv, const PtrSet& out,
                hipStream_t s);
// v = w / nrm[0] per right-hand side
void scale_by_inv_set(int nr, int64_t n, const PtrSetC& w, const PtrSetC& nrm, const PtrSet& v, hipStream_t s);

// ---- block (multi-right-hand-side) operations, S in {2, 4, 8, 16},
//      interleaved n x S vectors (device_block.hip) ----
// one wavefront per tile: tiles [tile0, tile0 + ntiles) of the level
void fwd_level_block(const Batch& b, int64_t tile0, int64_t ntiles, int S, const double* bin, double* yb, double* ubb,
                     bool coarse, hipStream_t s);
void bwd_level_block(const Batch& b, int64_t tile0, int64_t ntiles, int S, const double* yb, double* xb, bool coarse,
                     hipStream_t s);
// 16 right-hand sides on MFMA.  Forward: stage every supernode's input
// block of the level once (gather kernel, one workgroup per supernode of
// `sns`, gy workgroups per supernode each taking every gy-th run of 256
// block entries), then one 4-wave workgroup per wide tile (the first nwide
// tiles of the range) or one wave per narrow tile reads its B operands from
// the staged block.  Backward: one launch, each workgroup gathering its
// tile's input block into LDS a pass of columns at a time.
void fwd_level_mfma(const Batch& b, const int32_t* sns, int64_t nsn, int gy, int64_t tile0, int64_t ntiles,
                    int64_t nwide, const double* bin, double* yb, double* ubb, void* stage, bool coarse,
                    hipStream_t s);
void bwd_level_mfma(const Batch& b, int64_t tile0, int64_t ntiles, int64_t nwide, const double* yb, double* xb,
                    bool coarse, hipStream_t s);
// ---- block Gram-Schmidt of block GMRES (device_bgmres.hip): n x 16
//      interleaved complex blocks, X_j = X + j ldx (ldx in doubles) ----
// workgroups of bgs_dots (bgs_dots writes at most 16 blocks of partial sums
// per workgroup, or nb + 1 when that is more) and of bgs_mul
int bgs_wgs(int64_t n);
int bgs_mul_wgs(int64_t n);
// partial[(p * (nb + with_w) + j) * 256 + a * 16 + c] = sum over the rows of
// partial row p of conj(X_j[row][a]) W[row][c]; block nb is W itself
// (with_w).  Returns the number of partial rows (for bgs_reduce).
int bgs_dots(int64_t n, const double* X, int64_t ldx, int nb, bool with_w, const double* W, double* partial,
             hipStream_t s);
// out (and acc, = or +=) [j * 256 + e] = sum over nwg workgroups of the partials
void bgs_reduce(const double* partial, int nwg, int nbt, double* out, double* acc, bool accumulate, hipStream_t s);
// Y = (Y0 or 0) + sign sum_{j < nb} X_j C_j (C_j = C + 512 j doubles, 16 x
// 16 row-major); gram: per-workgroup partial Y^H Y (bgs_mul_wgs of them)
void bgs_mul(int64_t n, const double* X, int64_t ldx, int nb, const double* C, double sign, const double* Y0,
             double* Y, double* gram, hipStream_t s);
// G = L L^H on the leading s x s part: R = L^H, T = L^{-H}; status 0, or
// 1 + k if pivot k is not above tiny max_k ref[k][k] (ref null: tiny)
void chol16(const double* G, int s_act, const double* ref, double tiny, double* R, double* T, int* status,
            hipStream_t s);

// y = A x (or b - A x) for S interleaved vectors from the CSR copy of A.
// xr / xrows: XCD row ranges as for spmv (nullptr: plain order).
void csr_spmv_block(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const int64_t* xr,
                    int64_t xrows, int S, const double* x, const double* b, double* y, hipStream_t s);
void spmv_real_block(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, int S, const double* x,
                     double* y, hipStream_t s);
void prolong_block(int64_t n, const int64_t* ptr, const int32_t* idx, const double* w, int S, const double* xl,
                   const double* q, double* z, hipStream_t s);
// dst (interleaved) <- the S vectors src.p[r] (zeros for null entries)
void pack(int64_t n, int S, const PtrSetC& src, double* dst, hipStream_t s);
// dst.p[r] <- column r of src (skipped for null entries)
void unpack(int64_t n, int S, const double* src, const PtrSet& dst, hipStream_t s);
// out[0] = ||w||_2 (real, stored as complex with zero imaginary part)
void norm2(int64_t n, const double* w, double* partial, int nblk, double* out, hipStream_t s);
// v = alpha * w
void scale(int64_t n, const double* w, double alpha, double* v, hipStream_t s);
// x += Z y  (Z n x k column-major, y device)
void gemv_acc(int64_t n, const double* Z, int64_t ld, int k, const double* y, double* x, hipStream_t s);
void fill_zero(int64_t n_doubles, double* p, hipStream_t s);

// Fixed device scratch of the allocation-free coarse correction: a
// file-scope array of kScratchBytes per device.  scratch_init(device), with
// `device` current, looks up its device address once (hipGetSymbolAddress);
// scratch_ptr(device) returns it (nullptr before scratch_init).
constexpr size_t kScratchBytes = size_t(32) << 20;
hipError_t scratch_init(int device);
void* scratch_ptr(int device);
void copy(int64_t n_doubles, const double* src, double* dst, hipStream_t s);

}  // namespace dev
}  // namespace helm
