// Context of the C-ABI: host setup data and device-resident operators.
#pragma once

#include <hip/hip_runtime_api.h>

#include <chrono>
#include <deque>
#include <string>
#include <unordered_set>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace helm {

// A failing HIP call also sets the runtime's last error, which the next
// hipGetLastError would report again: it is cleared before the throw.
#define HELM_HIP(call)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) {                                                                         \
      (void)hipGetLastError();                                                                      \
      ::helm::fail(e_ == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EDEVICE,                          \
                   std::string(#call) + ": " + hipGetErrorString(e_));                              \
    }                                                                                               \
  } while (0)

// Owning device array.
template <class T>
struct DVec {
  T* p = nullptr;
  size_t n = 0;
  DVec() = default;
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
  ~DVec() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    reset();
    if (count == 0) return;
    HELM_HIP(hipMalloc((void**)&p, count * sizeof(T)));
    n = count;
  }
  void upload(const T* src, size_t count) {
    alloc(count);
    if (count) HELM_HIP(hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice));
  }
  void upload(const std::vector<T>& v) { upload(v.data(), v.size()); }
};

// Host description of a batch of factored matrices (solve layout).
struct BatchHost {
  int64_t npos = 0;                  // total positions (sum of matrix orders)
  std::vector<int32_t> c0, w, uoff, frow0;
  std::vector<int64_t> roff;
  std::vector<int32_t> rows, bidx, fcon_ptr, fcon_idx;
  // per front row its first two child-update indices (-1: none), or
  // (-2 - list start, 0) for a row with more than two (int2 pairs)
  std::vector<int32_t> fcon2;
  std::vector<dev::Tile> tf, tb;
  std::vector<dev::Task> kf, kb;      // workgroup tasks
  std::vector<int64_t> lev_f, lev_b;  // task ranges per level
  std::vector<int32_t> chunk_f, chunk_b;  // LDS input entries per level
  std::vector<int64_t> nwide_f, nwide_b;  // tiles of each level wider than 96 columns (they come first)
  std::vector<int64_t> nwide4_f, nwide4_b;  // of which those with four waves (wider than 384 columns, or root separators)
  // one-wave forward supernodes (their tiles close each level, in job
  // order); the tile kernel takes the first ktile_f tasks of a level
  std::vector<dev::SnJob> snj;
  std::vector<int64_t> snj_lev, ktile_f;
  std::vector<int32_t> gy_f;              // gather workgroups per supernode of each forward level
  std::vector<double> bytes_f, bytes_b;  // algorithmic bytes per level
  std::vector<double> pbytes_f, pbytes_b;  // of which panel bytes
  // staged 16-right-hand-side inputs of the forward sweep: supernodes of
  // every level, their column offsets in the level's staging block, the
  // largest block
  std::vector<int32_t> gsn_f;
  std::vector<int64_t> gsn_lev_f, goff_f;
  int64_t stage_cols = 0;
  int64_t nf = 0, nb = 0, nu = 0;     // panel entries (fwd, bwd), update entries
  int32_t max_front = 0;
  double flops = 0;
};

// Device copy of a batch.
struct BatchDev {
  DVec<dev::Tile> tf, tb;
  DVec<dev::Task> kf, kb;
  int c64 = 0;
  DVec<int32_t> c0, w, uoff, frow0, rows, bidx, fcon_ptr, fcon_idx, fcon2;
  DVec<int64_t> roff;
  DVec<unsigned char> pf, pb;  // panels, complex128 or complex64 entries
  DVec<double> ubuf, y, x;
  std::vector<int64_t> lev_f, lev_b;
  std::vector<int32_t> chunk_f, chunk_b;
  std::vector<int64_t> nwide_f, nwide_b, nwide4_f, nwide4_b;
  // 16-column level solves: tiles of each level taken four waves each (a
  // prefix of the level's tiles), chosen by timing at first use
  std::vector<int64_t> nw16_f, nw16_b;
  bool blk_tuned = false;
  std::vector<int32_t> gy_f;
  DVec<dev::SnJob> snj;
  std::vector<int64_t> snj_lev, ktile_f;
  int64_t npos = 0;
  std::vector<double> bytes_f, bytes_b;  // algorithmic bytes per level
  std::vector<double> pbytes_f, pbytes_b;  // of which panel bytes
  std::vector<int64_t> tiles_f, tiles_b;   // tile range of every level
  // multi-right-hand-side work vectors (interleaved, widest block so far)
  int blk_S = 0;
  DVec<double> ubuf_b, y_b, x_b;
  DVec<int32_t> gsn_f;
  DVec<int64_t> goff_f;
  std::vector<int64_t> gsn_lev_f;
  int64_t stage_cols = 0;
  DVec<unsigned char> stage;
  // > 0: grid of the single cooperative launch that runs the whole solve
  int coop = 0;
  // backward-sweep outputs inside a buffer shared by all subdomain batches
  // (each batch writes after the batches before it), else x / x_b
  double* xo = nullptr;
  double* xo_b = nullptr;
  double* xout() const { return xo ? xo : x.p; }
  double* xout_b() const { return xo_b ? xo_b : x_b.p; }
  dev::LevelRanges ranges{};
  dev::Batch view() const;
  void reset() {
    for (auto* v : {&c0, &w, &uoff, &frow0, &rows, &bidx, &fcon_ptr, &fcon_idx, &fcon2}) v->reset();
    for (auto* v : {&ubuf, &y, &x}) v->reset();
    pf.reset();
    pb.reset();
    tf.reset();
    tb.reset();
    kf.reset();
    kb.reset();
    c64 = 0;
    coop = 0;
    roff.reset();
    lev_f.clear();
    lev_b.clear();
    bytes_f.clear();
    bytes_b.clear();
    pbytes_f.clear();
    pbytes_b.clear();
    tiles_f.clear();
    tiles_b.clear();
    blk_S = 0;
    nw16_f.clear();
    nw16_b.clear();
    blk_tuned = false;
    ubuf_b.reset();
    y_b.reset();
    x_b.reset();
    gsn_f.reset();
    goff_f.reset();
    gsn_lev_f.clear();
    stage_cols = 0;
    stage.reset();
    npos = 0;
  }
};

// Event pairs around kernel launches; harvested at synchronisation points.
struct Profiler {
  bool on = false;
  helm_kernel_profile acc[HELM_K_COUNT] = {};
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, double>> pending;  // kernel id, bytes
  void begin(hipStream_t s);
  void end(int kid, double bytes, hipStream_t s);
  void harvest();  // stream must be synchronised
  void reset();
  ~Profiler();
};

// Subdomain batches whose local solves run concurrently, at most.
constexpr int kMaxBatches = 4;

struct Ctx {
  int device = -1;
  std::string err;
  bool assembled = false, precond_ready = false;
  Discretization D;
  // preconditioner (host)
  int32_t n_sub = 0, overlap = 0;
  std::vector<SubdomainHost> subs;
  std::vector<Symbolic> sym;
  bool two_level = false;
  CsrReal Z, ZT;
  Csr E;
  Symbolic Esym;
  helm_precond_stats stats{};
  // device operators
  // lanes per row of the CSR SpMV of A (plain order, XCD row ranges) and
  // of Z^T / Z, picked by timing at setup
  int g_A = dev::spmv_cfg(8, 1), g_X = dev::spmv_cfg(8, 1), g_ZT = 4, g_Zp = 4, g_AZ = 4;
  int spmv_kind = 1;   // in use: 1 CSR, 2 sliced ELL, 3 CSR over XCD row ranges, 4 split CSR
  int spmv_auto = 1;   // the fastest at assembly
  bool blk_xcd = false;     // multi-vector SpMV over XCD row ranges (faster on first use)
  bool blk_timed = false;   // blk_xcd has been timed for this matrix
  int blk_force = 0;        // 1 / 3: multi-vector SpMV order fixed by helm_set_spmv
  DVec<int64_t> A_xr;       // 9 row bounds: XCD k sweeps [A_xr[k], A_xr[k+1]), equal entries
  int64_t A_xrows = 0;      // longest of those ranges
  int64_t sell_nslices = 0;
  DVec<int64_t> sell_off;
  DVec<int32_t> sell_width, sell_perm, sell_col;
  DVec<double> sell_val;
  DVec<int64_t> A_ptr;
  DVec<int32_t> A_col;
  DVec<double> A_val;
  // split storage of A: real parts, plus imaginary parts as extra entries
  // flagged by bit 31 of the column index (only where they are nonzero)
  DVec<int64_t> S_ptr;
  DVec<int32_t> S_col;
  DVec<double> S_val;
  int64_t S_nnz = 0;
  int g_S = 0;  // its tile shape
  // the subdomains as nbatch consecutive batches of about equal factor size
  // whose level sweeps run on streams of their own (batch 0 on the caller's)
  BatchDev fine[kMaxBatches];
  int32_t nbatch = 1;
  BatchDev coarse;
  DVec<int64_t> pro_ptr;   // prolongation: global dof -> (position, weight)
  DVec<int32_t> pro_idx;
  DVec<double> pro_w;
  DVec<int64_t> Zp_ptr, ZT_ptr;
  // A Z (fine rows x coarse columns in the coarse solve's output order), split
  // real/imaginary storage: t = r - A q becomes one pass with q = Z x_c
  DVec<int64_t> AZ_ptr;
  DVec<int32_t> AZ_col;
  DVec<double> AZ_val;
  DVec<int32_t> Zp_col, ZT_col;
  DVec<double> Zp_val, ZT_val;
  // work vectors
  DVec<double> t, q, cvec;
  // GMRES work (restart gm_m, order gm_n)
  int gm_m = 0;
  int64_t gm_n = 0;
  DVec<double> V, Zk, w, partial, hcol, htmp, nrm, ydev, coef_w, coef_v;
  // 2-norms of single vectors (right-hand sides, residuals): partial sums,
  // the result and its pinned host copy
  DVec<double> npart, nval;
  double* nh_host = nullptr;
  // backward-sweep outputs of all batches in subdomain order (nbatch > 1)
  DVec<double> xall, xall_b;
  int xall_b_S = 0;
  hipStream_t sb[kMaxBatches] = {};  // streams of batches 1..nbatch-1
  hipEvent_t ev_fork = nullptr, ev_join[kMaxBatches] = {};
  hipEvent_t hev = nullptr;   // marks the Hessenberg column copy of a step
  double* h_host = nullptr;  // pinned
  Profiler prof;
  // pseudo-block GMRES work: Krylov bases bV/bZ/bw of the first blk_bases
  // right-hand sides (restart blk_m, order blk_n), and the buffers of blocks
  // up to blk_cap columns wide
  int blk_m = 0, blk_cap = 0, blk_bases = 0;
  int64_t blk_n = 0;
  DVec<double> bV[dev::kMaxBlock], bZ[dev::kMaxBlock], bw[dev::kMaxBlock];
  DVec<double> bhcol, bhtmp, bpartial, by, bX, bZb, bW, bq, bt, bcvec, bcoef_w, bcoef_v;
  double* bh_host = nullptr;  // pinned, kMaxBlock x (2 m + 4) complex
  // block GMRES (one Krylov basis of 16-column blocks shared by the block's
  // right-hand sides): bases V (m + 1 blocks) and Z_m (m blocks), W, the
  // block iterate X and right-hand sides B, reduction partials, coefficient
  // blocks, the 16 x 16 factors and their status; bg_host (pinned) receives
  // a step's Hessenberg block column
  int bg_m = 0;
  int64_t bg_n = 0;
  DVec<double> bgV, bgZ, bgW, bgX, bgB, bgpart, bgH, bgC;
  DVec<int> bgstat;
  double* bg_host = nullptr;
  int* bg_hstat = nullptr;
  // captured device work of block GMRES step j (per restart position),
  // valid for bg_graph_s active columns
  std::vector<hipGraphExec_t> bg_graph;
  int bg_graph_s = 0;
  // stream the graphs are captured on and replayed from (the caller's may be
  // the legacy null stream, which cannot be captured), joined to the
  // caller's stream by bg_ev[0] (caller -> graph) and bg_ev[1] (graph -> caller)
  hipStream_t bg_stream = nullptr;
  hipEvent_t bg_ev[2] = {};
  int64_t bg_fallbacks = 0;  // blocks handed to pseudo-block GMRES (dependent residuals)
  void free_bg_graphs();
  ~Ctx();
  void free_precond();
  void free_solve_work();
};

// solver.cpp: block work spaces (Krylov bases of the first `count` right-hand
// sides; buffers of blocks up to S columns wide) and their device bytes
size_t basis_bytes(int64_t n, int m);
size_t width_bytes(const Ctx& c, int m, int S);
void ensure_bases(Ctx& c, int m, int count);
void ensure_width(Ctx& c, int m, int S);

// factor_gpu.cpp: numeric factorisation of a set of matrices on the device,
// the panels of matrix i written from pf[i] / pb[i] on (device memory
// allocated by the caller; complex64 unless prec is kC128); pivots returned
// in num.  Fronts of at least split_min rows (none if negative) are
// factorised by several workgroups each.  scratch_bytes: the device memory
// it held besides the panels.
void factor_batch_device(const std::vector<const Csr*>& As, const std::vector<const Symbolic*>& Ss,
                         dev::FactorPrecision prec, int32_t split_min, const std::vector<void*>& pf,
                         const std::vector<void*>& pb, std::vector<NumericOut>& num, int32_t& n_perturbed,
                         double& scratch_bytes);

// solver.cpp
void layout_batch(const std::vector<const Symbolic*>& Ss, const std::vector<const std::vector<int64_t>*>& in_idx,
                  const std::vector<NumericOut>& num, int64_t sn_jobs_min, bool c64, BatchHost& B);
void precond_setup(Ctx& c, const int32_t* tet_part, int32_t n_sub, int32_t overlap, const helm_mesh* coarse,
                   const helm_precond_opts* opts);
void upload_matrix(Ctx& c);
void apply_A(Ctx& c, const double* x, double* y, hipStream_t s);
void apply_oras(Ctx& c, const double* r, double* z, const double* q, hipStream_t s);
void apply_coarse(Ctx& c, const double* r, double* q, hipStream_t s);
size_t coarse_scratch_bytes(const Ctx& c);
void apply_coarse_scratch(Ctx& c, const double* r, double* q, hipStream_t s, void* scratch);
void apply_precond(Ctx& c, const double* r, double* z, hipStream_t s);
int solve(Ctx& c, int32_t nrhs, const double* B, double tol, const helm_solve_opts* opts, double* U, hipStream_t s,
          helm_solve_info* info);

// Continuous-batching server over one context (solver.cpp).
struct Server {
  struct Request {
    const double* b;
    double* u;
    int64_t tag;
    std::chrono::steady_clock::time_point t0;
  };
  struct Slot {
    bool busy = false, conv = false;
    const double* b = nullptr;
    double* u = nullptr;
    int64_t tag = 0;
    std::chrono::steady_clock::time_point t0;
    double bnorm = 0, rel = 0;
    int its = 0, jj = 0;
    std::vector<cplx> H, g, sn, y;
    std::vector<double> cs;
  };
  Ctx& c;
  hipStream_t s;
  int m = 50, maxit = 1000, slots_n = 0;  // slots_n: slots at most (each opened on demand)
  double budget = 0;  // device bytes the slots' bases and block buffers may hold
  bool dcgs2 = true;
  double tol = 1e-6;
  std::deque<Request> queue;
  std::vector<Slot> slot;
  std::vector<int> act;
  hipEvent_t done_ev = nullptr;
  bool inflight = false;
  Server(Ctx& ctx, const helm_server_opts* o, hipStream_t st);
  ~Server();
  void submit(const double* b, double* u, int64_t tag);
  int launch();
  void finish(std::vector<helm_server_event>& out);
  void admit(std::vector<helm_server_event>& out);
  void emit(std::vector<helm_server_event>& out, const helm_server_event& e);
  std::unordered_set<int64_t> live;  // tags queued or in flight
  bool open_slot(int q);
  double bytes_for(int bases, int width) const;
  double held() const;
  bool start_cycle(int q, std::vector<helm_server_event>& out);
  int active() const {
    int a = 0;
    for (auto& z : slot) a += z.busy;
    return a;
  }
};

}  // namespace helm
