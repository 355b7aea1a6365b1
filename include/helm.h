/*
 * helm.h -- C-ABI of libhelm: ORAS-preconditioned GMRES for the 3D Helmholtz
 * equation on one MI355X (gfx950).
 *
 * Method (Dolean, Jolivet, Tournier, Operto, "Iterative frequency-domain
 * seismic wave solvers based on multi-level domain-decomposition
 * preconditioners"):
 *   - (Delta + k(x)^2) u = b, k = omega / c(x), c complex in attenuating media,
 *     homogeneous Dirichlet on the top face (z = min z; z is depth) and
 *     first-order absorbing conditions on the other boundary faces (eq. eqh);
 *   - P1/P2 Lagrange finite elements on tetrahedra, A u = b (eq. eq1);
 *   - right-preconditioned GMRES stopped at ||A x - b|| / ||b|| <= tol
 *     (Section "Numerical experiments");
 *   - one-level ORAS  M1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i (eq. oras) with
 *     impedance local matrices, and the two-level preconditioner
 *     M^{-1} = M1^{-1}(I - A Q) + Q, Q = Z E^{-1} Z^T, E = Z^T A Z (eq. 2lvl).
 *
 * Conventions
 *   - complex arrays are interleaved (re, im) doubles;
 *   - time dependence exp(-i omega t): absorbing condition d_n u = i k u and
 *     the weak form A = -K + M_{k^2} + i B_k;
 *   - dof numbering: P1 = vertices in input order; P2 = vertices, then edges
 *     sorted by (min vertex id, max vertex id), the edge dof at its midpoint;
 *   - Dirichlet dofs are kept as unknowns with identity rows and columns;
 *   - every call returns an int status, 0 = HELM_OK, negative = error; the
 *     message of the last error is returned by helm_last_error;
 *   - the caller owns every buffer it passes; the library keeps no caller
 *     pointer after a call returns; the library owns all memory it allocates;
 *   - a context is not thread-safe; distinct contexts may be used from
 *     distinct threads.
 */
#ifndef HELM_H
#define HELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HELM_OK = 0,
  HELM_EINVAL = -1,     /* bad argument, bad mesh, zero-volume tet          */
  HELM_ESINGULAR = -2,  /* zero pivot in a frontal matrix                   */
  HELM_ENOCONV = -3,    /* maxit reached; U holds the last iterates         */
  HELM_ENUMERIC = -4,   /* NaN/Inf met in the iteration                     */
  HELM_ENOMEM = -5,     /* host or device allocation failed                 */
  HELM_ESTATE = -6,     /* call made in the wrong order or on a host-only
                           context                                          */
  HELM_EDEVICE = -7     /* HIP runtime error                                */
};

typedef struct helm_ctx helm_ctx;

/* Tetrahedral mesh, host arrays (read during the call only). */
typedef struct helm_mesh {
  int64_t n_nodes;
  const double* xyz;       /* [n_nodes][3], metres, z = depth             */
  int64_t n_tets;
  const int64_t* tets;     /* [n_tets][4] vertex ids; any orientation      */
  int32_t order;           /* 1 (P1) or 2 (P2)                             */
} helm_mesh;

typedef struct helm_precond_opts {
  int32_t leaf_size;       /* nested-dissection leaf size, 0 = default     */
  int32_t factor_c64;      /* subdomain factor precision:
                              0: complex128 factorisation and panels;
                              1: complex64 factorisation (fronts, Schur
                                 complements and panels in complex64, the
                                 frontal updates on FP32 MFMA accumulating
                                 in FP32), complex64 panels;
                              2: complex128 factorisation, panels rounded
                                 once to complex64.
                              With complex64 panels the single-RHS solves
                              accumulate in FP64 and the 16-RHS block
                              solves on FP32 MFMA; the coarse factors stay
                              complex128.  Other values: HELM_EINVAL      */
  int32_t coarse_leaf_size;  /* leaf size of the coarse ordering, 0 = 256  */
  int32_t tile_rows;       /* rows per solve tile of the subdomain factors:
                              16, 32 or 64; 0 = 64                         */
  int32_t coarse_tile_rows;  /* same for the coarse factor; 0 = 16         */
  int32_t sn_jobs_min;     /* complex128 panels: a forward level with at least
                              this many supernodes of <= 64 pivots (and
                              64-row tiles) solves those with one wave per
                              supernode instead of one per tile; 0 = 6144,
                              -1 = never                                  */
  int32_t batches;         /* the subdomains as 1 .. 4 consecutive batches
                              of about equal factor size whose level
                              sweeps run concurrently, each on a stream of
                              its own (one after the other while
                              helm_profile is on); 0 = 2; other values
                              fail with HELM_EINVAL                       */
  int32_t perturb_pivots;  /* a pivot with |p| <= 1000 eps max|a_ij| of its
                              matrix (16 FP32 eps in a complex64
                              factorisation; zero to working precision, after
                              partial pivoting inside the front) makes
                              helm_precond_setup fail with HELM_ESINGULAR;
                              1: replace it by sqrt(eps) max|a_ij| instead,
                              count it in helm_precond_stats.n_perturbed
                              and return HELM_OK                          */
  int32_t coarse_launch;   /* coarse solve: 0 = the faster of the two forms
                              as timed at setup; 1 = one launch per level;
                              2 = one cooperative launch with a grid
                              barrier per level (HELM_EINVAL where the
                              device cannot co-schedule it).  The
                              cooperative form is used only after its
                              result on a fixed right-hand side matched the
                              per-level launches at setup (to 1e-13; with
                              2 a mismatch fails with HELM_EDEVICE)        */
  int32_t split_front_rows;  /* device factorisation: frontal matrices of at
                              least this many rows are spread over several
                              workgroups (a sequence of launches per
                              level), smaller ones take one workgroup each;
                              0 = 256, -1 = never.  The factors are the
                              same either way                              */
} helm_precond_opts;

enum {
  HELM_SOLVE_X0 = 1,       /* read U as the initial guess                  */
  HELM_SOLVE_CGS2 = 2,     /* classic CGS2 (three passes over the Krylov
                              basis per step) instead of the default
                              delayed CGS2 (two passes; the second
                              orthogonalisation of v_j is folded into step
                              j + 1), for single and pseudo-block solves  */
  HELM_SOLVE_BLOCK_GMRES = 4,  /* block > 1: block GMRES instead of pseudo-
                              block GMRES: the block's right-hand sides share
                              one block Krylov space (restart = blocks of
                              16 columns), orthogonalised by block CGS2 on
                              MFMA (two passes of tall-skinny contractions)
                              and CholQR2; the block Hessenberg least
                              squares runs on the host in FP64 (Householder).
                              Columns whose true residual reaches tol leave
                              the block at a restart; residuals that are
                              linearly dependent fall back to pseudo-block
                              GMRES.  Device memory: 16 n (2 m + 4) x 16
                              bytes.  iterations counts block steps       */
  HELM_SOLVE_GRAPHS = 8    /* with HELM_SOLVE_BLOCK_GMRES: replay each
                              block step's device work (preconditioner,
                              product with A, Gram-Schmidt, copy of the
                              Hessenberg column) from a HIP graph captured
                              on its first use (one graph per step index;
                              kept until the preconditioner changes).
                              Measured on ROCm 7.2: once a process has
                              replayed such graphs, its later eager solves
                              (other contexts included) run 11-17 % slower,
                              and at the mid size the replayed steps are no
                              faster than eager ones                      */
};

typedef struct helm_solve_opts {
  int32_t restart;         /* GMRES(m) restart length, 1..50, 0 = 50       */
  int32_t maxit;           /* total Arnoldi steps per RHS, 0 = 1000        */
  int32_t flags;           /* HELM_SOLVE_*                                 */
  int32_t block;           /* right-hand sides advanced together (pseudo-
                              block GMRES, one pass over A and the factors
                              per step for the whole block), 1..16; 0 or 1
                              = one at a time.  The first solve with a
                              block wider than 8 on a factored operator
                              first times, per level of the local solves,
                              which tiles take four waves each (about
                              0.1 s at one million unknowns); the
                              environment variable HELM_BLOCK_SPLIT = 0, 1,
                              2 or 3 fixes the choice instead: the tiles
                              wider than 96 columns; those wider than 384
                              and the root separators'; none; all         */
} helm_solve_opts;

typedef struct helm_solve_info {
  int32_t iterations;      /* Arnoldi steps over all restarts              */
  int32_t converged;       /* 1 if the true relative residual <= tol       */
  double relres;           /* true ||b - A u|| / ||b|| at exit            */
  double seconds;          /* wall time of this RHS (device-synchronised)  */
} helm_solve_info;

/* Serving: continuous batching of single-right-hand-side requests over one
 * factored operator (Section "Numerical experiments": many sources per
 * operator).  Up to 16 requests are in flight as slots of a pseudo-block
 * GMRES; a request waiting in the queue takes the first slot that frees up,
 * at the next Arnoldi step, while the others continue their own cycles. */
typedef struct helm_server helm_server;

typedef struct helm_server_opts {
  int32_t slots;           /* requests in flight at most, 1..16; 0 = 16;
                              each slot opens only when its memory fits
                              (mem_bytes)                                  */
  int32_t restart;         /* GMRES(m) restart length, 1..50, 0 = 50       */
  int32_t maxit;           /* Arnoldi steps per request, 0 = 1000          */
  int32_t flags;           /* HELM_SOLVE_CGS2: classic CGS2; other bits
                              are ignored                                  */
  double tol;              /* true relative residual, 0 = 1e-6             */
  double mem_bytes;        /* device memory the server may hold for its
                              slots (each slot's Krylov basis, 16 (2 m + 2) n
                              bytes, plus the block buffers of the widest
                              block in flight); 0 = three quarters of the
                              free device memory at creation plus what the
                              context already holds for slots of the same
                              restart (opened by an earlier server).  A
                              request is
                              admitted into a slot only when that slot's
                              memory fits (slots open lowest first and are
                              kept once opened); otherwise it stays queued */
} helm_server_opts;

typedef struct helm_server_event {
  int64_t tag;             /* the caller's tag of the finished request     */
  int32_t iterations;      /* Arnoldi steps it took                        */
  int32_t converged;       /* 1 if the true relative residual <= tol       */
  int32_t status;          /* HELM_OK, HELM_ENOCONV or HELM_ENUMERIC        */
  int32_t reserved;
  double relres;           /* true ||b - A u|| / ||b|| at exit            */
  double seconds;          /* host wall time from submit to completion     */
} helm_server_event;

typedef struct helm_precond_stats {
  int32_t n_sub;           /* subdomains                                   */
  int32_t n_coarse;        /* coarse unknowns (0 = one-level)              */
  int64_t n_local_total;   /* sum of local sizes n_i                       */
  int64_t factor_entries;  /* stored fine-level factor entries (L + U)     */
  int64_t coarse_entries;  /* stored coarse factor entries                 */
  int32_t levels_fwd;      /* batched forward-solve launches               */
  int32_t levels_bwd;      /* batched backward-solve launches              */
  int32_t max_front;       /* largest frontal matrix order                 */
  int32_t n_supernodes;    /* fine-level supernodes                        */
  double setup_seconds;    /* wall time of the last helm_precond_setup     */
  double factor_flops;     /* complex multiply-adds x 8 in the factorisation */
  int32_t factor_c64;      /* fine factor precision as run: 0, 1 or 2 (see
                              helm_precond_opts.factor_c64)               */
  int32_t coarse_grid;     /* workgroups of the one-launch cooperative coarse
                              solve; 0 = one launch per level              */
  int32_t n_perturbed;     /* tiny pivots replaced by sqrt(eps) max|a_ij|
                              (only with perturb_pivots)                  */
  double factor_seconds;   /* wall time of the numeric factorisation       */
  int32_t batches;         /* subdomain batches (1 .. 4)                   */
  int32_t reserved;
  double factor_scratch_bytes;  /* device memory the numeric factorisation
                              held besides the panels (fronts, Schur
                              complements, inputs), peak over the fine and
                              coarse factorisations; freed when setup
                              returns                                      */
} helm_precond_stats;

/* Create a context on HIP device `device_ordinal`; -1 creates a host-only
 * context that can assemble and analyse but not solve (used to inspect the
 * setup without a GPU).  *out is NULL on failure. */
int helm_create(helm_ctx** out, int device_ordinal);

/* Free every host and device resource of the context; NULL is accepted.
 * A server still open on the context loses its solver state (in-flight work
 * is waited for); its handle must still be released with
 * helm_server_destroy, and every other call on it returns HELM_ESTATE. */
void helm_destroy(helm_ctx* ctx);

/* Message of the last failing call on ctx (or of helm_create when ctx is
 * NULL); never NULL, owned by the library. */
const char* helm_last_error(const helm_ctx* ctx);

/* Assemble A of eq. eq1 for mesh, complex velocity c_tet (interleaved
 * c128[n_tets], constant per tet) and angular frequency omega (rad/s).
 * Tets are re-oriented if needed; a degenerate tet gives HELM_EINVAL.
 * Invalidates any earlier preconditioner. */
int helm_assemble(helm_ctx* ctx, const helm_mesh* mesh, const double* c_tet, double omega);

/* Number of global dofs n (after helm_assemble). */
int helm_ndof(const helm_ctx* ctx, int64_t* n);

/* Dof coordinates, caller-allocated host f64[n][3]. */
int helm_dof_coords(const helm_ctx* ctx, double* xyz);

/* Load of a point source b = delta(x - xs): F_i = phi_i(xs), zero on
 * Dirichlet dofs.  b is a caller-allocated host c128[n]. */
int helm_point_source(const helm_ctx* ctx, const double* xs, double* b);

/* Number of stored entries of A (CSR, after Dirichlet elimination). */
int helm_matrix_nnz(const helm_ctx* ctx, int64_t* nnz);

/* Copy A to caller-allocated host CSR arrays: rowptr i64[n+1],
 * col i32[nnz] (ascending per row), val c128[nnz]. */
int helm_matrix_csr(const helm_ctx* ctx, int64_t* rowptr, int32_t* col, double* val);

/* Build the preconditioner (eqs. oras and 2lvl): tet_part[n_tets] holds the
 * non-overlapping subdomain id (0..n_sub-1) of every tet, overlap the number
 * of element layers added by vertex adjacency, coarse the P1 coarse mesh
 * (NULL = one-level ORAS; its order field is ignored).  Local matrices carry
 * the impedance condition on artificial faces, the partition of unity is
 * chi_i = max(0, 1 - l/overlap) normalised, local solves are LU factors
 * (nested-dissection multifrontal, partial pivoting inside each front) and
 * the coarse matrix E = Z^T A Z is factored the same way, all on the device.
 * On a host-only context the numeric factorisation is skipped (assembly,
 * decomposition and symbolic analysis run, and the statistics report their
 * sizes).  HELM_ESINGULAR: a zero or tiny pivot (see perturb_pivots). */
int helm_precond_setup(helm_ctx* ctx, const int32_t* tet_part, int32_t n_sub, int32_t overlap,
                       const helm_mesh* coarse, const helm_precond_opts* opts);

int helm_precond_stats_get(const helm_ctx* ctx, helm_precond_stats* stats);

/* Subdomain i after setup: local size, then (when the pointers are not
 * NULL) its global dofs (i64[n_i], ascending), partition-of-unity weights
 * (f64[n_i]) and local matrix in CSR over local indices
 * (rowptr i64[n_i+1], col i32[nnz_i], val c128[nnz_i]).  Pass col == NULL
 * to read only nnz_i from rowptr[n_i]. */
int helm_subdomain_size(const helm_ctx* ctx, int32_t i, int64_t* n_i, int64_t* nnz_i);
int helm_subdomain_get(const helm_ctx* ctx, int32_t i, int64_t* dofs, double* D,
                       int64_t* rowptr, int32_t* col, double* val);

/* Coarse interpolation Z (real CSR n x n_c: rowptr i64[n+1], col i32, val f64)
 * after a two-level setup. */
int helm_coarse_nnz(const helm_ctx* ctx, int64_t* n_c, int64_t* nnz);
int helm_coarse_get(const helm_ctx* ctx, int64_t* rowptr, int32_t* col, double* val);

/* --- Device operations (device pointers to c128[n]; stream = hipStream_t or
 *     NULL for the null stream).  Asynchronous with respect to the host. --- */

/* SpMV storage used by every single-vector product with A: 0 = the fastest
 * as timed at helm_assemble (default), 1 = CSR in dof order, 2 = sliced ELL
 * (64-row slices of rows taken in Morton order of the dof positions), 3 = CSR
 * with each XCD sweeping its own contiguous row range (ranges of equal entry
 * counts), 4 = split CSR in dof order (real parts as real entries, nonzero
 * imaginary parts as extra real entries flagged in the column index; A is
 * complex only on the absorbing boundary, so 12 B per entry instead of 20).
 * Kinds 1 and 3 also fix the order of the multi-right-hand-side products
 * (otherwise the faster one as timed on first use).  HELM_EINVAL for any
 * other kind. */
int helm_set_spmv(helm_ctx* ctx, int kind);

/* y = A x  (complex SpMV). */
int helm_apply_A(helm_ctx* ctx, const void* x, void* y, void* stream);

/* z = M^{-1} r (two-level when a coarse mesh was given, else one-level). */
int helm_apply_precond(helm_ctx* ctx, const void* r, void* z, void* stream);

/* z = M1^{-1} r, the one-level ORAS part only. */
int helm_apply_oras(helm_ctx* ctx, const void* r, void* z, void* stream);

/* q = Z E^{-1} Z^T r (two-level setup only). */
int helm_apply_coarse(helm_ctx* ctx, const void* r, void* q, void* stream);

/* q = Z E^{-1} Z^T r exactly as helm_apply_coarse, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): it calls no hipMalloc, hipFree or other
 * allocating routine and records no timing events.  Its work vectors (Z^T r
 * and the coarse solve's forward, backward and update vectors) live in a
 * fixed device scratch of 32 MiB per GPU, set up by helm_create and held
 * until the process ends; a coarse problem whose work vectors exceed it
 * (about 16 (3 n_c + update entries) bytes) fails with HELM_EINVAL.  Every
 * call on a GPU shares that GPU's scratch: calls that overlap on one GPU
 * (other streams, other threads or contexts) race and must be serialised by
 * the caller.  Nothing in the scratch needs clearing between calls (every
 * work vector is written before it is read). */
int helm_apply_coarse_noalloc(helm_ctx* ctx, const void* r, void* q, void* stream);

/* Solve A U = B for nrhs right-hand sides with right-preconditioned GMRES.
 * B and U are device arrays c128, column-major n x nrhs; U is read as the
 * initial guess iff opts->flags has HELM_SOLVE_X0.  info (host, nrhs
 * entries, may be NULL) receives per-RHS results.  Returns HELM_OK when
 * every RHS reached the true relative residual tol, HELM_ENOCONV when some
 * did not (U then holds the last iterates).  ||b|| = 0 gives U = 0 in 0
 * iterations.  The call returns after the work on `stream` is complete. */
int helm_solve(helm_ctx* ctx, int32_t nrhs, const void* B, double tol, const helm_solve_opts* opts,
               void* U, void* stream, helm_solve_info* info);

/* --- Kernel timing (HIP events around every launch of the per-iteration
 *     kernels, on the stream they run on).  Algorithmic bytes count each
 *     stored factor entry (16 B), matrix entry (20 B) and vector entry the
 *     kernel must touch once. --- */

enum {
  HELM_K_TRSV_FWD = 0,    /* batched forward level solves, fine subdomains  */
  HELM_K_TRSV_BWD = 1,    /* batched backward level solves, fine subdomains */
  HELM_K_SPMV = 2,        /* A x and r - A x                               */
  HELM_K_COARSE = 3,      /* Z^T r, coarse solves, Z y                      */
  HELM_K_PROLONG = 4,     /* partition-of-unity prolongation                */
  HELM_K_GS = 5,          /* CGS2 dots, updates, norm, scaling              */
  HELM_K_COUNT = 6
};

/* Server on a context with a factored preconditioner, running on `stream`
 * (NULL = the null stream).  Its slots use the context's multi-right-hand-
 * side work space: while a server exists, helm_solve, helm_assemble and
 * helm_precond_setup on the same context return HELM_ESTATE.  *out is NULL on failure (HELM_ENOMEM when no slot
 * fits in opts->mem_bytes or in device memory). */
int helm_server_create(helm_ctx* ctx, const helm_server_opts* opts, void* stream, helm_server** out);

/* Queues one request: b (device c128[n], read) and u (device c128[n],
 * written with the solution); both must stay valid until the request's
 * completion event.  The tag names the request in its completion event, so
 * a tag still queued or in flight is refused (HELM_EINVAL).  Never blocks. */
int helm_server_submit(helm_server* srv, const void* b, void* u, int64_t tag);

/* Enqueues one Arnoldi step for every active slot on the server's stream
 * and returns without waiting; *active (may be NULL) receives the number of
 * slots stepped (0: nothing in flight). */
int helm_server_launch(helm_server* srv, int32_t* active);

/* Waits for the launched step, advances every slot's least-squares problem,
 * finishes cycles and requests, admits queued requests into free slots, and
 * writes up to `cap` completion events (host array) with their count in
 * *count.  Events beyond cap are kept for the next call. */
int helm_server_finish(helm_server* srv, helm_server_event* events, int32_t cap, int32_t* count);

/* Queued and in-flight requests. */
int helm_server_status(const helm_server* srv, int32_t* queued, int32_t* active);

/* Slots opened so far (their memory is held) and the device bytes the server
 * holds for them (any pointer may be NULL). */
int helm_server_memory(const helm_server* srv, int32_t* slots_open, double* bytes);

/* Frees the server (pending requests are dropped); NULL is accepted. */
void helm_server_destroy(helm_server* srv);

typedef struct helm_kernel_profile {
  int64_t launches;       /* timed launches since the last reset           */
  double milliseconds;    /* summed event-to-event time                    */
  double bytes;           /* summed algorithmic bytes                      */
} helm_kernel_profile;

/* Turn per-launch timing on (1) or off (0); both reset the counters. */
int helm_profile_enable(helm_ctx* ctx, int on);

/* Copy the HELM_K_COUNT counters (completed work only: call after
 * helm_solve returned or after synchronising the stream). */
int helm_profile_read(helm_ctx* ctx, helm_kernel_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
