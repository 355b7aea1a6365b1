// extern "C" entry points of libhelm (declared in include/helm.h).  Every
// call converts internal exceptions into a status code and keeps the message
// for helm_last_error.
#include <algorithm>
#include <cstring>
#include <memory>
#include <new>

#include "ctx.hpp"

using namespace helm;

struct helm_server;

struct helm_ctx {
  Ctx c;
  int servers = 0;                 // live servers on this context
  std::vector<helm_server*> srvs;  // them (detached when the context goes first)
};

struct helm_server {
  helm_ctx* ctx;                   // null once the context was destroyed
  std::unique_ptr<Server> srv;
  std::vector<helm_server_event> pending;  // completions not yet reported
};

namespace {
// A server whose context was destroyed: every call but destroy fails.
int detached(const helm_server* s) { return !s->ctx || !s->srv ? HELM_ESTATE : HELM_OK; }
}  // namespace

namespace {

thread_local std::string g_create_err;

template <class F>
int guarded(helm_ctx* h, F&& f) {
  if (!h) return HELM_EINVAL;
  try {
    if (h->c.device >= 0) HELM_HIP(hipSetDevice(h->c.device));
    int r = f(h->c);
    if (r == HELM_OK) h->c.err.clear();
    return r;
  } catch (const Error& e) {
    h->c.err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    h->c.err = "host allocation failed";
    return HELM_ENOMEM;
  } catch (const std::exception& e) {
    h->c.err = e.what();
    return HELM_EINVAL;
  }
}

template <class F>
int guarded_const(const helm_ctx* h, F&& f) {
  return guarded(const_cast<helm_ctx*>(h), std::forward<F>(f));
}

void need(bool ok, int code, const char* msg) {
  if (!ok) fail(code, msg);
}

}  // namespace

extern "C" {

int helm_create(helm_ctx** out, int device_ordinal) {
  if (!out) return HELM_EINVAL;
  *out = nullptr;
  try {
    if (device_ordinal >= 0) {
      int count = 0;
      if (hipGetDeviceCount(&count) != hipSuccess || device_ordinal >= count)
        fail(HELM_EDEVICE, "no HIP device " + std::to_string(device_ordinal));
      HELM_HIP(hipSetDevice(device_ordinal));
      // the device's fixed scratch (allocation-free entry point): its address,
      // once per device, with the device current
      HELM_HIP(dev::scratch_init(device_ordinal));
    } else if (device_ordinal != -1) {
      fail(HELM_EINVAL, "device_ordinal must be >= 0, or -1 for a host-only context");
    }
    helm_ctx* h = new helm_ctx;
    h->c.device = device_ordinal;
    *out = h;
    g_create_err.clear();
    return HELM_OK;
  } catch (const Error& e) {
    g_create_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_err = "host allocation failed";
    return HELM_ENOMEM;
  }
}

void helm_destroy(helm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->c.device >= 0) (void)hipSetDevice(ctx->c.device);
  // servers still open on this context lose their solver state now (their
  // handles stay valid for helm_server_destroy, every other call fails)
  for (helm_server* s : ctx->srvs) {
    if (s->srv && s->srv->inflight) (void)hipEventSynchronize(s->srv->done_ev);
    s->srv.reset();
    s->ctx = nullptr;
  }
  delete ctx;
}

const char* helm_last_error(const helm_ctx* ctx) {
  if (!ctx) return g_create_err.c_str();
  return ctx->c.err.c_str();
}

int helm_assemble(helm_ctx* ctx, const helm_mesh* mesh, const double* c_tet, double omega) {
  return guarded(ctx, [&](Ctx& c) {
    need(ctx->servers == 0, HELM_ESTATE, "a server is using this context");
    need(mesh && c_tet, HELM_EINVAL, "mesh and c_tet are required");
    need(omega > 0, HELM_EINVAL, "omega must be positive");
    c.free_precond();
    c.assembled = false;
    build_discretization(c.D, *mesh, c_tet, omega);
    if (c.device >= 0) upload_matrix(c);
    c.assembled = true;
    return HELM_OK;
  });
}

int helm_ndof(const helm_ctx* ctx, int64_t* n) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(n, HELM_EINVAL, "null output");
    *n = c.D.n;
    return HELM_OK;
  });
}

int helm_dof_coords(const helm_ctx* ctx, double* xyz) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(xyz, HELM_EINVAL, "null output");
    for (int64_t d = 0; d < c.D.n; ++d) c.D.dof_coord(d, xyz + 3 * d);
    return HELM_OK;
  });
}

int helm_point_source(const helm_ctx* ctx, const double* xs, double* b) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(xs && b, HELM_EINVAL, "null argument");
    double lam[4], phi[10];
    int64_t t = locate_point(c.D.xyz, c.D.tets, xs, lam);
    need(t >= 0, HELM_EINVAL, "source point outside the mesh");
    std::memset(b, 0, sizeof(double) * 2 * c.D.n);
    basis_values(c.D.order, lam, phi);
    for (int a = 0; a < c.D.nloc; ++a) {
      int64_t d = c.D.tet_dofs[(size_t)t * c.D.nloc + a];
      if (!c.D.dir_mask[d]) b[2 * d] = phi[a];
    }
    return HELM_OK;
  });
}

int helm_matrix_nnz(const helm_ctx* ctx, int64_t* nnz) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(nnz, HELM_EINVAL, "null output");
    *nnz = c.D.A.nnz();
    return HELM_OK;
  });
}

int helm_matrix_csr(const helm_ctx* ctx, int64_t* rowptr, int32_t* col, double* val) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(rowptr && col && val, HELM_EINVAL, "null output");
    std::memcpy(rowptr, c.D.A.ptr.data(), sizeof(int64_t) * (c.D.n + 1));
    std::memcpy(col, c.D.A.col.data(), sizeof(int32_t) * c.D.A.nnz());
    std::memcpy(val, c.D.A.val.data(), sizeof(cplx) * c.D.A.nnz());
    return HELM_OK;
  });
}

int helm_precond_setup(helm_ctx* ctx, const int32_t* tet_part, int32_t n_sub, int32_t overlap,
                       const helm_mesh* coarse, const helm_precond_opts* opts) {
  return guarded(ctx, [&](Ctx& c) {
    need(ctx->servers == 0, HELM_ESTATE, "a server is using this context");
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(tet_part, HELM_EINVAL, "tet_part is required");
    try {
      precond_setup(c, tet_part, n_sub, overlap, coarse, opts);
    } catch (...) {
      c.free_precond();
      throw;
    }
    return HELM_OK;
  });
}

int helm_precond_stats_get(const helm_ctx* ctx, helm_precond_stats* stats) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(stats, HELM_EINVAL, "null output");
    *stats = c.stats;
    return HELM_OK;
  });
}

int helm_subdomain_size(const helm_ctx* ctx, int32_t i, int64_t* n_i, int64_t* nnz_i) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(i >= 0 && i < c.n_sub, HELM_EINVAL, "subdomain index out of range");
    if (n_i) *n_i = (int64_t)c.subs[i].dofs.size();
    if (nnz_i) *nnz_i = c.subs[i].A.nnz();
    return HELM_OK;
  });
}

int helm_subdomain_get(const helm_ctx* ctx, int32_t i, int64_t* dofs, double* D, int64_t* rowptr, int32_t* col,
                       double* val) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(i >= 0 && i < c.n_sub, HELM_EINVAL, "subdomain index out of range");
    const SubdomainHost& S = c.subs[i];
    if (dofs) std::memcpy(dofs, S.dofs.data(), sizeof(int64_t) * S.dofs.size());
    if (D) std::memcpy(D, S.D.data(), sizeof(double) * S.D.size());
    if (rowptr) std::memcpy(rowptr, S.A.ptr.data(), sizeof(int64_t) * S.A.ptr.size());
    if (col) std::memcpy(col, S.A.col.data(), sizeof(int32_t) * S.A.col.size());
    if (val) std::memcpy(val, S.A.val.data(), sizeof(cplx) * S.A.val.size());
    return HELM_OK;
  });
}

int helm_coarse_nnz(const helm_ctx* ctx, int64_t* n_c, int64_t* nnz) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.precond_ready && c.two_level, HELM_ESTATE, "no coarse level");
    if (n_c) *n_c = c.Z.m;
    if (nnz) *nnz = (int64_t)c.Z.col.size();
    return HELM_OK;
  });
}

int helm_coarse_get(const helm_ctx* ctx, int64_t* rowptr, int32_t* col, double* val) {
  return guarded_const(ctx, [&](Ctx& c) {
    need(c.precond_ready && c.two_level, HELM_ESTATE, "no coarse level");
    need(rowptr && col && val, HELM_EINVAL, "null output");
    std::memcpy(rowptr, c.Z.ptr.data(), sizeof(int64_t) * c.Z.ptr.size());
    std::memcpy(col, c.Z.col.data(), sizeof(int32_t) * c.Z.col.size());
    std::memcpy(val, c.Z.val.data(), sizeof(double) * c.Z.val.size());
    return HELM_OK;
  });
}

int helm_set_spmv(helm_ctx* ctx, int kind) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(kind >= 0 && kind <= 4, HELM_EINVAL, "kind must be 0, 1, 2, 3 or 4");
    c.spmv_kind = kind == 0 ? c.spmv_auto : kind;
    c.blk_force = kind == 1 || kind == 3 ? kind : 0;
    return HELM_OK;
  });
}

int helm_apply_A(helm_ctx* ctx, const void* x, void* y, void* stream) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.assembled, HELM_ESTATE, "call helm_assemble first");
    need(x && y, HELM_EINVAL, "null vector");
    apply_A(c, (const double*)x, (double*)y, (hipStream_t)stream);
    HELM_HIP(hipGetLastError());
    return HELM_OK;
  });
}

int helm_apply_precond(helm_ctx* ctx, const void* r, void* z, void* stream) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(r && z, HELM_EINVAL, "null vector");
    apply_precond(c, (const double*)r, (double*)z, (hipStream_t)stream);
    HELM_HIP(hipGetLastError());
    return HELM_OK;
  });
}

int helm_apply_oras(helm_ctx* ctx, const void* r, void* z, void* stream) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(r && z, HELM_EINVAL, "null vector");
    apply_oras(c, (const double*)r, (double*)z, nullptr, (hipStream_t)stream);
    HELM_HIP(hipGetLastError());
    return HELM_OK;
  });
}

int helm_apply_coarse(helm_ctx* ctx, const void* r, void* q, void* stream) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.precond_ready && c.two_level, HELM_ESTATE, "no coarse level");
    need(r && q, HELM_EINVAL, "null vector");
    apply_coarse(c, (const double*)r, (double*)q, (hipStream_t)stream);
    HELM_HIP(hipGetLastError());
    return HELM_OK;
  });
}

int helm_apply_coarse_noalloc(helm_ctx* ctx, const void* r, void* q, void* stream) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.precond_ready && c.two_level, HELM_ESTATE, "no coarse level");
    need(r && q, HELM_EINVAL, "null vector");
    const size_t need_b = coarse_scratch_bytes(c);
    if (need_b > dev::kScratchBytes)
      fail(HELM_EINVAL, "the coarse correction needs " + std::to_string(need_b) +
                            " bytes of work space, more than the fixed scratch of " +
                            std::to_string(dev::kScratchBytes) + " bytes; use helm_apply_coarse");
    void* scratch = dev::scratch_ptr(c.device);
    need(scratch != nullptr, HELM_ESTATE, "device scratch not initialised");
    apply_coarse_scratch(c, (const double*)r, (double*)q, (hipStream_t)stream, scratch);
    HELM_HIP(hipGetLastError());
    return HELM_OK;
  });
}

int helm_solve(helm_ctx* ctx, int32_t nrhs, const void* B, double tol, const helm_solve_opts* opts, void* U,
               void* stream, helm_solve_info* info) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(ctx->servers == 0, HELM_ESTATE, "a server is using this context");
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(nrhs >= 0, HELM_EINVAL, "nrhs must be >= 0");
    need(nrhs == 0 || (B && U), HELM_EINVAL, "null vector");
    return solve(c, nrhs, (const double*)B, tol, opts, (double*)U, (hipStream_t)stream, info);
  });
}

int helm_profile_enable(helm_ctx* ctx, int on) {
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    c.prof.reset();
    c.prof.on = on != 0;
    return HELM_OK;
  });
}

int helm_profile_read(helm_ctx* ctx, helm_kernel_profile* out) {
  return guarded(ctx, [&](Ctx& c) {
    need(out, HELM_EINVAL, "null output");
    if (!c.prof.pending.empty()) c.prof.harvest();
    for (int k = 0; k < HELM_K_COUNT; ++k) out[k] = c.prof.acc[k];
    return HELM_OK;
  });
}


int helm_server_create(helm_ctx* ctx, const helm_server_opts* opts, void* stream, helm_server** out) {
  if (!out) return HELM_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&](Ctx& c) {
    need(c.device >= 0, HELM_ESTATE, "host-only context");
    need(c.precond_ready, HELM_ESTATE, "call helm_precond_setup first");
    need(ctx->servers == 0, HELM_ESTATE, "a server already uses this context");
    need(!opts || (opts->slots >= 0 && opts->slots <= 16), HELM_EINVAL, "slots must be 0..16");
    need(!opts || opts->tol >= 0, HELM_EINVAL, "tol must be >= 0");
    need(!opts || opts->mem_bytes >= 0, HELM_EINVAL, "mem_bytes must be >= 0");
    std::unique_ptr<helm_server> h(new helm_server);
    h->ctx = ctx;
    h->srv.reset(new Server(c, opts, (hipStream_t)stream));
    ctx->servers++;
    ctx->srvs.push_back(h.get());
    *out = h.release();
    return HELM_OK;
  });
}

int helm_server_submit(helm_server* srv, const void* b, void* u, int64_t tag) {
  if (!srv) return HELM_EINVAL;
  if (detached(srv)) return HELM_ESTATE;
  return guarded(srv->ctx, [&](Ctx&) {
    need(b && u, HELM_EINVAL, "null vector");
    srv->srv->submit((const double*)b, (double*)u, tag);
    return HELM_OK;
  });
}

int helm_server_launch(helm_server* srv, int32_t* active) {
  if (!srv) return HELM_EINVAL;
  if (detached(srv)) return HELM_ESTATE;
  return guarded(srv->ctx, [&](Ctx&) {
    need(!srv->srv->inflight, HELM_ESTATE, "a step is already launched");
    const int a = srv->srv->launch();
    if (active) *active = a;
    return HELM_OK;
  });
}

int helm_server_finish(helm_server* srv, helm_server_event* events, int32_t cap, int32_t* count) {
  if (!srv) return HELM_EINVAL;
  if (detached(srv)) return HELM_ESTATE;
  return guarded(srv->ctx, [&](Ctx&) {
    need(cap >= 0 && (cap == 0 || events), HELM_EINVAL, "bad event buffer");
    srv->srv->finish(srv->pending);
    const int32_t k = std::min<int32_t>(cap, (int32_t)srv->pending.size());
    for (int32_t i = 0; i < k; ++i) events[i] = srv->pending[i];
    srv->pending.erase(srv->pending.begin(), srv->pending.begin() + k);
    if (count) *count = k;
    return HELM_OK;
  });
}

int helm_server_status(const helm_server* srv, int32_t* queued, int32_t* active) {
  if (!srv) return HELM_EINVAL;
  if (detached(srv)) return HELM_ESTATE;
  if (queued) *queued = (int32_t)srv->srv->queue.size();
  if (active) *active = srv->srv->active();
  return HELM_OK;
}

int helm_server_memory(const helm_server* srv, int32_t* slots_open, double* bytes) {
  if (!srv) return HELM_EINVAL;
  if (detached(srv)) return HELM_ESTATE;
  if (slots_open) *slots_open = std::min(srv->srv->slots_n, srv->ctx->c.blk_bases);
  if (bytes) *bytes = srv->srv->held();
  return HELM_OK;
}

void helm_server_destroy(helm_server* srv) {
  if (!srv) return;
  if (srv->ctx) {
    if (srv->ctx->c.device >= 0) (void)hipSetDevice(srv->ctx->c.device);
    if (srv->srv && srv->srv->inflight) (void)hipEventSynchronize(srv->srv->done_ev);
    srv->ctx->servers--;
    auto& v = srv->ctx->srvs;
    v.erase(std::remove(v.begin(), v.end(), srv), v.end());
  }
  delete srv;
}

}  // extern "C"
