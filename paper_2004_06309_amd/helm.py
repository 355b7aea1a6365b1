"""ctypes binding of libhelm (include/helm.h).

Argument marshalling only: every step of the solver runs in the library
(host C++ setup, HIP kernels on the GPU).  Device vectors are torch tensors
of dtype complex128 (interleaved re/im doubles); torch only provides device
memory and streams.  Importing this module fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhelm.so")

HELM_OK = 0
HELM_EINVAL = -1
HELM_ESINGULAR = -2
HELM_ENOCONV = -3
HELM_ENUMERIC = -4
HELM_ENOMEM = -5
HELM_ESTATE = -6
HELM_EDEVICE = -7
HELM_SOLVE_X0 = 1
HELM_SOLVE_CGS2 = 2
HELM_SOLVE_BLOCK_GMRES = 4
HELM_SOLVE_GRAPHS = 8

_ERRNAMES = {-1: "EINVAL", -2: "ESINGULAR", -3: "ENOCONV", -4: "ENUMERIC", -5: "ENOMEM", -6: "ESTATE",
             -7: "EDEVICE"}


class HelmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"HELM_{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.c_void_p), ("n_tets", C.c_int64), ("tets", C.c_void_p),
                ("order", C.c_int32)]


class PrecondOpts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("factor_c64", C.c_int32), ("coarse_leaf_size", C.c_int32),
                ("tile_rows", C.c_int32), ("coarse_tile_rows", C.c_int32),
                ("sn_jobs_min", C.c_int32), ("batches", C.c_int32), ("perturb_pivots", C.c_int32),
                ("coarse_launch", C.c_int32), ("split_front_rows", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("flags", C.c_int32), ("block", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("seconds", C.c_double)]


class PrecondStats(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("n_coarse", C.c_int32), ("n_local_total", C.c_int64),
                ("factor_entries", C.c_int64), ("coarse_entries", C.c_int64), ("levels_fwd", C.c_int32),
                ("levels_bwd", C.c_int32), ("max_front", C.c_int32), ("n_supernodes", C.c_int32),
                ("setup_seconds", C.c_double), ("factor_flops", C.c_double), ("factor_c64", C.c_int32),
                ("coarse_grid", C.c_int32), ("n_perturbed", C.c_int32),
                ("factor_seconds", C.c_double), ("batches", C.c_int32), ("reserved", C.c_int32),
                ("factor_scratch_bytes", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32), ("flags", C.c_int32),
                ("tol", C.c_double), ("mem_bytes", C.c_double)]


class ServerEvent(C.Structure):
    _fields_ = [("tag", C.c_int64), ("iterations", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("relres", C.c_double), ("seconds", C.c_double)]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("milliseconds", C.c_double), ("bytes", C.c_double)]


KERNELS = ["trsv_fwd", "trsv_bwd", "spmv", "coarse", "prolong", "gs"]

EXPORTS = {
    "helm_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "helm_destroy": (None, [C.c_void_p]),
    "helm_last_error": (C.c_char_p, [C.c_void_p]),
    "helm_assemble": (C.c_int, [C.c_void_p, C.POINTER(Mesh), C.c_void_p, C.c_double]),
    "helm_ndof": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "helm_dof_coords": (C.c_int, [C.c_void_p, C.c_void_p]),
    "helm_point_source": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_matrix_nnz": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "helm_matrix_csr": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_precond_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Mesh),
                                     C.POINTER(PrecondOpts)]),
    "helm_precond_stats_get": (C.c_int, [C.c_void_p, C.POINTER(PrecondStats)]),
    "helm_subdomain_size": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "helm_subdomain_get": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "helm_coarse_nnz": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "helm_coarse_get": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_set_spmv": (C.c_int, [C.c_void_p, C.c_int]),
    "helm_apply_A": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_apply_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_apply_oras": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_apply_coarse": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_apply_coarse_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "helm_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.POINTER(SolveOpts), C.c_void_p,
                             C.c_void_p, C.POINTER(SolveInfo)]),
    "helm_server_create": (C.c_int, [C.c_void_p, C.POINTER(ServerOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "helm_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "helm_server_launch": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "helm_server_finish": (C.c_int, [C.c_void_p, C.POINTER(ServerEvent), C.c_int32, C.POINTER(C.c_int32)]),
    "helm_server_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "helm_server_memory": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "helm_server_destroy": (None, [C.c_void_p]),
    "helm_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "helm_profile_read": (C.c_int, [C.c_void_p, C.POINTER(KernelProfile)]),
}

_lib = None
# every open context and server, so a program can release them (and their
# device memory) at a point of its choosing rather than at interpreter exit
_live_ctx = weakref.WeakSet()
_live_srv = weakref.WeakSet()


def close_all():
    """Destroys every server, then every context, still open (frees their
    device memory now)."""
    for s in list(_live_srv):
        s.close()
    for h in list(_live_ctx):
        h.close()


def load():
    """Load libhelm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: run `python -m paper_2004_06309_amd.build` first")
        lib = C.CDLL(_LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _mesh(xyz, tets, order):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int64)
    m = Mesh(xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data, int(order))
    return m, (xyz, tets)


def _dev_ptr(t, numel=None, device=None, name="vector"):
    """Device pointer of a contiguous complex128 GPU tensor, after checking
    what the kernels assume: dtype, device, and (when given) its number of
    entries.  The library reads and writes exactly that many entries, so a
    short or complex64 tensor would be accessed out of bounds."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex128:
        raise ValueError(f"{name} must be complex128, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if device is not None and device >= 0 and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Helm:
    """One solver context (helm_ctx).  device=-1 gives a host-only context."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.helm_create(C.byref(h), device)
        if rc != HELM_OK:
            raise HelmError(rc, self.lib.helm_last_error(None).decode())
        self.h = h
        self.device = device
        self._keep = []
        self._servers = weakref.WeakSet()
        _live_ctx.add(self)

    def close(self):
        """Destroys the context, its servers first."""
        for srv in list(getattr(self, "_servers", ())):
            srv.close()
        if getattr(self, "h", None):
            self.lib.helm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != HELM_OK and rc not in allow:
            raise HelmError(rc, self.lib.helm_last_error(self.h).decode())
        return rc

    # ---- setup -------------------------------------------------------------
    def assemble(self, xyz, tets, order, c_tet, omega):
        m, keep = _mesh(xyz, tets, order)
        c = np.ascontiguousarray(np.asarray(c_tet, dtype=np.complex128))
        self._check(self.lib.helm_assemble(self.h, C.byref(m), _ptr(c), float(omega)))
        n = C.c_int64()
        self._check(self.lib.helm_ndof(self.h, C.byref(n)))
        self.n = n.value
        return self.n

    def dof_coords(self):
        out = np.empty((self.n, 3))
        self._check(self.lib.helm_dof_coords(self.h, _ptr(out)))
        return out

    def point_source(self, xs):
        xs = np.ascontiguousarray(xs, dtype=np.float64)
        b = np.empty(self.n, dtype=np.complex128)
        self._check(self.lib.helm_point_source(self.h, _ptr(xs), _ptr(b)))
        return b

    def matrix_csr(self):
        nnz = C.c_int64()
        self._check(self.lib.helm_matrix_nnz(self.h, C.byref(nnz)))
        ptr = np.empty(self.n + 1, dtype=np.int64)
        col = np.empty(nnz.value, dtype=np.int32)
        val = np.empty(nnz.value, dtype=np.complex128)
        self._check(self.lib.helm_matrix_csr(self.h, _ptr(ptr), _ptr(col), _ptr(val)))
        return ptr, col, val

    def precond_setup(self, part, n_sub, overlap, coarse_xyz=None, coarse_tets=None, leaf_size=0, c64=False,
                      coarse_leaf_size=0, tile_rows=0, coarse_tile_rows=0, sn_jobs_min=0,
                      batches=0, perturb_pivots=False, coarse_launch=0, split_front_rows=0):
        """helm_precond_setup: subdomains from the tet partition `part` with
        `overlap` layers, the optional P1 coarse mesh, then the factorisation.
        c64: complex64 factors (True or 1: factorised in complex64 on FP32
        MFMA; 2: factorised in complex128 and rounded once; False or 0:
        complex128); tile_rows / coarse_tile_rows: 16, 32 or 64
        (0: 64 / 16); sn_jobs_min: one-wave supernode jobs threshold (0:
        default, -1: never); batches: 1 to 4 subdomain batches whose level
        sweeps run concurrently (0: 2); perturb_pivots: replace zero or tiny
        pivots and count them instead of failing with HELM_ESINGULAR;
        coarse_launch: 0 timed, 1 per-level launches, 2 one cooperative
        launch for the coarse solve; split_front_rows: fronts of at least
        this many rows factorised by several workgroups each (0: 256, -1:
        never)."""
        part = np.ascontiguousarray(part, dtype=np.int32)
        if c64 not in (False, True, 0, 1, 2):
            raise ValueError("c64 must be False/True or 0, 1, 2")
        opts = PrecondOpts(int(leaf_size), int(c64), int(coarse_leaf_size), int(tile_rows),
                           int(coarse_tile_rows), int(sn_jobs_min), int(batches),
                           1 if perturb_pivots else 0, int(coarse_launch), int(split_front_rows))
        cm = None
        if coarse_xyz is not None:
            cm, keep = _mesh(coarse_xyz, coarse_tets, 1)
            self._keep = keep
        self._check(self.lib.helm_precond_setup(self.h, _ptr(part), int(n_sub), int(overlap),
                                                C.byref(cm) if cm is not None else None, C.byref(opts)))
        self.two_level = cm is not None

    def stats(self):
        s = PrecondStats()
        self._check(self.lib.helm_precond_stats_get(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in PrecondStats._fields_ if f != "reserved"}

    def subdomain(self, i):
        n_i, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.helm_subdomain_size(self.h, int(i), C.byref(n_i), C.byref(nnz)))
        dofs = np.empty(n_i.value, dtype=np.int64)
        D = np.empty(n_i.value)
        ptr = np.empty(n_i.value + 1, dtype=np.int64)
        col = np.empty(nnz.value, dtype=np.int32)
        val = np.empty(nnz.value, dtype=np.complex128)
        self._check(self.lib.helm_subdomain_get(self.h, int(i), _ptr(dofs), _ptr(D), _ptr(ptr), _ptr(col),
                                                _ptr(val)))
        return dofs, D, (ptr, col, val)

    def coarse_Z(self):
        nc, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.helm_coarse_nnz(self.h, C.byref(nc), C.byref(nnz)))
        ptr = np.empty(self.n + 1, dtype=np.int64)
        col = np.empty(nnz.value, dtype=np.int32)
        val = np.empty(nnz.value)
        self._check(self.lib.helm_coarse_get(self.h, _ptr(ptr), _ptr(col), _ptr(val)))
        return nc.value, (ptr, col, val)

    # ---- device operations (torch complex128 tensors) -----------------------
    def set_spmv(self, kind):
        """0: fastest storage as timed at assembly, 1: CSR, 2: sliced ELL in
        Morton row order, 3: CSR with XCD row ranges, 4: split real/imaginary
        CSR (1 and 3 also fix the multi-vector SpMV's order)."""
        self._check(self.lib.helm_set_spmv(self.h, int(kind)))

    def _vec(self, t, name, count=1):
        return _dev_ptr(t, count * self.n, self.device, name)

    def apply_A(self, x, y, stream=None):
        self._check(self.lib.helm_apply_A(self.h, self._vec(x, "x"), self._vec(y, "y"), _stream(stream)))

    def apply_precond(self, r, z, stream=None):
        self._check(self.lib.helm_apply_precond(self.h, self._vec(r, "r"), self._vec(z, "z"), _stream(stream)))

    def apply_oras(self, r, z, stream=None):
        self._check(self.lib.helm_apply_oras(self.h, self._vec(r, "r"), self._vec(z, "z"), _stream(stream)))

    def apply_coarse(self, r, q, stream=None):
        self._check(self.lib.helm_apply_coarse(self.h, self._vec(r, "r"), self._vec(q, "q"), _stream(stream)))

    def apply_coarse_noalloc(self, r, q, stream=None):
        """apply_coarse with its work vectors in the library's fixed device
        scratch (no device allocation)."""
        self._check(self.lib.helm_apply_coarse_noalloc(self.h, self._vec(r, "r"), self._vec(q, "q"),
                                                        _stream(stream)))

    def solve(self, B, U, tol=1e-6, restart=50, maxit=1000, x0=False, stream=None, block=1, classic_cgs2=False,
              block_gmres=False, graphs=False):
        """Solve A U = B; B, U are (n,) or (nrhs, n) complex128 GPU tensors
        (each RHS contiguous); `block` right-hand sides are advanced together.
        `classic_cgs2` selects three-pass CGS2 (default: delayed CGS2);
        `block_gmres` one shared block Krylov space per block (block CGS2 on
        MFMA) instead of pseudo-block GMRES, `graphs` its steps replayed
        from captured HIP graphs.
        Returns (status, [info dicts])."""
        if B.dim() not in (1, 2) or tuple(U.shape) != tuple(B.shape):
            raise ValueError(f"B {tuple(B.shape)} and U {tuple(U.shape)} must both be (n,) or (nrhs, n)")
        nrhs = 1 if B.dim() == 1 else B.shape[0]
        if B.shape[-1] != self.n:
            raise ValueError(f"right-hand sides have {B.shape[-1]} entries, the operator {self.n}")
        info = (SolveInfo * max(nrhs, 1))()
        flags = ((HELM_SOLVE_X0 if x0 else 0) | (HELM_SOLVE_CGS2 if classic_cgs2 else 0)
                 | (HELM_SOLVE_BLOCK_GMRES if block_gmres else 0) | (HELM_SOLVE_GRAPHS if graphs else 0))
        opts = SolveOpts(int(restart), int(maxit), flags, int(block))
        rc = self._check(self.lib.helm_solve(self.h, nrhs, self._vec(B, "B", nrhs), float(tol), C.byref(opts),
                                             self._vec(U, "U", nrhs), _stream(stream), info), allow=(HELM_ENOCONV,))
        return rc, [{f: getattr(info[i], f) for f, _ in SolveInfo._fields_} for i in range(nrhs)]

    # ---- kernel timing -----------------------------------------------------
    def profile(self, on: bool):
        """Time every launch of the per-iteration kernels with HIP events."""
        self._check(self.lib.helm_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        out = (KernelProfile * len(KERNELS))()
        self._check(self.lib.helm_profile_read(self.h, out))
        return {k: {"launches": out[i].launches, "ms": out[i].milliseconds, "bytes": out[i].bytes}
                for i, k in enumerate(KERNELS)}


class Server:
    """Continuous-batching server over a Helm context (helm_server_*):
    submit(b, u, tag) queues a request; launch() enqueues one Arnoldi step
    for every slot in flight; finish() waits for it and returns the
    completion events as dicts.  Keeps the submitted tensors alive until
    their completion."""

    def __init__(self, helm, slots=0, restart=50, maxit=1000, tol=1e-6, stream=None, classic_cgs2=False,
                 mem_bytes=0.0):
        self.helm = helm
        self.lib = helm.lib
        opts = ServerOpts(int(slots), int(restart), int(maxit), HELM_SOLVE_CGS2 if classic_cgs2 else 0, float(tol),
                          float(mem_bytes))
        out = C.c_void_p()
        helm._check(self.lib.helm_server_create(helm.h, C.byref(opts), _stream(stream), C.byref(out)))
        self.h = out
        self._alive = {}
        self._ev = (ServerEvent * 64)()
        _live_srv.add(self)
        helm._servers.add(self)

    def submit(self, b, u, tag):
        """Queues b -> u under `tag`; the library refuses a tag that is still
        queued or in flight, so the tensors kept alive here are keyed by it."""
        pb = self.helm._vec(b, "b")
        pu = self.helm._vec(u, "u")
        self.helm._check(self.lib.helm_server_submit(self.h, pb, pu, int(tag)))
        self._alive[int(tag)] = (b, u)

    def launch(self):
        a = C.c_int32()
        self.helm._check(self.lib.helm_server_launch(self.h, C.byref(a)))
        return a.value

    def finish(self):
        out = []
        while True:
            k = C.c_int32()
            self.helm._check(self.lib.helm_server_finish(self.h, self._ev, len(self._ev), C.byref(k)))
            for i in range(k.value):
                e = self._ev[i]
                out.append({f: getattr(e, f) for f, _ in ServerEvent._fields_ if f != "reserved"})
                self._alive.pop(e.tag, None)
            if k.value < len(self._ev):
                return out

    def status(self):
        q, a = C.c_int32(), C.c_int32()
        self.lib.helm_server_status(self.h, C.byref(q), C.byref(a))
        return q.value, a.value

    def memory(self):
        """(slots opened, device bytes held for them)."""
        k, b = C.c_int32(), C.c_double()
        self.helm._check(self.lib.helm_server_memory(self.h, C.byref(k), C.byref(b)))
        return k.value, b.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.helm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(w, device=0, leaf_size=0, c64=False, **opts):
    """Helm context assembled and preconditioned for a workloads.Workload;
    opts: coarse_leaf_size, tile_rows, coarse_tile_rows,
    sn_jobs_min, batches (see precond_setup)."""
    h = Helm(device)
    h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    h.precond_setup(w.part, w.n_sub, w.overlap, w.coarse_xyz, w.coarse_tets, leaf_size, c64, **opts)
    return h


def load_vector(h: Helm, w):
    """Right-hand side of a workload (point or nodal source), host complex128."""
    if w.source_point is not None:
        return h.point_source(w.source_point)
    b = np.zeros(h.n, dtype=np.complex128)
    b[w.source_node] = 1.0
    return b
