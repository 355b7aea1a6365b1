"""Oracle: the ORAS preconditioner with its subdomain factors held by a pool
of worker processes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The arithmetic is that of ``precond.Oras``: every worker builds the local
impedance matrices A_i of its subdomains with ``dd.local_matrix`` and factors
them with SuperLU; the one-level application (eq. oras)

    z = sum_i R_i^T D_i A_i^{-1} R_i r

reads r from shared memory, each worker writes A_i^{-1} R_i r of its
subdomains into a shared buffer, and the parent forms the weighted sum in
subdomain order, so the result equals ``Oras.one_level`` bit for bit.  The
coarse level (eq. 2lvl) runs in the parent as in ``Oras``.  Only the memory
of the factors is spread over processes: a mid-size problem whose 64
factorisations do not fit one process's share of memory, or a timing of the
oracle on all host cores, uses this.  Workers are forked, so the creating
process must not have initialised a GPU.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time
from multiprocessing import shared_memory

import numpy as np
import scipy.sparse.linalg as spla

from . import coarse, dd, fem


def _worker(conn, problem, subs, mine, offs, shm_r, shm_y, n, ny, verbose):
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except Exception:  # noqa: BLE001
        pass
    r_sh = shared_memory.SharedMemory(name=shm_r)
    y_sh = shared_memory.SharedMemory(name=shm_y)
    r = np.ndarray((n,), dtype=np.complex128, buffer=r_sh.buf)
    y = np.ndarray((ny,), dtype=np.complex128, buffer=y_sh.buf)
    lus, times = {}, {}
    for i in mine:
        t0 = time.perf_counter()
        Ai = dd.local_matrix(problem, subs[i]).tocsc()
        t1 = time.perf_counter()
        lus[i] = spla.splu(Ai)
        t2 = time.perf_counter()
        times[i] = {"local_matrix_s": t1 - t0, "factor_s": t2 - t1, "n_i": int(Ai.shape[0]),
                    "lu_nnz": int(lus[i].L.nnz + lus[i].U.nnz)}
        if verbose:
            print(f"[oracle pool] subdomain {i}: n_i {Ai.shape[0]}, factor {t2 - t1:.1f} s", flush=True)
    conn.send(("ready", times))
    while True:
        msg = conn.recv()
        if msg == "close":
            break
        if msg == "solve":
            ts = {}
            for i in mine:
                t0 = time.perf_counter()
                s = subs[i]
                y[offs[i]:offs[i] + s.dofs.size] = lus[i].solve(np.ascontiguousarray(r[s.dofs]))
                ts[i] = time.perf_counter() - t0
            conn.send(("done", ts))
    del r, y
    r_sh.close()
    y_sh.close()
    conn.close()


class PoolOras:
    """ORAS preconditioner (one- or two-level) of a Problem, local factors in
    `workers` processes (each owns a fixed set of subdomains, assigned
    largest first to the least loaded worker); `only` restricts the
    subdomains that are factored (a timing sample)."""

    def __init__(self, problem: fem.Problem, part, n_sub, delta, coarse_mesh=None, workers=None, only=None,
                 verbose=False):
        self.problem = problem
        self.subs = dd.decompose(problem, np.asarray(part), n_sub, delta)
        self.only = list(range(n_sub)) if only is None else list(only)
        n = problem.n
        sizes = [self.subs[i].dofs.size for i in self.only]
        self.offs = {}
        o = 0
        for i, sz in zip(self.only, sizes):
            self.offs[i] = o
            o += sz
        ny = max(o, 1)
        if workers is None:
            workers = len(os.sched_getaffinity(0))
        workers = max(1, min(workers, len(self.only)))
        self.workers = workers
        load = [0] * workers
        mine = [[] for _ in range(workers)]
        for i in sorted(self.only, key=lambda i: -self.subs[i].dofs.size):
            k = int(np.argmin(load))
            mine[k].append(i)
            load[k] += self.subs[i].dofs.size
        self._shm_r = shared_memory.SharedMemory(create=True, size=16 * n)
        self._shm_y = shared_memory.SharedMemory(create=True, size=16 * ny)
        self._r = np.ndarray((n,), dtype=np.complex128, buffer=self._shm_r.buf)
        self._y = np.ndarray((ny,), dtype=np.complex128, buffer=self._shm_y.buf)
        ctx = mp.get_context("fork")
        self._conns, self._procs = [], []
        t0 = time.perf_counter()
        for k in range(workers):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(b, problem, self.subs, mine[k], self.offs, self._shm_r.name,
                                                   self._shm_y.name, n, ny, verbose), daemon=True)
            p.start()
            self._conns.append(a)
            self._procs.append(p)
        self.sub_times = {}
        for a in self._conns:
            tag, times = a.recv()
            self.sub_times.update(times)
        self.factor_wall_s = time.perf_counter() - t0
        self.last_solve_times = {}
        self.Z = self.E = self.Elu = None
        if coarse_mesh is not None:
            self.Z, _ = coarse.interpolation(problem, *coarse_mesh)
            self.E = coarse.galerkin(problem.A, self.Z)
            self.Elu = spla.splu(self.E)

    def one_level(self, r):
        self._r[:] = r
        for a in self._conns:
            a.send("solve")
        self.last_solve_times = {}
        for a in self._conns:
            tag, ts = a.recv()
            self.last_solve_times.update(ts)
        z = np.zeros(self.problem.n, dtype=np.complex128)
        for i in self.only:  # subdomain order, as Oras.one_level
            s = self.subs[i]
            z[s.dofs] += s.D * self._y[self.offs[i]:self.offs[i] + s.dofs.size]
        return z

    def solve_each(self, r):
        """Local solves of r on one worker at a time (no other solve running):
        {subdomain: seconds}, the uncontended single-core times."""
        self._r[:] = r
        ts = {}
        for a in self._conns:
            a.send("solve")
            tag, t = a.recv()
            ts.update(t)
        return ts

    def coarse_correction(self, r):
        return self.Z @ self.Elu.solve(self.Z.T @ r)

    def apply(self, r):
        r = np.asarray(r, dtype=np.complex128)
        if self.Z is None:
            return self.one_level(r)
        q = self.coarse_correction(r)
        return self.one_level(r - self.problem.A @ q) + q

    def close(self):
        for a in getattr(self, "_conns", []):
            try:
                a.send("close")
            except (OSError, BrokenPipeError):
                pass
        for p in getattr(self, "_procs", []):
            p.join(timeout=30)
        self._conns, self._procs = [], []
        for name in ("_r", "_y"):
            if hasattr(self, name):
                delattr(self, name)
        for shm in (getattr(self, "_shm_r", None), getattr(self, "_shm_y", None)):
            if shm is not None:
                shm.close()
                shm.unlink()
        self._shm_r = self._shm_y = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
