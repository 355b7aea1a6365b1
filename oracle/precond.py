"""Oracle: one- and two-level ORAS preconditioners and the full solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

One level (eq. oras):   M_1^{-1} r = sum_i R_i^T D_i A_i^{-1} R_i r.
Two levels (eq. 2lvl):  M^{-1} r = M_1^{-1} (r - A q) + q,  q = Z E^{-1} Z^T r.
The local and coarse solves are direct (the paper's local solves use a sparse
direct solver); here SuperLU through scipy.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import coarse, dd, fem
from .gmres import gmres


class Oras:
    """ORAS preconditioner of a Problem for a given non-overlapping tet partition."""

    def __init__(self, problem: fem.Problem, part, n_sub, delta, coarse_mesh=None, factor=True,
                 only=None):
        self.problem = problem
        self.subs = dd.decompose(problem, np.asarray(part), n_sub, delta)
        self.only = list(range(n_sub)) if only is None else list(only)
        for i in self.only:
            s = self.subs[i]
            s.A = dd.local_matrix(problem, s).tocsc()
            s.lu = spla.splu(s.A) if factor else None
        self.Z = self.E = self.Elu = None
        if coarse_mesh is not None:
            self.Z, _ = coarse.interpolation(problem, *coarse_mesh)
            self.E = coarse.galerkin(problem.A, self.Z)
            self.Elu = spla.splu(self.E)

    def local_solve(self, i, rloc):
        return self.subs[i].lu.solve(np.asarray(rloc, dtype=np.complex128))

    def one_level(self, r):
        z = np.zeros(self.problem.n, dtype=np.complex128)
        for i in self.only:
            s = self.subs[i]
            z[s.dofs] += s.D * self.local_solve(i, r[s.dofs])
        return z

    def coarse_correction(self, r):
        return self.Z @ self.Elu.solve(self.Z.T @ r)

    def apply(self, r):
        r = np.asarray(r, dtype=np.complex128)
        if self.Z is None:
            return self.one_level(r)
        q = self.coarse_correction(r)
        return self.one_level(r - self.problem.A @ q) + q


def solve(problem: fem.Problem, b, precond=None, tol=1e-6, restart=50, maxit=1000, **kw):
    A = problem.A
    return gmres(lambda v: A @ v, b, None if precond is None else precond.apply, tol, restart, maxit, **kw)


def build(workload, factor=True, only=None):
    """Problem, load vector and preconditioner for a workloads.Workload."""
    P = fem.Problem(workload.xyz, workload.tets, workload.order, workload.c_tet, workload.omega)
    if workload.source_point is not None:
        b = P.point_source(workload.source_point)
    else:
        b = P.nodal_source(workload.source_node)
    cm = None if workload.coarse_xyz is None else (workload.coarse_xyz, workload.coarse_tets)
    M = Oras(P, workload.part, workload.n_sub, workload.overlap, cm, factor=factor, only=only)
    return P, b, M
