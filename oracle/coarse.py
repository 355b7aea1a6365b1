"""Oracle: coarse space of the two-level preconditioner (eq. 2lvl).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

M^{-1} = M_1^{-1}(I - A Q) + Q with Q = Z E^{-1} Z^T and E = Z^T A Z, where Z
carries the P1 finite-element space of a coarse mesh Gamma_H into the fine
space.  Readings: Z (n x n_c) is the prolongation, Z[j, l] = phi^H_l(x_j) for
fine dof position x_j and coarse P1 basis function phi^H_l; the transpose is
the plain (unconjugated) one, so E stays complex symmetric; coarse nodes on
the Dirichlet top face are not unknowns; fine Dirichlet rows of Z are zero;
barycentric values below 1e-12 in magnitude are snapped to 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def interpolation(problem: fem.Problem, cxyz, ctets):
    """Z as a real CSR matrix (n x n_c) and the coarse node id of each column."""
    cxyz = np.asarray(cxyz, dtype=np.float64)
    ctets = np.asarray(ctets, dtype=np.int64)
    pts = problem.dofs.coords()
    t, lam = fem.locate_points(cxyz, ctets, pts)
    if np.any(t < 0):
        raise ValueError("fine dof outside the coarse mesh")
    lam[np.abs(lam) < 1e-12] = 0.0
    ztop = cxyz[:, 2].min()
    free = cxyz[:, 2] != ztop
    col_of_node = np.full(cxyz.shape[0], -1, dtype=np.int64)
    col_of_node[free] = np.arange(free.sum())
    rows = np.repeat(np.arange(pts.shape[0]), 4)
    nodes = ctets[t].ravel()
    vals = lam.ravel()
    keep = (col_of_node[nodes] >= 0) & (vals != 0.0) & ~problem.dir_mask[rows]
    Z = sp.csr_matrix((vals[keep], (rows[keep], col_of_node[nodes[keep]])),
                      shape=(pts.shape[0], int(free.sum())))
    Z.sum_duplicates()
    return Z, np.nonzero(free)[0]


def galerkin(A, Z):
    """E = Z^T A Z (plain transpose)."""
    return (Z.T @ A @ Z).tocsc()
