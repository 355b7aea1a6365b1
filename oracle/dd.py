"""Oracle: overlapping decomposition, R_i, D_i and impedance local matrices A_i.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows the construction of the one-level ORAS preconditioner (eq. oras):
M_1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i over an overlapping decomposition
{Gamma_i} of the mesh, with Boolean restrictions R_i, diagonal partition-of-
unity matrices D_i and local Helmholtz matrices A_i carrying absorbing
(impedance) conditions on the subdomain interfaces.  Readings (the paper
defers the details to its citation of Bonazzoli et al. 2018):

* Gamma_i^(0) = tets with part == i; one overlap layer adds every tet sharing
  a vertex with the current set; Gamma_i = Gamma_i^(delta);
* local dofs = dofs of Gamma_i's tets in ascending global order;
* l(j) = smallest layer l such that dof j belongs to a tet of Gamma_i^(l);
  chi_i(j) = max(0, 1 - l(j)/delta) (chi_i = 1 for delta = 0) and
  D_i(j) = chi_i(j) / sum_k chi_k(j);
* A_i is assembled from Gamma_i's tets only; physical boundary faces keep
  their condition, and the artificial faces (faces of exactly one Gamma_i tet
  that are interior to the global mesh) receive the same first-order
  impedance term i int k u v as the physical absorbing faces, with the k of
  their tet.  Dirichlet dofs keep identity rows/columns.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import fem


def grow_layers(tets, nv, part, i, delta):
    """Tet layer index of Gamma_i^(l) for l = 0..delta: -1 if not in Gamma_i."""
    layer = np.full(tets.shape[0], -1, dtype=np.int64)
    layer[part == i] = 0
    for l in range(1, delta + 1):
        cur = layer >= 0
        verts = np.zeros(nv, dtype=bool)
        verts[tets[cur].ravel()] = True
        touch = verts[tets].any(axis=1)
        layer[touch & ~cur] = l
    return layer


@dataclass
class Subdomain:
    tets: np.ndarray  # tet indices of Gamma_i
    dofs: np.ndarray  # global dofs, ascending (R_i)
    level: np.ndarray  # l(j) per local dof
    chi: np.ndarray  # chi_i per local dof
    D: np.ndarray = None  # partition of unity per local dof
    A: sp.csr_matrix = None  # local impedance matrix
    art_faces: np.ndarray = None


def decompose(problem: fem.Problem, part, n_sub, delta):
    """Subdomains with their dofs, layers, chi and D (no matrices yet)."""
    tets = problem.tets
    nv = problem.xyz.shape[0]
    tet_dofs = problem.dofs.tet_dofs
    subs = []
    chi_sum = np.zeros(problem.n)
    for i in range(n_sub):
        layer = grow_layers(tets, nv, part, i, delta)
        st = np.nonzero(layer >= 0)[0]
        lev_g = np.full(problem.n, np.iinfo(np.int64).max)
        np.minimum.at(lev_g, tet_dofs[st].ravel(), np.repeat(layer[st], tet_dofs.shape[1]))
        dofs = np.nonzero(lev_g < np.iinfo(np.int64).max)[0]
        level = lev_g[dofs]
        if delta == 0:
            chi = np.ones(dofs.size)
        else:
            chi = np.maximum(0.0, 1.0 - level / delta)
        chi_sum[dofs] += chi
        subs.append(Subdomain(st, dofs, level, chi))
    for s in subs:
        s.D = s.chi / chi_sum[s.dofs]
    return subs


def local_matrix(problem: fem.Problem, sub: Subdomain):
    """A_i: Helmholtz operator of Gamma_i with impedance on its artificial faces."""
    tets = problem.tets
    nv = problem.xyz.shape[0]
    faces, owner = fem.tet_faces(tets[sub.tets])
    owner = sub.tets[owner]
    cnt_loc, keys_loc = fem.face_counts(faces, nv)
    # global multiplicity of each local face
    gk_sorted = problem.global_face_keys_sorted()
    gcount = np.searchsorted(gk_sorted, keys_loc, side="right") - np.searchsorted(gk_sorted, keys_loc, side="left")
    once = cnt_loc == 1
    artificial = once & (gcount == 2)
    physical = once & (gcount == 1)
    ztop = problem.xyz[:, 2].min()
    dirich = np.all(problem.xyz[faces, 2] == ztop, axis=1)
    imp = artificial | (physical & ~dirich)
    _, K, Mk2, Bk = fem.assemble_parts(problem.xyz, tets, problem.order, problem.c_tet, problem.omega,
                                       tet_subset=sub.tets, imp_faces=faces[imp], imp_owner=owner[imp],
                                       dofs=problem.dofs)
    Aglob = -K + Mk2 + 1j * Bk
    R = restriction(sub.dofs, problem.n)
    Aloc = (R @ Aglob @ R.T).tocsr()
    mask = problem.dir_mask[sub.dofs]
    sub.art_faces = faces[artificial]
    return fem.apply_dirichlet(Aloc, mask)


def restriction(dofs, n):
    """Boolean R_i (n_i x n): (R_i x)[k] = x[dofs[k]]."""
    m = dofs.size
    return sp.csr_matrix((np.ones(m), (np.arange(m), dofs)), shape=(m, n))


def artificial_dofs(problem: fem.Problem, sub: Subdomain):
    """Global dofs on the artificial interface faces of Gamma_i."""
    if sub.art_faces is None or len(sub.art_faces) == 0:
        return np.zeros(0, dtype=np.int64)
    return np.unique(problem.dofs.face_dofs(sub.art_faces).ravel())
