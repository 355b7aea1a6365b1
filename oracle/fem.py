"""Oracle: Lagrange P1/P2 finite elements for (Delta + k^2) u = b (eqs. eqh, eq1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Problem (Section "Iterative solver ..."): find u with (Delta + k(x)^2) u = b in
the box Omega, k = omega / c(x), c complex in attenuating media, homogeneous
Dirichlet on the top face and first-order absorbing conditions on the five
other faces.  Readings of the paper used here (it is silent on them):

* time dependence exp(-i omega t): the absorbing condition is d_n u = i k u;
* weak form, taken literally from eq. eqh:
      -int grad u . grad v + int k^2 u v + int_{absorbing} i k u v = int b v,
  i.e. A = -K + M_{k^2} + i B_k;
* c is constant per tet; each absorbing face uses its tet's k;
* all integrals are exact: every integrand is a polynomial in the barycentric
  coordinates, integrated with  int_T lambda^alpha = d! |T| alpha! / (|alpha|+d)!;
* Dirichlet dofs stay unknowns with identity rows/columns and zero load;
* dofs: P1 = vertices in input order; P2 = vertices, then the edges sorted by
  (min vertex, max vertex); the edge dof sits at the edge midpoint.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# Polynomials in barycentric coordinates: dict {exponent tuple: Fraction}.
# ----------------------------------------------------------------------------

def poly_mul(p, q):
    r = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(a + b for a, b in zip(ea, eb))
            r[e] = r.get(e, 0) + ca * cb
    return r


def poly_diff(p, k):
    """Partial derivative with respect to lambda_k (lambdas treated as independent)."""
    r = {}
    for e, c in p.items():
        if e[k] > 0:
            e2 = list(e)
            e2[k] -= 1
            r[tuple(e2)] = r.get(tuple(e2), 0) + c * e[k]
    return r


def poly_integral_per_measure(p):
    """(1/|simplex|) * integral over a d-simplex, d = nvar - 1, exact."""
    d = len(next(iter(p))) - 1 if p else 0
    tot = Fraction(0)
    for e, c in p.items():
        num = factorial(d)
        for a in e:
            num *= factorial(a)
        tot += Fraction(c) * Fraction(num, factorial(sum(e) + d))
    return tot


def lagrange_basis(order, nvar):
    """Barycentric-monomial form of the P1/P2 Lagrange basis on a simplex with
    nvar vertices.  P2 order: vertex functions l_i(2 l_i - 1), then edge
    functions 4 l_i l_j for (i, j) in lexicographic order."""
    basis = []
    one = lambda i: tuple(1 if k == i else 0 for k in range(nvar))
    two = lambda i: tuple(2 if k == i else 0 for k in range(nvar))
    for i in range(nvar):
        if order == 1:
            basis.append({one(i): Fraction(1)})
        else:
            basis.append({two(i): Fraction(2), one(i): Fraction(-1)})
    if order == 2:
        for i in range(nvar):
            for j in range(i + 1, nvar):
                e = tuple(1 if k in (i, j) else 0 for k in range(nvar))
                basis.append({e: Fraction(4)})
    return basis


def local_edges(nvar):
    return [(i, j) for i in range(nvar) for j in range(i + 1, nvar)]


def reference_tensors(order):
    """Per-unit-measure element tensors (exact fractions converted to float):

    Mref[a, b]        = int_T phi_a phi_b / |T|
    Kref[k, l, a, b]  = int_T (d phi_a / d l_k)(d phi_b / d l_l) / |T|
    Bref[a, b]        = int_F psi_a psi_b / |F|   (face basis, 3 vertices)
    Fref[a]           = int_T phi_a / |T|
    Gref[a]           = int_F psi_a / |F|

    With grad phi = sum_k (d phi / d l_k) grad l_k the stiffness is
    K_e[a, b] = |T| sum_{k,l} (grad l_k . grad l_l) Kref[k, l, a, b].
    """
    tb = lagrange_basis(order, 4)
    fb = lagrange_basis(order, 3)
    nl = len(tb)
    M = np.array([[float(poly_integral_per_measure(poly_mul(p, q))) for q in tb] for p in tb])
    dtb = [[poly_diff(p, k) for k in range(4)] for p in tb]
    K = np.zeros((4, 4, nl, nl))
    for k in range(4):
        for l in range(4):
            for a in range(nl):
                for b in range(nl):
                    pr = poly_mul(dtb[a][k], dtb[b][l])
                    K[k, l, a, b] = float(poly_integral_per_measure(pr)) if pr else 0.0
    B = np.array([[float(poly_integral_per_measure(poly_mul(p, q))) for q in fb] for p in fb])
    F = np.array([float(poly_integral_per_measure(p)) for p in tb])
    G = np.array([float(poly_integral_per_measure(p)) for p in fb])
    return M, K, B, F, G


_REF_CACHE = {}


def ref(order):
    if order not in _REF_CACHE:
        _REF_CACHE[order] = reference_tensors(order)
    return _REF_CACHE[order]


def eval_basis(order, lam):
    """Lagrange basis values at barycentric points lam (n, nvar) -> (n, nloc)."""
    lam = np.asarray(lam, dtype=np.float64)
    nvar = lam.shape[1]
    if order == 1:
        return lam.copy()
    out = [lam[:, i] * (2 * lam[:, i] - 1) for i in range(nvar)]
    out += [4 * lam[:, i] * lam[:, j] for i, j in local_edges(nvar)]
    return np.stack(out, axis=1)


# ----------------------------------------------------------------------------
# Mesh topology and dof numbering
# ----------------------------------------------------------------------------

class Dofs:
    """Dof numbering of a tetrahedral mesh (P1: vertices; P2: + sorted edges)."""

    def __init__(self, xyz, tets, order):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.order = order
        nv = self.xyz.shape[0]
        self.nv = nv
        if order == 1:
            self.edges = np.zeros((0, 2), dtype=np.int64)
            self.tet_dofs = self.tets.copy()
        else:
            le = local_edges(4)
            pairs = np.stack([np.sort(self.tets[:, [i, j]], axis=1) for i, j in le], axis=1)  # (nt,6,2)
            keys = pairs[..., 0] * nv + pairs[..., 1]
            ukeys, inv = np.unique(keys.ravel(), return_inverse=True)  # sorted = lexicographic
            self.edges = np.stack([ukeys // nv, ukeys % nv], axis=1)
            self.tet_dofs = np.concatenate([self.tets, nv + inv.reshape(-1, 6)], axis=1)
        self.n = nv + self.edges.shape[0]

    def edge_id(self, a, b):
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        keys = self.edges[:, 0] * self.nv + self.edges[:, 1]
        pos = np.searchsorted(keys, lo * self.nv + hi)
        assert np.all(keys[pos] == lo * self.nv + hi)
        return self.nv + pos

    def coords(self):
        if self.order == 1:
            return self.xyz.copy()
        mid = 0.5 * (self.xyz[self.edges[:, 0]] + self.xyz[self.edges[:, 1]])
        return np.concatenate([self.xyz, mid], axis=0)

    def face_dofs(self, faces):
        """Dofs of triangles given by vertex triples (sorted ascending)."""
        if self.order == 1:
            return faces.copy()
        e = [self.edge_id(faces[:, i], faces[:, j]) for i, j in local_edges(3)]
        return np.concatenate([faces, np.stack(e, axis=1)], axis=1)


_FACE_OPP = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]


def tet_faces(tets):
    """All faces (nt*4, 3) sorted vertex triples and their owning tet index."""
    f = np.concatenate([tets[:, list(o)] for o in _FACE_OPP], axis=0)
    owner = np.tile(np.arange(tets.shape[0]), 4)
    return np.sort(f, axis=1), owner


def face_counts(faces, nv):
    keys = (faces[:, 0] * nv + faces[:, 1]) * nv + faces[:, 2]
    _, inv, cnt = np.unique(keys, return_inverse=True, return_counts=True)
    return cnt[inv], keys


def boundary_faces(xyz, tets):
    """Faces appearing in exactly one tet; returns (faces, owner, is_dirichlet).
    A boundary face is Dirichlet when all its vertices lie on the top face
    z == min z, otherwise it is absorbing."""
    faces, owner = tet_faces(tets)
    cnt, _ = face_counts(faces, xyz.shape[0])
    b = cnt == 1
    faces, owner = faces[b], owner[b]
    ztop = xyz[:, 2].min()
    dirich = np.all(xyz[faces, 2] == ztop, axis=1)
    return faces, owner, dirich


def dirichlet_dofs(dofs: Dofs, bfaces, dirich):
    mask = np.zeros(dofs.n, dtype=bool)
    if np.any(dirich):
        mask[dofs.face_dofs(bfaces[dirich]).ravel()] = True
    return mask


# ----------------------------------------------------------------------------
# Element and face matrices
# ----------------------------------------------------------------------------

def tet_geometry(xyz, tets):
    """Volumes |T| and barycentric gradients grad lambda_k (nt, 4, 3)."""
    p = xyz[tets]
    J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    vol = np.abs(det) / 6.0
    Jinv = np.linalg.inv(J)  # rows of Jinv are grad lambda_1..3
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    return vol, g


def element_matrices(xyz, tets, order):
    """Stiffness K_e and mass M_e (unit coefficient) for every tet."""
    Mref, Kref, *_ = ref(order)
    vol, g = tet_geometry(xyz, tets)
    G = np.einsum("tkd,tld->tkl", g, g)
    K = vol[:, None, None] * np.einsum("tkl,klab->tab", G, Kref)
    M = vol[:, None, None] * Mref[None]
    return K, M


def face_areas(xyz, faces):
    p = xyz[faces]
    return 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), axis=1)


def face_matrices(xyz, faces, order):
    _, _, Bref, _, _ = ref(order)
    return face_areas(xyz, faces)[:, None, None] * Bref[None]


# ----------------------------------------------------------------------------
# Assembly
# ----------------------------------------------------------------------------

def _coo(n, dofs_e, vals_e):
    nl = dofs_e.shape[1]
    rows = np.repeat(dofs_e, nl, axis=1).ravel()
    cols = np.tile(dofs_e, (1, nl)).ravel()
    return sp.coo_matrix((vals_e.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def wavenumber(c_tet, omega):
    return omega / np.asarray(c_tet, dtype=np.complex128)


def assemble_parts(xyz, tets, order, c_tet, omega, tet_subset=None, imp_faces=None, imp_owner=None, dofs=None):
    """Assemble -K, M_{k^2} and i B_k separately (global dofs of the full mesh).

    tet_subset restricts the volume terms to a subset of tets; imp_faces /
    imp_owner give the faces carrying the impedance term and the tet whose k
    they use.  Returns (dofs, K, Mk2, Bk) with A = -K + Mk2 + 1j * Bk.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    if dofs is None:
        dofs = Dofs(xyz, tets, order)
    k = wavenumber(c_tet, omega)
    sel = np.arange(tets.shape[0]) if tet_subset is None else np.asarray(tet_subset)
    Ke, Me = element_matrices(xyz, tets[sel], order)
    K = _coo(dofs.n, dofs.tet_dofs[sel], Ke)
    Mk2 = _coo(dofs.n, dofs.tet_dofs[sel], Me * (k[sel] ** 2)[:, None, None])
    if imp_faces is not None and len(imp_faces):
        Be = face_matrices(xyz, imp_faces, order) * k[imp_owner][:, None, None]
        Bk = _coo(dofs.n, dofs.face_dofs(imp_faces), Be)
    else:
        Bk = sp.csr_matrix((dofs.n, dofs.n), dtype=np.complex128)
    return dofs, K, Mk2, Bk


def apply_dirichlet(A, mask):
    """Zero the rows and columns of Dirichlet dofs and put 1 on their diagonal."""
    keep = sp.diags((~mask).astype(np.float64))
    return (keep @ A @ keep + sp.diags(mask.astype(np.float64))).tocsr()


class Problem:
    """Global system A u = b of eq. eq1 for a mesh, velocity and frequency."""

    def __init__(self, xyz, tets, order, c_tet, omega):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.order = order
        self.c_tet = np.asarray(c_tet, dtype=np.complex128)
        self.omega = float(omega)
        self.k = wavenumber(self.c_tet, self.omega)
        bf, bown, bdir = boundary_faces(self.xyz, self.tets)
        self.bfaces, self.bowner, self.bdir = bf, bown, bdir
        dofs, K, Mk2, Bk = assemble_parts(self.xyz, self.tets, order, self.c_tet, omega,
                                          imp_faces=bf[~bdir], imp_owner=bown[~bdir])
        self.dofs = dofs
        self.n = dofs.n
        self.K, self.Mk2, self.Bk = K, Mk2, Bk
        self.dir_mask = dirichlet_dofs(dofs, bf, bdir)
        self.A = apply_dirichlet(-K + Mk2 + 1j * Bk, self.dir_mask)
        self._gface_keys = None

    def global_face_keys_sorted(self):
        if self._gface_keys is None:
            f, _ = tet_faces(self.tets)
            _, keys = face_counts(f, self.xyz.shape[0])
            self._gface_keys = np.sort(keys)
        return self._gface_keys

    def point_source(self, xs):
        """Load F_i = phi_i(x_s) of b = delta(x - x_s); zero on Dirichlet dofs."""
        t, lam = locate_points(self.xyz, self.tets, np.asarray(xs, dtype=np.float64)[None, :])
        if t[0] < 0:
            raise ValueError("source point outside the mesh")
        F = np.zeros(self.n, dtype=np.complex128)
        F[self.dofs.tet_dofs[t[0]]] = eval_basis(self.order, lam)[0]
        F[self.dir_mask] = 0.0
        return F

    def nodal_source(self, node):
        F = np.zeros(self.n, dtype=np.complex128)
        F[node] = 1.0
        F[self.dir_mask] = 0.0
        return F


# ----------------------------------------------------------------------------
# Point location (shared by sources and the coarse interpolation)
# ----------------------------------------------------------------------------

def locate_points(xyz, tets, pts, tol=1e-10):
    """For each point, the first tet (in index order) containing it and its
    barycentric coordinates; -1 if none.  Uniform-bucket search."""
    xyz = np.asarray(xyz, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    p = xyz[tets]
    J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)
    lo, hi = p.min(axis=1), p.max(axis=1)
    glo, ghi = xyz.min(axis=0), xyz.max(axis=0)
    nb = max(1, int(round(tets.shape[0] ** (1 / 3) / 2)))
    width = (ghi - glo) / nb + 1e-300
    blo = np.clip(np.floor((lo - glo) / width - 1e-9).astype(np.int64), 0, nb - 1)
    bhi = np.clip(np.floor((hi - glo) / width + 1e-9).astype(np.int64), 0, nb - 1)
    # bucket -> candidate tets, as a CSR list built from all (tet, bucket) pairs
    span = bhi - blo
    pair_t, pair_b = [], []
    for di in range(span[:, 0].max() + 1):
        for dj in range(span[:, 1].max() + 1):
            for dk in range(span[:, 2].max() + 1):
                m = (span[:, 0] >= di) & (span[:, 1] >= dj) & (span[:, 2] >= dk)
                t = np.nonzero(m)[0]
                pair_t.append(t)
                pair_b.append((blo[t, 0] + di) + nb * ((blo[t, 1] + dj) + nb * (blo[t, 2] + dk)))
    pair_t, pair_b = np.concatenate(pair_t), np.concatenate(pair_b)
    o = np.lexsort((pair_t, pair_b))
    pair_t, pair_b = pair_t[o], pair_b[o]
    cptr = np.searchsorted(pair_b, np.arange(nb ** 3 + 1))
    pb = np.clip(np.floor((pts - glo) / width).astype(np.int64), 0, nb - 1)
    pkey = pb[:, 0] + nb * (pb[:, 1] + nb * pb[:, 2])
    found = np.full(pts.shape[0], -1, dtype=np.int64)
    lam_out = np.zeros((pts.shape[0], 4))
    order = np.argsort(pkey, kind="stable")
    bounds = np.searchsorted(pkey[order], np.arange(nb ** 3 + 1))
    for b in range(nb ** 3):
        idx = order[bounds[b]:bounds[b + 1]]
        ct = pair_t[cptr[b]:cptr[b + 1]]
        if idx.size == 0 or ct.size == 0:
            continue
        d = pts[idx][:, None, :] - p[ct][None, :, 0, :]  # (np, nc, 3)
        l123 = np.einsum("cij,pcj->pci", Jinv[ct], d)
        lam = np.concatenate([1 - l123.sum(axis=2, keepdims=True), l123], axis=2)
        ok = np.all(lam >= -tol, axis=2)
        has = ok.any(axis=1)
        first = np.argmax(ok, axis=1)
        sel = idx[has]
        found[sel] = ct[first[has]]
        lam_out[sel] = lam[has, first[has]]
    return found, lam_out
