"""Pins of the oracle's discretisation (eqs. eqh, eq1) against mathematics.

Each test checks the oracle against something other than itself: textbook
closed forms, quadrature that bypasses the exact monomial formula, invariants
of the weak form, and the O(h^{p+1}) L2 convergence of a manufactured
solution that satisfies the paper's boundary conditions.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from paper_2004_06309_amd import workloads as wl
from tests.quadrature import tet_rule, tri_rule

RNG = np.random.default_rng(1234)
RAND_TET = np.array([[0.1, 0.2, 0.05], [1.3, 0.1, 0.2], [0.3, 1.1, -0.1], [0.2, 0.4, 0.9]])


def _nodes_bary(order, nvar):
    I = np.eye(nvar)
    if order == 1:
        return I
    return np.concatenate([I, [0.5 * (I[i] + I[j]) for i, j in fem.local_edges(nvar)]])


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("nvar", [3, 4])
def test_basis_is_nodal(order, nvar):
    """phi_a(node_b) = delta_ab at vertices and edge midpoints (Lagrange basis)."""
    V = fem.eval_basis(order, _nodes_bary(order, nvar))
    assert np.allclose(V, np.eye(V.shape[0]), atol=1e-15)


@pytest.mark.parametrize("order", [1, 2])
def test_element_matrices_vs_quadrature(order):
    """Exact monomial integration == collapsed Gauss-Jacobi quadrature on a
    skewed tet, with gradients taken by central differences in x."""
    xyz = RAND_TET
    tets = np.array([[0, 1, 2, 3]])
    K, M = fem.element_matrices(xyz, tets, order)
    lam, w = tet_rule(6)
    vol = abs(np.linalg.det((xyz[1:] - xyz[0]).T)) / 6
    phi = fem.eval_basis(order, lam)
    Mq = vol * 6 * np.einsum("q,qa,qb->ab", w, phi, phi)
    assert np.allclose(M[0], Mq, rtol=1e-13, atol=1e-15 * vol)
    # physical points of the quadrature nodes, gradients by differences
    X = lam @ xyz
    T = np.stack([xyz[1] - xyz[0], xyz[2] - xyz[0], xyz[3] - xyz[0]], axis=1)
    Tinv = np.linalg.inv(T)

    def basis_at(P):
        l123 = (P - xyz[0]) @ Tinv.T
        return fem.eval_basis(order, np.concatenate([1 - l123.sum(1, keepdims=True), l123], axis=1))

    eps = 1e-5
    grads = np.stack([(basis_at(X + eps * e) - basis_at(X - eps * e)) / (2 * eps) for e in np.eye(3)], axis=2)
    Kq = vol * 6 * np.einsum("q,qad,qbd->ab", w, grads, grads)
    assert np.allclose(K[0], Kq, rtol=1e-8, atol=1e-8 * np.abs(Kq).max())


def test_p2_mass_textbook():
    """P2 tet mass matrix = |T|/420 x the classical integer table."""
    t = np.array([[6, 1, 1, 1, -4, -4, -4, -6, -6, -6],
                  [1, 6, 1, 1, -4, -6, -6, -4, -4, -6],
                  [1, 1, 6, 1, -6, -4, -6, -4, -6, -4],
                  [1, 1, 1, 6, -6, -6, -4, -6, -4, -4],
                  [-4, -4, -6, -6, 32, 16, 16, 16, 16, 8],
                  [-4, -6, -4, -6, 16, 32, 16, 16, 8, 16],
                  [-4, -6, -6, -4, 16, 16, 32, 8, 16, 16],
                  [-6, -4, -4, -6, 16, 16, 8, 32, 16, 16],
                  [-6, -4, -6, -4, 16, 8, 16, 16, 32, 16],
                  [-6, -6, -4, -4, 8, 16, 16, 16, 16, 32]]) / 420.0
    M, *_ = fem.ref(2)
    assert np.allclose(M, t, atol=1e-16)


@pytest.mark.parametrize("order", [1, 2])
def test_stiffness_invariants(order):
    """K_e 1 = 0, K_e symmetric positive semi-definite with a 1-dim kernel."""
    K, M = fem.element_matrices(RAND_TET, np.array([[0, 1, 2, 3]]), order)
    K = K[0]
    assert np.allclose(K.sum(axis=1), 0, atol=1e-13 * np.abs(K).max())
    assert np.allclose(K, K.T, atol=0)
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1]


def test_basis_integrals():
    """int phi_vertex = -|T|/20, int phi_edge = |T|/5 (P2 tet);
    face P2: vertex 0, edge |F|/3; P1: |T|/4 and |F|/3."""
    _, _, _, F2, G2 = fem.ref(2)
    _, _, _, F1, G1 = fem.ref(1)
    assert np.allclose(F2, [-1 / 20] * 4 + [1 / 5] * 6, atol=1e-16)
    assert np.allclose(G2, [0] * 3 + [1 / 3] * 3, atol=1e-16)
    assert np.allclose(F1, 0.25) and np.allclose(G1, 1 / 3)
    lam, w = tri_rule(5)
    phi = fem.eval_basis(2, lam)
    B = fem.ref(2)[2]
    assert np.allclose(B, 2 * np.einsum("q,qa,qb->ab", w, phi, phi), atol=1e-15)


@pytest.fixture(scope="module")
def tiny_problem():
    w = wl.tiny()
    return w, fem.Problem(w.xyz, w.tets, w.order, w.c_tet, w.omega)


def test_assembly_complex_symmetric(tiny_problem):
    _, P = tiny_problem
    assert abs(P.A - P.A.T).max() == 0.0


def test_assembly_integrals(tiny_problem):
    """1^T M_{k^2} 1 = int k^2 = |Omega| k^2; 1^T B_k 1 = k |absorbing area|
    = 5 km^2 k; K 1 = 0 (constants are in the kernel of the Laplacian)."""
    w, P = tiny_problem
    k = w.omega / w.c_tet[0]
    one = np.ones(P.n)
    assert np.isclose(one @ (P.Mk2 @ one), 1e9 * k ** 2, rtol=1e-12)
    assert np.isclose(one @ (P.Bk @ one), 5e6 * k, rtol=1e-12)
    assert np.abs(P.K @ one).max() < 1e-9 * abs(P.K).max()


def test_dof_counts():
    """Kuhn counts: 16^3 -> 24,576 tets / 4,913 P1 dofs (289 on the top face)."""
    w = wl.tiny()
    P = fem.Problem(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    assert w.tets.shape[0] == 24576 and P.n == 4913 and P.dir_mask.sum() == 17 * 17
    xyz, tets = wl.kuhn_mesh(8, 8, 2, 800, 800, 200)
    D = fem.Dofs(xyz, tets, 2)
    assert D.n == 17 * 17 * 5  # P2 nodes on a refined lattice


def test_dense_lu_agrees_with_superlu(tiny_problem):
    """Direct SuperLU solve == dense LAPACK solve on the tiny system."""
    w, P = tiny_problem
    b = P.nodal_source(w.source_node)
    u1 = spla.spsolve(P.A.tocsc(), b)
    u2 = np.linalg.solve(P.A.toarray(), b)
    assert np.linalg.norm(u1 - u2) <= 1e-10 * np.linalg.norm(u2)


def test_reciprocity(tiny_problem):
    """A symmetric => Green's function symmetric: u_a[b] = u_b[a]."""
    w, P = tiny_problem
    lu = spla.splu(P.A.tocsc())
    a, b = 722, 3001
    ea = np.zeros(P.n, complex); ea[a] = 1
    eb = np.zeros(P.n, complex); eb[b] = 1
    assert np.isclose(lu.solve(ea)[b], lu.solve(eb)[a], rtol=1e-10)


def test_point_source_is_basis_evaluation():
    """F_i = phi_i(x_s): partition of unity (sum = 1 away from Dirichlet), and
    at a vertex the load is the unit vector of that vertex."""
    w = wl.small_box(order=2)
    P = fem.Problem(w.xyz, w.tets, 2, w.c_tet, w.omega)
    F = P.point_source(w.source_point)
    assert np.isclose(F.sum(), 1.0) and np.count_nonzero(F) <= 10
    v = 200
    assert not P.dir_mask[v]
    Fv = P.point_source(w.xyz[v])
    assert np.isclose(Fv[v], 1) and np.isclose(np.abs(Fv).sum(), 1)


# ---------------------------------------------------------------------------
# Manufactured solution: u* = sin(kz z) exp(i (kx x + ky y)), kx^2+ky^2+kz^2 = k^2
# satisfies (Delta + k^2) u* = 0 and u* = 0 on the top face z = 0.
# ---------------------------------------------------------------------------

L = 1000.0
C = 2000.0
FREQ = 1.0


def _wavevector():
    k = 2 * np.pi * FREQ / C
    kx, ky = k / 3, 2 * k / 5
    kz = np.sqrt(k ** 2 - kx ** 2 - ky ** 2)
    return k, kx, ky, kz


def _u(P):
    k, kx, ky, kz = _wavevector()
    return np.sin(kz * P[:, 2]) * np.exp(1j * (kx * P[:, 0] + ky * P[:, 1]))


def _grad_u(P):
    k, kx, ky, kz = _wavevector()
    e = np.exp(1j * (kx * P[:, 0] + ky * P[:, 1]))
    s, c = np.sin(kz * P[:, 2]), np.cos(kz * P[:, 2])
    return np.stack([1j * kx * s * e, 1j * ky * s * e, kz * c * e], axis=1)


def _manufactured_error(nx, order):
    xyz, tets = wl.kuhn_mesh(nx, nx, nx, L, L, L)
    c = np.full(tets.shape[0], C, dtype=complex)
    omega = 2 * np.pi * FREQ
    P = fem.Problem(xyz, tets, order, c, omega)
    k = omega / C
    # boundary data g = d_n u* - i k u* on the absorbing faces, load -int g phi
    lam_f, w_f = tri_rule(8)
    faces = P.bfaces[~P.bdir]
    fd = P.dofs.face_dofs(faces)
    pts = np.einsum("qv,fvd->fqd", lam_f, xyz[faces])
    cen = pts.mean(axis=1)
    normal = np.zeros_like(cen)
    for d in range(3):
        normal[np.isclose(cen[:, d], 0.0), d] = -1.0
        normal[np.isclose(cen[:, d], L), d] = 1.0
    flat = pts.reshape(-1, 3)
    g = (np.einsum("fqd,fd->fq", _grad_u(flat).reshape(pts.shape), normal)
         - 1j * k * _u(flat).reshape(pts.shape[:2]))
    area = fem.face_areas(xyz, faces)
    phi_f = fem.eval_basis(order, lam_f)
    load = np.zeros(P.n, dtype=complex)
    np.add.at(load, fd, -2 * area[:, None] * np.einsum("q,fq,qa->fa", w_f, g, phi_f))
    load[P.dir_mask] = 0
    uh = spla.spsolve(P.A.tocsc(), load)
    # L2 error by quadrature
    lam_t, w_t = tet_rule(6)
    vol, _ = fem.tet_geometry(xyz, tets)
    X = np.einsum("qv,tvd->tqd", lam_t, xyz[tets])
    phi = fem.eval_basis(order, lam_t)
    uq = np.einsum("qa,ta->tq", phi, uh[P.dofs.tet_dofs])
    ex = _u(X.reshape(-1, 3)).reshape(uq.shape)
    err2 = np.sum(6 * vol[:, None] * w_t[None, :] * np.abs(uq - ex) ** 2)
    return np.sqrt(err2)


@pytest.mark.parametrize("order,levels,rate", [(1, (4, 8, 16), 2.0), (2, (2, 4, 8), 3.0)])
def test_manufactured_convergence_rate(order, levels, rate):
    """L2 error of the discrete solution decays as h^{p+1} (p = 1, 2)."""
    errs = [_manufactured_error(n, order) for n in levels]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > rate - 0.25, (errs, rates)
    assert rates[-1] < rate + 0.5, (errs, rates)
