"""Pins of the oracle's decomposition, preconditioners and GMRES (eqs. oras, 2lvl).

Checked against identities that hold exactly: the partition of unity sums to
the identity, ORAS with one subdomain is A^{-1}, the coarse correction with
Z = I is A^{-1}, Galerkin E equals the directly assembled coarse operator on
nested meshes in a homogeneous medium, the Arnoldi relation, orthonormality,
and the least-squares optimality of the Givens solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import coarse, dd, fem, precond
from oracle.gmres import gmres
from paper_2004_06309_amd import workloads as wl


@pytest.fixture(scope="module")
def small():
    w = wl.small_box(n=(6, 6, 4), order=2, n_parts=(2, 2, 1), overlap=2)
    P, b, M = precond.build(w)
    return w, P, b, M


def test_partition_of_unity(small):
    """sum_i R_i^T D_i R_i = I."""
    w, P, b, M = small
    s = np.zeros(P.n)
    for sub in M.subs:
        np.add.at(s, sub.dofs, sub.D)
    assert np.abs(s - 1).max() < 1e-15


def test_pou_zero_on_artificial_interface(small):
    w, P, b, M = small
    for sub in M.subs:
        art = dd.artificial_dofs(P, sub)
        assert art.size > 0
        pos = np.searchsorted(sub.dofs, art)
        assert np.all(sub.D[pos] == 0)
        assert np.all(sub.level[pos] == w.overlap)


def test_local_rows_match_global_inside(small):
    """Rows of A_i for dofs with l(j) <= delta-1 equal the rows of A."""
    w, P, b, M = small
    for sub in M.subs:
        inner = np.nonzero(sub.level <= w.overlap - 1)[0]
        Ai = sub.A.tocsr()[inner]
        Ag = P.A[sub.dofs[inner]]
        # every nonzero of these global rows lies inside the subdomain
        assert np.isclose(abs(Ag).sum(), abs(Ag[:, sub.dofs]).sum())
        assert abs(Ai - Ag[:, sub.dofs]).max() <= 1e-12 * abs(Ag).max()


def test_local_matrices_symmetric(small):
    w, P, b, M = small
    for sub in M.subs:
        assert abs(sub.A - sub.A.T).max() <= 1e-15 * abs(sub.A).max()


def test_oras_one_subdomain_is_exact():
    """N_d = 1: M_1^{-1} = A^{-1}, GMRES converges in one iteration."""
    w = wl.small_box(n=(6, 5, 4), order=2, n_parts=(1, 1, 1), overlap=1, coarse=False)
    P, b, M = precond.build(w)
    assert len(M.subs) == 1 and M.subs[0].dofs.size == P.n
    assert np.allclose(M.subs[0].D, 1.0)
    r = precond.solve(P, b, M, tol=1e-10)
    assert r.converged and r.iterations == 1


def test_two_level_identity_coarse_space_is_exact():
    """Coarse mesh = fine P1 mesh => Z = I (on non-Dirichlet dofs), Q = A^{-1}."""
    w = wl.small_box(n=(4, 4, 4), order=1, n_parts=(2, 2, 1), overlap=1, coarse=False)
    w.coarse_xyz, w.coarse_tets = w.xyz, w.tets
    P, b, M = precond.build(w)
    Zd = M.Z.toarray()
    free = ~P.dir_mask
    assert np.allclose(Zd[free][:, :], np.eye(P.n)[free][:, free], atol=0)
    r = precond.solve(P, b, M, tol=1e-10)
    assert r.converged and r.iterations == 1


def test_coarse_interpolation_reproduces_linears():
    """Nested Kuhn meshes: Z (coarse nodal values of a linear l) = fine nodal
    values of l, for l vanishing on the top face."""
    w = wl.small_box(n=(6, 6, 4), order=2, coarse=True)
    P = fem.Problem(w.xyz, w.tets, 2, w.c_tet, w.omega)
    Z, cols = coarse.interpolation(P, w.coarse_xyz, w.coarse_tets)
    lin = lambda X: 0.3 * X[:, 2]  # linear, zero on the top face
    fine = lin(P.dofs.coords())
    assert np.allclose(Z @ lin(w.coarse_xyz[cols]), fine, atol=1e-12 * np.abs(fine).max())


def test_galerkin_equals_coarse_assembly():
    """Homogeneous medium, nested meshes: E = Z^T A Z equals the P1 matrix
    assembled directly on the coarse mesh (top nodes removed)."""
    w = wl.small_box(n=(6, 6, 4), order=2, coarse=True)
    c = np.full(w.tets.shape[0], 2300.0 * (1 - 0.01j))
    P = fem.Problem(w.xyz, w.tets, 2, c, w.omega)
    Z, cols = coarse.interpolation(P, w.coarse_xyz, w.coarse_tets)
    E = coarse.galerkin(P.A, Z)
    Pc = fem.Problem(w.coarse_xyz, w.coarse_tets, 1, np.full(w.coarse_tets.shape[0], c[0]), w.omega)
    Ac = Pc.A.tocsr()[cols][:, cols]
    assert abs(E - Ac).max() <= 1e-12 * abs(Ac).max()


@pytest.fixture(scope="module")
def tiny():
    w = wl.tiny()
    P, b, M = precond.build(w)
    return w, P, b, M


def test_unpreconditioned_gmres_matches_direct(tiny):
    w, P, b, M = tiny
    r = gmres(lambda v: P.A @ v, b, None, tol=1e-10, restart=400, maxit=4000)
    u = spla.spsolve(P.A.tocsc(), b)
    assert r.converged
    assert np.linalg.norm(r.x - u) <= 1e-7 * np.linalg.norm(u)


def test_arnoldi_relation_and_orthonormality(tiny):
    """A Z_m = V_{m+1} H_m and V^H V = I for the preconditioned Arnoldi process.
    MGS loses orthogonality roughly like eps / (relative residual), so the
    orthonormality bound is checked at the paper's tolerance 1e-6."""
    w, P, b, M = tiny
    r = precond.solve(P, b, M, tol=1e-10, restart=60, keep_arnoldi=True)
    V, Z, H = r.arnoldi["V"], r.arnoldi["Z"], r.arnoldi["H"]
    lhs = P.A @ Z
    assert np.linalg.norm(lhs - V @ H) <= 1e-12 * np.linalg.norm(lhs)
    # z_j = M^{-1} v_j
    assert np.linalg.norm(Z[:, 3] - M.apply(V[:, 3])) < 1e-13 * np.linalg.norm(Z[:, 3])
    r = precond.solve(P, b, M, tol=1e-6, restart=60, keep_arnoldi=True)
    V = r.arnoldi["V"]
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() < 1e-8


def test_givens_solution_is_least_squares(tiny):
    """Rotated solution y minimises ||beta e_1 - H y|| (compare with lstsq):
    the residual estimate equals that minimum."""
    w, P, b, M = tiny
    r = precond.solve(P, b, M, tol=1e-8, restart=60, keep_arnoldi=True)
    H = r.arnoldi["H"]
    k = H.shape[1]
    rhs = np.zeros(k + 1, complex)
    rhs[0] = np.linalg.norm(b)
    y, res, *_ = np.linalg.lstsq(H, rhs, rcond=None)
    assert np.isclose(np.sqrt(res[0]) / np.linalg.norm(b), r.history[-1], rtol=1e-8)


def test_history_monotone_and_estimate_matches_true(tiny):
    w, P, b, M = tiny
    r = precond.solve(P, b, M)
    h = np.array(r.history)
    assert np.all(np.diff(h) <= 1e-15)
    assert r.relres <= 1e-6 and h[-1] <= 1e-6
    assert abs(r.relres - h[-1]) < 0.05 * h[-1] + 1e-9


def test_two_level_beats_one_level():
    """The paper's claim: the two-level preconditioner needs fewer iterations.
    Checked where the P1 coarse mesh resolves the wavelength (1.25 Hz on the
    scaled-down thrust model, >= 2 coarse nodes per wavelength)."""
    w = wl.mid(scale=4, n_parts=(4, 4, 1), freq=1.25)
    P, b, M2 = precond.build(w)
    r2 = precond.solve(P, b, M2)
    M2.Z = None  # same local solves, no coarse correction
    r1 = precond.solve(P, b, M2)
    assert r2.converged and r1.converged
    assert r2.iterations < r1.iterations


def test_attenuation_lowers_iterations():
    """The paper's claim: physical attenuation reduces the iteration count."""
    its = []
    for att in (0.0, 0.05):
        w = wl.small_box(n=(8, 8, 6), size=(1600.0, 1600.0, 1200.0), order=2, freq=6.0,
                         n_parts=(2, 2, 2), overlap=1, attenuation=att, coarse=False)
        P, b, M = precond.build(w)
        its.append(precond.solve(P, b, M).iterations)
    assert its[1] < its[0], its


def _box_id(i, n_parts):
    return i % n_parts[0], (i // n_parts[0]) % n_parts[1], i // (n_parts[0] * n_parts[1])


@pytest.mark.parametrize("order", [1, 2])
def test_interface_impedance_term_on_box_subdomains(order):
    """The artificial-face term of the ORAS local matrices (eq. oras; the
    local problems carry the same absorbing condition as the physical
    boundary).  The Lagrange basis sums to one and K 1 = 0, so
        1^T A_i 1 = k_i^2 |Gamma_i| + i k_i |boundary of Gamma_i off the top|,
    the imaginary part counting every impedance face once.  With overlap 0 and
    a velocity constant on each box subdomain, Gamma_i is its box and both
    sides follow from the box extents.  Checked on the six subdomains of the
    lower layer of a 3x2x2 split (four corners, two edge boxes; none touches
    the Dirichlet top).  A dropped interface term (Neumann interfaces), a
    flipped sign, or the neighbour's k on the interface would each miss by far
    more than the tolerance (asserted below)."""
    n_parts = (3, 2, 2)
    size = (600.0, 400.0, 400.0)
    w = wl.small_box(n=(6, 4, 4), size=size, order=order, n_parts=n_parts, overlap=0, coarse=False)
    c_sub = (2000.0 + 250.0 * np.arange(w.n_sub)) * (1 - 0.02j)
    c = c_sub[w.part]
    P = fem.Problem(w.xyz, w.tets, order, c, w.omega)
    subs = dd.decompose(P, w.part, w.n_sub, 0)
    hx, hy, hz = (s / p for s, p in zip(size, n_parts))
    checked = 0
    for i, s in enumerate(subs):
        ix, iy, iz = _box_id(i, n_parts)
        if iz == 0:
            continue  # touches the Dirichlet top
        Ai = dd.local_matrix(P, s)
        one = np.ones(s.dofs.size)
        got = one @ (Ai @ one)
        k = w.omega / c_sub[i]
        vol = hx * hy * hz
        faces = [(hy * hz, ix, n_parts[0]), (hx * hz, iy, n_parts[1]), (hx * hy, iz, n_parts[2])]
        area = 2 * (hx * hy + hy * hz + hx * hz)
        expect = k * k * vol + 1j * k * area
        assert abs(got - expect) <= 1e-11 * abs(expect), (i, got, expect)
        # the same sum under plausible misreadings of the interface term
        phys = sum(a * ((j == 0) + (j == n - 1)) for a, j, n in faces)
        art = area - phys
        wrong = [k * k * vol + 1j * k * phys,  # no interface term
                 k * k * vol + 1j * k * (phys - art)]  # interface term with the wrong sign
        for nb in (i - 1, i + 1):  # interface term with a neighbour box's k
            if 0 <= nb < w.n_sub:
                wrong.append(k * k * vol + 1j * (k * phys + w.omega / c_sub[nb] * art))
        for v in wrong:
            assert abs(got - v) > 1e-3 * abs(expect)
        checked += 1
    assert checked == 6


def _boundary_area_off_top(xyz, tets):
    """Area of the faces that belong to exactly one tet, excluding faces on
    z = min z: plain enumeration with a dictionary."""
    count = {}
    for t in tets.tolist():
        for f in ((t[0], t[1], t[2]), (t[0], t[1], t[3]), (t[0], t[2], t[3]), (t[1], t[2], t[3])):
            key = tuple(sorted(f))
            count[key] = count.get(key, 0) + 1
    ztop = xyz[:, 2].min()
    area = 0.0
    for key, cnt in count.items():
        if cnt != 1:
            continue
        p = xyz[list(key)]
        if np.all(p[:, 2] == ztop):
            continue
        area += 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
    return area


@pytest.mark.parametrize("order,overlap", [(1, 1), (2, 2)])
def test_interface_impedance_term_with_overlap(order, overlap):
    """Same identity for overlapping subdomains in a homogeneous medium:
    1^T A_i 1 = k^2 |Gamma_i| + i k |boundary of Gamma_i off the top|, with
    the volume summed over Gamma_i's tets and the boundary area found by
    enumerating the faces of Gamma_i that belong to one of its tets only (the
    artificial faces of the grown region, jagged at its edges, plus its
    physical absorbing faces).  Subdomains of the lower layer only (away
    from the Dirichlet top)."""
    w = wl.small_box(n=(6, 6, 6), size=(600.0, 600.0, 600.0), order=order, n_parts=(2, 2, 2), overlap=overlap,
                     coarse=False)
    c0 = 2400.0 * (1 - 0.03j)
    P = fem.Problem(w.xyz, w.tets, order, np.full(w.n_tets, c0), w.omega)
    subs = dd.decompose(P, w.part, w.n_sub, overlap)
    k = w.omega / c0
    checked = 0
    for i, s in enumerate(subs):
        if _box_id(i, (2, 2, 2))[2] == 0:
            continue
        T = w.tets[s.tets]
        p = w.xyz[T]
        vol = np.abs(np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])).sum() / 6
        assert w.xyz[np.unique(T), 2].min() > 0  # away from the top
        area = _boundary_area_off_top(w.xyz, T)
        Ai = dd.local_matrix(P, s)
        one = np.ones(s.dofs.size)
        got = one @ (Ai @ one)
        expect = k * k * vol + 1j * k * area
        assert abs(got - expect) <= 1e-11 * abs(expect), (i, got, expect)
        checked += 1
    assert checked == 4


def test_pool_oras_equals_sequential_oras(small):
    """The pooled oracle (factors in single-threaded worker processes)
    applies the same one- and two-level preconditioner as Oras, bit for bit
    when Oras also factors with one BLAS thread (threaded BLAS inside
    SuperLU only reorders sums)."""
    from threadpoolctl import threadpool_limits

    from oracle.pool import PoolOras

    w, P, b, _ = small
    with threadpool_limits(1):
        M = precond.Oras(P, w.part, w.n_sub, w.overlap, (w.coarse_xyz, w.coarse_tets))
    pm = PoolOras(P, w.part, w.n_sub, w.overlap, (w.coarse_xyz, w.coarse_tets), workers=2)
    try:
        r = wl.random_vector(P.n, 3)
        assert np.array_equal(pm.one_level(r), M.one_level(r))
        assert np.array_equal(pm.apply(r), M.apply(r))
        assert len(pm.sub_times) == w.n_sub
        ro = precond.solve(P, b, M)
        rp = precond.solve(P, b, pm)
        assert rp.iterations == ro.iterations and np.array_equal(rp.x, ro.x)
    finally:
        pm.close()
