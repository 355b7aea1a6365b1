"""Host-side checks of libhelm (no GPU): exported symbols, and the setup the
library builds on the host (assembly, subdomains, partition of unity, coarse
interpolation, point source) against the oracle, entry by entry.  Error paths
that the host can force are checked here too."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import coarse as ocoarse
from oracle import dd as odd
from oracle import fem
from paper_2004_06309_amd import workloads as wl

helm = pytest.importorskip("paper_2004_06309_amd.helm")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = helm.load()
    header = open(os.path.join(ROOT, "include", "helm.h")).read()
    declared = set(re.findall(r"\b(helm_[A-Za-z_0-9]+)\s*\(", header))
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(helm.EXPORTS), declared ^ set(helm.EXPORTS)


def _csr(h):
    ptr, col, val = h.matrix_csr()
    return sp.csr_matrix((val, col, ptr), shape=(h.n, h.n))


CASES = {
    "tiny_p1": lambda: wl.tiny(),
    "small_p2": lambda: wl.small_box(n=(6, 6, 4), order=2, n_parts=(2, 2, 1), overlap=2),
    "small_p2_ragged": lambda: wl.small_box(n=(5, 3, 4), order=2, n_parts=(3, 2, 1), overlap=1, coarse=False),
    "adapted_p2": lambda: wl.adapted_box(lx=2000.0, ly=2000.0, lz=1000.0, n0=(2, 2, 1), freq=3.0, n_parts=(2, 2, 1)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    w = CASES[request.param]()
    P = fem.Problem(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    h = helm.Helm(-1)
    h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    h.precond_setup(w.part, w.n_sub, w.overlap, w.coarse_xyz, w.coarse_tets)
    return w, P, h


def test_assembly_matches_oracle(case):
    w, P, h = case
    assert h.n == P.n
    A = _csr(h)
    diff = abs(A - P.A).max()
    assert diff <= 1e-13 * abs(P.A).max(), diff
    # no stored entry outside the oracle's pattern (Dirichlet couplings removed)
    assert A.nnz == (P.A != 0).sum()


def test_dof_coordinates_match_oracle(case):
    w, P, h = case
    assert np.array_equal(h.dof_coords(), P.dofs.coords())


def test_subdomains_match_oracle(case):
    w, P, h = case
    subs = odd.decompose(P, w.part, w.n_sub, w.overlap)
    for i, s in enumerate(subs):
        dofs, D, (ptr, col, val) = h.subdomain(i)
        assert np.array_equal(dofs, s.dofs)
        assert np.allclose(D, s.D, rtol=0, atol=1e-15)
        Ai = sp.csr_matrix((val, col, ptr), shape=(dofs.size, dofs.size))
        Ao = odd.local_matrix(P, s)
        assert abs(Ai - Ao).max() <= 1e-13 * abs(Ao).max()


def test_coarse_interpolation_matches_oracle(case):
    w, P, h = case
    if w.coarse_xyz is None:
        pytest.skip("one-level case")
    nc, (ptr, col, val) = h.coarse_Z()
    Zo, _ = ocoarse.interpolation(P, w.coarse_xyz, w.coarse_tets)
    Z = sp.csr_matrix((val, col, ptr), shape=(h.n, nc))
    assert Z.shape == Zo.shape
    assert abs(Z - Zo).max() <= 1e-14


def test_point_source_matches_oracle(case):
    w, P, h = case
    xs = np.array([w.xyz[:, 0].max() * 0.41, w.xyz[:, 1].max() * 0.53, w.xyz[:, 2].max() * 0.37])
    assert np.allclose(h.point_source(xs), P.point_source(xs), rtol=0, atol=1e-14)


def test_stats_are_consistent(case):
    w, P, h = case
    st = h.stats()
    assert st["n_sub"] == w.n_sub
    assert st["factor_entries"] > 0 and st["levels_fwd"] >= 1
    assert st["n_local_total"] == sum(h.subdomain(i)[0].size for i in range(w.n_sub))


def test_mid_sizes():
    """Mid workload: 80x80x20 Kuhn P2 mesh -> 161^2 * 41 dofs."""
    w = wl.mid()
    h = helm.Helm(-1)
    assert h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega) == 161 * 161 * 41


# ---- error paths ----------------------------------------------------------

def test_degenerate_tet_is_rejected():
    w = wl.small_box(n=(2, 2, 2), order=1, coarse=False)
    tets = w.tets.copy()
    tets[3, 3] = tets[3, 2]  # repeated vertex: zero volume
    h = helm.Helm(-1)
    with pytest.raises(helm.HelmError) as e:
        h.assemble(w.xyz, tets, 1, w.c_tet, w.omega)
    assert e.value.code == helm.HELM_EINVAL


def test_bad_partition_is_rejected():
    w = wl.small_box(n=(2, 2, 2), order=1, coarse=False)
    h = helm.Helm(-1)
    h.assemble(w.xyz, w.tets, 1, w.c_tet, w.omega)
    part = w.part.copy()
    part[0] = 99
    with pytest.raises(helm.HelmError) as e:
        h.precond_setup(part, w.n_sub, 1)
    assert e.value.code == helm.HELM_EINVAL


def test_call_order_and_host_only_context():
    h = helm.Helm(-1)
    with pytest.raises(helm.HelmError) as e:
        h.precond_setup(np.zeros(3, np.int32), 1, 1)
    assert e.value.code == helm.HELM_ESTATE
    lib = helm.load()
    assert lib.helm_solve(h.h, 0, None, 1e-6, None, None, None, None) == helm.HELM_ESTATE
    assert lib.helm_apply_A(h.h, None, None, None) == helm.HELM_ESTATE
    assert b"host-only" in lib.helm_last_error(h.h) or b"assemble" in lib.helm_last_error(h.h)
    h.close()
    h.close()  # NULL-safe destroy


def test_create_rejects_bad_ordinal():
    with pytest.raises(helm.HelmError):
        helm.Helm(-7)


def test_bad_tile_rows_are_rejected():
    w = wl.small_box(n=(2, 2, 2), order=1, coarse=False)
    h = helm.Helm(-1)
    h.assemble(w.xyz, w.tets, 1, w.c_tet, w.omega)
    for kw in ({"tile_rows": 48}, {"coarse_tile_rows": 8}, {"coarse_launch": 3}):
        with pytest.raises(helm.HelmError) as e:
            h.precond_setup(w.part, w.n_sub, 1, **kw)
        assert e.value.code == helm.HELM_EINVAL


def test_shorter_tiles_store_fewer_triangle_zeros():
    """Tiles of the diagonal blocks stop at their last row, so shorter tiles
    store a subset of the entries of taller ones; the analysis is unchanged."""
    w = wl.small_box(n=(6, 6, 4), order=2, n_parts=(2, 2, 1), overlap=2)
    st = {}
    for tr in (16, 64):
        h = helm.Helm(-1)
        h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
        h.precond_setup(w.part, w.n_sub, w.overlap, w.coarse_xyz, w.coarse_tets, tile_rows=tr,
                        coarse_tile_rows=tr)
        st[tr] = h.stats()
    assert st[16]["factor_entries"] < st[64]["factor_entries"]
    assert st[16]["coarse_entries"] <= st[64]["coarse_entries"]
    for k in ("n_local_total", "levels_fwd", "levels_bwd", "max_front", "n_supernodes"):
        assert st[16][k] == st[64][k]


def test_server_needs_a_device_context():
    h = helm.Helm(-1)
    lib = helm.load()
    out = __import__("ctypes").c_void_p()
    assert lib.helm_server_create(h.h, None, None, __import__("ctypes").byref(out)) == helm.HELM_ESTATE
    assert not out.value
    lib.helm_server_destroy(None)  # NULL-safe
    assert lib.helm_server_submit(None, None, None, 0) == helm.HELM_EINVAL


def test_batch_options_on_a_host_context():
    """The subdomain-batch and one-wave-job options are accepted by a
    host-only context, which analyses one batch and reports it."""
    w = wl.small_box(n=(4, 4, 2), order=2, n_parts=(2, 2, 1), overlap=1, coarse=False)
    for kw in ({}, {"batches": 1}, {"batches": 4}, {"sn_jobs_min": -1}, {"sn_jobs_min": 1}):
        h = helm.Helm(-1)
        h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
        h.precond_setup(w.part, w.n_sub, w.overlap, **kw)
        st = h.stats()
        assert st["batches"] == 1 and st["n_sub"] == 4 and st["factor_entries"] > 0
    for bad in (-1, 5):
        h = helm.Helm(-1)
        h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
        with pytest.raises(helm.HelmError, match="batches"):
            h.precond_setup(w.part, w.n_sub, w.overlap, batches=bad)


def test_factor_precision_and_split_options_on_a_host_context():
    """factor_c64 0/1/2 and split_front_rows -1/0/k are accepted by a
    host-only context (which runs the symbolic analysis only); other values
    fail with HELM_EINVAL."""
    w = wl.small_box(n=(4, 4, 2), order=2, n_parts=(2, 2, 1), overlap=1, coarse=False)

    def setup(**kw):
        h = helm.Helm(-1)
        h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
        h.precond_setup(w.part, w.n_sub, w.overlap, **kw)
        return h.stats()

    for mode in (0, 1, 2):
        assert setup(c64=mode)["factor_c64"] == mode
    for split in (-1, 0, 1, 300):
        assert setup(split_front_rows=split)["factor_entries"] > 0
    with pytest.raises(ValueError, match="c64"):
        setup(c64=3)
    h = helm.Helm(-1)
    h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    opts = helm.PrecondOpts(0, 3, 0, 0, 0, 0, 0, 0, 0, 0)
    rc = h.lib.helm_precond_setup(h.h, helm._ptr(np.ascontiguousarray(w.part, dtype=np.int32)), w.n_sub, w.overlap,
                                  None, __import__("ctypes").byref(opts))
    assert rc == helm.HELM_EINVAL
    with pytest.raises(helm.HelmError, match="split_front_rows"):
        setup(split_front_rows=-2)


def test_binding_rejects_vectors_the_kernels_would_overrun():
    """Wrong dtype, wrong length, mismatched shapes and host tensors are
    refused by the binding before any pointer reaches the library."""
    torch = pytest.importorskip("torch")
    w = wl.small_box(n=(2, 2, 2), order=1, coarse=False)
    h = helm.Helm(-1)
    n = h.assemble(w.xyz, w.tets, 1, w.c_tet, w.omega)
    good = torch.zeros(n, dtype=torch.complex128)
    for bad, msg in ((torch.zeros(n, dtype=torch.complex64), "complex128"),
                     (torch.zeros(n - 1, dtype=torch.complex128), "entries"),
                     (torch.zeros(2 * n, dtype=torch.complex128)[::2], "contiguous"),
                     (np.zeros(n, np.complex128), "torch tensor"),
                     (good, "GPU tensor")):
        with pytest.raises(ValueError, match=msg):
            h.apply_A(bad, good)
    with pytest.raises(ValueError, match="must both be"):
        h.solve(torch.zeros(2, n, dtype=torch.complex128), torch.zeros(n, dtype=torch.complex128))
    with pytest.raises(ValueError, match="entries"):
        h.solve(torch.zeros(2, n + 1, dtype=torch.complex128), torch.zeros(2, n + 1, dtype=torch.complex128))
