"""The allocation-free coarse correction (helm_apply_coarse_noalloc) against
helm_apply_coarse, through the C-ABI: two calls in a row on one GPU, the
second on a smaller coarse problem (the fixed scratch keeps the first call's
contents), each compared with the allocating entry point and with the
oracle's q = Z E^{-1} Z^T r (eq. 2lvl)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import precond as opre  # noqa: E402
from paper_2004_06309_amd import helm  # noqa: E402
from paper_2004_06309_amd import workloads as wl  # noqa: E402


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def test_noalloc_coarse_matches_allocating_entry_point():
    cases = [("mid/4", wl.mid(scale=4, n_parts=(4, 4, 1))),
             ("small", wl.small_box(n=(6, 6, 4), order=2, n_parts=(2, 2, 1), overlap=2))]
    for name, w in cases:
        print(f"[noalloc] {name}", flush=True)
        sys.stdout.flush()
        P, b, M = opre.build(w)
        h = helm.from_workload(w)
        r = wl.random_vector(P.n, 31)
        q_ref = torch.empty(P.n, dtype=torch.complex128, device="cuda")
        q_new = torch.full((P.n,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
        h.apply_coarse(_dev(r), q_ref)
        h.apply_coarse_noalloc(_dev(r), q_new)
        torch.cuda.synchronize()
        a, c = q_new.cpu().numpy(), q_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.abs(a - c).max() <= 1e-14 * np.abs(c).max()
        qo = M.coarse_correction(r)
        assert np.abs(a - qo).max() <= 1e-9 * np.abs(qo).max()
        # repeated call on the same scratch: same result
        h.apply_coarse_noalloc(_dev(r), q_new)
        torch.cuda.synchronize()
        assert np.array_equal(q_new.cpu().numpy(), a)
        h.close()
