"""Input generators: the h-adapted meshes (bisection of a Kuhn mesh to the
local wavelength) are conforming, cover the box, are positively oriented and
meet their size target; the structured generators keep their counts."""
import numpy as np
import pytest

from paper_2004_06309_amd import workloads as wl


def _faces(tets):
    f = np.sort(np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 3]], tets[:, [1, 2, 3]]]),
                axis=1)
    return np.unique(f, axis=0, return_counts=True)


def _check_mesh(xyz, tets, box):
    u, cnt = _faces(tets)
    assert cnt.max() == 2  # no face shared by three tets
    # faces of one tet lie on the box surface: no hanging vertices inside
    P = xyz[u[cnt == 1]]
    on = np.zeros(P.shape[0], dtype=bool)
    for d in range(3):
        for v in (0.0, box[d]):
            on |= np.all(np.abs(P[:, :, d] - v) < 1e-9 * max(box), axis=1)
    assert on.all()
    p = xyz[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6
    assert vol.min() > 0
    assert np.isclose(vol.sum(), np.prod(box), rtol=1e-12)
    assert np.unique(tets).size == xyz.shape[0]  # every vertex is used


@pytest.mark.parametrize("freq", [2.0, 4.0])
def test_adapted_mesh_is_conforming_and_meets_the_size_target(freq):
    box = (2000.0, 2000.0, 1000.0)
    w = wl.adapted_box(*box, n0=(2, 2, 1), freq=freq, n_parts=(2, 2, 1))
    _check_mesh(w.xyz, w.tets, box)
    _check_mesh(w.coarse_xyz, w.coarse_tets, box)
    model = wl.ThrustModel.draw(*box, 12, 0)
    e = np.concatenate([w.tets[:, [i, j]] for i in range(4) for j in range(i + 1, 4)])
    a, b = w.xyz[e[:, 0]], w.xyz[e[:, 1]]
    # the refinement edges meet lambda/4; the other edges of a tet are at
    # most its refinement edge (the longest of a Kuhn-bisection tet)
    lam4 = model.velocity(0.5 * (a + b)) / (4 * freq)
    assert np.percentile(np.linalg.norm(a - b, axis=1) / lam4, 99) <= 1.0 + 1e-12
    # graded: slow layers get smaller tets than fast ones
    c = w.c_tet.real
    p = w.xyz[w.tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6
    assert vol[c <= 2500].mean() < vol[c >= 4500].mean()


def test_adapted_mesh_is_deterministic_and_finer_at_higher_frequency():
    w1 = wl.adapted_box(2000.0, 2000.0, 1000.0, n0=(2, 2, 1), freq=3.0)
    w2 = wl.adapted_box(2000.0, 2000.0, 1000.0, n0=(2, 2, 1), freq=3.0)
    assert np.array_equal(w1.tets, w2.tets) and np.array_equal(w1.xyz, w2.xyz)
    w3 = wl.adapted_box(2000.0, 2000.0, 1000.0, n0=(2, 2, 1), freq=6.0)
    assert w3.tets.shape[0] > 2 * w1.tets.shape[0]


def test_subdomains_of_adapted_mesh_are_uneven():
    w = wl.adapted_box(8000.0, 8000.0, 2000.0, n0=(4, 4, 1), freq=2.0, n_parts=(4, 4, 1))
    counts = np.bincount(w.part, minlength=w.n_sub)
    assert counts.min() > 0 and counts.max() > 1.5 * counts.min()
