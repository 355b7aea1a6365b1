"""Seeded synthetic inputs: meshes, velocity models, partitions, source points.

This module produces *inputs* only.  It holds none of the solver's arithmetic
(no basis functions, no element integrals, no boundary classification), so both
the C-ABI library and the CPU oracle can be fed from it without sharing method
code.  Every random draw is made here from ``numpy.random.default_rng(seed)``
and handed to the solver as plain arrays.

Workloads follow the paper's setting (Section "Numerical experiments"): a
layered, folded and faulted acoustic velocity model standing in for the
SEG/EAGE Overthrust model, tetrahedral meshes of a box whose top face is the
free surface (z = 0, z is depth), box subdomains and point sources.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# Kuhn split of the unit cube: one tetrahedron per permutation of the axes,
# each following a monotone lattice path from corner (0,0,0) to (1,1,1).
_KUHN_PATHS = []
for _perm in itertools.permutations(range(3)):
    _c = [0, 0, 0]
    _path = [tuple(_c)]
    for _ax in _perm:
        _c[_ax] += 1
        _path.append(tuple(_c))
    _KUHN_PATHS.append(_path)


def kuhn_mesh(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float):
    """Structured box mesh [0,lx]x[0,ly]x[0,lz], each hex cut into 6 Kuhn tets.

    Node (i, j, k) has index i + (nx+1)*(j + (ny+1)*k) and coordinates
    (i*lx/nx, j*ly/ny, k*lz/nz); z is depth and the top face is z = 0.  Tets
    are returned positively oriented.  Refining (nx, ny, nz) by 2 gives a mesh
    nested in the coarser one.
    """
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    xyz = np.stack([ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")], axis=1).astype(np.float64)
    # order="F" makes i fastest, matching the index formula above
    xyz *= np.array([lx / nx, ly / ny, lz / nz])

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(order="F"), cj.ravel(order="F"), ck.ravel(order="F")

    def nid(a, b, c):
        return a + (nx + 1) * (b + (ny + 1) * c)

    tets = []
    for path in _KUHN_PATHS:
        tets.append(np.stack([nid(ci + p[0], cj + p[1], ck + p[2]) for p in path], axis=1))
    # cell-major order: the 6 tets of a cell are consecutive
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int64)
    return xyz, orient_positive(xyz, tets)


def orient_positive(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap two vertices of every negatively oriented tet (input hygiene)."""
    p = xyz[tets]
    d = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    t = tets.copy()
    neg = d < 0
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t


def tet_centroids(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    return xyz[tets].mean(axis=1)


@dataclass
class ThrustModel:
    """Parameters of the layered/folded/faulted model (all drawn from one seed)."""

    lx: float
    ly: float
    lz: float
    n_layers: int
    amp: np.ndarray = field(default_factory=lambda: np.zeros(3))
    wavelength: np.ndarray = field(default_factory=lambda: np.ones(3))
    theta: np.ndarray = field(default_factory=lambda: np.zeros(3))
    phase: np.ndarray = field(default_factory=lambda: np.zeros(3))
    fault_point: np.ndarray = field(default_factory=lambda: np.zeros(3))
    fault_strike: float = 0.0
    fault_dip_deg: float = 60.0
    fault_throw: float = 200.0

    @classmethod
    def draw(cls, lx, ly, lz, n_layers, seed=0):
        rng = np.random.default_rng(seed)
        amp = rng.uniform(50.0, 300.0, 3)
        wavelength = rng.uniform(2000.0, 6000.0, 3)
        theta = rng.uniform(0.0, np.pi, 3)
        phase = rng.uniform(0.0, 2 * np.pi, 3)
        fx = rng.uniform(0.3, 0.7) * lx
        fy = rng.uniform(0.3, 0.7) * ly
        strike = rng.uniform(0.0, np.pi)
        return cls(lx, ly, lz, n_layers, amp, wavelength, theta, phase,
                   np.array([fx, fy, 0.0]), strike)

    def layer_velocities(self) -> np.ndarray:
        nl = self.n_layers
        return 2000.0 + 4000.0 * np.arange(nl) / (nl - 1)

    def velocity(self, pts: np.ndarray) -> np.ndarray:
        """Real velocity at points (x, y, depth)."""
        x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
        fold = np.zeros_like(x)
        for a, lam, th, ph in zip(self.amp, self.wavelength, self.theta, self.phase):
            fold += a * np.sin(2 * np.pi * (x * np.cos(th) + y * np.sin(th)) / lam + ph)
        # Fault plane through fault_point, trace along the strike direction,
        # dipping at fault_dip_deg towards +h.  Points above it are the
        # hanging wall; a thrust (reverse) fault raises it, so its interfaces
        # sit fault_throw shallower than on the footwall.
        h = np.array([-np.sin(self.fault_strike), np.cos(self.fault_strike)])
        dist = (x - self.fault_point[0]) * h[0] + (y - self.fault_point[1]) * h[1]
        hanging = z < np.tan(np.deg2rad(self.fault_dip_deg)) * dist
        shift = fold - np.where(hanging, self.fault_throw, 0.0)
        nl = self.n_layers
        z0 = self.lz * np.arange(1, nl) / nl  # nl-1 interfaces
        below = (z[:, None] > (z0[None, :] + shift[:, None])).sum(axis=1)
        return self.layer_velocities()[below]


def box_partition(xyz: np.ndarray, tets: np.ndarray, nparts: tuple[int, int, int]) -> np.ndarray:
    """Non-overlapping subdomain id per tet: boxes of the bounding box, by centroid."""
    c = tet_centroids(xyz, tets)
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    idx = []
    for d in range(3):
        t = (c[:, d] - lo[d]) / (hi[d] - lo[d]) * nparts[d]
        idx.append(np.clip(np.floor(t).astype(np.int64), 0, nparts[d] - 1))
    return (idx[0] + nparts[0] * (idx[1] + nparts[1] * idx[2])).astype(np.int32)


def nearest_node(xyz: np.ndarray, point) -> int:
    d = np.linalg.norm(xyz - np.asarray(point, dtype=np.float64)[None, :], axis=1)
    return int(np.argmin(d))


@dataclass
class Workload:
    """One solver configuration: fine mesh, coefficients, decomposition, source."""

    name: str
    xyz: np.ndarray
    tets: np.ndarray
    order: int
    c_tet: np.ndarray  # complex velocity per tet
    omega: float
    part: np.ndarray
    n_sub: int
    overlap: int
    coarse_xyz: np.ndarray | None
    coarse_tets: np.ndarray | None
    source_point: np.ndarray | None  # load F_i = phi_i(x_s) when given
    source_node: int | None  # load F = e_node when given (P1 nodal source)
    restart: int = 50
    tol: float = 1e-6

    @property
    def n_tets(self):
        return self.tets.shape[0]


def tiny(nx: int = 16, n_parts=(2, 2, 2), overlap: int = 1, freq: float = 4.0,
         c0: complex = 2000.0 * (1 - 0.01j)) -> Workload:
    """1 km cube, 16^3 hexes -> 24,576 P1 tets, homogeneous attenuating medium,
    unit source at the node nearest (500, 500, 100) m, one-level ORAS on 2x2x2 boxes."""
    xyz, tets = kuhn_mesh(nx, nx, nx, 1000.0, 1000.0, 1000.0)
    c = np.full(tets.shape[0], c0, dtype=np.complex128)
    part = box_partition(xyz, tets, n_parts)
    node = nearest_node(xyz, (500.0, 500.0, 100.0))
    return Workload("tiny", xyz, tets, 1, c, 2 * np.pi * freq, part, int(np.prod(n_parts)), overlap,
                    None, None, None, node)


def mid(scale: int = 1, freq: float = 5.0, n_parts=(8, 8, 1), overlap: int = 2,
        two_level: bool = True, seed: int = 0, n_layers: int = 12) -> Workload:
    """8x8x2 km thrust model, (80x80x20)/scale hexes -> Kuhn tets, P2, source at
    (4000, 4000, 10) m, 8x8x1 boxes, overlap 2, P1 coarse mesh at twice the
    element size (nested).  scale > 1 shrinks the mesh for quick tests."""
    nx, ny, nz = 80 // scale, 80 // scale, 20 // scale
    xyz, tets = kuhn_mesh(nx, ny, nz, 8000.0, 8000.0, 2000.0)
    model = ThrustModel.draw(8000.0, 8000.0, 2000.0, n_layers, seed)
    c = model.velocity(tet_centroids(xyz, tets)).astype(np.complex128)
    part = box_partition(xyz, tets, n_parts)
    cx = cy = None
    if two_level:
        cx, cy = kuhn_mesh(nx // 2, ny // 2, nz // 2, 8000.0, 8000.0, 2000.0)
    return Workload("mid" if scale == 1 else f"mid/{scale}", xyz, tets, 2, c, 2 * np.pi * freq, part,
                    int(np.prod(n_parts)), overlap, cx, cy, np.array([4000.0, 4000.0, 10.0]), None)


def small_box(n=(6, 5, 4), size=(600.0, 500.0, 400.0), order=2, freq=3.0, n_parts=(2, 2, 1), overlap=1,
              seed=5, attenuation=0.02, coarse=True) -> Workload:
    """A few-hundred-tet box with a random per-tet velocity (2000-3000 m/s),
    used for ragged/edge-case parity tests.  Even n gives a nested coarse mesh."""
    rng = np.random.default_rng(seed)
    xyz, tets = kuhn_mesh(*n, *size)
    c = rng.uniform(2000.0, 3000.0, tets.shape[0]) * (1 - 1j * attenuation)
    part = box_partition(xyz, tets, n_parts)
    cx = cy = None
    if coarse and all(v % 2 == 0 for v in n):
        cx, cy = kuhn_mesh(n[0] // 2, n[1] // 2, n[2] // 2, *size)
    src = np.array([size[0] * 0.37, size[1] * 0.61, size[2] * 0.29])
    return Workload("small", xyz, tets, order, c.astype(np.complex128), 2 * np.pi * freq, part,
                    int(np.prod(n_parts)), overlap, cx, cy, src, None)


def surface_sources(lx: float, ly: float, n_side: int, depth: float = 10.0) -> np.ndarray:
    """n_side x n_side point sources on a regular grid at the given depth
    (cell centres of an n_side x n_side partition of the top face)."""
    xs = (np.arange(n_side) + 0.5) * lx / n_side
    ys = (np.arange(n_side) + 0.5) * ly / n_side
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, depth)], axis=1)


# ---- h-adapted meshes (conforming bisection of a Kuhn mesh) ----------------

def _kuhn_tagged(nx, ny, nz, lx, ly, lz):
    """Kuhn mesh with every tet as its monotone lattice path (x0 .. x3, from
    the cell's lower corner to its upper corner) and bisection tag 3 (its
    refinement edge is the cell diagonal x0-x3)."""
    xyz, _ = kuhn_mesh(nx, ny, nz, lx, ly, lz)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(order="F"), cj.ravel(order="F"), ck.ravel(order="F")

    def nid(a, b, c):
        return a + (nx + 1) * (b + (ny + 1) * c)

    tets = [np.stack([nid(ci + p[0], cj + p[1], ck + p[2]) for p in path], axis=1) for path in _KUHN_PATHS]
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int64)
    return xyz, tets, np.full(tets.shape[0], 3, dtype=np.int8)


def _edge_keys(a, b, n_max):
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    return lo * n_max + hi


def bisect_to_size(xyz, tets, tags, target, max_passes=200):
    """Refines a tagged simplicial mesh by newest-vertex bisection (the
    tagged-simplex rule of Maubach: the refinement edge of (x0..x3; k) is
    x0-xk; its children are (x0..x_{k-1}, z, x_{k+1}..x3) and
    (x1..xk, z, x_{k+1}..x3) with tag k-1, or 3 after 1) until every
    refinement edge is at most target(midpoint) long, bisecting further any
    tet that holds a hanging vertex on one of its edges (closure), so the
    result is conforming.  target: callable on an (m, 3) array of points."""
    xyz = [np.asarray(xyz, dtype=np.float64)]
    nv = xyz[0].shape[0]
    tets = np.asarray(tets, dtype=np.int64).copy()
    tags = np.asarray(tags, dtype=np.int8).copy()
    mid_of = {}  # edge key -> midpoint vertex id
    n_max = np.int64(1) << np.int64(31)
    pairs = [(i, j) for i in range(4) for j in range(i + 1, 4)]
    for _ in range(max_passes):
        P = np.concatenate(xyz)
        k = tags.astype(np.int64)
        a, b = tets[:, 0], tets[np.arange(tets.shape[0]), k]
        mid = 0.5 * (P[a] + P[b])
        mark = np.linalg.norm(P[a] - P[b], axis=1) > target(mid)
        if mid_of:
            known = np.fromiter(mid_of.keys(), dtype=np.int64)
            for (i, j) in pairs:
                mark |= np.isin(_edge_keys(tets[:, i], tets[:, j], n_max), known)
        if not mark.any():
            break
        idx = np.nonzero(mark)[0]
        keys = _edge_keys(a[idx], b[idx], n_max)
        uk, inv = np.unique(keys, return_inverse=True)
        zid = np.empty(uk.size, dtype=np.int64)
        for q, key in enumerate(uk.tolist()):
            v = mid_of.get(key)
            if v is None:
                v = nv
                nv += 1
                mid_of[key] = v
            zid[q] = v
        # coordinates of the new midpoints (in creation order)
        created = [(key, mid_of[key]) for key in uk.tolist() if mid_of[key] >= P.shape[0]]
        if created:
            created.sort(key=lambda t: t[1])
            lo = np.array([c[0] // n_max for c in created], dtype=np.int64)
            hi = np.array([c[0] % n_max for c in created], dtype=np.int64)
            xyz.append(0.5 * (P[lo] + P[hi]))
        z = zid[inv]
        T = tets[idx]
        kk = k[idx]
        c1 = T.copy()
        c1[np.arange(idx.size), kk] = z
        # (x1..xk, z, x_{k+1}..x3), by tag
        c2 = np.empty_like(T)
        for kr in (1, 2, 3):
            s_ = kk == kr
            c2[s_] = np.concatenate([T[s_][:, 1:kr + 1], z[s_][:, None], T[s_][:, kr + 1:]], axis=1)
        nt = np.where(kk > 1, kk - 1, 3).astype(np.int8)
        keep = np.ones(tets.shape[0], dtype=bool)
        keep[idx] = False
        tets = np.concatenate([tets[keep], c1, c2])
        tags = np.concatenate([tags[keep], nt, nt])
    else:
        raise RuntimeError("bisection did not finish")
    P = np.concatenate(xyz)
    return P, orient_positive(P, tets), tags


def adapted_box(lx=8000.0, ly=8000.0, lz=2000.0, n0=(4, 4, 1), freq=2.0, per_wavelength=4.0, coarse_factor=2.0,
                n_parts=(4, 4, 1), overlap=2, order=2, n_layers=12, seed=0, source=None):
    """Thrust model meshed to the local wavelength: a Kuhn mesh of n0 cells
    bisected until every edge is at most c(x) / (per_wavelength f) long
    (edges in slow layers get short, fast ones long), P2, box subdomains of
    uneven size, two-level ORAS on the same bisection at coarse_factor x the
    edge length (not nested in general: the coarse basis is located by
    point search)."""
    model = ThrustModel.draw(lx, ly, lz, n_layers, seed)

    def target(scale):
        return lambda p: scale * model.velocity(p) / (per_wavelength * freq)

    x0, t0, g0 = _kuhn_tagged(*n0, lx, ly, lz)
    xyz, tets, _ = bisect_to_size(x0, t0, g0, target(1.0))
    cx, ct, _ = bisect_to_size(x0, t0, g0, target(coarse_factor))
    c = model.velocity(tet_centroids(xyz, tets)).astype(np.complex128)
    part = box_partition(xyz, tets, n_parts)
    src = np.array([lx / 2, ly / 2, 10.0]) if source is None else np.asarray(source, dtype=np.float64)
    return Workload("adapted", xyz, tets, order, c, 2 * np.pi * freq, part, int(np.prod(n_parts)), overlap,
                    cx, ct, src, None)


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded complex test vector (standard normal real and imaginary parts),
    the input of the preconditioner-application parity checks."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def sample_dofs(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of distinct dof indices."""
    return np.sort(np.random.default_rng(seed).choice(n, count, replace=False))


def thrust_box(nxy: int, nz: int, freq: float, n_parts=(8, 8, 1), overlap: int = 2, two_level: bool = True,
               seed: int = 0, n_layers: int = 12, name: str = "thrust") -> Workload:
    """The 8 x 8 x 2 km thrust model (as in mid) on an nxy x nxy x nz Kuhn
    mesh, P2, at frequency freq, source at (4000, 4000, 10) m, box
    subdomains, and (nxy, nz even) the nested P1 coarse mesh at twice the
    element size."""
    xyz, tets = kuhn_mesh(nxy, nxy, nz, 8000.0, 8000.0, 2000.0)
    model = ThrustModel.draw(8000.0, 8000.0, 2000.0, n_layers, seed)
    c = model.velocity(tet_centroids(xyz, tets)).astype(np.complex128)
    part = box_partition(xyz, tets, n_parts)
    cx = cy = None
    if two_level:
        cx, cy = kuhn_mesh(nxy // 2, nxy // 2, nz // 2, 8000.0, 8000.0, 2000.0)
    return Workload(f"{name} {nxy}x{nxy}x{nz} at {freq:g} Hz", xyz, tets, 2, c, 2 * np.pi * freq, part,
                    int(np.prod(n_parts)), overlap, cx, cy, np.array([4000.0, 4000.0, 10.0]), None)
