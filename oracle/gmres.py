"""Oracle: right-preconditioned restarted GMRES (Krylov solver of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper solves A u = b with GMRES (Saad's textbook) preconditioned by M^{-1}
and stops when ||A x - b|| / ||b|| <= 1e-6 (experiments section).  Readings:
right preconditioning (so the Arnoldi estimate tracks that true residual),
restart m, x0 = 0 unless given, modified Gram-Schmidt with the Hermitian
inner product, complex Givens rotations
    r = sqrt(|a|^2 + |b|^2), c = |a| / r, s = (a / |a|) conj(b) / r
    (c = 0, s = 1 when a = 0),
convergence declared on the estimate |g_{j+1}| <= tol ||b|| and confirmed with
the true residual; a failed confirmation restarts.  Iterations count Arnoldi
steps over all restarts.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    converged: bool
    relres: float
    history: list = field(default_factory=list)  # residual estimates / ||b||
    restarts: int = 0
    arnoldi: dict = field(default_factory=dict)  # V, Z, H of the last cycle (for tests)


def givens(a, b):
    """Complex rotation (c, s) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if a == 0:
        return 0.0, 1.0 + 0j
    r = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    return abs(a) / r, (a / abs(a)) * np.conj(b) / r


def gmres(matvec, b, precond=None, tol=1e-6, restart=50, maxit=1000, x0=None, keep_arnoldi=False):
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    if precond is None:
        precond = lambda v: v.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return GmresResult(np.zeros(n, dtype=np.complex128), 0, True, 0.0)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    its = 0
    hist = []
    restarts = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return GmresResult(x, its, True, beta / bnorm, hist, restarts)
        if its >= maxit:
            return GmresResult(x, its, False, beta / bnorm, hist, restarts)
        m = restart
        V = np.zeros((n, m + 1), dtype=np.complex128)
        Zs = np.zeros((n, m), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        H_arnoldi = np.zeros((m + 1, m), dtype=np.complex128)  # before rotations
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            Zs[:, j] = precond(V[:, j])
            w = matvec(Zs[:, j])
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            its += 1
            k = j + 1
            Hraw = H[: j + 2, j].copy()
            for i in range(j):  # previous rotations
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            hist.append(abs(g[j + 1]) / bnorm)
            breakdown = Hraw[-1] == 0
            if not breakdown:
                V[:, j + 1] = w / Hraw[-1]
            H_arnoldi[: j + 2, j] = Hraw
            if abs(g[j + 1]) <= tol * bnorm or its >= maxit or breakdown:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Zs[:, :k] @ y
        restarts += 1
        arn = {}
        if keep_arnoldi:
            arn = {"V": V[:, : k + 1], "Z": Zs[:, :k], "H": H_arnoldi[: k + 1, :k]}
        rt = b - matvec(x)
        rel = np.linalg.norm(rt) / bnorm
        if rel <= tol:
            return GmresResult(x, its, True, rel, hist, restarts, arn)
        if its >= maxit:
            return GmresResult(x, its, False, rel, hist, restarts, arn)
