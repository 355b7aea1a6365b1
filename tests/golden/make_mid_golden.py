"""Writes tests/golden/mid_oracle.json: the CPU oracle's results on the mid
workload (8x8x2 km thrust model, 80x80x20 Kuhn hexes, P2, 1,062,761 dofs,
f = 5 Hz, 64 box subdomains with overlap 2, two-level ORAS with the nested
40x40x10 P1 coarse mesh; source phi_i(4000, 4000, 10 m)).

Calls only the oracle (and the seeded input generators): nothing here comes
from the HIP library.  Stored values:

* the right-preconditioned GMRES(50) solve at relative residual 1e-6
  (Section "Numerical experiments" stopping rule): iteration count, true
  relative residual, ||x||_2 and x at a seeded sample of dofs;
* for a seeded vector r: the coarse correction q = Z E^{-1} Z^T r (eq. 2lvl),
  the one-level ORAS application M_1^{-1} r (eq. oras) and the two-level
  application M^{-1} r (eq. 2lvl), each as its 2-norm and its values at a
  seeded sample of dofs.

The 64 SuperLU factorisations take about 60 GB, so the local solves run in
the oracle's process pool (``oracle.pool``, single-threaded workers: the same
arithmetic as the sequential oracle, bit for bit).  Run on a host with that
much memory and a few cores:

    python tests/golden/make_mid_golden.py [--workers 16]

About five minutes with 16 workers.
"""
import argparse
import json
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fem, precond  # noqa: E402
from oracle.pool import PoolOras  # noqa: E402
from paper_2004_06309_amd import workloads as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mid_oracle.json")
SEED_R, SEED_SX, SEED_SR = 21, 11, 12
N_SAMPLE = 512


def log(*a):
    rss = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 2**20
    print(f"[{time.strftime('%H:%M:%S')} rss {rss:.1f} GB]", *a, flush=True)


def cplx(v):
    return {"re": [float(t) for t in np.real(v)], "im": [float(t) for t in np.imag(v)]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    args = ap.parse_args()
    from threadpoolctl import threadpool_limits

    threadpool_limits(1)
    t0 = time.time()
    w = wl.mid()
    log("workload", w.name, "tets", w.n_tets)
    P = fem.Problem(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    b = P.point_source(w.source_point)
    log(f"assembled, n = {P.n}")
    M = PoolOras(P, w.part, w.n_sub, w.overlap, (w.coarse_xyz, w.coarse_tets), workers=args.workers, verbose=True)
    t_setup = time.time() - t0
    log(f"oracle setup {t_setup:.0f} s ({args.workers} workers)")
    t1 = time.time()
    calls = [0]

    def precond_logged(v):
        calls[0] += 1
        if calls[0] % 10 == 0:
            log(f"preconditioner application {calls[0]}")
        return M.apply(v)

    class _P:
        apply = staticmethod(precond_logged)

    res = precond.solve(P, b, _P, tol=w.tol, restart=w.restart, maxit=1000)
    t_solve = time.time() - t1
    log(f"solve: its {res.iterations} relres {res.relres:.3e} converged {res.converged} ({t_solve:.0f} s)")
    sx = wl.sample_dofs(P.n, N_SAMPLE, SEED_SX)
    r = wl.random_vector(P.n, SEED_R)
    sr = wl.sample_dofs(P.n, N_SAMPLE, SEED_SR)
    q = M.coarse_correction(r)
    z1 = M.one_level(r)
    z2 = z1 if M.Z is None else M.one_level(r - P.A @ q) + q
    log("applications done")
    out = {
        "workload": "mid: 8x8x2 km thrust model (12 layers, seed 0), 80x80x20 Kuhn hexes, P2, f = 5 Hz, "
                    "8x8x1 box subdomains, overlap 2, nested 40x40x10 P1 coarse mesh, "
                    "source phi_i(4000, 4000, 10 m)",
        "n": int(P.n),
        "nnz": int(P.A.nnz),
        "tol": w.tol,
        "restart": w.restart,
        "solve": {
            "iterations": int(res.iterations),
            "restarts": int(res.restarts),
            "converged": bool(res.converged),
            "relres": float(res.relres),
            "x_norm": float(np.linalg.norm(res.x)),
            "b_norm": float(np.linalg.norm(b)),
            "sample_seed": SEED_SX,
            "x_sample": cplx(res.x[sx]),
        },
        "apply": {
            "r_seed": SEED_R,
            "sample_seed": SEED_SR,
            "q_norm": float(np.linalg.norm(q)),
            "q_sample": cplx(q[sr]),
            "oras_norm": float(np.linalg.norm(z1)),
            "oras_sample": cplx(z1[sr]),
            "precond_norm": float(np.linalg.norm(z2)),
            "precond_sample": cplx(z2[sr]),
        },
        "n_sample": N_SAMPLE,
        "oracle_seconds": {"setup": t_setup, "solve": t_solve, "workers": args.workers},
    }
    M.close()
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    log("wrote", OUT)


if __name__ == "__main__":
    main()
