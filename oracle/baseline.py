"""Timing of the CPU oracle on the host's cores (a bounded sample).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``): run as a child process
of the benchmark, never by the library.

    python -m oracle.baseline --iterations 92 [--restart 50] [--sample 8]

Prints one JSON object.  The oracle is timed as it stands (SuperLU local
solves, SciPy SpMV, MGS), single-threaded per process:

* the subdomains are classed by how many sides of their box touch the domain
  boundary (interior / edge / corner); a sample of each class, one subdomain
  per core, is factored in a pool of worker processes (oracle.pool) and its
  local solves are timed twice: one worker at a time (the single-core times)
  and all workers at once (the times when every core works, memory bandwidth
  shared); sums over all subdomains use the class means times the class
  counts;
* the SpMV with A (twice per iteration in the two-level method), the coarse
  correction and MGS at the mean Krylov dimension of GMRES(m) over the given
  iteration count are timed in this process, single-threaded;
* single core: seconds per iteration = estimated sum of the uncontended
  local solves + the rest; all cores: the concurrent local-solve times spread
  over the host's cores (largest first, least-loaded core) + the rest;
* setup seconds: assembly + decomposition (timed) + the factorisations,
  timed concurrently (so the single-core sum is an upper bound), summed
  (single core) or spread over the cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import time

import numpy as np


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def mean_krylov_dim(iterations, restart):
    """Mean number of basis vectors MGS orthogonalises against per step of
    GMRES(restart) over `iterations` steps (step j of a cycle: j + 1)."""
    dims = []
    left = iterations
    while left > 0:
        k = min(restart, left)
        dims.extend(range(1, k + 1))
        left -= k
    return float(np.mean(dims)) if dims else 1.0


def box_class(i, n_parts):
    """0 interior, 1 edge, 2 corner: sides of the box subdomain i on the
    lateral boundary of an n_parts[0] x n_parts[1] layout."""
    ix, iy = i % n_parts[0], (i // n_parts[0]) % n_parts[1]
    return int(ix in (0, n_parts[0] - 1)) + int(iy in (0, n_parts[1] - 1))


def lpt_makespan(times, cores):
    load = [0.0] * cores
    for t in sorted(times, reverse=True):
        k = int(np.argmin(load))
        load[k] += t
    return max(load)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iterations", type=float, required=True, help="GMRES iterations of the timed solve")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--sample", type=int, default=0, help="subdomains factored and timed; 0: one per core")
    ap.add_argument("--cores", type=int, default=0, help="0: the cores this process may use, at most 16")
    args = ap.parse_args()
    from threadpoolctl import threadpool_limits

    threadpool_limits(1)
    import scipy.sparse.linalg as spla

    from oracle import coarse, fem
    from oracle.pool import PoolOras
    from paper_2004_06309_amd import workloads as wl

    cores = args.cores or min(16, len(os.sched_getaffinity(0)))
    nsample = args.sample or cores
    t0 = time.perf_counter()
    w = wl.mid()
    P = fem.Problem(w.xyz, w.tets, w.order, w.c_tet, w.omega)
    t_asm = time.perf_counter() - t0
    n_parts = (8, 8, 1)
    cls = np.array([box_class(i, n_parts) for i in range(w.n_sub)])
    counts = np.bincount(cls, minlength=3)
    rng = np.random.default_rng(7)
    # sample proportional to the class counts, at least one per class
    want = np.maximum(1, np.round(nsample * counts / counts.sum()).astype(int))
    sample = []
    for c in range(3):
        ids = np.nonzero(cls == c)[0]
        sample += sorted(rng.choice(ids, min(want[c], ids.size), replace=False).tolist())
    t1 = time.perf_counter()
    pool = PoolOras(P, w.part, w.n_sub, w.overlap, None, workers=min(cores, len(sample)), only=sample)
    t_pool = time.perf_counter() - t1
    r = wl.random_vector(P.n, 0)
    pool.one_level(r)  # first solve (warm)
    reps = 3
    sol = {i: 0.0 for i in sample}   # one worker at a time
    solc = {i: 0.0 for i in sample}  # all workers at once
    for _ in range(reps):
        for i, t in pool.solve_each(r).items():
            sol[i] += t / reps
        pool.one_level(r)
        for i, t in pool.last_solve_times.items():
            solc[i] += t / reps
    fac = {i: pool.sub_times[i]["factor_s"] + pool.sub_times[i]["local_matrix_s"] for i in sample}
    pool.close()
    # class means -> every subdomain
    est_sol, est_solc, est_fac = [], [], []
    for i in range(w.n_sub):
        same = [j for j in sample if cls[j] == cls[i]]
        est_sol.append(np.mean([sol[j] for j in same]))
        est_solc.append(np.mean([solc[j] for j in same]))
        est_fac.append(np.mean([fac[j] for j in same]))
    # the rest of an iteration, single-threaded in this process
    t = time.perf_counter()
    for _ in range(reps):
        y = P.A @ r
    t_spmv = (time.perf_counter() - t) / reps
    Z, _ = coarse.interpolation(P, w.coarse_xyz, w.coarse_tets)
    t = time.perf_counter()
    Elu = spla.splu(coarse.galerkin(P.A, Z))
    t_efac = time.perf_counter() - t
    t = time.perf_counter()
    for _ in range(reps):
        q = Z @ Elu.solve(Z.T @ r)
    t_coarse = (time.perf_counter() - t) / reps
    jbar = mean_krylov_dim(int(round(args.iterations)), args.restart)
    jb = int(round(jbar))
    V = rng.standard_normal((P.n, jb)) + 1j * rng.standard_normal((P.n, jb))
    t = time.perf_counter()
    wv = y.copy()
    for i in range(jb):
        h = np.vdot(V[:, i], wv)
        wv = wv - h * V[:, i]
    t_mgs = (time.perf_counter() - t) * jbar / jb
    rest = 2 * t_spmv + t_coarse + t_mgs  # A z, r - A q, coarse, MGS
    per_it_1 = float(np.sum(est_sol)) + rest
    per_it_all = lpt_makespan(est_solc, cores) + rest
    setup_1 = t_asm + float(np.sum(est_fac)) + t_efac
    setup_all = t_asm + lpt_makespan(est_fac, cores) + t_efac
    its = args.iterations
    out = {
        "cpu_model": cpu_model(),
        "cores_available": len(os.sched_getaffinity(0)),
        "single_core": {"cores": 1, "seconds_per_iteration": per_it_1, "iterations_per_s": 1.0 / per_it_1,
                        "solves_per_s": 1.0 / (per_it_1 * its), "setup_s": setup_1},
        "all_cores": {"cores": cores, "seconds_per_iteration": per_it_all, "iterations_per_s": 1.0 / per_it_all,
                      "solves_per_s": 1.0 / (per_it_all * its), "setup_s": setup_all},
        "parts_s": {"assembly_and_decomposition": t_asm, "local_solves_sum": float(np.sum(est_sol)),
                    "spmv": t_spmv, "coarse_correction": t_coarse, "coarse_factor": t_efac,
                    "mgs_at_mean_dim": t_mgs, "mean_krylov_dim": jbar},
        "sample": {"subdomains": [int(i) for i in sample], "class_counts": counts.tolist(),
                   "solve_s": {int(i): sol[i] for i in sample},
                   "solve_concurrent_s": {int(i): solc[i] for i in sample},
                   "factor_s": {int(i): fac[i] for i in sample},
                   "pool_wall_s": t_pool},
        "wall_s": time.perf_counter() - t0,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
