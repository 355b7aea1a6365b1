"""Benchmark: ORAS-preconditioned GMRES solves of the 3D Helmholtz equation on
one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config mid|tiny]

A step is one full solve (right-preconditioned GMRES to 1e-6 true relative
residual, complex128) of the workload's point-source right-hand side, with
the operator, the factored two-level preconditioner and the right-hand side
already resident in HBM.  Setup (assembly, analysis, factorisation) happens
before the timed region and is reported separately.  Prints one JSON line.

Workload "mid": 8 x 8 x 2 km synthetic thrust-layered model (12 layers,
folded and faulted, seed 0), 80 x 80 x 20 hexes cut into 768,000 Kuhn tets,
P2 (1,062,761 dofs), f = 5 Hz, source at (4000, 4000, 10) m, 8 x 8 x 1 box
subdomains with 2 overlap layers, two-level ORAS with the nested 40 x 40 x 10
P1 coarse mesh, GMRES(50).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
ROOT = os.path.dirname(os.path.abspath(__file__))
# rocprofv3 FETCH_SIZE/WRITE_SIZE per dispatch, scaled by a device copy of
# known size; valid only for the kernel sources they were measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mid_c128.json")
# what one timed launch of each profiled kernel class is
LAUNCH_UNIT = {"trsv_fwd": "one level of the forward sweep of one of the two subdomain batches (fwd_level_kernel, or "
                           "fwd_sn_kernel on levels with one-wave supernode jobs), timed with the batches one after "
                           "the other",
               "trsv_bwd": "one level of the backward sweep of one of the two subdomain batches (bwd_level_kernel), "
                           "timed with the batches one after the other"}
TRAFFIC_KERNEL = {"trsv_fwd": ("trsv_fwd",), "trsv_bwd": ("trsv_bwd",),
                  "spmv": ("spmv_kernel<", "sell_kernel")}


def kernel_source_hash():
    """SHA-256 of the kernel source and of the host code that shapes the
    launches (what the committed counters depend on)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("device.hip", "solver.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2004_06309_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernels changed since it was taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != kernel_source_hash():
        return None
    for name, e in t.items():
        if isinstance(e, dict) and "fetch_bytes" in e and name.startswith(TRAFFIC_KERNEL.get(kernel, ("?",))):
            return e["fetch_bytes"] + e["write_bytes"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def adapted_operator():
    """The unstructured h-adapted operator: the 8 x 8 x 2 km thrust model
    bisected to a quarter of the local wavelength at 5.5 Hz (about 3M P2
    dofs; the frequency is chosen so the lambda/4 mesh has that size), 128
    box subdomains of uneven size, two-level ORAS with a non-nested coarse
    bisection mesh, complex64 subdomain factors.  Returns (workload, context,
    mesh seconds)."""
    from paper_2004_06309_amd import helm
    from paper_2004_06309_amd import workloads as wl

    t0 = time.perf_counter()
    w = wl.adapted_box(freq=5.5, n0=(4, 4, 1), n_parts=(8, 8, 2))
    t_mesh = time.perf_counter() - t0
    return w, helm.from_workload(w, c64=True), t_mesh


def run_adapted_batch(nrhs, w, h, t_mesh):
    """Batching on the h-adapted operator: nrhs point sources on a 10 m-depth
    grid in blocks of 16."""
    import torch

    from paper_2004_06309_amd import helm
    from paper_2004_06309_amd import workloads as wl

    st = h.stats()
    side = int(np.ceil(np.sqrt(nrhs)))
    pts = wl.surface_sources(8000.0, 8000.0, side)[:nrhs]
    Bb = torch.from_numpy(np.stack([h.point_source(p) for p in pts])).to("cuda")
    Ub = torch.zeros_like(Bb)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    rc, info = h.solve(Bb, Ub, tol=w.tol, restart=w.restart, block=16)
    e1.record()
    torch.cuda.synchronize()
    if rc != helm.HELM_OK:
        raise RuntimeError(f"adapted batched solve did not converge: {info}")
    tb = e0.elapsed_time(e1) / 1e3
    counts = np.bincount(w.part, minlength=w.n_sub)
    its = [i["iterations"] for i in info]
    return {"workload": f"adapted: {w.tets.shape[0]} tets (bisection to lambda/4 at 5.5 Hz), P2, {h.n} dofs, "
                        f"128 subdomains ({counts.min()}-{counts.max()} tets), coarse {st['n_coarse']} unknowns",
            "nrhs": nrhs, "block": 16, "precond_precision": "c64 factors, FP64 FGMRES",
            "solves_per_s": nrhs / tb, "iterations_per_s": float(np.sum(its)) / tb, "mean_iterations": float(np.mean(its)),
            "seconds": tb, "max_relres": max(i["relres"] for i in info), "setup_s": st["setup_seconds"],
            "mesh_s": t_mesh, "factor_GB": st["factor_entries"] * 8 / 1e9}


def run_serving(n_requests, rate, adapted=None, seed=3):
    """Continuous batching over three resident operators of the thrust model:
    3 Hz on the 40 x 40 x 10 P2 mesh, 5 Hz on the 80 x 80 x 20 one and the
    h-adapted 3M-dof operator (`adapted` = (workload, context), or left out),
    all with complex64 subdomain factors (FP64 FGMRES and coarse solve), one
    server and stream each, 16 slots.  Requests arrive as a seeded Poisson
    process, each for one operator with 1-16 point sources at random surface
    positions (10 m deep); a request is done when all its sources are.
    Reports solves/s over the makespan and request latency (arrival to last
    source done)."""
    import torch

    from paper_2004_06309_amd import helm
    from paper_2004_06309_amd import workloads as wl

    ops = [wl.mid(scale=2, freq=3.0), wl.mid()]
    ctxs = [helm.from_workload(w, c64=True) for w in ops]
    if adapted is not None:
        ops.append(adapted[0])
        ctxs.append(adapted[1])
    servers, streams = [], []
    for w, h in zip(ops, ctxs):
        st = torch.cuda.Stream()
        streams.append(st)
        servers.append(helm.Server(h, slots=16, restart=w.restart, tol=w.tol, stream=st))
    rng = np.random.default_rng(seed)
    t_arr = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    op_of = rng.integers(0, len(ops), n_requests)
    nsrc = rng.integers(1, 17, n_requests)
    reqs = []  # (arrival, op, [tags])
    B, U, tag = {}, {}, 0
    for r in range(n_requests):
        h = ctxs[op_of[r]]
        tags = []
        for _ in range(nsrc[r]):
            xs = np.array([rng.uniform(100.0, 7900.0), rng.uniform(100.0, 7900.0), 10.0])
            B[tag] = torch.from_numpy(h.point_source(xs)).to("cuda")
            U[tag] = torch.zeros_like(B[tag])
            tags.append(tag)
            tag += 1
        reqs.append((float(t_arr[r]), int(op_of[r]), tags))
    torch.cuda.synchronize()
    done_at, its, nxt = {}, {}, 0
    t0 = time.perf_counter()
    while len(done_at) < tag:
        now = time.perf_counter() - t0
        while nxt < n_requests and reqs[nxt][0] <= now:
            _, op, tags = reqs[nxt]
            for t in tags:
                servers[op].submit(B[t], U[t], t)
            nxt += 1
        stepped = sum(s_.launch() for s_ in servers)
        for s_ in servers:
            for e in s_.finish():
                if e["status"] != helm.HELM_OK:
                    raise RuntimeError(f"served solve failed: {e}")
                done_at[e["tag"]] = time.perf_counter() - t0
                its[e["tag"]] = e["iterations"]
        if stepped == 0 and nxt < n_requests:
            time.sleep(max(0.0, min(0.01, reqs[nxt][0] - (time.perf_counter() - t0))))
    makespan = max(done_at.values()) - reqs[0][0]
    lat = np.array([max(done_at[t] for t in tags) - a for a, _, tags in reqs])
    for s_ in servers:
        s_.close()
    return {"requests": n_requests, "solves": tag, "arrival_rate_per_s": rate,
            "operators": [f"{w.name}: {h.n} dofs, f={w.omega / (2 * np.pi):.1f} Hz" for w, h in zip(ops, ctxs)],
            "sources_per_request": "1-16",
            "slots_per_operator": 16, "precond_precision": "c64 factors, FP64 FGMRES",
            "solves_per_s": tag / makespan, "makespan_s": makespan,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            "mean_iterations": float(np.mean(list(its.values())))}


def cpu_baseline(w, iters_per_solve):
    """Times the CPU oracle (single thread) on a bounded sample of the same
    workload and scales it to GMRES iterations per second: one of the
    subdomain factorisations and local solves (scaled by the number of
    subdomains), the full-size SpMV, the coarse correction and MGS at the
    mean Krylov dimension of the measured solves."""
    from threadpoolctl import threadpool_limits

    from oracle import coarse as ocoarse
    from oracle import dd as odd
    from oracle import fem
    import scipy.sparse.linalg as spla

    with threadpool_limits(1):
        t0 = time.perf_counter()
        P = fem.Problem(w.xyz, w.tets, w.order, w.c_tet, w.omega)
        subs = odd.decompose(P, w.part, w.n_sub, w.overlap)
        mid = w.n_sub // 2 + int(np.sqrt(w.n_sub)) // 2  # an interior subdomain
        s = subs[mid]
        lu = spla.splu(odd.local_matrix(P, s).tocsc())
        rng = np.random.default_rng(0)
        r = rng.standard_normal(P.n) + 1j * rng.standard_normal(P.n)
        reps = 3
        t = time.perf_counter()
        for _ in range(reps):
            z = np.zeros(P.n, dtype=np.complex128)
            z[s.dofs] += s.D * lu.solve(r[s.dofs])
        t_loc = (time.perf_counter() - t) / reps
        t = time.perf_counter()
        for _ in range(reps):
            y = P.A @ r
        t_spmv = (time.perf_counter() - t) / reps
        t_coarse = 0.0
        if w.coarse_xyz is not None:
            Z, _ = ocoarse.interpolation(P, w.coarse_xyz, w.coarse_tets)
            Elu = spla.splu(ocoarse.galerkin(P.A, Z))
            t = time.perf_counter()
            for _ in range(reps):
                q = Z @ Elu.solve(Z.T @ r)
            t_coarse = (time.perf_counter() - t) / reps + t_spmv  # plus r - A q
        jbar = max(1, int(round(iters_per_solve / 2)))
        V = rng.standard_normal((P.n, jbar)) + 0j
        t = time.perf_counter()
        wv = y.copy()
        for i in range(jbar):
            h = np.vdot(V[:, i], wv)
            wv = wv - h * V[:, i]
        t_gs = time.perf_counter() - t
        per_it = w.n_sub * t_loc + t_spmv + t_coarse + t_gs
        total = time.perf_counter() - t0
    return {
        "value": 1.0 / per_it,
        "unit": "GMRES iterations/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle single-threaded: 1 of {w.n_sub} subdomain LU solves (x{w.n_sub}), full SpMV, "
                   f"coarse correction, MGS at j={jbar}; {total:.1f} s of CPU work"),
        "seconds_per_iteration": per_it,
        "solves_per_s": 1.0 / (per_it * iters_per_solve),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="mid", choices=["mid", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the complex64-factor measurement")
    ap.add_argument("--nrhs", type=int, default=16, help="right-hand sides of the batched measurement (0: skip)")
    ap.add_argument("--block", type=int, default=16, help="right-hand sides advanced together")
    ap.add_argument("--adapted-nrhs", type=int, default=32,
                    help="right-hand sides of the h-adapted batching measurement (0: skip)")
    ap.add_argument("--serve", type=int, default=24,
                    help="requests of the serving measurement (Poisson arrivals over three operators; 0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2.0,
                    help="mean request arrivals per second (the default offers more than the device serves)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        x = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_06309_amd import helm
    from paper_2004_06309_amd import workloads as wl

    w = wl.mid() if args.config == "mid" else wl.tiny()
    log(f"[bench] workload {w.name}: {w.tets.shape[0]} tets, P{w.order}")
    stream = torch.cuda.current_stream()

    def setup(c64):
        t0 = time.perf_counter()
        h = helm.Helm(0)
        h.assemble(w.xyz, w.tets, w.order, w.c_tet, w.omega)
        t_asm = time.perf_counter() - t0
        h.precond_setup(w.part, w.n_sub, w.overlap, w.coarse_xyz, w.coarse_tets, c64=c64)
        st = h.stats()
        log(f"[bench] setup ({'c64' if c64 else 'c128'} factors) {time.perf_counter() - t0:.1f} s, stats {st}")
        return h, st, t_asm

    def run(h, B, U, steps, warmup, tag):
        def one_solve():
            U.zero_()
            rc, info = h.solve(B, U, tol=w.tol, restart=w.restart, stream=stream)
            if rc != helm.HELM_OK:
                raise RuntimeError(f"solve did not converge: {info}")
            return info[0]

        for i in range(warmup):
            inf = one_solve()
            log(f"[bench] {tag} warmup {i}: {inf}")
        torch.cuda.synchronize()
        # the timed solves run without the per-launch profiling events (they
        # add a few microseconds between launches); one more solve with them
        # gives the per-kernel breakdown
        times, its = [], []
        for i in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            inf = one_solve()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
            its.append(inf["iterations"])
            log(f"[bench] {tag} step {i}: {inf['iterations']} its, {times[-1] * 1e3:.1f} ms, "
                f"relres {inf['relres']:.2e}")
        torch.cuda.synchronize()
        h.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        one_solve()
        e1.record(stream)
        torch.cuda.synchronize()
        prof = h.profile_read()
        prof["_solve_s"] = e0.elapsed_time(e1) / 1e3
        h.profile(False)
        return times, its, prof

    def local_solves(h, prof, reps=20, c64=False):
        """Wall time of one-level ORAS applications (both subdomain batches'
        forward and backward sweeps, concurrent on two streams, then the
        prolongation) against their algorithmic bytes from the profile."""
        applies = max(prof["prolong"]["launches"], 1)
        panel = 0.5 if c64 else 1.0  # the profile counts complex128 panel bytes
        by = (panel * (prof["trsv_fwd"]["bytes"] + prof["trsv_bwd"]["bytes"]) + prof["prolong"]["bytes"]) / applies
        r = torch.randn(h.n, dtype=torch.complex128, device="cuda")
        z = torch.empty_like(r)
        for _ in range(2):
            h.apply_oras(r, z, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            h.apply_oras(r, z, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        return {"us_per_apply": us, "bytes_per_apply": by, "GBps": by / (us * 1e-6) / 1e9,
                "frac_of_hbm_peak": by / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}

    h, st, t_asm = setup(False)
    b = helm.load_vector(h, w)
    B = torch.from_numpy(b).to("cuda")
    U = torch.zeros_like(B)
    t_start = time.perf_counter()
    times, its, prof = run(h, B, U, args.steps, args.warmup, "fp64")
    wall = time.perf_counter() - t_start
    total_t = float(np.sum(times))
    total_its = int(np.sum(its))
    its_per_s = total_its / total_t
    solves_per_s = len(times) / total_t
    # dominant kernel by summed time
    dom = max(("trsv_fwd", "trsv_bwd", "spmv", "gs"), key=lambda k: prof[k]["ms"])
    pk = prof[dom]
    avg_ms = pk["ms"] / max(pk["launches"], 1)
    avg_bytes = pk["bytes"] / max(pk["launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    prof_solve_s = prof.pop("_solve_s")  # the profiled solve (batches one after the other)
    kernels = {k: {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / max(v["launches"], 1),
                   "share_of_solve": v["ms"] / 1e3 / prof_solve_s,
                   "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
               for k, v in prof.items()}
    loc = local_solves(h, prof)
    out = {
        "metric": "GMRES iterations/s and solves/s at 1e-6 rel. residual (fp32 vs fp64 precond); p50/p99",
        "value": its_per_s,
        "unit": "GMRES iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total_t / len(times),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: 8x8x2 km thrust model, 80x80x20 hex -> Kuhn tets, P2, "
                               f"{h.n} dofs, f=5 Hz, 64 subdomains overlap 2, two-level ORAS (P1 coarse "
                               f"{st['n_coarse']} unknowns), GMRES(50), tol 1e-6, 1 RHS"
                   if w.name == "mid" else f"{w.name}: {h.n} P1 dofs, 8 subdomains, one-level ORAS",
                   "precond_precision": "fp64 (complex128 factors)", "nrhs": 1},
        "solves_per_s": solves_per_s,
        "iterations_per_solve": float(np.mean(its)),
        "p50_ms": 1e3 * float(np.percentile(times, 50)),
        "p99_ms": 1e3 * float(np.percentile(times, 99)),
        "setup_s": st["setup_seconds"] + t_asm,
        "factorisation": {"seconds": st["factor_seconds"], "on": "host" if st["factor_on_host"] else "device",
                          "flops": st["factor_flops"],
                          "tflops": st["factor_flops"] / max(st["factor_seconds"], 1e-9) / 1e12,
                          "frac_fp64_mfma_peak": st["factor_flops"] / max(st["factor_seconds"], 1e-9) / 78.6e12},
        "factor_GB": st["factor_entries"] * 16 / 1e9,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 counters, copy-calibrated)",
                     "avg_launch_us": 1e3 * avg_ms, "avg_bytes_per_launch": avg_bytes,
                     "launch": LAUNCH_UNIT.get(dom, "one launch")},
        "kernels": kernels,
        "local_solves": loc,
        "wall_s_timed": wall,
    }
    def run_batched(hh, tag):
        """Pseudo-block solves: args.nrhs point sources on a 10 m-depth grid,
        args.block right-hand sides advanced together."""
        side = int(round(np.sqrt(args.nrhs)))
        pts = wl.surface_sources(8000.0, 8000.0, side)[: args.nrhs]
        Bb = torch.from_numpy(np.stack([hh.point_source(p) for p in pts])).to("cuda")
        Ub = torch.zeros_like(Bb)
        hh.solve(Bb[:1].contiguous(), Ub[:1], tol=w.tol, restart=w.restart, block=1)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        Ub.zero_()
        e0.record(stream)
        rc, info = hh.solve(Bb, Ub, tol=w.tol, restart=w.restart, stream=stream, block=args.block)
        e1.record(stream)
        torch.cuda.synchronize()
        if rc != helm.HELM_OK:
            raise RuntimeError(f"batched solve did not converge: {info}")
        tb = e0.elapsed_time(e1) / 1e3
        its_b = [i["iterations"] for i in info]
        log(f"[bench] {tag} batched: {args.nrhs} rhs in blocks of {args.block}: {tb:.3f} s, its {its_b}")
        return {"nrhs": args.nrhs, "block": args.block, "solves_per_s": args.nrhs / tb,
                "iterations_per_s": float(np.sum(its_b)) / tb, "mean_iterations": float(np.mean(its_b)),
                "seconds": tb, "max_relres": max(i["relres"] for i in info)}

    if args.nrhs > 0:
        out["batched_fp64"] = run_batched(h, "fp64")
        out["batched_fp64"]["speedup_vs_single_fp64"] = out["batched_fp64"]["solves_per_s"] / solves_per_s
    if not args.no_fp32:
        # the metric's other line: complex64 subdomain factors, FP64 FGMRES,
        # FP64 coarse solve; error reported against the FP64-factor result
        u64 = U.clone()
        h.close()
        torch.cuda.empty_cache()
        h32, st32, _ = setup(True)
        U32 = torch.zeros_like(B)
        t32, it32, prof32 = run(h32, B, U32, args.steps, args.warmup, "fp32")
        prof32.pop("_solve_s")
        loc32 = local_solves(h32, prof32, c64=True)
        tt = float(np.sum(t32))
        k32 = {k: {"avg_us": 1e3 * v["ms"] / max(v["launches"], 1),
                   "GBps": (v["bytes"] / 2 / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and k.startswith("trsv")
                   else ((v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None)}
               for k, v in prof32.items()}
        out["fp32_precond"] = {
            "iterations_per_s": int(np.sum(it32)) / tt,
            "solves_per_s": len(t32) / tt,
            "iterations_per_solve": float(np.mean(it32)),
            "p50_ms": 1e3 * float(np.percentile(t32, 50)),
            "p99_ms": 1e3 * float(np.percentile(t32, 99)),
            "rel_l2_vs_fp64_factors": float(torch.linalg.norm(U32 - u64) / torch.linalg.norm(u64)),
            "factor_GB": st32["factor_entries"] * 8 / 1e9,
            "speedup_vs_fp64": (len(t32) / tt) / solves_per_s,
            "kernels": k32,
            "local_solves": loc32,
        }
        if args.nrhs > 0:
            out["batched_fp32"] = run_batched(h32, "fp32")
            out["batched_fp32"]["speedup_vs_single_fp64"] = out["batched_fp32"]["solves_per_s"] / solves_per_s
        h32.close()
    # the extra lines below are reported, and a failure there is recorded
    # instead of hiding the main result
    adapted = None
    if (args.adapted_nrhs > 0 or args.serve > 0) and args.config == "mid":
        torch.cuda.empty_cache()
        try:
            adapted = adapted_operator()
        except Exception as e:  # noqa: BLE001
            out["batched_adapted"] = {"error": repr(e)}
    if args.adapted_nrhs > 0 and adapted is not None:
        log(f"[bench] adapted batching: {args.adapted_nrhs} rhs")
        try:
            out["batched_adapted"] = run_adapted_batch(args.adapted_nrhs, *adapted)
        except Exception as e:  # noqa: BLE001
            out["batched_adapted"] = {"error": repr(e)}
        log(f"[bench] adapted batching: {out['batched_adapted']}")
    if args.serve > 0 and args.config == "mid":
        log(f"[bench] serving: {args.serve} requests at {args.serve_rate}/s")
        try:
            out["serving"] = run_serving(args.serve, args.serve_rate, None if adapted is None else adapted[:2])
        except Exception as e:  # noqa: BLE001
            out["serving"] = {"error": repr(e)}
        log(f"[bench] serving: {out['serving']}")
    if adapted is not None:
        adapted[1].close()
    del adapted
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, float(np.mean(its)))
    print(json.dumps(out), flush=True)
    del B, U
    release_device_state()


def release_device_state():
    """Frees every solver context and server and torch's cached blocks, then
    synchronises, so no device object is left for interpreter teardown (a
    profiler that finalises at exit then sees no late hipFree)."""
    import gc

    import torch

    from paper_2004_06309_amd import helm

    helm.close_all()
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    try:
        import psutil

        kids = psutil.Process().children(recursive=True)
        log(f"[bench] child processes at exit: {[(k.pid, k.name()) for k in kids]}")
    except Exception:  # noqa: BLE001
        pass


if __name__ == "__main__":
    main()
