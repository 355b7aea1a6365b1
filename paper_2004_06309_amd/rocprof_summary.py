"""Summarise rocprofv3 CSV output of a bench run into a short text table.

    python -m paper_2004_06309_amd.rocprof_summary --trace DIR/mid_kernel_trace.csv \
        [--fetch DIR/mid_counter_collection.csv --write DIR/mid_counter_collection.csv \
         --copy-fetch ... --copy-write ...] [--level-group NAME=K1+K2] [--row KERNEL] \
        --out profiles/<name>.md --command "<cmd>"

Kernel-trace statistics are grouped by kernel (template arguments kept, so
fine and coarse level solves are separate rows).  With counter files, the
per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) are scaled by what the same
counters read for a device copy of known size, and averaged per dispatch.
A level group pools kernels that share the levels of one sweep (the tile
kernel and the one-wave supernode kernel of the forward sweep), each level
being one launch of one of them, and reports them per launch: over all
launches, and over the isolated ones (no other kernel running at the same
time, as when the subdomain batches are timed one after the other).
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import re


def short_name(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "")
    n = re.sub(r"HIP_vector_type<(\w+), 2u>", r"\g<1>2", n)
    m = re.match(r"(?:void )?(?:[\w:]+::)?(\w+(?:<[^()]*>)?)\(", n)
    return re.sub(r"\s+>", ">", m.group(1)) if m else n[:60]


def trace_stats(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[short_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return d


def isolated_stats(path):
    """Durations of the launches that overlap no other kernel in time (the
    ones not sharing the device with a launch on another stream)."""
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
                for r in csv.DictReader(open(path)))
    d = collections.defaultdict(list)
    reach = -1  # latest end among earlier launches
    for i, (a, b, k) in enumerate(ev):
        nxt = ev[i + 1][0] if i + 1 < len(ev) else None
        if a >= reach and (nxt is None or nxt >= b):
            d[k].append(b - a)
        reach = max(reach, b)
    return d


def counter_sums(path, counter):
    """kernel -> [dispatches, summed counter value]"""
    acc = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        k = short_name(r["Kernel_Name"])
        acc[k][0] += 1
        acc[k][1] += float(r["Counter_Value"])
    return acc


def counter_means(path, counter):
    return {k: v[1] / v[0] for k, v in counter_sums(path, counter).items()}


def mfma_table(path, simds, xcds, command):
    """MFMA busy fraction per kernel: SQ_VALU_MFMA_BUSY_CYCLES summed over the
    kernel's dispatches / (device cycles x SIMDs), the device cycles being
    GRBM_GUI_ACTIVE / xcds (the counter sums the dies: it advances by about
    xcds x the shader clock per ns, shown in the last column)."""
    busy = collections.defaultdict(float)
    gui = collections.defaultdict(float)
    ns = collections.defaultdict(float)
    calls = collections.Counter()
    for r in csv.DictReader(open(path)):
        k = short_name(r["Kernel_Name"])
        if r["Counter_Name"] == "SQ_VALU_MFMA_BUSY_CYCLES":
            busy[k] += float(r["Counter_Value"])
        elif r["Counter_Name"] == "GRBM_GUI_ACTIVE":
            gui[k] += float(r["Counter_Value"])
            ns[k] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            calls[k] += 1
    lines = ["# rocprofv3 MFMA counters", "", f"Command: `{command}`", "",
             f"MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {xcds} x {simds} SIMDs), summed over each "
             f"kernel's dispatches (counters serialise the dispatches).  GRBM_GUI_ACTIVE sums the {xcds} XCDs: it "
             f"advances by about {xcds} x 2.4 cycles per ns (last column).", "",
             "| kernel | calls | avg us | MFMA busy | GUI cycles / ns |", "|---|---|---|---|---|"]
    for k in sorted(busy, key=lambda k: -busy[k]):
        if busy[k] <= 0 or calls[k] == 0:
            continue
        lines.append(f"| `{k}` | {calls[k]} | {ns[k] / calls[k] / 1e3:.1f} | {busy[k] * xcds / (gui[k] * simds):.3f} | "
                     f"{gui[k] / ns[k]:.2f} |")
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--mfma", help="counter CSV with SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE per dispatch")
    ap.add_argument("--simds", type=int, default=1024, help="SIMDs of the device (MI355X: 256 CUs x 4)")
    ap.add_argument("--xcds", type=int, default=8,
                    help="dies whose GRBM_GUI_ACTIVE counts are summed (MI355X: 8 XCDs)")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, default=2.0 ** 30)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--json-out")
    ap.add_argument("--level-group", action="append", default=[],
                    help="NAME=K1+K2: kernels sharing the levels of one sweep, reported per level")
    ap.add_argument("--row", action="append", default=[],
                    help="kernel listed in the traffic table even when outside the 16 largest")
    args = ap.parse_args()
    groups = {}
    for g in args.level_group:
        name, ks = g.split("=", 1)
        groups[name] = [k.strip() for k in ks.split("+")]
    if args.mfma:
        lines = mfma_table(args.mfma, args.simds, args.xcds, args.command)
        open(args.out, "w").write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    st = trace_stats(args.trace)
    total = sum(sum(v) for v in st.values())
    lines = [f"# rocprofv3 kernel summary", "", f"Command: `{args.command}`", "",
             "| kernel | calls | avg us | total ms | share |", "|---|---|---|---|---|"]
    for k in sorted(st, key=lambda k: -sum(st[k]))[:24]:
        v = st[k]
        lines.append(f"| `{k}` | {len(v)} | {sum(v) / len(v) / 1e3:.1f} | {sum(v) / 1e6:.2f} | "
                     f"{100 * sum(v) / total:.1f}% |")
    if groups:
        iso = isolated_stats(args.trace)
        lines += ["", "Per level solve (each level of a sweep is one launch of one of the group's kernels; the "
                      "isolated launches share the device with no other kernel, as in the profiled solve, where "
                      "the subdomain batches run one after the other):", "",
                  "| group | kernels | launches | avg us | isolated launches | avg us isolated |",
                  "|---|---|---|---|---|---|"]
        for name, ks in groups.items():
            t = sum(sum(st.get(k, [])) for k in ks)
            n = sum(len(st.get(k, [])) for k in ks)
            ti = sum(sum(iso.get(k, [])) for k in ks)
            ni = sum(len(iso.get(k, [])) for k in ks)
            lines.append(f"| {name} | {' + '.join('`' + k + '`' for k in ks)} | {n} | {t / max(n, 1) / 1e3:.1f} | "
                         f"{ni} | {ti / max(ni, 1) / 1e3:.1f} |")
    out = {}
    if args.fetch and args.write and args.copy_fetch and args.copy_write:
        cf = max(counter_means(args.copy_fetch, "FETCH_SIZE").values())
        cw = max(counter_means(args.copy_write, "WRITE_SIZE").values())
        sf = args.copy_bytes / (cf * 1024.0)
        sw = args.copy_bytes / (cw * 1024.0)
        fe = counter_means(args.fetch, "FETCH_SIZE")
        wr = counter_means(args.write, "WRITE_SIZE")
        lines += ["", f"HBM traffic per dispatch (FETCH_SIZE x {sf:.3f}, WRITE_SIZE x {sw:.3f}; factors from a "
                      f"{args.copy_bytes / 2**30:.0f} GiB device copy):", "",
                  "| kernel | fetch MB | write MB |", "|---|---|---|"]
        top = sorted(fe, key=lambda k: -fe[k])[:16]
        for k in top + [k for k in args.row if k in fe and k not in top]:
            lines.append(f"| `{k}` | {fe[k] * 1024 * sf / 1e6:.2f} | {wr.get(k, 0.0) * 1024 * sw / 1e6:.2f} |")
        for k in fe:  # every kernel's figures go into the JSON
            out[k] = {"fetch_bytes": fe[k] * 1024 * sf, "write_bytes": wr.get(k, 0.0) * 1024 * sw}
        if groups:
            fs = counter_sums(args.fetch, "FETCH_SIZE")
            ws = counter_sums(args.write, "WRITE_SIZE")
            lines += ["", "Per level solve:", "", "| group | fetch MB | write MB |", "|---|---|---|"]
            for name, ks in groups.items():
                na = sum(fs[k][0] for k in ks if k in fs)
                nw = sum(ws[k][0] for k in ks if k in ws)
                f = sum(fs[k][1] for k in ks if k in fs) * 1024 * sf / max(na, 1)
                w = sum(ws[k][1] for k in ks if k in ws) * 1024 * sw / max(nw, 1)
                out[name] = {"fetch_bytes": f, "write_bytes": w}
                lines.append(f"| {name} | {f / 1e6:.2f} | {w / 1e6:.2f} |")
        out["_scale"] = {"fetch": sf, "write": sw}
        import hashlib
        import os
        hs = hashlib.sha256()
        for f in ("device.hip", "solver.cpp"):  # kernels and the host code that shapes their launches
            hs.update(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f), "rb").read())
        out["sources_sha256"] = hs.hexdigest()
    open(args.out, "w").write("\n".join(lines) + "\n")
    if args.json_out:
        json.dump(out, open(args.json_out, "w"), indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
