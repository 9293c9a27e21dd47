"""HBM traffic (and matrix-core / vector-ALU use) of a kernel from rocprofv3
counter runs.

Two separate `rocprofv3 --pmc` runs of the same command (FETCH_SIZE, then
WRITE_SIZE; both in KiB per dispatch) are reduced to bytes per launch of one
kernel.  Each counter is scaled by what it reads for a plain copy kernel of known
size that ran in the same process (the benchmark's `--calibrate-copy`: a
`torch.neg` of a float32 buffer, which reads and writes the buffer once).

    python -m paper_2308_08410_amd.profiling \\
        --fetch out/pmc_fetch --write out/pmc_write \\
        --kernel k_sweep --copy-mib 256 --out profiles/k_sweep_shell500k_traffic.md

The summary written is Markdown with one fenced JSON block; `bench.py` reads it
and reports the traffic only while the kernel sources still hash the same.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))


def _kernel_text(src: str, name: str) -> str:
    """Source text of one __global__ function template (from its template line to
    the closing brace at column 0)."""
    m = re.search(r"\n((?:template <[^\n]*>\n)?__global__[^\n]*?\s+" + re.escape(name) + r"\(.*?\n}\n)",
                  src, re.S)
    if not m:
        raise KeyError(name)
    return m.group(1)


def source_hash(kernel: str = "k_sweep", source: str = "eikonal.hip") -> str:
    """Hash of what a kernel is compiled from: its own text, the queue-push
    helpers and the local solver."""
    with open(os.path.join(_HERE, "csrc", source)) as f:
        eik = f.read()
    with open(os.path.join(_HERE, "csrc", "local_solve.h")) as f:
        ls = f.read()
    i = eik.find("constexpr int kPushCap")
    j = eik.index("__global__", i) if i >= 0 else 0
    h = hashlib.sha256()
    for part in (eik[max(i, 0):j], _kernel_text(eik, kernel), ls):
        h.update(part.encode())
    return h.hexdigest()[:16]


def _counter_csv(path):
    if os.path.isfile(path):
        return path
    hits = sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *counter_collection.csv under {path}")
    return hits[-1]


def per_kernel(path, counter):
    """{kernel name: [value per dispatch]} for one counter (values summed over
    the rows a dispatch may be split into)."""
    rows = {}
    with open(_counter_csv(path), newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            key = (r.get("Dispatch_Id") or r.get("Correlation_Id"), r["Kernel_Name"])
            rows[key] = rows.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (_, name), v in rows.items():
        out.setdefault(name, []).append(v)
    return out


def _mean_of(d, substr):
    vals = [v for name, vs in d.items() if substr in name for v in vs]
    if not vals:
        raise KeyError(f"no dispatch of a kernel matching {substr!r}")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_path, write_path, kernel="k_sweep", copy_substr="neg", copy_mib=256, match=None):
    """match: the substring that selects the kernel's dispatches (default: its
    name; e.g. one template instance)."""
    fetch = per_kernel(fetch_path, "FETCH_SIZE")
    write = per_kernel(write_path, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    f_k, n_f = _mean_of(fetch, match or kernel)
    w_k, n_w = _mean_of(write, match or kernel)
    f_c, _ = _mean_of(fetch, copy_substr)
    w_c, _ = _mean_of(write, copy_substr)
    sf, sw = copy_kib / f_c, copy_kib / w_c
    return dict(kernel=kernel, match=match or kernel, dispatches=[n_f, n_w], fetch_kib_raw=f_k, write_kib_raw=w_k,
                copy_fetch_kib_raw=f_c, copy_write_kib_raw=w_c, copy_mib=copy_mib,
                fetch_scale=sf, write_scale=sw,
                bytes_per_launch=1024.0 * (f_k * sf + w_k * sw),
                source_hash=source_hash(kernel))


def mfma(path, kernel, source="ecg.hip", peak_tflops=2500.0, match=None):
    """Matrix-core use of one kernel from a `--pmc MfmaFlopsBF16 MfmaUtil` run:
    executed bf16 MFMA flops per dispatch, their rate over the dispatch's
    duration, and the fraction of cycles the matrix units were busy."""
    flops, util, dur = {}, {}, {}
    with open(_counter_csv(path), newline="") as f:
        for r in csv.DictReader(f):
            if (match or kernel) not in r["Kernel_Name"]:
                continue
            d = r.get("Dispatch_Id") or r.get("Correlation_Id")
            v = float(r["Counter_Value"])
            if r["Counter_Name"] == "MfmaFlopsBF16":
                flops[d] = flops.get(d, 0.0) + v
            elif r["Counter_Name"] == "MfmaUtil":
                util[d] = v
            dur[d] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    if not flops:
        raise KeyError(f"no MfmaFlopsBF16 rows for {kernel!r}")
    n = len(flops)
    f_avg = sum(flops.values()) / n
    t_avg = sum(dur[d] for d in flops) / n
    return dict(kernel=kernel, dispatches=n, mfma_flops_per_launch=f_avg,
                avg_duration_s_under_counters=t_avg, achieved_tflops=f_avg / t_avg / 1e12,
                peak_tflops=peak_tflops, frac=f_avg / t_avg / 1e12 / peak_tflops,
                mfma_busy_pct=sum(util.values()) / max(len(util), 1),
                source_hash=source_hash(kernel, source))


# Quarter-rate transcendental peak of the VALU (exp2, rcp, ...): 256 CUs x 4 SIMDs
# x 4 lanes per clock x 2.4 GHz.
PEAK_TRANS_OPS = 256 * 4 * 4 * 2.4e9


def valu(path, kernel, source="ecg.hip"):
    """Vector-ALU use of one kernel from a `--pmc SQ_INSTS_VALU SQ_INSTS_VALU_TRANS_F32
    VALUBusy` run: VALU and FP32 transcendental instructions per dispatch (wave
    instructions; x64 lanes for operations), the transcendental rate over the
    dispatch's duration against the quarter-rate peak, and VALUBusy (percent of
    the dispatch's GPU time the CUs' vector ALUs issue)."""
    cnt = {"SQ_INSTS_VALU": {}, "SQ_INSTS_VALU_TRANS_F32": {}, "VALUBusy": {}}
    dur = {}
    with open(_counter_csv(path), newline="") as f:
        for r in csv.DictReader(f):
            if kernel not in r["Kernel_Name"] or r["Counter_Name"] not in cnt:
                continue
            d = r.get("Dispatch_Id") or r.get("Correlation_Id")
            c = cnt[r["Counter_Name"]]
            c[d] = c.get(d, 0.0) + float(r["Counter_Value"])
            dur[d] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    ds = sorted(set(cnt["SQ_INSTS_VALU"]) & set(cnt["SQ_INSTS_VALU_TRANS_F32"]))
    if not ds:
        raise KeyError(f"no VALU counter rows for {kernel!r}")
    n = len(ds)
    v = sum(cnt["SQ_INSTS_VALU"][d] for d in ds) / n
    tr = sum(cnt["SQ_INSTS_VALU_TRANS_F32"][d] for d in ds) / n
    t = sum(dur[d] for d in ds) / n
    busy = [cnt["VALUBusy"][d] for d in ds if d in cnt["VALUBusy"]]
    rate = 64.0 * tr / t
    return dict(kernel=kernel, dispatches=n, valu_insts_per_launch=v, trans_insts_per_launch=tr,
                trans_ops_per_launch=64.0 * tr, avg_duration_s_under_counters=t,
                trans_ops_per_s=rate, trans_peak_ops_per_s=PEAK_TRANS_OPS, trans_frac=rate / PEAK_TRANS_OPS,
                valu_busy_pct=sum(busy) / len(busy) if busy else None,
                source_hash=source_hash(kernel, source))


def trace_table(stats_csv, top=12):
    """Markdown table of the most expensive kernels of a `rocprofv3 --kernel-trace
    --stats` run (names shortened to the function and its template arguments)."""
    rows = []
    with open(stats_csv, newline="") as f:
        for r in csv.DictReader(f):
            name = r["Name"]
            short = re.sub(r"^void ", "", name.replace("(anonymous namespace)::", ""))
            short = re.sub(r"\(.*$", "", short)
            rows.append((short, int(r["Calls"]), float(r["TotalDurationNs"]) * 1e-6,
                         float(r["AverageNs"]) * 1e-3, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for short, calls, tot, avg, pct in rows[:top]:
        out.append(f"| {short} | {calls} | {tot:.3f} | {avg:.2f} | {pct:.2f} |")
    return "\n".join(out)


def read_summary(path):
    """The JSON block of a summary written by this module, or None."""
    try:
        with open(path) as f:
            txt = f.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    return json.loads(m.group(1)) if m else None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--mfma", help="a --pmc MfmaFlopsBF16 MfmaUtil run (instead of --fetch/--write)")
    ap.add_argument("--valu", help="a --pmc SQ_INSTS_VALU SQ_INSTS_VALU_TRANS_F32 VALUBusy run")
    ap.add_argument("--kernel", default="k_sweep")
    ap.add_argument("--match", default=None, help="substring selecting the kernel's dispatches "
                                                  "(default: --kernel)")
    ap.add_argument("--source", default=None, help="source file of --kernel for the hash "
                                                   "(default: eikonal.hip for traffic, ecg.hip otherwise)")
    ap.add_argument("--trace", help="a --kernel-trace --stats run's *_kernel_stats.csv: print its table")
    ap.add_argument("--copy", default="neg")
    ap.add_argument("--copy-mib", type=float, default=256)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="", help="the profiled command, recorded in the summary")
    args = ap.parse_args(argv)
    if args.trace:
        table = trace_table(args.trace)
        with open(args.out, "w") as f:
            f.write(table + "\n")
        print(table)
        return
    if args.mfma:
        t = mfma(args.mfma, args.kernel, source=args.source or "ecg.hip", match=args.match)
        with open(args.out, "w") as f:
            f.write(f"# Matrix-core use: {args.kernel}\n\n")
            f.write("One rocprofv3 counter run (derived counters MfmaFlopsBF16 = 512 x\n"
                    "SQ_INSTS_VALU_MFMA_MOPS_BF16, MfmaUtil = MFMA-busy cycles over active cycles x SIMDs).\n\n")
            if args.command:
                f.write("Commands (repository root, on the MI355X):\n\n")
                for line in args.command.split(";;"):
                    f.write(f"    {line.strip()}\n")
                f.write("\n")
            f.write(f"Per launch: {t['mfma_flops_per_launch'] / 1e9:.3f} GFLOP executed on the matrix cores, "
                    f"{t['achieved_tflops']:.2f} TFLOP/s over the counted dispatch time "
                    f"({100 * t['frac']:.3f}% of the {t['peak_tflops']:.0f} TFLOP/s bf16 dense peak); "
                    f"MFMA busy {t['mfma_busy_pct']:.3f}% of cycles.\n\n")
            f.write("```json\n" + json.dumps(t, indent=1) + "\n```\n")
        print(json.dumps(t))
        return
    if args.valu:
        t = valu(args.valu, args.kernel)
        with open(args.out, "w") as f:
            f.write(f"# Vector-ALU use: {args.kernel}\n\n")
            f.write("One rocprofv3 counter run (SQ_INSTS_VALU and SQ_INSTS_VALU_TRANS_F32 in wave\n"
                    "instructions; VALUBusy = percent of GPU time the vector ALUs issue).  The\n"
                    "transcendental peak is quarter rate: 256 CUs x 4 SIMDs x 4 lanes x 2.4 GHz.\n\n")
            if args.command:
                f.write("Commands (repository root, on the MI355X):\n\n")
                for line in args.command.split(";;"):
                    f.write(f"    {line.strip()}\n")
                f.write("\n")
            busy = t["valu_busy_pct"]
            f.write(f"Per launch: {t['valu_insts_per_launch'] / 1e6:.2f}M VALU wave instructions, "
                    f"{t['trans_insts_per_launch'] / 1e6:.3f}M of them FP32 transcendental "
                    f"({t['trans_ops_per_launch'] / 1e9:.3f} G lane operations, "
                    f"{100 * t['trans_frac']:.1f}% of the transcendental peak over the counted dispatch time); "
                    f"VALUBusy {'n/a' if busy is None else f'{busy:.1f}%'}.\n\n")
            f.write("```json\n" + json.dumps(t, indent=1) + "\n```\n")
        print(json.dumps(t))
        return
    if not (args.fetch and args.write):
        ap.error("--fetch and --write are required without --mfma or --valu")
    t = traffic(args.fetch, args.write, args.kernel, args.copy, args.copy_mib, match=args.match)
    with open(args.out, "w") as f:
        f.write(f"# HBM traffic per launch: {args.kernel}\n\n")
        f.write("Two rocprofv3 counter runs of the same command, FETCH_SIZE then WRITE_SIZE (KiB per\n"
                "dispatch), each scaled by the same counter on a plain copy of known size\n"
                f"(`{args.copy}`, {args.copy_mib:g} MiB read and written) in the same process.\n\n")
        if args.command:
            f.write("Commands (repository root, on the MI355X):\n\n")
            for line in args.command.split(";;"):
                f.write(f"    {line.strip()}\n")
            f.write("\n")
        f.write(f"Per launch: {t['bytes_per_launch'] / 1e6:.2f} MB "
                f"(fetch {t['fetch_kib_raw']:.0f} KiB x {t['fetch_scale']:.3f}, "
                f"write {t['write_kib_raw']:.0f} KiB x {t['write_scale']:.3f}).\n\n")
        f.write("```json\n" + json.dumps(t, indent=1) + "\n```\n")
    print(json.dumps(t))


if __name__ == "__main__":
    sys.exit(main())
