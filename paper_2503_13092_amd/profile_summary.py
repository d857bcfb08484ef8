"""Turns rocprofv3 CSV output of the benchmark into the short text summaries
kept under profiles/ and the per-launch HBM traffic that bench.py reports.

Three profiler runs of the same benchmark command feed it (print them with
--print-commands): a kernel trace with statistics, a FETCH_SIZE pass and a
WRITE_SIZE pass.  Counters are read per dispatch in KiB.  They are scaled by
what the same counter reads for the benchmark's own 2 GiB device-to-device
copy (the copy-ceiling probe), whose true traffic is 2 GiB read and 2 GiB
written, so that the reported bytes are HBM bytes.
"""
import argparse
import csv
import json
import os
import statistics

from .build_lib import ROOT, kernel_source_hash

COPY_BYTES = 2 << 30            # one copy-ceiling probe: 2 GiB read + 2 GiB written
COPY_KERNEL = "__amd_rocclr_copyBuffer"
BENCH = "python $REPO/bench.py --steps {steps} --warmup 2 --no-plain --no-cpu-baseline --no-serve"


SQ_SETS = (
    "SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
    "SQ_ACTIVE_INST_SCA SQ_ACTIVE_INST_ANY",
    "SQ_INSTS_VALU SQ_THREAD_CYCLES_VALU SQ_LDS_BANK_CONFLICT SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 "
    "SQ_INSTS_VALU_MUL_F64 SQ_BUSY_CYCLES SQ_INSTS_LDS",
    "SQ_WAVES SQ_INSTS_SALU SQ_INSTS_SMEM SQ_INST_CYCLES_SMEM SQ_INSTS_BRANCH SQ_LEVEL_WAVES SQ_CYCLES "
    "SQ_INSTS_VALU_CVT",
)
SQ_BENCH = "python $REPO/bench.py --steps 3 --warmup 1 --no-plain --no-cpu-baseline --no-serve --no-copy-ceiling"


def sq_commands(config: int = 1):
    bench = SQ_BENCH + ("" if config == 1 else f" --config {config} --no-dv1")
    return [f"rocprofv3 --pmc {c} --output-format csv -d $OUT/pmc_sq{k} -o sq -- {bench}"
            for k, c in enumerate(SQ_SETS)]


def commands(steps: int = 10, config: int = 1):
    """The three profiler runs, each started in /tmp with TMPDIR=/tmp, $REPO
    set to the repository root and $OUT to the output directory; the trace
    run's stdout (the benchmark's JSON line) goes to $OUT/prof_bench.json."""
    bench = BENCH.format(steps=steps) + ("" if config == 1 else f" --config {config} --no-dv1")
    d = "$OUT"
    return {
        "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d {d}/prof_trace -o trace -- {bench}"
                 f" > {d}/prof_bench.json",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/prof_fetch -o fetch -- {bench}",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/prof_write -o write -- {bench}",
    }


def _find(d: str, suffix: str) -> str:
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _counter(d: str, name: str):
    """Per-kernel lists of one counter's per-dispatch values (KiB)."""
    out = {}
    with open(_find(d, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == name:
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _copy_factor(vals):
    """Bytes per counted KiB from the largest copy dispatches (the 2 GiB probes)."""
    top = max(vals)
    big = [v for v in vals if v >= 0.9 * top]
    return COPY_BYTES / (statistics.median(big) * 1024.0), len(big)


def _match(names, key):
    hits = [n for n in names if key in n]
    if len(hits) != 1:
        raise KeyError(f"{key!r} matches {hits}")
    return hits[0]


def summarize(trace_dir, fetch_dir, write_dir, kernel_key, name, workload, algorithmic_bytes,
              out_dir, steps=10, config=1, src=None):
    with open(_find(trace_dir, "_kernel_stats.csv")) as f:
        stats = list(csv.DictReader(f))
    kname = _match([r["Name"] for r in stats], kernel_key)
    kstat = next(r for r in stats if r["Name"] == kname)
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")
    ff, nf = _copy_factor(fetch[COPY_KERNEL])
    fw, nw = _copy_factor(write[COPY_KERNEL])
    kf = statistics.mean(fetch[_match(fetch, kernel_key)])
    kw = statistics.mean(write[_match(write, kernel_key)])
    fetch_b, write_b = kf * 1024.0 * ff, kw * 1024.0 * fw
    cmds = commands(steps=steps, config=config)
    src = src or kernel_source_hash()
    avg_ns = float(kstat["AverageNs"])

    lines = [f"# {name}", "",
             f"Workload: {workload}.  Kernel source hash {src}.", "",
             "Commands (each in /tmp with `TMPDIR=/tmp`, `$REPO` = repository root, `$OUT` = output "
             "directory):", ""]
    lines += [f"    {c}" for c in cmds.values()]
    lines += ["", "## Kernel time (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in stats[:8]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {r['Percentage']} |")
    lines += ["", "## HBM traffic of the dominant kernel (FETCH_SIZE, WRITE_SIZE passes)", "",
              f"Copy calibration: the 2 GiB copy reads {COPY_BYTES / 1024 / ff:,.0f} KiB of FETCH_SIZE "
              f"(factor {ff:.3f}, {nf} dispatches) and {COPY_BYTES / 1024 / fw:,.0f} KiB of WRITE_SIZE "
              f"(factor {fw:.3f}, {nw} dispatches).", "",
              "| quantity | per launch |", "|---|---|",
              f"| FETCH_SIZE (counter) | {kf:,.1f} KiB |",
              f"| WRITE_SIZE (counter) | {kw:,.1f} KiB |",
              f"| HBM read (scaled) | {fetch_b / 1e6:,.2f} MB |",
              f"| HBM write (scaled) | {write_b / 1e6:,.2f} MB |",
              f"| HBM total | {(fetch_b + write_b) / 1e6:,.2f} MB |",
              f"| algorithmic bytes | {algorithmic_bytes / 1e6:,.2f} MB |",
              f"| traffic / algorithmic | {(fetch_b + write_b) / algorithmic_bytes:.3f} |",
              f"| avg duration | {avg_ns / 1e3:.1f} us |",
              f"| achieved (algorithmic / duration) | {algorithmic_bytes / avg_ns:,.1f} GB/s |", ""]
    sq = {}
    for k in range(len(SQ_SETS)):
        d = os.path.join(os.path.dirname(trace_dir), f"pmc_sq{k}")
        if os.path.isdir(d):
            with open(_find(d, "_counter_collection.csv")) as f:
                for r in csv.DictReader(f):
                    if kernel_key in r["Kernel_Name"]:
                        sq.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if sq:
        m = {k: statistics.mean(v) for k, v in sq.items()}
        g = lambda k: m.get(k, float("nan"))
        lines += ["## Issue and stall counters of the dominant kernel (SQ, per dispatch)", "",
                  "Commands:", ""] + [f"    {c}" for c in sq_commands(config)] + ["", "| counter | value |", "|---|---|"]
        lines += [f"| {k} | {v:.4g} |" for k, v in sorted(m.items())]
        lines += ["", "| derived | value |", "|---|---|",
                  f"| wave cycles waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES) | {g('SQ_WAIT_ANY') / g('SQ_WAVE_CYCLES'):.3f} |",
                  f"| wave cycles issuing (SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES) | "
                  f"{g('SQ_ACTIVE_INST_ANY') / g('SQ_WAVE_CYCLES'):.3f} |",
                  f"| active lanes per VALU instruction (SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU) | "
                  f"{g('SQ_THREAD_CYCLES_VALU') / g('SQ_ACTIVE_INST_VALU'):.1f} of 64 |",
                  f"| VALU instructions per event-batch launch | {g('SQ_INSTS_VALU'):.4g} |",
                  f"| FP64 add+mul+fma share of VALU | "
                  f"{(g('SQ_INSTS_VALU_ADD_F64') + g('SQ_INSTS_VALU_MUL_F64') + g('SQ_INSTS_VALU_FMA_F64')) / g('SQ_INSTS_VALU'):.3f} |",
                  ""]
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"{name}.md"), "w") as f:
        f.write("\n".join(lines))
    tj = os.path.join(out_dir, "traffic.json")
    d = json.load(open(tj)) if os.path.exists(tj) else {}
    d[name] = dict(kernel=kernel_key_id(kernel_key), config=config, source_hash=src,
                   bytes_per_launch=round(fetch_b + write_b),
                   read_bytes=round(fetch_b), write_bytes=round(write_b),
                   fetch_factor=round(ff, 4), write_factor=round(fw, 4),
                   avg_ns=round(avg_ns), workload=workload, summary=f"{name}.md")
    with open(tj, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    return d


def kernel_key_id(key: str) -> str:
    """Short name of a kernel instantiation: k_track<block, candidate rows,
    fused vertexing, Dv1, vertex extras>, k_vertex<block, extras>."""
    if key.startswith("k_track<"):
        f = [x.strip() for x in key[len("k_track<"):-1].split(",")]
        return "k_track" + ("_fused" if f[2] == "true" else "") + ("_dv1" if f[3] == "true" else "")
    if key.startswith("k_vertex<"):
        return "k_vertex"
    return key


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--print-commands", action="store_true")
    ap.add_argument("--print-sq-commands", action="store_true")
    ap.add_argument("--dir", default="prof_out", help="output directory of the profiler runs ($OUT)")
    ap.add_argument("--kernel", default="k_track<256, false, true, false, false>")
    ap.add_argument("--name", default="k_track_fused_throughput_10k")
    ap.add_argument("--algorithmic-bytes", type=float, default=None,
                    help="per launch; default: read from the benchmark JSON line in <dir>/prof_bench.json")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--workload", default=None, help="workload text (default: the benchmark line's)")
    args = ap.parse_args()
    if args.print_commands:
        for k, c in commands(args.steps, args.config).items():
            print(f"{k}\t{c}")
        return
    if args.print_sq_commands:
        for c in sq_commands(args.config):
            print(c)
        return
    ab = args.algorithmic_bytes
    workload = src = None
    bj = os.path.join(args.dir, "prof_bench.json")
    if os.path.exists(bj):
        line = [l for l in open(bj) if l.startswith("{")][-1]
        b = json.loads(line)
        ab = ab or b["roofline"]["algorithmic_bytes_per_launch"]
        workload = args.workload or b["config"]["workload"]
        src = b.get("kernel_source")     # the source the profiled run was built from
    if ab is None:
        raise SystemExit("algorithmic bytes unknown: pass --algorithmic-bytes or provide prof_bench.json")
    summarize(os.path.join(args.dir, "prof_trace"), os.path.join(args.dir, "prof_fetch"),
              os.path.join(args.dir, "prof_write"), args.kernel, args.name, workload or "benchmark batch",
              ab, os.path.join(ROOT, "profiles"), args.steps, args.config, src)


if __name__ == "__main__":
    main()
