"""Summaries of rocprofv3 output for the library's kernels.

Turns the CSV files of

    rocprofv3 --kernel-trace --stats --output-format csv -d DIR/solve -o run -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch -o run -- python3 bench.py --mode kernels
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write -o run -- python3 bench.py --mode kernels
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/cfetch -o run -- python3 bench.py --mode copy
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/cwrite -o run -- python3 bench.py --mode copy

into a short markdown summary and a traffic record (bytes per launch of the
dominant kernel, byte counters scaled by what they read for a copy of known
size). The record carries a hash of the kernel sources so that a benchmark can
tell when the counters no longer describe the kernel it runs.

    python -m paper_1608_03630_amd.profiling DIR OUT.md TRAFFIC.json KERNEL_SUBSTRING GRID_SIZE FAMILY N
    python -m paper_1608_03630_amd.profiling counters DIR OUT.md   # SQ counter passes (SQ_PASSES), L2 pass
"""
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/interp.hip", "csrc/common.hpp"]


def source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def counter_per_dispatch(path, name_sub, grid_size=None):
    vals = collections.defaultdict(list)
    for r in _rows(path):
        if name_sub in r["Kernel_Name"] and (grid_size is None or r["Grid_Size"] == str(grid_size)):
            vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}


def trace_average_ns(path, name_sub, grid_size=None):
    d = []
    for r in _rows(path):
        gsz = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        if name_sub in r["Kernel_Name"] and (grid_size is None or gsz == grid_size):
            d.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return (sum(d) / len(d), len(d)) if d else (None, 0)


def summarize(pdir, out_md, out_json, kernel_sub, grid_size, family, n, copy_bytes=256 * 1024 * 1024):
    stats = _rows(os.path.join(pdir, "solve", "run_kernel_stats.csv"))
    avg_ns, count = trace_average_ns(os.path.join(pdir, "solve", "run_kernel_trace.csv"), kernel_sub, grid_size)
    fetch, _ = counter_per_dispatch(os.path.join(pdir, "fetch", "run_counter_collection.csv"), kernel_sub, grid_size)
    write, _ = counter_per_dispatch(os.path.join(pdir, "write", "run_counter_collection.csv"), kernel_sub, grid_size)
    cf, _ = counter_per_dispatch(os.path.join(pdir, "cfetch", "run_counter_collection.csv"), "copyBuffer")
    cw, _ = counter_per_dispatch(os.path.join(pdir, "cwrite", "run_counter_collection.csv"), "copyBuffer")
    fetch_scale = (copy_bytes / 1024.0) / cf["FETCH_SIZE"]
    write_scale = (copy_bytes / 1024.0) / cw["WRITE_SIZE"]
    rd = fetch["FETCH_SIZE"] * 1024.0 * fetch_scale
    wr = write["WRITE_SIZE"] * 1024.0 * write_scale
    rec = {
        "kernel": kernel_sub, "kernel_family": family, "n": n, "grid_size": grid_size,
        "bytes_read_per_launch": rd, "bytes_written_per_launch": wr, "bytes_per_launch": rd + wr,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "trace_avg_ms": avg_ns / 1e6 if avg_ns else None, "trace_launches": count,
        "source_sha": source_hash(),
    }
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# rocprofv3 summary: {family} kernel at {n}^3", ""]
    lines += ["Commands (from the repository root; `DIR` is the output folder):", "", "```"]
    lines += [l.strip() for l in __doc__.splitlines() if l.strip().startswith("rocprofv3")]
    lines += ["```", "", f"Dominant kernel `{kernel_sub}` (grid size {grid_size}): {count} dispatches in the solve "
              f"trace, average {avg_ns / 1e6:.4f} ms." if avg_ns else "", ""]
    lines += [f"Byte counters per dispatch: FETCH_SIZE {fetch['FETCH_SIZE']:.0f} KiB, WRITE_SIZE "
              f"{write['WRITE_SIZE']:.0f} KiB. A {copy_bytes // 2**20} MiB copy reads FETCH_SIZE "
              f"{cf['FETCH_SIZE']:.0f} KiB and WRITE_SIZE {cw['WRITE_SIZE']:.0f} KiB, so the scale factors are "
              f"{fetch_scale:.3f} (fetch) and {write_scale:.3f} (write): {rd / 1e6:.1f} MB read + {wr / 1e6:.1f} MB "
              f"written per launch.", ""]
    lines += ["Top kernels of the solve (`--stats`):", "", "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in stats[:14]:
        name = r["Name"].replace("regk::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    lines += ["", f"Kernel source hash: `{rec['source_sha']}`.", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    return rec


# instruction and stall counters of the gather kernels, two passes of at
# most eight SQ counters each (rocprofv3 does not split passes itself)
SQ_PASSES = [
    ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU",
     "SQ_ACTIVE_INST_LDS", "SQ_BUSY_CYCLES"],
    ["SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
     "SQ_ACTIVE_INST_ANY", "SQ_LDS_IDX_ACTIVE"],
]
L2_PASS = ["TCC_HIT_sum", "TCC_MISS_sum", "TCC_REQ_sum"]
GATHER_KERNELS = [("k_tiled_canon<float, 0, 1>", "state step (interp)", 20.0),
                  ("k_tiled_canon<float, 1, 1>", "adjoint step", 24.0),
                  ("k_tiled_canon<float, 2, 1>", "incremental-state step", 44.0),
                  ("k_backtrace_canon", "backtrace (LDS tiles)", 24.0),
                  ("k_floor_bounds<float>", "floor bounds of D", 12.0),
                  ("k_b_assemble<float>", "b assembly (17 levels)", 16.0 * 17 + 12.0)]


def counters_summary(pdir, out_md, n=256, passes=("sq1", "sq2")):
    """Per-dispatch averages of the SQ counters of the gather kernels (and the
    kernel-trace times of the same dispatches) as a markdown table."""
    trace = os.path.join(pdir, "solve", "run_kernel_trace.csv")
    N = n ** 3
    rows = []
    for sub, what, bpp in GATHER_KERNELS:
        vals = {}
        for ps in passes:
            v, _ = counter_per_dispatch(os.path.join(pdir, ps, "run_counter_collection.csv"), sub)
            vals.update(v)
        avg_ns, cnt = trace_average_ns(trace, sub)
        rows.append((sub, what, bpp, vals, avg_ns, cnt))
    lines = [f"# Instruction and stall counters of the gather kernels at {n}^3", "",
             "Commands (from the repository root; `DIR` is the output folder):", "", "```",
             "rocprofv3 --kernel-trace --stats --output-format csv -d DIR/solve -o run -- python3 bench.py --steps 1 "
             "--warmup 0 --no-cpu-baseline"]
    for i, ps in enumerate(passes):
        lines.append(f"rocprofv3 --pmc {' '.join(SQ_PASSES[i])} --output-format csv -d DIR/{ps} -o run -- "
                     "python3 bench.py --mode kernels")
    lines += ["```", "", "Per dispatch (counters summed over the device, averaged over the dispatches of "
              "`--mode kernels`; time from the solve's kernel trace):", ""]
    cols = SQ_PASSES[0][1:] + ["SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_WAIT_INST_ANY", "SQ_LDS_IDX_ACTIVE"]
    lines.append("| kernel | us | GB/s (alg.) | VALU/pt | LDS/pt | " + " | ".join(c.replace("SQ_", "") for c in cols) + " |")
    lines.append("|---" * (5 + len(cols)) + "|")
    for sub, what, bpp, vals, avg_ns, cnt in rows:
        us = avg_ns / 1e3 if avg_ns else float("nan")
        gbs = bpp * N / (avg_ns * 1e-9) / 1e9 if avg_ns else float("nan")
        vpp = vals.get("SQ_INSTS_VALU", float("nan")) * 64 / N
        lpp = vals.get("SQ_INSTS_LDS", float("nan")) * 64 / N
        cells = [f"{vals[c]:.3g}" if c in vals else "-" for c in cols]
        lines.append(f"| {what} `{sub}` | {us:.1f} | {gbs:.0f} | {vpp:.0f} | {lpp:.0f} | " + " | ".join(cells) + " |")
    lines += ["", "VALU/pt and LDS/pt are lane instructions per grid point (wave instructions x 64 / n^3).", ""]
    # the three limits of each kernel against its time
    lines += ["Limits per launch (MI355X: 256 CUs at 2.4 GHz; one wave64 VALU instruction per clock per CU with "
              "packed FP32 off; LDS index unit busy for SQ_LDS_IDX_ACTIVE cycles summed over the CUs; HBM at "
              "8 TB/s for the algorithmic bytes):", "",
              "| kernel | us | VALU floor us | LDS busy us | HBM floor us | time / largest |", "|---|---|---|---|---|---|"]
    cu_hz = 256 * 2.4e9
    for sub, what, bpp, vals, avg_ns, cnt in rows:
        us = avg_ns / 1e3 if avg_ns else float("nan")
        valu = vals.get("SQ_INSTS_VALU", float("nan")) / cu_hz * 1e6
        lds = vals.get("SQ_LDS_IDX_ACTIVE", float("nan")) / cu_hz * 1e6
        hbm = bpp * N / 8e12 * 1e6
        top = max(x for x in (valu, lds, hbm) if x == x)
        lines.append(f"| {what} | {us:.1f} | {valu:.1f} | {lds:.1f} | {hbm:.1f} | {us / top:.2f} |")
    lines.append("")
    l2 = os.path.join(pdir, "l2", "run_counter_collection.csv")
    if os.path.exists(l2):
        lines += ["L2 (TCC) requests and hit rate per dispatch, from a pass of its own:", "", "```",
                  f"rocprofv3 --pmc {' '.join(L2_PASS)} --output-format csv -d DIR/l2 -o run -- python3 bench.py "
                  "--mode kernels", "```", "",
                  "| kernel | L2 requests | requests/pt | hit rate |", "|---|---|---|---|"]
        for sub, what, bpp, _, _, _ in rows:
            v, _ = counter_per_dispatch(l2, sub)
            hit, miss, req = v.get("TCC_HIT_sum"), v.get("TCC_MISS_sum"), v.get("TCC_REQ_sum")
            if hit is None or miss is None or req is None:
                continue
            rate = hit / (hit + miss) if hit + miss > 0 else float("nan")
            lines.append(f"| {what} | {req:.3g} | {req / N:.2f} | {rate:.3f} |")
        lines.append("")
    with open(out_md, "w") as f:
        f.write("\n".join(lines))


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "counters":
        counters_summary(a[1], a[2])
    else:
        print(json.dumps(summarize(a[0], a[1], a[2], a[3], int(a[4]), a[5], int(a[6])), indent=1))
