"""Summaries of rocprofv3 runs of the library (kernel times and HBM traffic).

    # a plain device copy of known size, for the counter calibration
    rocprofv3 --pmc FETCH_SIZE -d D -o calf --output-format csv -- \\
        python -m paper_2204_06979_amd.profile_summary copy
    # the summary (markdown to stdout; traffic per stage merged into a JSON file)
    python -m paper_2204_06979_amd.profile_summary summarize --stats S_kernel_stats.csv \\
        --fetch F_counter_collection.csv --write W_counter_collection.csv \\
        --cal-fetch CF_counter_collection.csv --cal-write CW_counter_collection.csv \\
        --workload single/mixed --traffic-json profiles/traffic.json --command "..."

FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch.  Each is scaled by
the ratio of the bytes a plain copy of known size moves to what the same
counter reports for that copy.  Per-step figures divide a kernel's total over
the run by the number of steps in it: one step is one run of the whole path
(one solve, one batch, or one sliding-window solve), and every step starts
the threshold search once (one k_sure_init dispatch per step).
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys
from collections import defaultdict

COPY_BYTES = 256 * 1024 * 1024

# kernel-name fragment -> stage of the solve
STAGE_OF = [
    ("k_gram", "gram"), ("k_small", "small"), ("k_project", "project"), ("k_ritz", "project"),
    ("k_dwt_level", "dwt"), ("k_sure", "sure"), ("k_copy_f64", "sure"), ("k_idwt_level", "idwt"),
    ("k_backproject", "backproject"), ("k_blend_axis", "backproject"), ("k_blend_f32", "backproject"),
    ("k_upload", "setup"), ("k_l1l1", "l1l1"), ("k_vdwt", "dwt"), ("k_vidwt", "idwt"),
    ("k_forpdn_filter", "smoother"), ("k_forpdn_lambda", "threshold"),
    ("k_adj_", "adjoint"), ("k_chunk_reduce", "adjoint"), ("k_polar", "polar"),
]


def stage_of(name: str) -> str:
    for frag, st in STAGE_OF:
        if frag in name:
            return st
    return "other"


def short(name: str) -> str:
    n = name.replace("void ", "").replace("hyres::", "").replace("(anonymous namespace)::", "")
    i = n.find("(")
    return n[:i] if i > 0 else n


def read_stats(path):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["Percentage"])))
    return rows


def read_counter(path, counter):
    """kernel name -> (dispatches, total counter value in KiB)."""
    tot = defaultdict(lambda: [0, 0.0])
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            e = tot[r["Kernel_Name"]]
            e[0] += 1
            e[1] += float(r["Counter_Value"])
    return {k: tuple(v) for k, v in tot.items()}


def copy_factor(path, counter):
    """Bytes moved per KiB reported, from the largest-value dispatch of the copy run."""
    best = 0.0
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                best = max(best, float(r["Counter_Value"]))
    return COPY_BYTES / best if best > 0 else None


def summarize(a) -> int:
    stats = read_stats(a.stats)
    fetch = read_counter(a.fetch, "FETCH_SIZE") if a.fetch else {}
    write = read_counter(a.write, "WRITE_SIZE") if a.write else {}
    cf = copy_factor(a.cal_fetch, "FETCH_SIZE") if a.cal_fetch else None
    cw = copy_factor(a.cal_write, "WRITE_SIZE") if a.cal_write else None
    def steps_of(counts):
        # one threshold-search start per cube group and solve
        s = sum(c for n, c in counts if "k_sure_init" in n)
        s = s or sum(c for n, c in counts if "k_small" in n) or 1
        return max(1, s // max(1, a.groups))
    solves_t = steps_of([(n, c) for n, c, *_ in stats])
    solves_f = steps_of([(n, v[0]) for n, v in fetch.items()])
    solves_w = steps_of([(n, v[0]) for n, v in write.items()])
    out = []
    out.append("# rocprofv3 summary: %s\n" % a.workload)
    if a.command:
        out.append("Commands (run from the repository root):\n")
        for c in a.command:
            out.append("    %s" % c)
        out.append("")
    out.append("Steps in the profiled run: %d (threshold-search starts / %d cube group%s per solve).\n"
               % (solves_t, a.groups, "" if a.groups == 1 else "s"))
    for n in a.note or []:
        out.append(n + "\n")
    out.append("| kernel | stage | calls | avg us | us per step | % time |")
    out.append("|---|---|---|---|---|---|")
    for name, calls, total, avg, pct in sorted(stats, key=lambda r: -r[2]):
        out.append("| %s | %s | %d | %.1f | %.1f | %.2f |" % (short(name), stage_of(name), calls, avg / 1e3,
                                                               total / 1e3 / solves_t, pct))
    traffic = defaultdict(float)
    if fetch or write:
        out.append("")
        out.append("HBM traffic per step (counter KiB x calibration: FETCH %s B/KiB, WRITE %s B/KiB, "
                   "from a %d MiB copy):\n" % ("%.1f" % cf if cf else "n/a", "%.1f" % cw if cw else "n/a",
                                               COPY_BYTES >> 20))
        out.append("| kernel | stage | FETCH KiB/step | WRITE KiB/step | bytes/step (calibrated) |")
        out.append("|---|---|---|---|---|")
        names = sorted(set(fetch) | set(write), key=lambda n: -(fetch.get(n, (0, 0))[1] + write.get(n, (0, 0))[1]))
        for n in names:
            fk = fetch.get(n, (0, 0.0))[1] / solves_f
            wk = write.get(n, (0, 0.0))[1] / solves_w
            b = (fk * cf if cf else 0.0) + (wk * cw if cw else 0.0)
            traffic[stage_of(n)] += b
            out.append("| %s | %s | %.0f | %.0f | %.3e |" % (short(n), stage_of(n), fk, wk, b))
        if a.traffic_json and cf and cw:
            try:
                with open(a.traffic_json) as f:
                    t = json.load(f)
            except (OSError, ValueError):
                t = {}
            t[a.workload] = {st: {"bytes": b} for st, b in traffic.items() if st not in ("setup", "other")}
            with open(a.traffic_json, "w") as f:
                json.dump(t, f, indent=1, sort_keys=True)
                f.write("\n")
    print("\n".join(out))
    return 0


def copy_run() -> int:
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes" % COPY_BYTES, flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    s = sub.add_parser("summarize")
    s.add_argument("--stats", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--cal-fetch")
    s.add_argument("--cal-write")
    s.add_argument("--workload", required=True)
    s.add_argument("--traffic-json")
    s.add_argument("--command", action="append")
    s.add_argument("--note", action="append", help="a line of text under the step count")
    s.add_argument("--groups", type=int, default=1, help="cube groups per solve (each starts its own search)")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        return copy_run()
    return summarize(a)


if __name__ == "__main__":
    sys.exit(main())
