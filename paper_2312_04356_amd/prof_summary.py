"""Summarises a rocprofv3 kernel trace (CSV output) next to bench.py JSON lines.

    python -m paper_2312_04356_amd.prof_summary <kernel_trace.csv> <bench_under_rocprof.json> \
        <bench_plain.json> "<command>" > summary.md

For every kernel family the bench line reports (launches per step x steps), the
last that-many dispatches in the trace are the bench's live-profiled steps (the
last GPU work of a bench run); their rocprofv3 average duration is set beside the
HIP-event average of a plain bench run (no profiler attached: under rocprofv3 the
events also count the profiler's own per-dispatch work).  Whole-run totals follow,
then the last profiled step launch by launch (grid, registers, LDS, duration).
"""
import csv
import json
import re
import sys
from collections import defaultdict


def family(name):
    n = re.sub(r"\(.*", "", name)
    n = n.replace("void ", "").replace("nj::", "")
    n = re.sub(r"k_ntt_col<\d+, (false|true)(, (false|true))?>", r"k_ntt_col<\1>", n)
    n = re.sub(r"k_ntt_tile_md<(false|true)>", "k_ntt_tile_md", n)
    n = n.strip()
    if n == "k_ntt_tile_gal":  # ModUp's inverse tile pass through X -> X^g
        return "k_ntt_tile<true>"
    # the same families the library's HIP-event counters use
    if n.startswith("k_bconv"):
        return "k_bconv"
    if n.startswith("k_key_ip") or n.startswith("k_ntt_ip"):
        return "k_key_ip"
    if n.startswith("k_bsgs_mac"):
        return "k_pmac"
    if n in OTHER or n.startswith("k_lift_col"):
        return "other"
    return n


# kernels the library times together under "other"
OTHER = ("k_moddown_multi", "k_automorph_multi", "k_automorph_acc", "k_tensor", "k_mul_int",
         "k_add_int", "k_zero", "k_ntt_tile_rs")


def main(trace, bench_json, plain_json, command):
    rows = list(csv.DictReader(open(trace)))
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    plain = json.loads(open(plain_json).read().strip().splitlines()[-1])
    steps = bench["steps"]
    by = defaultdict(list)
    for r in rows:
        by[family(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    print("# rocprofv3 kernel summary: %s" % bench["config"]["workload"])
    print()
    print("Command (repository root; rocprofv3 run from /tmp):")
    print()
    print("    " + command)
    print()
    print("bench.py under rocprofv3: %.4f ms per step, %d steps.  Plain bench.py run (same call, no profiler): "
          "%.4f ms per step; dominant kernel %s, %.2f us per launch (HIP events), %.1f GB/s algorithmic "
          "(%.1f%% of 8 TB/s)."
          % (bench["value"], steps, plain["value"], plain["roofline"]["kernel"], plain["roofline"]["avg_launch_us"],
             plain["roofline"]["achieved"], 100 * plain["roofline"]["frac"]))
    print()
    print("## Live-profiled steps: rocprofv3 kernel durations vs the plain run's HIP events")
    print()
    print("| kernel | launches/step | rocprofv3 avg us | HIP-event avg us (plain run) | ms/step (plain run) |")
    print("|---|---|---|---|---|")
    for k, v in sorted(plain["pipeline"]["kernels"].items(), key=lambda kv: -kv[1]["ms_per_step"]):
        n = int(round(bench["pipeline"]["kernels"].get(k, v)["launches_per_step"] * steps))
        d = by.get(k, [])[-n:] if n else []
        avg = sum(d) / len(d) / 1e3 if d else float("nan")
        print("| %s | %.0f | %.2f | %.2f | %.3f |" % (k, v["launches_per_step"], avg, v["avg_launch_us"], v["ms_per_step"]))
    print()
    print("## Whole run (setup, key switches, warmup, timed and profiled steps)")
    print()
    print("| kernel family | dispatches | total ms | avg us |")
    print("|---|---|---|---|")
    tot = sum(sum(v) for v in by.values())
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:16]:
        print("| %s | %d | %.3f | %.2f |" % (k, len(v), sum(v) / 1e6, sum(v) / len(v) / 1e3))
    print()
    print("Total kernel time %.3f ms." % (tot / 1e6))
    # the last profiled step, launch by launch (the trace's final dispatches)
    per_step = int(round(sum(v["launches_per_step"] for v in bench["pipeline"]["kernels"].values())))
    last = rows[-per_step:] if per_step else []
    if last:
        print()
        print("## The last profiled step, launch by launch (%d launches, %.3f ms of kernel time)"
              % (len(last), sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in last) / 1e6))
        print()
        print("| # | kernel | blocks (x, y, z) | threads | VGPR | LDS B | us |")
        print("|---|---|---|---|---|---|---|")
        for i, r in enumerate(last):
            wg = int(r["Workgroup_Size_X"])
            blocks = (int(r["Grid_Size_X"]) // wg, int(r["Grid_Size_Y"]), int(r["Grid_Size_Z"]))
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("nj::", "").strip()
            print("| %d | %s | %d, %d, %d | %d | %s | %s | %.1f |"
                  % (i, name, blocks[0], blocks[1], blocks[2], wg, r["VGPR_Count"], r["LDS_Block_Size"],
                     (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], sys.argv[3], sys.argv[4])
