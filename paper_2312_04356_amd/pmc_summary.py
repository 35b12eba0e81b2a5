"""Summarises rocprofv3 counter runs (CSV output) of bench.py next to its JSON line.

    python -m paper_2312_04356_amd.pmc_summary <pmc_root> <bench_plain.json> "<commands>" > summary.md

<pmc_root> holds the counter directories the passes wrote: pmc_FETCH_SIZE, pmc_WRITE_SIZE,
pmc_VALUBusy (bench.py under --pmc) and pmc_copy_FETCH_SIZE, pmc_copy_WRITE_SIZE (the
device-to-device copies of `bench.py --copy-calibration`, 128 MiB read and 128 MiB written
per launch).  For every kernel family the bench line reports, the last
launches_per_step x (steps) dispatches are the bench's last steps; their counters are
averaged per launch.  HBM bytes per launch = FETCH_SIZE and WRITE_SIZE scaled by the copy
kernel's known bytes over what the same counters read for it.  The last line,
`traffic-record: {...}`, is what bench.py reads back as `roofline.traffic` while the
library's sources still have the digest it records.
"""
import csv
import json
import sys

from paper_2312_04356_amd.prof_summary import family

COPY_BYTES = 128 * 2 ** 20  # bytes read and bytes written per calibration copy
COPY_KERNEL = "copyBuffer"  # the runtime's device-to-device copy kernel


def per_dispatch(path):
    """{dispatch id: (family, {counter: value})} in dispatch order"""
    out = {}
    for r in csv.DictReader(open(path)):
        d = int(r["Dispatch_Id"])
        if d not in out:
            out[d] = (family(r["Kernel_Name"]), {})
        out[d][1][r["Counter_Name"]] = out[d][1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [out[d] for d in sorted(out)]


def copy_factor(root, counter):
    rows = [c[counter] for f, c in per_dispatch("%s/pmc_copy_%s/run_counter_collection.csv" % (root, counter))
            if COPY_KERNEL in f]
    rows = [v for v in rows if v >= 0.25 * max(rows)]  # the 128 MiB copies (not the small ones torch adds)
    return COPY_BYTES / (sum(rows) / len(rows) * 1024.0), sum(rows) / len(rows)


def last_of(disp, fam, n, counter):
    vals = [c[counter] for f, c in disp if f == fam and counter in c]
    vals = vals[-n:] if n else []
    return sum(vals) / len(vals) if vals else float("nan")


def main(root, plain_json, commands):
    plain = json.loads(open(plain_json).read().strip().splitlines()[-1])
    steps = plain["steps"]
    ff, fcopy = copy_factor(root, "FETCH_SIZE")
    fw, wcopy = copy_factor(root, "WRITE_SIZE")
    fetch = per_dispatch("%s/pmc_FETCH_SIZE/run_counter_collection.csv" % root)
    write = per_dispatch("%s/pmc_WRITE_SIZE/run_counter_collection.csv" % root)
    valu = per_dispatch("%s/pmc_VALUBusy/run_counter_collection.csv" % root)
    print("# rocprofv3 counters: %s" % plain["config"]["workload"])
    print()
    print("Commands (repository root; rocprofv3 run from /tmp, each pass its own run):")
    print()
    for line in commands.split(";;"):
        print("    " + line.strip())
    print()
    print("Copy calibration (bench.py --copy-calibration: device-to-device copies, %d MiB read + %d MiB written "
          "per launch): FETCH_SIZE reads %.0f KiB (factor %.4f), WRITE_SIZE %.0f KiB (factor %.4f)."
          % (COPY_BYTES >> 20, COPY_BYTES >> 20, fcopy, ff, wcopy, fw))
    print()
    print("| kernel | launches/step | kernel I/O MB/launch | HBM read MB/launch | HBM written MB/launch | "
          "HBM total / kernel I/O | VALUBusy % | VALU instr / launch (M) |")
    print("|---|---|---|---|---|---|---|---|")
    rows = {}
    for k, v in sorted(plain["pipeline"]["kernels"].items(), key=lambda kv: -kv[1]["ms_per_step"]):
        n = int(round(v["launches_per_step"] * steps))
        alg = v["gbs"] * v["avg_launch_us"] * 1e3  # input + output bytes per launch (library's count)
        rd = last_of(fetch, k, n, "FETCH_SIZE") * 1024 * ff
        wr = last_of(write, k, n, "WRITE_SIZE") * 1024 * fw
        vb = last_of(valu, k, n, "VALUBusy")
        vi = last_of(valu, k, n, "SQ_INSTS_VALU")
        rows[k] = {"read": rd, "write": wr, "alg": alg}
        print("| %s | %.0f | %.1f | %.1f | %.1f | %.2f | %.1f | %.2f |"
              % (k, v["launches_per_step"], alg / 1e6, rd / 1e6, wr / 1e6, (rd + wr) / alg, vb, vi / 1e6))
    print()
    dom = plain["roofline"]["kernel"]
    r = rows.get(dom)
    if r:
        print("Dominant kernel %s: %.0f bytes of HBM traffic per launch (read %.0f + written %.0f) against %.0f "
              "bytes of kernel input and output and %.0f algorithmic bytes (the switching keys it reads)."
              % (dom, r["read"] + r["write"], r["read"], r["write"], r["alg"],
                 plain["roofline"].get("algorithmic_bytes_per_launch", float("nan"))))
    print()
    rec = {"source_sha16": plain["pipeline"]["source_sha16"], "workload": plain["config"]["workload"],
           "kernels": {k: {"hbm_bytes_per_launch": round(v["read"] + v["write"]), "read": round(v["read"]),
                           "written": round(v["write"])} for k, v in rows.items()}}
    print("traffic-record: " + json.dumps(rec))


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], sys.argv[3])
