"""Turns rocprofv3 output into the short text records kept under profiles/.

  python -m paper_1902_01715_amd.profile_records traffic WORKLOAD COPY_DOUBLES FETCH_DB WRITE_DB CMD
      HBM bytes per launch of q = K p (k_sell_spmv_dot) from a FETCH_SIZE run and a
      WRITE_SIZE run (`rocprofv3 --pmc <counter> -d DIR -o NAME`, DIR/NAME_results.db).
      Both counters read in KiB per dispatch at a granularity of their own; each is
      scaled by what it reads for k_copy, which moves COPY_DOUBLES doubles in and the
      same out, in the same run.  Writes profiles/k_sell_spmv_dot_<WORKLOAD>_traffic.json
      with the SHA-256 of kernels_solve.hip, so a later change to the kernels retires it.
      CMD is the profiled command with PMC in place of the counter name.

  python -m paper_1902_01715_amd.profile_records stats KERNEL_STATS_CSV N
      The N most expensive kernels of a `rocprofv3 --kernel-trace --stats
      --output-format csv` run as a markdown table (names without the namespace and
      parameter list; template arguments kept).
"""
import csv
import hashlib
import json
import os
import re
import sqlite3
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS = os.path.join(ROOT, "paper_1902_01715_amd", "csrc", "kernels_solve.hip")


def short_name(s):
    s = s.replace("aspamg::(anonymous namespace)::", "").replace("void ", "")
    depth = 0
    for j, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return s[:j]
    return s


def counter_by_kernel(db):
    """Counter values of one --pmc run, grouped by kernel name without template arguments."""
    con = sqlite3.connect(db)
    out = {}
    for name, value in con.execute("select name, counter_value from pmc_events"):
        base = re.split(r"[(<]", short_name(name))[0]
        out.setdefault(base, []).append(value)
    con.close()
    return out


def traffic(workload, copy_doubles, fetch_db, write_db, cmd):
    F, W = counter_by_kernel(fetch_db), counter_by_kernel(write_db)
    copy_kib = copy_doubles * 8 / 1024
    fetch_copy, write_copy = statistics.median(F["k_copy"]), statistics.median(W["k_copy"])
    ff, wf = copy_kib / fetch_copy, copy_kib / write_copy
    fk, wk = statistics.median(F["k_sell_spmv_dot"]), statistics.median(W["k_sell_spmv_dot"])
    rec = {
        "kernel": "k_sell_spmv_dot", "workload": workload,
        "command_fetch": cmd.replace("PMC", "FETCH_SIZE"), "command_write": cmd.replace("PMC", "WRITE_SIZE"),
        "calibration": {"kernel": "k_copy", "bytes": copy_doubles * 8, "fetch_kib": fetch_copy,
                        "write_kib": write_copy, "fetch_factor": ff, "write_factor": wf},
        "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
        "launches": len(F["k_sell_spmv_dot"]),
        "bytes_per_launch": (fk * ff + wk * wf) * 1024,
        "kernels_solve_sha256": hashlib.sha256(open(KERNELS, "rb").read()).hexdigest(),
    }
    path = os.path.join(ROOT, "profiles", f"k_sell_spmv_dot_{workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec, indent=1))


def stats(path, n):
    rows = list(csv.DictReader(open(path)))
    print("| kernel | calls | average us | total ms | % |")
    print("|---|---|---|---|---|")
    for r in rows[:n]:
        print(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")


def main(argv):
    if len(argv) == 6 and argv[0] == "traffic":
        traffic(argv[1], int(argv[2]), argv[3], argv[4], argv[5])
    elif len(argv) == 3 and argv[0] == "stats":
        stats(argv[1], int(argv[2]))
    else:
        sys.exit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
