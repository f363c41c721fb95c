"""Turns rocprofv3 output into the short text records kept under profiles/.

  python -m paper_1902_01715_amd.profile_records traffic WORKLOAD COPY_DOUBLES FETCH_DB WRITE_DB CMD
      HBM bytes per launch of q = K p (k_sell_spmv_dot) from a FETCH_SIZE run and a
      WRITE_SIZE run (`rocprofv3 --pmc <counter> -d DIR -o NAME`, DIR/NAME_results.db).
      Both counters read in KiB per dispatch at a granularity of their own; each is
      scaled by what it reads for k_copy, which moves COPY_DOUBLES doubles in and the
      same out, in the same run.  Writes profiles/k_sell_spmv_dot_<WORKLOAD>_traffic.json
      with the SHA-256 of kernels_solve.hip, so a later change to the kernels retires it.
      CMD is the profiled command with PMC in place of the counter name.

  python -m paper_1902_01715_amd.profile_records spmm WORKLOAD BENCH_OUT TRACE_CSV FETCH_DB WRITE_DB TCC_DB CMD
      One PCG iteration of the FP32-cycle batch solve, launch by launch: the fused
      K P product with its dot (FP64) and every block SpMM of the V-cycle, labelled
      with its level and operator, with the algorithmic bytes of the launch (the
      block values and column indices once, the gathered X once, W and Y), the
      measured FETCH_SIZE / WRITE_SIZE (scaled by k_copy of the same run, whose
      write counter reads the bytes it moved), the L2 hit rate
      (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)) and the duration of the same
      launch in a --kernel-trace run.  BENCH_OUT is a file that holds the JSON line
      of the batch benchmark (its "levels" give the block counts).  The iteration
      taken is the one between the third and fourth fused K P launches.  Writes
      profiles/k_bsr_spmm_<WORKLOAD>_traffic.json and prints a markdown table.

  python -m paper_1902_01715_amd.profile_records levels WORKLOAD COPY_DOUBLES BENCH_OUT TRACE_CSV FETCH_DB WRITE_DB TCC_DB CMD
      Every V-cycle product per level and precision as `bench.py --level-table`
      launches it (aspamg_time_operator: one warm-up launch, then the timed ones),
      in four runs of the same command: --kernel-trace, FETCH_SIZE, WRITE_SIZE and
      TCC_HIT_sum/TCC_MISS_sum.  The table's launches are the last ones of each run;
      each product gets the median over its timed launches of the duration and of
      the counters (FETCH and WRITE scaled by k_copy of COPY_DOUBLES doubles, as
      for `traffic`), its algorithmic bytes from the benchmark line and the kernel
      each run launched (the layouts are chosen by timing at set-up, so a run may
      pick another layout for a product near a tie; such rows are flagged).
      Writes profiles/k_sell_spmv_<WORKLOAD>_levels_traffic.json and prints a
      markdown table.

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


BATCH_KERNELS = os.path.join(ROOT, "paper_1902_01715_amd", "csrc", "kernels_batch.hip")
SPMM_RE = re.compile(r"k_bsr_spmm<(float|double), (true|false), (true|false), (\d+), (\d+)>")


def dispatches_db(db):
    """[(name, {counter: value})] of one --pmc run in dispatch order."""
    con = sqlite3.connect(db)
    rows = {}
    for did, name, cn, cv in con.execute("select dispatch_id, name, counter_name, counter_value from pmc_events"):
        rows.setdefault(did, [short_name(name), {}])[1][cn] = cv
    con.close()
    return [tuple(rows[d]) for d in sorted(rows)]


def dispatches_trace(path):
    """[(name, duration ns)] of a --kernel-trace csv in dispatch order."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
    return [(short_name(r["Kernel_Name"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows]


def iteration_window(names):
    """Indices of one FP32-cycle PCG iteration: from the third fused K P launch
    (k_bsr_spmm with the dot) up to the fourth."""
    kp = [i for i, n in enumerate(names) if (m := SPMM_RE.match(n)) and m.group(3) == "true"]
    return list(range(kp[2], kp[3]))


def cycle_labels(levels, tail):
    """Operators of the batch V-cycle in launch order: per level G, G^T, A, R,
    (the coarser levels), P, A, G, G^T; the dense tail is one dense product."""
    def walk(l):
        if l == tail:
            return [(l, "dense")]
        return ([(l, "G"), (l, "GT"), (l, "A"), (l, "R")] + walk(l + 1) +
                [(l, "P"), (l, "A"), (l, "G"), (l, "GT")])
    return walk(0)


def spmm_bytes(levels, l, op, size, k):
    """Algorithmic bytes of Y = alpha M X (+ W) over k columns of type size."""
    L = levels[l]
    n, nc = L["n"], L["n_coarse"]
    nnzb, rows, cols = {"A": (L["nnzb_A"], n, n), "G": (L["nnzb_G"], n, n), "GT": (L["nnzb_G"], n, n),
                        "R": (L["nnzb_P"], nc, n), "P": (L["nnzb_P"], n, nc), "KP": (L["nnzb_A"], n, n)}[op]
    vec = 3 * k * size
    return nnzb * (9 * size + 4) + (rows + 1) * 4 + cols * vec + rows * vec


def spmm(workload, bench_out, trace_csv, fetch_db, write_db, tcc_db, cmd):
    bench = None
    for line in open(bench_out):
        if line.startswith("{") and '"levels"' in line:
            bench = json.loads(line)
    levels, k = bench["levels"], bench["config"]["rhs"]
    F, W, T = dispatches_db(fetch_db), dispatches_db(write_db), dispatches_db(tcc_db)
    D = dispatches_trace(trace_csv)
    # k_copy reads what it writes: pair its launches of the two runs in order
    cf = [c["FETCH_SIZE"] for n, c in F if n == "k_copy"]
    cw = [c["WRITE_SIZE"] for n, c in W if n == "k_copy"]
    if not cf or len(cf) != len(cw):
        raise SystemExit("the FETCH and WRITE runs launch k_copy differently")
    ff = statistics.median(w / f for f, w in zip(cf, cw))
    launches = []
    wins = [iteration_window([n for n, _ in src]) for src in (F, W, T, D)]
    seqs = [[src[i] for i in w] for src, w in zip((F, W, T, D), wins)]
    names = [n for n, _ in seqs[0]]
    if any([n for n, _ in sq] != names for sq in seqs[1:]):
        raise SystemExit("the four runs launch different sequences in the iteration")
    ntail = sum(1 for n in names if n.startswith("k_dense_gemm"))
    nspmm = sum(1 for n in names if SPMM_RE.match(n)) - 1
    tail = nspmm // 8
    labels = iter(cycle_labels(levels, tail))
    if ntail != 1 or nspmm != 8 * tail:
        raise SystemExit(f"unexpected cycle: {nspmm} products, {ntail} dense")
    total_ns = 0
    for (name, fc), (_, wc), (_, tc), (_, dur) in zip(*seqs):
        total_ns += dur
        m = SPMM_RE.match(name)
        if m is None and not name.startswith("k_dense_gemm"):
            launches.append({"kernel": name, "us": dur / 1e3})
            continue
        if m is not None and m.group(3) == "true":
            lev, op, size = 0, "KP", 8
        else:
            lev, op = next(labels)
            size = 4 if "float" in name else 8
        if op == "dense":
            launches.append({"kernel": name, "level": lev, "op": "dense tail", "us": dur / 1e3})
            continue
        if m.group(2) == "true" and op not in ("A", "P", "GT"):
            raise SystemExit(f"{name} labelled {op}")
        alg = spmm_bytes(levels, lev, op, size, k)
        if m.group(2) == "true":                 # W has the rows of the product (A, P, G^T: level n)
            alg += levels[lev]["n"] * 3 * k * size
        fetch = fc["FETCH_SIZE"] * ff * 1024
        write = wc["WRITE_SIZE"] * 1024
        hit, miss = tc["TCC_HIT_sum"], tc["TCC_MISS_sum"]
        launches.append({"kernel": name, "level": lev, "op": op, "bytes_alg": alg, "fetch": fetch, "write": write,
                         "measured_over_alg": (fetch + write) / alg, "l2_hit": hit / max(hit + miss, 1),
                         "us": dur / 1e3, "alg_GBps": alg / dur})
    rec = {"workload": workload, "rhs": k, "levels": levels, "command_pmc": cmd, "calibration": {"kernel": "k_copy", "fetch_factor": ff, "write_factor": 1.0},
           "iteration_us": total_ns / 1e3, "launches": launches,
           "kernels_batch_sha256": hashlib.sha256(open(BATCH_KERNELS, "rb").read()).hexdigest()}
    path = os.path.join(ROOT, "profiles", f"k_bsr_spmm_{workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print("| launch | level | operator | alg. MB | FETCH MB | WRITE MB | meas./alg. | L2 hit | us | alg. GB/s |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for x in launches:
        if "bytes_alg" in x:
            print(f"| `{x['kernel']}` | {x['level']} | {x['op']} | {x['bytes_alg'] / 1e6:.1f} | {x['fetch'] / 1e6:.1f} | "
                  f"{x['write'] / 1e6:.1f} | {x['measured_over_alg']:.2f} | {x['l2_hit']:.2f} | {x['us']:.1f} | "
                  f"{x['alg_GBps']:.0f} |")
        else:
            print(f"| `{x['kernel']}` | {x.get('level', '')} | {x.get('op', '')} | | | | | | {x['us']:.1f} | |")
    print(f"\niteration: {total_ns / 1e3:.1f} us")


def levels_traffic(workload, copy_doubles, bench_out, trace_csv, fetch_db, write_db, tcc_db, cmd):
    bench = None
    for line in open(bench_out):
        if line.startswith("{") and '"level_table"' in line:
            bench = json.loads(line)
    rows, reps = bench["level_table"], bench["level_table_reps"]
    per_row = reps + 1
    need = len(rows) * per_row
    F, W, T = dispatches_db(fetch_db), dispatches_db(write_db), dispatches_db(tcc_db)
    D = dispatches_trace(trace_csv)
    copy_kib = copy_doubles * 8 / 1024
    ff = copy_kib / statistics.median(c["FETCH_SIZE"] for n, c in F if n == "k_copy")
    wf = copy_kib / statistics.median(c["WRITE_SIZE"] for n, c in W if n == "k_copy")
    srcs = [F[-need:], W[-need:], T[-need:], D[-need:]]
    if any(len(x) != need for x in srcs):
        raise SystemExit("a run has fewer launches than the level table")
    out = []
    for i, row in enumerate(rows):
        parts = [x[i * per_row:(i + 1) * per_row] for x in srcs]
        names = [{n for n, _ in part} for part in parts]
        kind = "k_dense_gemv" if row["op"] == "dense" else "spmv"
        for ns in names:
            if len(ns) != 1 or kind not in next(iter(ns)):
                raise SystemExit(f"row {i} ({row['level']}, {row['prec']}, {row['op']}): launches {sorted(ns)}")
        kern = [next(iter(ns)) for ns in names]
        timed = [part[1:] for part in parts]
        fetch = statistics.median(c["FETCH_SIZE"] for _, c in timed[0]) * ff * 1024
        write = statistics.median(c["WRITE_SIZE"] for _, c in timed[1]) * wf * 1024
        hit = statistics.median(c["TCC_HIT_sum"] for _, c in timed[2])
        miss = statistics.median(c["TCC_MISS_sum"] for _, c in timed[2])
        us = statistics.median(d for _, d in timed[3]) / 1e3
        rec = {"level": row["level"], "prec": row["prec"], "op": row["op"], "per_cycle": row["per_cycle"],
               "kernel": kern[3], "bytes_alg": row["bytes"], "fetch": fetch, "write": write,
               "measured_over_alg": (fetch + write) / row["bytes"], "l2_hit": hit / max(hit + miss, 1),
               "us": us, "alg_GBps": row["bytes"] / (us * 1e3)}
        if len(set(kern)) != 1:
            rec["kernel_by_run"] = {"fetch": kern[0], "write": kern[1], "tcc": kern[2], "trace": kern[3]}
        out.append(rec)
    rec = {"workload": workload, "command_pmc": cmd, "reps": reps,
           "calibration": {"kernel": "k_copy", "bytes": copy_doubles * 8, "fetch_factor": ff, "write_factor": wf},
           "levels": bench["levels"], "products": out,
           "kernels_solve_sha256": hashlib.sha256(open(KERNELS, "rb").read()).hexdigest()}
    path = os.path.join(ROOT, "profiles", f"k_sell_spmv_{workload}_levels_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print("| level | prec | product | per cycle | kernel | alg. MB | FETCH MB | WRITE MB | meas./alg. | L2 hit | us | alg. GB/s |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for x in out:
        flag = " (layout differs between runs)" if "kernel_by_run" in x else ""
        print(f"| {x['level']} | {x['prec']} | {x['op']} | {x['per_cycle']} | `{x['kernel']}`{flag} | "
              f"{x['bytes_alg'] / 1e6:.1f} | {x['fetch'] / 1e6:.1f} | {x['write'] / 1e6:.1f} | "
              f"{x['measured_over_alg']:.2f} | {x['l2_hit']:.2f} | {x['us']:.1f} | {x['alg_GBps']:.0f} |")


def main(argv):
    if len(argv) == 6 and argv[0] == "traffic":
        traffic(argv[1], int(argv[2]), argv[3], argv[4], argv[5])
    elif len(argv) == 8 and argv[0] == "spmm":
        spmm(*argv[1:])
    elif len(argv) == 9 and argv[0] == "levels":
        levels_traffic(argv[1], int(argv[2]), *argv[3:])
    elif len(argv) == 3 and argv[0] == "stats":
        stats(argv[1], int(argv[2]))
    else:
        sys.exit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
