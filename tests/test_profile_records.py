"""The script that turns rocprofv3 output into the committed records: kernel
names shortened, counters grouped by kernel, the copy-kernel calibration and
the bytes per launch (checked on a small synthetic counter database and stats
CSV, no GPU)."""
import csv
import json
import sqlite3

from paper_1902_01715_amd import profile_records as pr


def test_short_name_keeps_template_arguments():
    long = ("void aspamg::(anonymous namespace)::k_pack_spmv<float, float, float, true, 2, false, "
            "unsigned short>(int, int const*, unsigned short const*)")
    assert pr.short_name(long) == "k_pack_spmv<float, float, float, true, 2, false, unsigned short>"
    assert pr.short_name("k_copy(long, double const*, double*)") == "k_copy"


def _db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table pmc_events (name text, counter_value real)")
    con.executemany("insert into pmc_events values (?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_record(tmp_path, monkeypatch):
    # copy of 1,000,000 doubles: FETCH reads half the bytes (factor 2), WRITE all (factor 1)
    kib = 8e6 / 1024
    dot = "void aspamg::(anonymous namespace)::k_sell_spmv_dot<unsigned short, 1>(int, int const*)"
    _db(tmp_path / "f.db", [("k_copy(long, double const*, double*)", kib / 2)] * 3 + [(dot, 100.0), (dot, 102.0), (dot, 101.0)])
    _db(tmp_path / "w.db", [("k_copy(long, double const*, double*)", kib)] * 3 + [(dot, 10.0)] * 3)
    monkeypatch.setattr(pr, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    pr.traffic("t", 1000000, str(tmp_path / "f.db"), str(tmp_path / "w.db"), "cmd PMC")
    rec = json.load(open(tmp_path / "profiles" / "k_sell_spmv_dot_t_traffic.json"))
    assert rec["launches"] == 3
    assert abs(rec["calibration"]["fetch_factor"] - 2.0) < 1e-12
    assert abs(rec["calibration"]["write_factor"] - 1.0) < 1e-12
    # median fetch 101 KiB x 2 + write 10 KiB x 1
    assert abs(rec["bytes_per_launch"] - (101.0 * 2 + 10.0) * 1024) < 1e-6
    assert rec["command_fetch"] == "cmd FETCH_SIZE" and rec["command_write"] == "cmd WRITE_SIZE"
    assert len(rec["kernels_solve_sha256"]) == 64


def test_stats_table(tmp_path, capsys):
    path = tmp_path / "s.csv"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void aspamg::(anonymous namespace)::k_fill(long, double*, double)", "Calls": 4,
                    "TotalDurationNs": 8000, "AverageNs": 2000, "Percentage": 75.0})
        w.writerow({"Name": "k_copy(long)", "Calls": 1, "TotalDurationNs": 1000, "AverageNs": 1000,
                    "Percentage": 25.0})
    pr.stats(str(path), 1)
    out = capsys.readouterr().out.splitlines()
    assert out[0].startswith("| kernel |") and len(out) == 3
    assert out[2] == "| `k_fill` | 4 | 2.00 | 0.01 | 75.00 |"


def test_cycle_labels_follow_the_v_cycle():
    got = pr.cycle_labels([{}] * 3, 2)
    assert got == [(0, "G"), (0, "GT"), (0, "A"), (0, "R"),
                   (1, "G"), (1, "GT"), (1, "A"), (1, "R"), (2, "dense"), (1, "P"), (1, "A"), (1, "G"), (1, "GT"),
                   (0, "P"), (0, "A"), (0, "G"), (0, "GT")]


def test_spmm_bytes_of_each_operator():
    lev = [{"n": 10, "n_coarse": 4, "nnzb_A": 50, "nnzb_G": 30, "nnzb_P": 12}]
    k, s = 4, 4                       # 4 FP32 columns: 48 B per gathered or written block row
    assert pr.spmm_bytes(lev, 0, "A", s, k) == 50 * 40 + 11 * 4 + 10 * 48 + 10 * 48
    assert pr.spmm_bytes(lev, 0, "GT", s, k) == 30 * 40 + 11 * 4 + 10 * 48 + 10 * 48
    assert pr.spmm_bytes(lev, 0, "R", s, k) == 12 * 40 + 5 * 4 + 10 * 48 + 4 * 48      # 4 rows, 10 columns
    assert pr.spmm_bytes(lev, 0, "P", s, k) == 12 * 40 + 11 * 4 + 4 * 48 + 10 * 48     # 10 rows, 4 columns


def test_spmm_record_labels_one_iteration(tmp_path, monkeypatch, capsys):
    ns = "void aspamg::(anonymous namespace)::"
    kp = ns + "k_bsr_spmm<double, false, true, 4, 1>(int)"
    plain, axpy = ns + "k_bsr_spmm<float, false, false, 4, 1>(int)", ns + "k_bsr_spmm<float, true, false, 4, 1>(int)"
    dense, copy = ns + "k_dense_gemm<float>(int)", ns + "k_copy(long, double const*, double*)"
    other = [ns + "k_col_finish(int)", ns + "k_col_update<float>(long)", ns + "k_col_finish(int)"]
    it = [kp] + other + [plain, plain, axpy, plain, dense, axpy, axpy, plain, axpy] + [ns + "k_col_rz<float>(long)"]
    seq = [copy, copy] + it * 4 + [kp]
    def db(path, counters):
        con = sqlite3.connect(path)
        con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, counter_value real)")
        for i, name in enumerate(seq):
            for c, v in counters(name).items():
                con.execute("insert into pmc_events values (?, ?, ?, ?)", (i + 1, name, c, v))
        con.commit()
        con.close()
    db(tmp_path / "f.db", lambda n: {"FETCH_SIZE": 50.0 if "k_copy" in n else 100.0})
    db(tmp_path / "w.db", lambda n: {"WRITE_SIZE": 100.0 if "k_copy" in n else 10.0})
    db(tmp_path / "t.db", lambda n: {"TCC_HIT_sum": 3.0, "TCC_MISS_sum": 1.0})
    with open(tmp_path / "trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i, name in enumerate(seq):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": 1000 * i,
                        "End_Timestamp": 1000 * i + 500})
    levels = [{"n": 10, "n_coarse": 4, "nnzb_A": 50, "nnzb_G": 30, "nnzb_P": 12},
              {"n": 4, "n_coarse": 0, "nnzb_A": 16, "nnzb_G": 0, "nnzb_P": 0}]
    (tmp_path / "bench.out").write_text("[bench] x\n" + json.dumps({"levels": levels, "config": {"rhs": 4}}) + "\n")
    monkeypatch.setattr(pr, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    pr.spmm("t", str(tmp_path / "bench.out"), str(tmp_path / "trace.csv"), str(tmp_path / "f.db"),
            str(tmp_path / "w.db"), str(tmp_path / "t.db"), "cmd PMC")
    rec = json.load(open(tmp_path / "profiles" / "k_bsr_spmm_t_traffic.json"))
    ops = [(x.get("level"), x.get("op")) for x in rec["launches"] if "op" in x]
    assert ops == [(0, "KP"), (0, "G"), (0, "GT"), (0, "A"), (0, "R"), (1, "dense tail"), (0, "P"), (0, "A"),
                   (0, "G"), (0, "GT")]
    assert abs(rec["calibration"]["fetch_factor"] - 2.0) < 1e-12
    a = [x for x in rec["launches"] if x.get("op") == "A"][0]
    assert a["fetch"] == 100.0 * 2 * 1024 and a["write"] == 10.0 * 1024 and a["l2_hit"] == 0.75
    # A with the fused axpy: the matrix, row pointers, x, y and w
    assert a["bytes_alg"] == 50 * 40 + 11 * 4 + 3 * 10 * 48
    assert rec["iteration_us"] == 14 * 0.5


def test_levels_record_takes_the_table_launches(tmp_path, monkeypatch, capsys):
    ns = "void aspamg::(anonymous namespace)::"
    sell, pack = ns + "k_sell_spmv<float, float, float, 4>(int)", ns + "k_pack_spmv<float, float, float, 2>(int)"
    dense, copy = ns + "k_dense_gemv<float>(int)", ns + "k_copy(long, double const*, double*)"
    rows = [{"level": 0, "prec": 32, "op": "residual A", "per_cycle": 1, "ms": 0.1, "bytes": 4.0e6, "GBps": 40.0},
            {"level": 0, "prec": 32, "op": "G", "per_cycle": 2, "ms": 0.05, "bytes": 2.0e6, "GBps": 40.0},
            {"level": 1, "prec": 32, "op": "dense", "per_cycle": 1, "ms": 0.01, "bytes": 1.0e5, "GBps": 10.0}]
    reps = 3
    # set-up and solve launches first (k_copy among them), then warm-up + reps per row
    head = [copy, sell, copy, pack]
    table = [sell] * (reps + 1) + [pack] * (reps + 1) + [dense] * (reps + 1)
    seq = head + table
    def db(path, counters):
        con = sqlite3.connect(path)
        con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, counter_value real)")
        for i, name in enumerate(seq):
            for c, v in counters(i, name).items():
                con.execute("insert into pmc_events values (?, ?, ?, ?)", (i + 1, name, c, v))
        con.commit()
        con.close()
    kib = 8e6 / 1024                      # k_copy of 1,000,000 doubles
    # the warm-up launch of each row reads a cold cache: 10x the counts, ignored by the median
    warm = {len(head) + r * (reps + 1) for r in range(3)}
    db(tmp_path / "f.db", lambda i, n: {"FETCH_SIZE": kib / 2 if "k_copy" in n else (1000.0 if i in warm else 100.0 + i % 2)})
    db(tmp_path / "w.db", lambda i, n: {"WRITE_SIZE": kib if "k_copy" in n else 20.0})
    db(tmp_path / "t.db", lambda i, n: {"TCC_HIT_sum": 9.0, "TCC_MISS_sum": 1.0})
    with open(tmp_path / "trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i, name in enumerate(seq):
            # the trace run chose the sliced layout for G
            name = sell if name == pack and i >= len(head) else name
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": 10000 * i,
                        "End_Timestamp": 10000 * i + 2000})
    (tmp_path / "bench.out").write_text("[bench] x\n" + json.dumps({"levels": [{"n": 1}], "level_table": rows,
                                                                    "level_table_reps": reps}) + "\n")
    monkeypatch.setattr(pr, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    pr.main(["levels", "t", "1000000", str(tmp_path / "bench.out"), str(tmp_path / "trace.csv"),
             str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(tmp_path / "t.db"), "cmd PMC"])
    rec = json.load(open(tmp_path / "profiles" / "k_sell_spmv_t_levels_traffic.json"))
    a, g, d = rec["products"]
    assert abs(rec["calibration"]["fetch_factor"] - 2.0) < 1e-12 and abs(rec["calibration"]["write_factor"] - 1.0) < 1e-12
    # median of the timed launches only (the warm-up's 1000 KiB left out)
    assert a["fetch"] in (100.0 * 2 * 1024, 101.0 * 2 * 1024) and a["write"] == 20.0 * 1024
    assert abs(a["measured_over_alg"] - (a["fetch"] + a["write"]) / 4.0e6) < 1e-12
    assert a["l2_hit"] == 0.9 and a["us"] == 2.0 and a["alg_GBps"] == 4.0e6 / 2000
    assert "kernel_by_run" not in a and a["kernel"].startswith("k_sell_spmv")
    assert g["kernel_by_run"]["fetch"].startswith("k_pack_spmv") and g["kernel_by_run"]["trace"].startswith("k_sell_spmv")
    assert d["op"] == "dense" and d["kernel"].startswith("k_dense_gemv")
    assert "layout differs between runs" in capsys.readouterr().out


def test_levels_record_rejects_a_misaligned_run(tmp_path, monkeypatch):
    ns = "void aspamg::(anonymous namespace)::"
    sell, dense = ns + "k_sell_spmv<float, float, float, 4>(int)", ns + "k_dense_gemv<float>(int)"
    copy = ns + "k_copy(long, double const*, double*)"
    rows = [{"level": 0, "prec": 32, "op": "G", "per_cycle": 2, "ms": 0.05, "bytes": 2.0e6, "GBps": 40.0},
            {"level": 1, "prec": 32, "op": "dense", "per_cycle": 1, "ms": 0.01, "bytes": 1.0e5, "GBps": 10.0}]
    seq = [copy] + [sell] * 2 + [dense] * 3          # one launch short in the first row: misaligned by one
    con = sqlite3.connect(tmp_path / "x.db")
    con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, counter_value real)")
    for i, name in enumerate(seq):
        for c in ("FETCH_SIZE", "WRITE_SIZE", "TCC_HIT_sum", "TCC_MISS_sum"):
            con.execute("insert into pmc_events values (?, ?, ?, ?)", (i + 1, name, c, 1.0))
    con.commit()
    con.close()
    with open(tmp_path / "trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i, name in enumerate(seq):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": 0, "End_Timestamp": 1})
    (tmp_path / "b.out").write_text(json.dumps({"levels": [], "level_table": rows, "level_table_reps": 2}) + "\n")
    monkeypatch.setattr(pr, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    db = str(tmp_path / "x.db")
    try:
        pr.levels_traffic("t", 1000, str(tmp_path / "b.out"), str(tmp_path / "trace.csv"), db, db, db, "cmd")
    except SystemExit as e:
        assert "row 0" in str(e)
    else:
        raise AssertionError("a misaligned run was accepted")
