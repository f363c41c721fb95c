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
