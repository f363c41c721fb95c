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
