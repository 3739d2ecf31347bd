"""bench.py command-line contract on the host (no GPU): several GPUs are
refused with a message and a nonzero exit status before any GPU work; the
profile summarisers turn a rocpd-style database and counter CSVs into the
summaries kept under profiles/."""
import csv
import json
import os
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_stats_summary_from_a_database(tmp_path):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table k (name text, total_calls int, total_duration real, average real, percentage real)")
    con.execute("create view top_kernels as select * from k order by total_duration desc")
    con.executemany("insert into k values (?, ?, ?, ?, ?)",
                    [("kernel_a", 10, 300.0, 30.0, 75.0), ("kernel_b", 5, 100.0, 20.0, 25.0)])
    con.commit()
    con.close()
    out = tmp_path / "s.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-stats", str(db), str(out),
                        "Title", "cmd", "note"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    txt = out.read_text()
    assert txt.startswith("# Title") and "    cmd" in txt
    rows = [l for l in txt.splitlines() if l.startswith("| 10 ") or l.startswith("| 5 ")]
    assert rows[0].startswith("| 10 | 30.00 | 0.300 | 75.00% | `kernel_a`")
    assert rows[1].startswith("| 5 | 20.00 | 0.100 | 25.00% | `kernel_b`")


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path):
    def write(path, rows):
        with open(path, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
            w.writeheader()
            for r in rows:
                w.writerow(r)
    fetch, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    brick = "void chns::k_brick_o4<3, 8, double, 0, false, true>(args)"
    comb = "void chns::k_combine<double, 1, 0>(args)"
    # the copy reads 131072 KiB by the counter: fetch factor 2; writes are exact
    write(fetch, [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": 131072.0},
                  {"Kernel_Name": brick, "Counter_Value": 100.0}, {"Kernel_Name": brick, "Counter_Value": 300.0},
                  {"Kernel_Name": comb, "Counter_Value": 10.0}])
    write(wr, [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": 262144.0},
               {"Kernel_Name": brick, "Counter_Value": 50.0}, {"Kernel_Name": brick, "Counter_Value": 50.0},
               {"Kernel_Name": comb, "Counter_Value": 5.0}])
    prefix = tmp_path / "pp_apply"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-pmc", str(fetch), str(wr),
                        str(prefix), "c1", "c2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    d = json.loads((tmp_path / "pp_apply_fp64_l7_pmc.json").read_text())
    assert d["fetch_factor"] == 2.0 and d["write_factor"] == 1.0
    assert d["brick_fetch_bytes"] == 200.0 * 2.0 * 1024
    assert d["brick_write_bytes"] == 50.0 * 1024
    assert d["combine_fetch_bytes"] == 10.0 * 2.0 * 1024 and d["combine_write_bytes"] == 5.0 * 1024
    assert d["bytes_per_launch"] == (400.0 + 50.0 + 20.0 + 5.0) * 1024
    assert (tmp_path / "pp_apply_fp32_l7_pmc.json").exists()
