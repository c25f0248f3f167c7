"""CPU tests of the rocprofv3 summariser behind profiles/ (profile_sweep.py).

The traffic figure scales the sweep kernel's FETCH_SIZE / WRITE_SIZE by what
the same counters read for the 512 MiB calibration copy.  Only that copy (the
first dispatch of the profiled process) may calibrate: the step itself clones
states with copy kernels of the same size, and summing those in would halve
the reported traffic.
"""
import json
import os
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table pmc_events(name, counter_name, counter_value, dispatch_id)")
    con.executemany("insert into pmc_events values(?,?,?,?)", [(n, counter, v, d) for n, v, d in rows])
    con.commit()
    con.close()


def test_traffic_calibrates_on_first_dispatch_only(tmp_path):
    copy_kib = 512 * 1024
    # FETCH_SIZE reads half the copy's bytes, WRITE_SIZE all of them; the
    # step's own 512 MiB clone (k_copy) and small runtime copies follow.
    _db(tmp_path / "fetch.db", "FETCH_SIZE", [
        ("__amd_rocclr_copyBuffer", copy_kib / 2, 1),
        ("void k_sweep_reg_real_exact<float, float, 4, true, 2>(...)", 1000.0, 5),
        ("void k_sweep_reg_real_exact<float, float, 4, true, 2>(...)", 3000.0, 6),
        ("void k_copy<float>(...)", copy_kib / 2, 7),
        ("__amd_rocclr_copyBuffer", 4.0, 8),
        ("void k_sweep_reg_states<float, float, 4, true, 2>(...)", 9000.0, 9),
    ])
    _db(tmp_path / "write.db", "WRITE_SIZE", [
        ("__amd_rocclr_copyBuffer", copy_kib, 1),
        ("void k_sweep_reg_real_exact<float, float, 4, true, 2>(...)", 2000.0, 5),
        ("void k_sweep_reg_real_exact<float, float, 4, true, 2>(...)", 2000.0, 6),
        ("void k_copy<float>(...)", copy_kib, 7),
    ])
    out = tmp_path / "traffic.json"
    subprocess.check_call([sys.executable, os.path.join(ROOT, "profile_sweep.py"), "summarize", "--kind", "traffic",
                           "--out", str(out), str(tmp_path / "fetch.db"), str(tmp_path / "write.db")])
    t = json.loads(out.read_text())
    assert t["launches"] == 2
    assert t["copy_scale_fetch"] == 2.0 and t["copy_scale_write"] == 1.0
    assert t["fetch_bytes_per_launch"] == 4000.0 * 1024 * 2.0 / 2
    assert t["write_bytes_per_launch"] == 4000.0 * 1024 / 2
    assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
