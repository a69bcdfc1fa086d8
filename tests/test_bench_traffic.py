"""bench.py --traffic-from: HBM bytes of the timed post-smoothing step from two
rocprofv3 counter databases, scaled by a reference copy of known size.  The
step's kernels share names with other levels' launches, so the step must be taken
from the probe's last dispatches, not from whichever kernel name was seen last."""
import json
import os
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY = 1 << 28  # bytes read and written by one reference copy


def make_db(path, counter, copy_kib, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    d = 0
    for _ in range(3):
        d += 1
        con.execute("insert into counters_collection values (?, ?, ?, ?)",
                    (d, "__amd_rocclr_copyBuffer", counter, copy_kib))
    for name, val in rows:
        d += 1
        con.execute("insert into counters_collection values (?, ?, ?, ?)", (d, name, counter, val))
    con.commit()
    con.close()


def test_step_is_taken_from_the_last_dispatches(tmp_path):
    start0 = "void amg::k_smooth_start<double, 2>(int, ...) [finest]"
    start1 = "void amg::k_smooth_start<double, 2>(int, ...) [level 1]"
    fin0 = "void amg::k_sell_smooth_finish<double, true>(int, ...)"
    fin1 = "void amg::k_smooth_finish<double, 4, false>(Rows, ...)"
    solve = [(start0, 1.0), (fin0, 2.0), (start1, 7.0), (fin1, 9.0)] * 3  # the solve's launches
    probe_f = [(start0, 100.0), (fin0, 200.0)] * 5  # the timed steps come last
    probe_w = [(start0, 40.0), (fin0, 60.0)] * 5
    fdb, wdb = str(tmp_path / "fetch.db"), str(tmp_path / "write.db")
    # the copy reads 256 MiB but FETCH_SIZE shows half of it (scale 2); WRITE_SIZE all of it
    make_db(fdb, "FETCH_SIZE", COPY / 1024 / 2, solve + probe_f)
    make_db(wdb, "WRITE_SIZE", COPY / 1024, solve + probe_w)
    out = str(tmp_path / "traffic.json")
    subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--traffic-from", fdb, wdb, "--traffic-file", out],
                   check=True, capture_output=True, cwd=ROOT)
    with open(out) as f:
        tr = json.load(f)
    assert tr["fetch_kib_per_dispatch"] == 300.0 and tr["write_kib_per_dispatch"] == 100.0
    assert tr["fetch_scale"] == 2.0 and tr["write_scale"] == 1.0
    assert tr["bytes_per_launch"] == 300.0 * 1024 * 2 + 100.0 * 1024
