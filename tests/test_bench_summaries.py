"""The benchmark's counter summaries without a GPU: a synthetic rocprofv3
result database (the counters_collection view's columns) is grouped into
transport passes (a pass opens at transport_kernel and holds the hand-off
kernels after it; the warm-up passes are skipped), and the atomic
calibration divides each counter by grid size x rounds."""
import json
import os
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _db(path, dispatches):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
                "grid_size integer, duration integer, counter_name text, value real)")
    for d, (k, g, t, cs) in enumerate(dispatches):
        for c, v in cs.items():
            con.execute("insert into counters_collection values (?,?,?,?,?,?)",
                        (d + 1, k, g, t, c, v))
    con.commit()
    con.close()


def _k(name):
    return f"void smc::(anonymous namespace)::{name}(smc::LaunchArgs)"


def _iteration(scale):
    return [(_k("reset_kernel<false>"), 256, 10, {"C": 1000.0}),
            (_k("transport_kernel<false>"), 1 << 20, 1000, {"C": 1.0 * scale}),
            (_k("order_count_kernel<false>"), 256, 10, {"C": 2.0 * scale}),
            ("void smc::order_scan_kernel(smc::LaunchArgs)", 64, 10, {"C": 3.0 * scale}),
            (_k("order_place_kernel<false>"), 256, 10, {"C": 4.0 * scale}),
            (_k("solo_kernel<false>"), 4096, 500, {"C": 5.0 * scale}),
            (_k("finalise_kernel<false>"), 256, 10, {"C": 1000.0})]


def test_passes_are_grouped_and_warmup_skipped(tmp_path):
    db = str(tmp_path / "r.db")
    _db(db, _iteration(100.0) + _iteration(1.0) + _iteration(2.0) + _iteration(7.0))
    passes = bench._transport_passes(bench._pmc_dispatches(db), warmup=1, steps=2)
    assert [len(p) for p in passes] == [5, 5]
    assert [sum(d[3]["C"] for d in p) for p in passes] == [15.0, 30.0]
    assert passes[0][0][0] == "transport_kernel<false>"
    assert passes[0][2][0] == "order_scan_kernel"


def test_counter_summary_and_atomic_calibration(tmp_path):
    db = str(tmp_path / "b.db")
    _db(db, _iteration(100.0) + _iteration(1.0) + _iteration(3.0))
    adb = str(tmp_path / "a.db")
    _db(adb, [("void smc::(anonymous namespace)::atomic_rate_kernel<false>(double*, unsigned "
               "long, unsigned int)", 1024, 2000, {"TCC_ATOMIC_sum": 1024 * 256 / 8.0}),
              ("void smc::(anonymous namespace)::atomic_rate_kernel<true>(double*, unsigned "
               "long, unsigned int)", 1024, 4000, {"TCC_ATOMIC_sum": 1024 * 256.0})])
    line = str(tmp_path / "line.json")
    with open(line, "w") as f:
        f.write("# log\n" + json.dumps({"segments_per_s": 1000.0, "ms_per_step": 10.0,
                                        "line_passes_per_s": 0.0,
                                        "config": {"packets_per_iteration": 1}}) + "\n")
    out = str(tmp_path / "s.json")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--counter-summary", out,
                        line, adb, db, "--warmup", "1", "--steps", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    s = json.load(open(out))
    assert s["per_pass"]["C"] == (15.0 + 45.0) / 2
    assert s["per_kernel"]["solo_kernel"]["C"] == (5.0 + 15.0) / 2
    assert s["segments_per_pass"] == 10.0
    assert s["per_segment"]["C"] == 3.0
    cal = s["atomic_calibration"]
    assert cal["window"]["TCC_ATOMIC_sum_per_add"] == 1.0 / 8.0
    assert cal["scattered"]["TCC_ATOMIC_sum_per_add"] == 1.0
    assert cal["window"]["adds_per_dispatch"] == 1024 * 256
