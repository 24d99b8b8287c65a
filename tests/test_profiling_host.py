"""Host logic of the rocprofv3 summaries (no GPU): counter scaling by the copy
calibration, per-kernel selection and the counted-vs-algorithmic table."""
import csv
import os

from paper_1701_04685_amd import profiling


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def _runs(tmp_path):
    copy_bytes = 1 << 29
    kib = copy_bytes / 1024.0
    # the copy kernel: FETCH_SIZE reads half its bytes, WRITE_SIZE all of them;
    # its first dispatch (a warm-up) is ignored
    cf = os.path.join(tmp_path, "cf.csv")
    cw = os.path.join(tmp_path, "cw.csv")
    _counter_csv(cf, [("elementwise_copy", "FETCH_SIZE", 1.0)] +
                 [("elementwise_copy", "FETCH_SIZE", kib / 2)] * 3)
    _counter_csv(cw, [("elementwise_copy", "WRITE_SIZE", 1.0)] + [("elementwise_copy", "WRITE_SIZE", kib)] * 3)
    # two kernels of one run: A reads 3 GiB-ish worth (counter reads half), writes 1;
    # B's dispatches differ, the median is taken
    f = os.path.join(tmp_path, "f.csv")
    w = os.path.join(tmp_path, "w.csv")
    _counter_csv(f, [("k_a<double, 1>", "FETCH_SIZE", 1000.0)] * 3 +
                 [("k_b<double, 2>", "FETCH_SIZE", v) for v in (400.0, 500.0, 9000.0)])
    _counter_csv(w, [("k_a<double, 1>", "WRITE_SIZE", 700.0)] * 3 +
                 [("k_b<double, 2>", "WRITE_SIZE", v) for v in (100.0, 200.0, 300.0)])
    return f, w, cf, cw, copy_bytes


def test_copy_calibration_scales(tmp_path):
    f, w, cf, cw, nb = _runs(str(tmp_path))
    d = profiling.traffic_summary("k_a<double, 1>", f, w, cf, cw, nb, "cmd")
    assert abs(d["fetch_scale"] - 2.0) < 1e-12 and abs(d["write_scale"] - 1.0) < 1e-12
    assert d["fetch_bytes"] == 2.0 * 1000.0 * 1024.0
    assert d["write_bytes"] == 700.0 * 1024.0
    assert d["dispatches"] == [3, 3]


def test_pass_table_ratios(tmp_path):
    f, w, cf, cw, nb = _runs(str(tmp_path))
    specs = [("k_a<double, 1>", "pass a", 2.0 * 1000.0 * 1024.0, 700.0 * 1024.0),
             ("k_b<double, 2>", "pass b", 1000.0 * 1024.0, 400.0 * 1024.0),
             ("k_missing", "absent", 1.0, 1.0)]
    text, d = profiling.pass_traffic_table(specs, f, w, cf, cw, nb, "title", "cmd")
    rows = {r["pass"]: r for r in d["rows"]}
    assert set(rows) == {"pass a", "pass b"}  # a kernel with no dispatches is left out
    assert rows["pass a"]["read_bytes"] == rows["pass a"]["alg_read_bytes"]
    assert rows["pass a"]["write_bytes"] == rows["pass a"]["alg_write_bytes"]
    # medians: FETCH 500 KiB x 2, WRITE 200 KiB x 1
    assert rows["pass b"]["read_bytes"] == 2.0 * 500.0 * 1024.0
    assert rows["pass b"]["write_bytes"] == 200.0 * 1024.0
    assert "pass b" in text and "ratio" in text
    assert d["fingerprint"] == profiling.source_fingerprint()
