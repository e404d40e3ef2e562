"""Host-side pieces of the measurement (no GPU): bench.py refuses more than one GPU before touching
one, and the counter record is built from rocprofv3's per-dispatch CSV rows by the copy-kernel
calibration (bytes = counter KiB x 1024 x the copy's true bytes / its counter bytes)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, v) in enumerate(rows):
            # a counter may come in several rows per dispatch (one per instance); they add up
            w.writerow([i + 1, name, counter, v / 2])
            w.writerow([i + 1, name, counter, v / 2])


def test_traffic_record_from_counter_rows(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2311_13798_amd import traffic_probe as tp
    mul = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
          "at::native::binary_internal::MulFunctor<float> > >(int)"
    fill = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float> >(int)"
    search = "void ebb::k_search<3, false>(ebb::SearchArgs)"
    # the copy reads 1 GiB but FETCH_SIZE shows half of it; WRITE_SIZE shows all of it
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", [(fill, 10.0), (mul, 524288.0), (search, 1000.0)])
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", [(fill, 1048576.0), (mul, 1048576.0), (search, 300.0)])
    out = str(tmp_path / "rec.json")
    rec = tp.write_record(str(tmp_path / "f"), str(tmp_path / "w"), out, 9, "cmd")
    assert rec == json.load(open(out))
    assert rec["source_sha256"] == tp.source_sha256()
    assert rec["copy_kernel"]["fetch_scale"] == 2.0 and rec["copy_kernel"]["write_scale"] == 1.0
    e = rec["launches"]["ebb::k_search<3, false>@k=9"]
    assert (e["fetch_KiB"], e["write_KiB"]) == (1000.0, 300.0)
    assert e["hbm_bytes"] == 1000 * 1024 * 2 + 300 * 1024
