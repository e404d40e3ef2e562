"""Host-side pieces of the measurement (no GPU): bench.py refuses more than one GPU before touching
one, its step plan keeps the run inside the wall budget, and the counter record is built from rocprofv3's per-dispatch CSV rows by the copy-kernel
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
    import bench as tp
    mul = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
          "at::native::binary_internal::MulFunctor<float> > >(int)"
    fill = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float> >(int)"
    search = "void ebb::k_search<3, false>(ebb::SearchArgs)"
    # the copy reads 1 GiB but FETCH_SIZE shows half of it; WRITE_SIZE shows all of it
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", [(fill, 10.0), (mul, 524288.0), (search, 1000.0)])
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", [(fill, 1048576.0), (mul, 1048576.0), (search, 300.0)])
    out = str(tmp_path / "rec.json")
    rec = tp.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), out, 9, "cmd")
    assert rec == json.load(open(out))
    assert rec["source_sha256"] == tp.source_sha256()
    assert rec["copy_kernel"]["fetch_scale"] == 2.0 and rec["copy_kernel"]["write_scale"] == 1.0
    e = rec["launches"]["ebb::k_search<3, false>@k=9"]
    assert (e["fetch_KiB"], e["write_KiB"]) == (1000.0, 300.0)
    assert e["hbm_bytes"] == 1000 * 1024 * 2 + 300 * 1024


def test_step_plan_keeps_the_wall_budget():
    sys.path.insert(0, ROOT)
    import bench
    # the first warmup and the first timed step always run
    assert bench.plan_warmups(5, 0, 0.0, -10.0, 20)
    assert bench.plan_timed(0, 20, 85.0, -10.0)
    # a second warmup only while all requested timed steps still fit after it
    assert not bench.plan_warmups(5, 1, 85.0, 200.0, 20)
    assert bench.plan_warmups(5, 1, 10.0, 250.0, 20)
    assert not bench.plan_warmups(1, 1, 1.0, 1e9, 20)
    # a timed step starts only while it is expected to end before the deadline
    assert bench.plan_timed(1, 20, 85.0, 86.0)
    assert not bench.plan_timed(1, 20, 85.0, 84.0)
    assert not bench.plan_timed(20, 20, 1.0, 1e9)
    # simulated driver command (--steps 20 --warmup 5) with 85 s steps after 90 s of start-up:
    # the measurement ends by the 300 s deadline plus at most one step
    t, warm, timed = 90.0, 0, 0
    while bench.plan_warmups(5, warm, 85.0 if warm else 0.0, 300.0 - t, 20):
        t += 85.0
        warm += 1
    while bench.plan_timed(timed, 20, 85.0, 300.0 - t):
        t += 85.0
        timed += 1
    assert (warm, timed) == (1, 1) and t <= 300.0 + 85.0


def test_kernel_hash_ignores_comments_but_not_code():
    sys.path.insert(0, ROOT)
    import bench as tp
    base = {"search.hip": "int f(int a) {\n  return a + 1; // one\n}\n", "build.h": "/* b */ int g;\n",
            "arena.h": "", "device_util.h": "", "common.h": ""}
    h0 = tp.source_sha256(base.get)
    recommented = dict(base, **{"search.hip": "// header\nint f(int a) {   return a + 1; /* one */ }\n"})
    assert tp.source_sha256(recommented.get) == h0
    changed = dict(base, **{"search.hip": "int f(int a) {\n  return a + 2; // one\n}\n"})
    assert tp.source_sha256(changed.get) != h0
