"""Host logic of bench.py, on the CPU: the algorithmic byte counts, the
timing summary, the kernel names it reports for the autotuner's variants (as
the step source dispatches them), the HBM counter and kernel-trace summaries
on synthetic rocprofv3 files, and the one-GPU guard."""
import csv
import json
import os
import re
import subprocess
import sys

import pytest

import bench


def test_algorithmic_bytes_per_node_update():
    # FP32: 4 (8K weights + K indices + 9 read + 9 written) + 32 B of owners
    assert bench.bytes_per_update(30, "f32", True) == 1184
    assert bench.bytes_per_update(12, "f32", False) == 504
    assert bench.bytes_per_update(20, "f32", False) == 792
    # FP64: 8 8K + 4K + 8 18 + 32
    assert bench.bytes_per_update(30, "f64", True) == 2216
    # adjoint: 8K (4 B + 10-bit position) + 8 row pointers + 3 x 36 B
    assert bench.adjoint_bytes_per_update(30) == pytest.approx(1420.0)


def test_timing_summary_is_median_min_max_per_step():
    s = bench.timing_summary([4.0, 2.0, 3.0, 5.0, 1.0], 10)
    assert s == {"replays": 5, "steps_per_replay": 10, "ms_per_step_median": 0.3,
                 "ms_per_step_min": 0.1, "ms_per_step_max": 0.5}


def test_kernel_names_follow_the_step_dispatch():
    """Each variant's name is the k_step32 / k_step32s instance that
    launch32_tuned starts for the headline configuration (MODE 0, no force,
    no walls, no recording)."""
    src = open(os.path.join(bench.ROOT, "paper_2306_01525_amd", "csrc", "step.hip")).read()
    body = src[src.index("void launch32_tuned("):]
    body = body[:body.index("\n}\n")]
    cases = dict(re.findall(r"case (\d+): (launch32s?<[^>]*>)", body))
    default = re.search(r"default: (launch32s?<[^>]*>)", body).group(1)
    for v in range(10):
        call = cases.get(str(v), default)
        args = [a.strip() for a in call[call.index("<") + 1:-1].split(",")][4:]
        if call.startswith("launch32s<"):
            nt, unroll = args[0], args[1] if len(args) > 1 else "1"
            want = "k_step32s<0, false, 0, false, %s, %s>" % (nt, unroll)
        else:
            want = "k_step32<0, false, 0, false, %s, %s>" % (args[0], args[1])
        assert bench.step_kernel_name(v) == want, (v, call)


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_scales_by_the_copy_kernel(tmp_path, monkeypatch):
    """FETCH_SIZE reads half the bytes of the copy kernel here, WRITE_SIZE all
    of them: the step's counters are scaled by those factors."""
    step = "void mlbm::(anonymous namespace)::k_step32s<0, false, 0, false, true, 2>(x)"
    copy = "void at::native::vectorized_elementwise_kernel<4, MulFunctor<float>>(y)"
    kib = bench.COPY_BYTES / 1024.0
    fetch, write = [], []
    for d in range(3):   # three dispatches of each, several rows per dispatch
        for part in (0.5, 0.5):
            fetch.append(dict(Dispatch_Id=str(10 + d), Kernel_Name=step,
                              Counter_Name="FETCH_SIZE", Counter_Value=str(1000.0 * part)))
            write.append(dict(Dispatch_Id=str(10 + d), Kernel_Name=step,
                              Counter_Name="WRITE_SIZE", Counter_Value=str(40.0 * part)))
        fetch.append(dict(Dispatch_Id=str(20 + d), Kernel_Name=copy,
                          Counter_Name="FETCH_SIZE", Counter_Value=str(kib / 2)))
        write.append(dict(Dispatch_Id=str(20 + d), Kernel_Name=copy,
                          Counter_Name="WRITE_SIZE", Counter_Value=str(kib)))
    _counter_csv(str(tmp_path / "fetch"), fetch)
    _counter_csv(str(tmp_path / "write"), write)
    out = tmp_path / "pmc.json"
    monkeypatch.setattr(bench, "PROFILE_PMC", str(out))
    bench.summarize_pmc(str(tmp_path / "fetch"), str(tmp_path / "write"), "cmd")
    d = json.loads(out.read_text())
    assert d["kernel"] == step and d["dispatches"] == 3
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    assert d["bytes_per_launch"] == pytest.approx(1000.0 * 1024 * 2 + 40.0 * 1024)
    assert d["kernel_hash"] == bench.step_kernel_hash()
    # the bench uses these bytes only while the hash matches the step source
    assert bench.load_traffic(1, 1) == pytest.approx(d["bytes_per_launch"])
    d["kernel_hash"] = "0" * 16
    out.write_text(json.dumps(d))
    assert bench.load_traffic(1, 1) is None


def test_trace_summary_keeps_every_step_kernel(tmp_path):
    """The trace summary lists the 40 longest kernels and then every further
    step-kernel instance (the autotuner's losing variants), nothing else."""
    rows = [dict(Name="k_other_%d(x)" % i, Calls="1", AverageNs=str(1e6 - i),
                 TotalDurationNs=str(1e6 - i), Percentage="1.0") for i in range(45)]
    rows += [dict(Name="void k_step32s<0, false, 0, false, true, 2>(x)", Calls="21",
                  AverageNs="46000", TotalDurationNs="966000", Percentage="0.03"),
             dict(Name="void k_adj_step<float>(x)", Calls="3", AverageNs="66000",
                  TotalDurationNs="198000", Percentage="0.01")]
    os.makedirs(tmp_path / "trace")
    with open(tmp_path / "trace" / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    out = tmp_path / "trace.txt"
    bench.summarize_trace(str(tmp_path / "trace"), "cmd", str(out))
    text = out.read_text()
    assert "k_other_39(" in text and "k_other_40(" not in text
    assert "k_step32s<0, false, 0, false, true, 2>" in text and "k_adj_step<float>" in text
    assert re.search(r"^21\s+46\.00\s", text, re.M)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
