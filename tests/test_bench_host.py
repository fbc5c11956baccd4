"""Host logic of bench.py, without a GPU: the one-GPU contract, the algorithmic
bytes of each launch kind, the source check of the traffic record and the CPU
baseline record."""
import glob
import importlib.util
import json
import os
import subprocess
import sys

from conftest import ROOT


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_site():
    b = load_bench()
    # couplings 24 B once, spins 16 B per replica, buffered draws 4 B per replica and sweep
    assert b.algorithmic_bytes_per_site("minstd", 1) == 40
    assert b.algorithmic_bytes_per_site("minstd", 2) == 56
    assert b.algorithmic_bytes_per_site("minstd", 2, 2) == 56  # two sweeps per launch move the same words
    assert b.algorithmic_bytes_per_site("philox", 2) == 56
    assert b.algorithmic_bytes_per_site("mt19937", 2) == 64
    assert b.algorithmic_bytes_per_site("mt19937", 2, 2) == 72
    assert b.algorithmic_bytes_per_site("parisi_rapuano", 1, 2) == 48


def test_traffic_record_needs_the_current_kernel_source_and_shape(monkeypatch):
    b = load_bench()
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_sweep_fused_c1_*.json")))
    assert paths, "the L=256 workload has committed counter records"
    with open(paths[0]) as f:
        rec = json.load(f)
    tile = rec["tile"]
    want = rec["hbm_bytes_per_launch"] if rec["kernel_source_sha"] == b.kernel_source_sha() else None
    assert b.load_traffic("c1", "fused2", tile) == want
    assert b.load_traffic("c1", "fused", tile) is None  # the record is of the two-sweep kernel
    assert b.load_traffic("c1", "fused2", tile[:4] + [tile[4] + 100] + tile[5:]) is None  # another band
    assert b.load_traffic("no-such-workload", "fused2", tile) is None
    monkeypatch.setattr(b, "kernel_source_sha", lambda: "0" * 16)
    assert b.load_traffic("c1", "fused2", tile) is None


def test_alu_roofline_figures():
    b = load_bench()
    assert b.VALU_PEAK_WAVE_INSTS == 614.4e9
    r = b.alu_roofline(614.4e6, 2.0)  # 614.4 M wave instructions in 2 ms: half the issue peak
    assert r["bound"] == "alu" and r["frac"] == 0.5 and r["peak"] == 614.4 and r["achieved"] == 307.2


def test_kernel_labels():
    b = load_bench()
    assert b.kernel_label("fused2", 2).startswith("sg::k_fused2")
    assert "odd sweep count" in b.kernel_label("fused2", 1)
    assert b.kernel_label("fused", 1).startswith("sg::k_fused ")
    assert b.kernel_label("twopass", 1).startswith("sg::k_twopass")


def test_cpu_baseline_record():
    b = load_bench()
    r = b.cpu_baseline("c0", 2, threads=3)
    assert r["kind"] == "oracle" and r["cores"] == 3 and r["unit"] == "ps/flip"
    assert r["value"] > 0 and "L=16" in r["sample"] and "bit-planes 0 and 63" in r["sample"]
    assert set(r["c0_L16_1000_sweeps"]) == {"threads_1", "threads_3"}
    assert r["cpu_model"] and r["nproc"] >= 1


def test_batch_bytes_count_two_sweep_rounds():
    b = load_bench()
    from paper_1411_0127_amd.serve import Job

    # 40 B per site and round; a round is two sweeps, an odd last sweep one round
    jobs = [Job(0, 32, 4, 1.0, 1, 2), Job(1, 64, 5, 1.0, 1, 2)]
    assert b.batch_bytes(jobs) == 40 * 32**3 * 2 + 40 * 64**3 * 3
