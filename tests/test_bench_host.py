"""Host logic of bench.py that needs no GPU: the lookup of the dominant
kernel's measured HBM traffic (valid only for the attention source it was
taken on) and the one-GPU guard."""
import hashlib
import os
import shutil
import subprocess
import sys

import bench


def _kv(path):
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_lookup_only_for_the_profiled_source(tmp_path, monkeypatch):
    assert bench.measured_traffic("bf16", 200) is None  # counters exist for S=1000 only
    assert bench.measured_traffic("fp8pv", 1000) is None  # and not for the FP8 P V kernel
    src = os.path.join(bench.ROOT, "paper_2509_25191_amd", "csrc", "attention.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for prec in ("bf16", "fp8"):
        path = os.path.join(bench.ROOT, "profiles", f"attn_{prec}_kernel_vggt_l_s1000_traffic.txt")
        if not os.path.exists(path):
            assert bench.measured_traffic(prec, 1000) is None
            continue
        kv = _kv(path)
        got = bench.measured_traffic(prec, 1000)
        if kv["attention_hip_sha256"] == digest:
            assert got == float(kv["hbm_bytes_per_launch"]) and got > 0
            assert abs(got - float(kv["fetch_bytes_per_launch"]) - float(kv["write_bytes_per_launch"])) <= 1e-6 * got
        else:
            assert got is None
    prof = os.path.join(bench.ROOT, "profiles", "attn_bf16_kernel_vggt_l_s1000_traffic.txt")
    # the same summary next to a different attention source is ignored
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2509_25191_amd" / "csrc").mkdir(parents=True)
    shutil.copy(prof, tmp_path / "profiles")
    (tmp_path / "paper_2509_25191_amd" / "csrc" / "attention.hip").write_bytes(open(src, "rb").read() + b"\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("bf16", 1000) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_plan_steps_fits_the_budget():
    # S=1000-sized steps (~190 s) against a few hundred seconds: one timed step, no warm-up
    assert bench.plan_steps(20, 5, 190.0, 350.0) == (1, 0)
    # a budget below one step still runs the one timed step
    assert bench.plan_steps(20, 5, 190.0, 10.0) == (1, 0)
    # small steps: everything requested fits
    assert bench.plan_steps(20, 5, 0.3, 350.0) == (20, 5)
    # timed steps are kept before warm-up steps
    assert bench.plan_steps(20, 5, 10.0, 220.0) == (20, 2)
    assert bench.plan_steps(20, 5, 10.0, 150.0) == (15, 0)
    # never more than requested
    assert bench.plan_steps(2, 1, 1.0, 1e6) == (2, 1)
    assert bench.plan_steps(3, 0, 0.0, 0.0) == (3, 0)


def test_forward_flops_matches_the_per_config_arithmetic():
    m = bench.synth.ModelConfig()
    # global attention dominates: 4 N^2 C per layer; at S=1000 about 187.4 PFLOP per forward
    f = bench.forward_flops(1000, 1374, m)
    assert abs(f / 1.874e17 - 1) < 0.01
    assert abs(bench.forward_flops(32, 1374, m) / 2.49e14 - 1) < 0.01


class _Ev:
    """Stands in for a device event that completes after n queries."""

    def __init__(self, n):
        self.n = n
        self.synced = False

    def query(self):
        self.n -= 1
        return self.n <= 0

    def synchronize(self):
        self.synced = True


def test_wait_ends_on_the_event_not_on_counted_launches(monkeypatch):
    # the wait ends when the event completes, whatever the timing record
    # holds (records may have been dropped or never taken)
    polls = []
    monkeypatch.setattr(bench.time, "sleep", lambda s: None)
    monkeypatch.setattr(bench.vg, "timing_poll", lambda h: polls.append(1) or (0, 0, 0))
    ev = _Ev(5)
    bench.wait_logged(ev, None, "t", 24, 0.0, every_s=0.0)
    assert ev.synced and ev.n <= 0 and len(polls) == 4
