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
    assert bench.measured_traffic("fp8", 200) is None  # counters exist for S=1000 only
    prof = os.path.join(bench.ROOT, "profiles", "attn_fp8_kernel_vggt_l_s1000_traffic.txt")
    src = os.path.join(bench.ROOT, "paper_2509_25191_amd", "csrc", "attention.hip")
    kv = _kv(prof)
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    got = bench.measured_traffic("fp8", 1000)
    if kv["attention_hip_sha256"] == digest:
        assert got == float(kv["hbm_bytes_per_launch"]) and got > 0
        assert abs(got - float(kv["fetch_bytes_per_launch"]) - float(kv["write_bytes_per_launch"])) <= 1e-6 * got
    else:
        assert got is None
    # the same summary next to a different attention source is ignored
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2509_25191_amd" / "csrc").mkdir(parents=True)
    shutil.copy(prof, tmp_path / "profiles")
    (tmp_path / "paper_2509_25191_amd" / "csrc" / "attention.hip").write_bytes(open(src, "rb").read() + b"\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fp8", 1000) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
