"""The benchmark's host-side contract, on the CPU: the one-GPU refusal and
the peeling byte model that its roofline figure divides by time, and when a
measured-traffic summary applies."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    for args in (["--gpus", "2"], ["--gpus", "8", "--workload", "peel_rmat24"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 2, (args, r.returncode, r.stderr)
        assert "one GPU" in r.stderr


def test_peel_byte_model():
    # |S_0..S_3| = 10, 4, 1, 0: 15 alive vertices over the rounds (10 in the
    # first step, which reads no list), 5 survivors, every vertex removed once
    sizes = [10, 4, 1, 0]
    dg = bench.peel_bytes("DG", 10, sizes, {"incidences": 0})
    assert dg == {"decide": 32 * 15 - 4 * 10 + 4 * 10, "update": 28 * 5, "reduce": 12 * 5}
    fd = bench.peel_bytes("FD", 10, sizes, {"incidences": 0})
    assert fd["update"] == 36 * 5 and fd["reduce"] == 20 * 5 and fd["decide"] == dg["decide"]
    assert bench.peel_bytes("DW", 10, sizes, {"incidences": 0}) == dg


def test_traffic_profile_applies_to_its_kernel_and_source(tmp_path, monkeypatch):
    # a measured-traffic summary counts only while the kernels' source has
    # the hash recorded with it, and only for the kernel it was taken on
    # (the pull class runs as k_pull<T> or, finalize fused, k_pull_fin<T>)
    import hashlib
    src = tmp_path / "paper_2504_09311_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "kernels.hip").write_text("// kernels\n")
    digest = hashlib.sha256((src / "kernels.hip").read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_pull_work_traffic.md").write_text(
        "# HBM traffic\n\n`traffic_bytes_per_launch: 1234`\n\n`source: kernels.hip`\n\n"
        f"`source_sha256: {digest}`\n\n`class: pull`\n\n`kernel_name: k_pull_fin<16>`\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("pull", "work", "k_pull_fin<16>") == 1234
    assert bench.measured_traffic("pull", "work") == 1234
    assert bench.measured_traffic("pull", "work", "k_pull<16>") is None
    assert bench.measured_traffic("pull", "other", "k_pull_fin<16>") is None
    (src / "kernels.hip").write_text("// kernels, changed\n")
    assert bench.measured_traffic("pull", "work", "k_pull_fin<16>") is None
