"""Host logic of bench.py (no GPU): the one-GPU refusal, the traffic records tied to the
kernel source they were measured on, and the roofline entry's arithmetic."""
import hashlib
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def _tree(tmp_path, source, records):
    csrc = tmp_path / "paper_2212_01309_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "kernels.hip").write_bytes(source)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hbm_traffic.md").write_text("# traffic\n\n```\n" + "\n".join(records) + "\n```\n")


def test_traffic_record_is_used_only_for_the_source_it_was_measured_on(tmp_path, monkeypatch):
    source = b"// kernels\n"
    sha = hashlib.sha256(source).hexdigest()[:16]
    _tree(tmp_path, source, [
        f"traffic: workload=medium kernel=k_row_fused_obj bytes_per_launch=28000000 kernels_sha={sha}",
        "traffic: workload=large kernel=k_row_fused_obj bytes_per_launch=127000000 kernels_sha=0123456789abcdef",
    ])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("medium", "k_row_fused_obj") == 28000000.0
    assert bench.measured_traffic("medium", "k_row_update<true>") is None   # no record for this kernel
    assert bench.measured_traffic("large", "k_row_fused_obj") is None       # measured on another source
    (tmp_path / "paper_2212_01309_amd" / "csrc" / "kernels.hip").write_bytes(source + b"// changed\n")
    assert bench.measured_traffic("medium", "k_row_fused_obj") is None      # the kernel changed since


def test_traffic_is_none_without_a_record(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2212_01309_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "kernels.hip").write_bytes(b"x")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("medium", "k_row_fused_obj") is None


@pytest.mark.parametrize("order,fused,kernel,per", [("object", True, "k_row_fused_obj", 8.0),
                                                     ("spectrum", True, "k_row_update<true>", 24.0),
                                                     ("spectrum", False, "k_row_update<false>", 16.0)])
def test_roofline_entry_from_algorithmic_bytes(order, fused, kernel, per, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))   # no traffic record here
    (tmp_path / "paper_2212_01309_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2212_01309_amd" / "csrc" / "kernels.hip").write_bytes(b"x")
    wl = types.SimpleNamespace(name="medium", batch=128, n=64, dose=1e4, sy=128, sx=128)
    n_freq, k, us = 12647, 256, 12.5
    r = bench.roofline(wl, n_freq, k, "accumulate", us, factored=True, fused=fused, order=order)
    assert r["kernel"] == kernel and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["algorithmic_bytes"] == per * n_freq * k
    assert r["achieved"] == pytest.approx(per * n_freq * k / (us * 1e-6) / 1e9)
    assert r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None
