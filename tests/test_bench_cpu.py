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
    (tmp_path / "profiles" / "records.md").write_text("# records\n\n```\n" + "\n".join(records) + "\n```\n")


def test_profile_records_are_used_only_for_the_source_they_were_measured_on(tmp_path, monkeypatch):
    source = b"// kernels\n"
    sha = hashlib.sha256(source).hexdigest()[:16]
    _tree(tmp_path, source, [
        f"traffic: workload=medium kernel=k_row_fused_obj bytes_per_launch=28000000 kernels_sha={sha}",
        "traffic: workload=large kernel=k_row_fused_obj bytes_per_launch=127000000 kernels_sha=0123456789abcdef",
        f"kernel_trace: workload=large kernel=k_row_fused_obj avg_us=28.5 kernels_sha={sha}",
    ])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_record("traffic", "medium", "k_row_fused_obj")["bytes_per_launch"] == "28000000"
    assert bench.profile_record("traffic", "medium", "k_row_update<true>") is None   # no record for this kernel
    assert bench.profile_record("traffic", "large", "k_row_fused_obj") is None       # measured on another source
    assert bench.profile_record("kernel_trace", "large", "k_row_fused_obj")["avg_us"] == "28.5"
    (tmp_path / "paper_2212_01309_amd" / "csrc" / "kernels.hip").write_bytes(source + b"// changed\n")
    assert bench.profile_record("traffic", "medium", "k_row_fused_obj") is None      # the kernel changed since
    assert bench.profile_record("kernel_trace", "large", "k_row_fused_obj") is None


@pytest.mark.parametrize("order,kernel,per", [("object", "k_row_fused_obj", 8.0),
                                              ("spectrum", "k_row_update<true>", 24.0)])
def test_roofline_entry_from_algorithmic_bytes(order, kernel, per, tmp_path, monkeypatch):
    source = b"x"
    sha = hashlib.sha256(source).hexdigest()[:16]
    # spectrum-order runs are recorded under "<workload>_spectrum"
    label = "medium" if order == "object" else "medium_spectrum"
    _tree(tmp_path, source, [f"kernel_trace: workload={label} kernel={kernel} avg_us=10.0 kernels_sha={sha}"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    wl = types.SimpleNamespace(name="medium", batch=128, n=64, dose=1e4, sy=128, sx=128)
    n_freq, k, ev = 12647, 256, 12.5
    r = bench.roofline(wl, n_freq, k, order, False, "fp32", ev)
    assert r["kernel"] == kernel and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["algorithmic_bytes"] == per * n_freq * k
    # the kernel-trace average is the divisor; the HIP-event figure is reported beside it
    assert r["avg_us"] == 10.0 and r["hip_event_us"] == ev
    assert r["achieved"] == pytest.approx(per * n_freq * k / (10.0 * 1e-6) / 1e9)
    assert r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None
    if order == "object":  # the previous image's column pass riding in the launch adds its bytes
        r = bench.roofline(wl, n_freq, k, order, False, "fp32", ev, display_bytes=1e6)
        assert r["algorithmic_bytes"] == per * n_freq * k + 1e6 and "column pass" in r["algorithmic_bytes_rule"]
    # without a trace record for this source the live HIP-event mean is used, and said so
    (tmp_path / "paper_2212_01309_amd" / "csrc" / "kernels.hip").write_bytes(b"y")
    r = bench.roofline(wl, n_freq, k, order, False, "fp32", ev)
    assert r["avg_us"] == ev and "HIP events" in r["avg_us_source"]
