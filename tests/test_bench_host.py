"""Host logic of bench.py (no GPU): the HBM traffic of a roofline object is
read from a committed rocprofv3 counter summary only while the kernel source
it was taken on is unchanged, and is scaled by the copy-kernel factors."""
import hashlib
import os

import pytest

import bench


def _setup(tmp_path, src_text, recorded_sha, fetch="1000.0", write="500.0", ff="0.5", wf="1.0"):
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_1106_2176_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text(src_text)
    (tmp_path / "profiles" / "k_traffic.txt").write_text(
        "# a comment: with a colon\n"
        f"source_sha256: {recorded_sha}\n"
        f"fetch_kib_per_dispatch: {fetch}\n"
        f"write_kib_per_dispatch: {write}\n"
        f"copy_fetch_factor: {ff}\n"
        f"copy_write_factor: {wf}\n")


def test_traffic_scaled_by_copy_factors(tmp_path, monkeypatch):
    src = "kernel source\n"
    _setup(tmp_path, src, hashlib.sha256(src.encode()).hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # (1000 / 0.5 + 500 / 1.0) KiB
    assert bench.traffic_from_profile("k.hip", "k_traffic.txt") == pytest.approx(2500.0 * 1024)


def test_traffic_null_when_the_kernel_changed(tmp_path, monkeypatch):
    _setup(tmp_path, "kernel source, edited\n", hashlib.sha256(b"kernel source\n").hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("k.hip", "k_traffic.txt") is None


def test_traffic_null_when_missing_or_malformed(tmp_path, monkeypatch):
    src = "kernel source\n"
    _setup(tmp_path, src, hashlib.sha256(src.encode()).hexdigest(), ff="0")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("k.hip", "k_traffic.txt") is None
    assert bench.traffic_from_profile("k.hip", "absent.txt") is None
    assert bench.traffic_from_profile("absent.hip", "k_traffic.txt") is None


def test_committed_profiles_name_their_kernel_sources():
    """Each committed counter summary records the hash of a kernel source
    that exists (whether it still matches is checked at bench time)."""
    prof = os.path.join(bench.ROOT, "profiles")
    for name, src in (("p2p_C2_traffic.txt", "p2p.hip"), ("m2l_bf16_C2_traffic.txt", "m2l.hip")):
        text = open(os.path.join(prof, name)).read()
        assert "source_sha256:" in text and "copy_fetch_factor:" in text
        assert os.path.exists(os.path.join(bench.ROOT, "paper_1106_2176_amd", "csrc", src))
