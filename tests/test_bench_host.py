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
    for name, src in (("p2p_C2_counters.txt", "p2p.hip"), ("m2l_bf16x3_C2_counters.txt", "m2l.hip"),
                      ("m2l_fp16x2_C2_counters.txt", "m2l.hip")):
        text = open(os.path.join(prof, name)).read()
        assert "source_sha256:" in text and "copy_fetch_factor:" in text
        assert os.path.exists(os.path.join(bench.ROOT, "paper_1106_2176_amd", "csrc", src))


def _fake_result(dom="M2L"):
    from paper_1106_2176_amd import inputs
    info = {"n": 1_000_000, "n_leaves": 32768, "levels": 5, "p2p_pairs": 773_617_576,
            "m2l_pairs": 6_039_504}
    st = {"gather": 0.0, "P2M": 0.05, "M2M": 0.04, "pack": 0.02, "M2L": 0.5, "L2L": 0.04,
          "L2P": 0.05, "P2P": 0.45, "combine": 0.04}
    return inputs.WORKLOADS["C2"], {"info": info, "dom": dom, "dom_ms": st[dom], "stages_ms": st,
                                    "build_ms": 0.1}


def test_rooflines_use_the_algorithmic_work_and_both_fp32_rates():
    wl, res = _fake_result()
    roof, other = bench.rooflines(wl, res, "mixed", "fp16x2", False)
    assert roof["kernel"].startswith("k_m2l_bf16<2,10,8,fp16>") and other["kernel"] == "k_p2p<float>"
    # 2 p^4 FLOP per M2L pair over the stage time, against the 16-bit MFMA peak
    assert roof["achieved"] == pytest.approx(2e4 * 6_039_504 / 0.5e-3 / 1e12)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 2500.0)
    assert roof["mfma_products_per_term"] == 3
    # 19 FLOP per P2P pair, against 157.3 and the unpacked 78.6 TFLOP/s
    assert other["achieved"] == pytest.approx(19 * 773_617_576 / 0.45e-3 / 1e12)
    assert other["frac_unpacked"] == pytest.approx(2 * other["frac"] * 157.3 / 157.2, rel=1e-3)
    roof64, _ = bench.rooflines(wl, res, "fp64", None, False)
    assert roof64["kernel"] == "k_m2l_f64<10>" and roof64["peak"] == 78.6


def test_tree_pass_bytes_per_particle():
    wl, res = _fake_result()
    tp = bench.tree_pass(wl, res, "mixed")
    # FP64 inputs, 16-byte records: 92 B build + 32 B P2M + 48 B L2P per
    # particle, plus the leaf coefficients written and read once (the combine
    # is part of the P2P kernel)
    assert tp["bytes"] == 1_000_000 * (92 + 32 + 48) + 2 * 32768 * 104 * 4
    assert tp["ms"] == pytest.approx(0.1 + 0.05 + 0.05)


def test_tree_pass_counters_read_from_the_committed_summary():
    tp = bench.tree_pass_counters()
    assert tp is not None, "the tree-pass summary no longer matches tree.hip / far.hip"
    for k in ("k_keys", "k_place", "k_fixup", "k_p2m", "k_l2p", "total"):
        assert tp[k]["us"] > 0 and tp[k]["measured_mb"] > 0 and tp[k]["algorithmic_mb"] > 0
    assert abs(sum(tp[k]["us"] for k in tp if k != "total") - tp["total"]["us"]) < 1.0
