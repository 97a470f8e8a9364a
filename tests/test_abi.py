"""The C-ABI library loads on a CPU-only host, exports every declared symbol
and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1106_2176_amd as fmm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fmm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = fmm.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(fmm.EXPORTED)


def test_status_strings_and_defaults():
    L = fmm.lib()
    assert L.fmm_status_string(0) == b"ok"
    assert b"invalid" in L.fmm_status_string(1)
    c = fmm.Config()
    L.fmm_config_default(ctypes.byref(c))
    assert c.abi_version == fmm.FMM_ABI_VERSION
    assert (c.p, c.leaf_max, c.max_level, c.precision, c.bf16_splits, c.m2l_fp16) == (8, 64, 10, 1, 3, 1)
    assert c.box_size == 1.0 and list(c.box_lo) == [0.0, 0.0, 0.0]
    # 6 int32 (24) + double[3] (24) + double (8) + 3 pointers (24) + int32[8] (32)
    assert ctypes.sizeof(fmm.Config) == 112


def _build(cfg, n=10, dtype=fmm.FMM_F64, pos=ctypes.c_void_p(16)):
    h = ctypes.c_void_p(None)
    return fmm.lib().fmm_build_tree(ctypes.byref(cfg) if cfg is not None else None, n, dtype, pos,
                                    None, ctypes.byref(h)), h


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("p", 0), ("p", 17), ("leaf_max", 0), ("max_level", -1),
    ("max_level", 11), ("precision", 7), ("bf16_splits", 4), ("box_size", 0.0),
    ("box_size", float("nan")),
])
def test_build_rejects_bad_config(field, value):
    cfg = fmm.make_config()
    setattr(cfg, field, value)
    rc, h = _build(cfg)
    assert rc == fmm.FMM_EINVAL
    assert not h.value
    assert fmm.lib().fmm_last_error_message()


@pytest.mark.parametrize("changes,status", [
    (dict(precision=1, m2l_fp16=0), fmm.FMM_EUNSUPPORTED),  # the adaptive mixed form is binary16 only
    (dict(m2l_rotation=1), fmm.FMM_EUNSUPPORTED),       # and use the dense M2L
    (dict(max_level=11), fmm.FMM_EINVAL),               # keys have 30 bits
])
def test_adaptive_config_checks(changes, status):
    cfg = fmm.make_config(precision="fp64", adaptive=True)
    assert cfg.adaptive == 1 and cfg.max_level == fmm.ADAPTIVE_MAX_LEVEL
    for k, v in changes.items():
        setattr(cfg, k, v)
    rc, h = _build(cfg)
    assert rc == status and not h.value


def test_profile_stages_past_the_last_stage_rejected():
    cfg = fmm.make_config(profile=True)
    cfg.profile_stages = 1 << 9
    rc, h = _build(cfg)
    assert rc == fmm.FMM_EINVAL and not h.value
    assert fmm.make_config(profile=True, profile_stages=["M2L", "P2P"]).profile_stages == (1 << 4) | (1 << 7)


def test_graph_and_profile_are_exclusive():
    cfg = fmm.make_config(graph=True, profile=True)
    rc, h = _build(cfg)
    assert rc == fmm.FMM_EINVAL and not h.value
    assert b"exclusive" in fmm.lib().fmm_last_error_message()


def test_build_rejects_bad_arguments():
    cfg = fmm.make_config()
    assert _build(None)[0] == fmm.FMM_EINVAL
    assert _build(cfg, n=0)[0] == fmm.FMM_EINVAL
    assert _build(cfg, n=2 ** 31)[0] == fmm.FMM_EINVAL
    assert _build(cfg, dtype=5)[0] == fmm.FMM_EINVAL
    assert _build(cfg, pos=None)[0] == fmm.FMM_EINVAL
    cfg.box_lo[1] = float("inf")
    assert _build(cfg)[0] == fmm.FMM_EINVAL


def test_other_entry_points_reject_null():
    L = fmm.lib()
    assert L.fmm_evaluate(None, None, None, None, 0, None) == fmm.FMM_EINVAL
    assert L.fmm_backward(None, None, None, None, None, None, None) == fmm.FMM_EINVAL
    assert L.fmm_tree_info(None, None) == fmm.FMM_EINVAL
    assert L.fmm_stage_times(None, None, 0) == fmm.FMM_EINVAL
    assert L.fmm_tree_export(None, None, None) == fmm.FMM_EINVAL
    assert L.fmm_tree_export_adaptive(None, None, None, None, None, None) == fmm.FMM_EINVAL
    L.fmm_tree_destroy(None)
    assert L.fmm_operator_host(0, 0, 0, None) == fmm.FMM_EINVAL
    with pytest.raises(fmm.FMMError):
        fmm.operator_host(4, 2, 171)  # the zero offset is not an M2L offset
