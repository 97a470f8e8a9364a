"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Tolerances (relative L2 over all checked outputs):
  tree build               bit-exact (level, leaf ranges, stable permutation)
  FP64 form vs oracle FMM  1e-10 for phi and E (same approximation, different
                           basis: spherical harmonics vs Cartesian Taylor)
  FP64 P2P vs oracle near  1e-12
  mixed form vs FP64 form  1e-6 for phi and for F = qE (precision-induced
                           error only; FP32 P2P, binary16- or bf16-split M2L,
                           FP32 fine levels)
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_1106_2176_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1106_2176_amd as fmm  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_eval(pos, q, p, leaf, precision, vec="field", part=None, **kw):
    with fmm.Tree(dev(pos), p=p, leaf_max=leaf, precision=precision, **kw) as t:
        phi, v = t.evaluate(dev(q), vec=vec, part=part)
        torch.cuda.synchronize()
        info = t.info()
    return phi.cpu().numpy().astype(np.float64), (None if v is None else v.cpu().numpy().astype(np.float64)), info


# mixed-form M2L encodings: binary16 (the default), and bf16 in 3 or 2 parts
ENCODINGS = {"fp16x2": dict(m2l_fp16=True), "bf16x3": dict(m2l_fp16=False, bf16_splits=3),
             "bf16x2": dict(m2l_fp16=False, bf16_splits=2)}


# ---------------------------------------------------------------- tree

@pytest.mark.parametrize("n,leaf,seed", [(1, 4, 1), (7, 4, 2), (10_000, 64, 1), (30_000, 16, 3),
                                         (5000, 5000, 4), (100_000, 32, 5)])
def test_tree_matches_oracle(oracle_mod, n, leaf, seed):
    pos, _ = inputs.particles(n, seed)
    if n > 10:
        pos[:5] = pos[5]        # duplicates: ties must keep input order
        pos[6] = [1.0, 0.0, 0.5]  # on the faces of the root cube
    lev, mx = oracle_mod.select_level(pos, leaf)
    _, start, perm = oracle_mod.tree(pos, lev)
    with fmm.Tree(dev(pos), p=4, leaf_max=leaf) as t:
        info = t.info()
        gperm, gstart = t.export()
    assert info["levels"] == lev
    assert info["max_leaf_count"] == mx
    np.testing.assert_array_equal(gstart.astype(np.int64), start)
    np.testing.assert_array_equal(gperm.astype(np.int64), perm)


def test_tree_float32_positions(oracle_mod):
    pos, _ = inputs.particles(20_000, 9, dtype="f32")
    lev, _ = oracle_mod.select_level(pos.astype(np.float64), 32)
    _, start, perm = oracle_mod.tree(pos.astype(np.float64), lev)
    with fmm.Tree(dev(pos), p=4, leaf_max=32) as t:
        gperm, gstart = t.export()
    np.testing.assert_array_equal(gperm.astype(np.int64), perm)
    np.testing.assert_array_equal(gstart.astype(np.int64), start)


def test_pair_counts(oracle_mod):
    pos, _ = inputs.particles(20_000, 10)
    lev, _ = oracle_mod.select_level(pos, 32)
    _, start, _ = oracle_mod.tree(pos, lev)
    side = 2 ** lev
    cnt = np.diff(start)
    # Morton -> (i,j,k) by bit extraction
    idx = np.arange(8 ** lev)
    ijk = np.zeros((8 ** lev, 3), dtype=np.int64)
    for b in range(lev):
        for a in range(3):
            ijk[:, a] |= ((idx >> (3 * b + a)) & 1) << b
    grid = np.zeros((side, side, side), dtype=np.int64)
    grid[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = cnt
    padded = np.pad(grid, 1)
    nsum = sum(padded[1 + dx:1 + dx + side, 1 + dy:1 + dy + side, 1 + dz:1 + dz + side]
               for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))
    want = int((grid * nsum).sum() - len(pos))
    with fmm.Tree(dev(pos), p=4, leaf_max=32) as t:
        info = t.info()
    assert info["p2p_pairs"] == want


# ------------------------------------------------------------------ P2P

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_near_field_matches_oracle(oracle_mod, precision, tol):
    pos, q = inputs.particles(20_000, 11, "u11")
    pos[10] = pos[11]  # a coincident pair contributes nothing
    ref = oracle_mod.fmm(pos, q, 4, 32)
    phi, E, _ = gpu_eval(pos, q, 4, 32, precision, part="near")
    assert rel_l2(phi, ref["phi_near"]) < tol
    assert rel_l2(E, ref["E_near"]) < tol


@pytest.mark.parametrize("n,leaf", [(1, 8), (2, 8), (300, 300), (900, 200), (3000, 700)])
def test_small_levels_equal_direct(oracle_mod, n, leaf):
    """L <= 1 (and a single leaf): the FMM is the direct sum."""
    pos, q = inputs.particles(n, 12)
    phi_d, E_d = oracle_mod.direct(pos, q)
    for precision, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        phi, E, info = gpu_eval(pos, q, 4, leaf, precision)
        assert info["levels"] <= 1
        if n == 1:
            assert phi[0] == 0 and np.all(E == 0)
            continue
        assert rel_l2(phi, phi_d) < tol
        assert rel_l2(E, E_d) < tol


# ------------------------------------------------------------ far field

@pytest.mark.parametrize("p", [1, 2, 4, 7])
def test_far_field_fp64_matches_oracle(oracle_mod, p):
    pos, q = inputs.particles(12_000, 13, "u11")
    ref = oracle_mod.fmm(pos, q, p, 24)
    assert ref["level"] >= 3
    phi, E, _ = gpu_eval(pos, q, p, 24, "fp64", part="far")
    assert rel_l2(phi, ref["phi_far"]) < 1e-10
    if p > 1:
        assert rel_l2(E, ref["E_far"]) < 1e-10
    else:
        assert np.max(np.abs(E)) < 1e-9 * np.max(np.abs(ref["E_near"]))


# ------------------------------------------------------------- whole FMM

def test_c1_fp64_and_mixed_vs_oracle(oracle_mod):
    pos, q = inputs.workload("C1")
    w = inputs.WORKLOADS["C1"]
    ref = oracle_mod.fmm(pos, q, w.p, w.leaf_max)
    phi_d, E_d = oracle_mod.direct(pos, q)
    phi, E, info = gpu_eval(pos, q, w.p, w.leaf_max, "fp64")
    assert info["levels"] == ref["level"] == 3
    assert rel_l2(phi, ref["phi"]) < 1e-10
    assert rel_l2(E, ref["E"]) < 1e-10
    for enc in ("fp16x2", "bf16x3", "bf16x2"):
        phm, Em, _ = gpu_eval(pos, q, w.p, w.leaf_max, "mixed", **ENCODINGS[enc])
        assert rel_l2(phm, phi) < 1e-6
        assert rel_l2(q[:, None] * Em, q[:, None] * E) < 1e-6
    # the FMM error itself is that of the oracle (p = 4)
    assert abs(rel_l2(phi, phi_d) - rel_l2(ref["phi"], phi_d)) < 1e-8


@pytest.mark.parametrize("p,leaf", [(3, 16), (6, 40), (9, 30)])
def test_fmm_fp64_matches_oracle_various(oracle_mod, p, leaf):
    pos, q = inputs.particles(15_000, 14 + p)
    ref = oracle_mod.fmm(pos, q, p, leaf)
    phi, E, info = gpu_eval(pos, q, p, leaf, "fp64")
    assert info["levels"] == ref["level"]
    assert rel_l2(phi, ref["phi"]) < 1e-10
    assert rel_l2(E, ref["E"]) < 1e-10


def test_c2_sampled_fp64_and_mixed(oracle_mod):
    """N = 1e6, p = 10, leaf <= 64 (full size) on 1000 sampled targets."""
    w = inputs.WORKLOADS["C2"]
    pos, q = inputs.workload("C2")
    t = inputs.targets(w.n, w.seed)
    ref = oracle_mod.fmm(pos, q, w.p, w.leaf_max, targets=t)
    phi_d, E_d = oracle_mod.direct(pos, q, t)
    phi, E, info = gpu_eval(pos, q, w.p, w.leaf_max, "fp64")
    assert info["levels"] == 5
    assert rel_l2(phi[t], ref["phi"]) < 1e-10
    assert rel_l2(E[t], ref["E"]) < 1e-10
    for enc in ("fp16x2", "bf16x3"):
        phm, Em, _ = gpu_eval(pos, q, w.p, w.leaf_max, "mixed", **ENCODINGS[enc])
        e_phi, e_F = rel_l2(phm, phi), rel_l2(q[:, None] * Em, q[:, None] * E)
        print("C2 mixed (%s) vs FP64 on all N: phi %.3e F %.3e" % (enc, e_phi, e_F))
        assert e_phi < 1e-6
        assert e_F < 1e-6
        # accuracy against the exact sum is the FMM truncation error of p = 10
        assert rel_l2(phm[t], phi_d) < 1e-6
        assert rel_l2(Em[t], E_d) < 1e-5


def test_c3_sampled_fp64_and_mixed(oracle_mod):
    """N = 1e7, p = 10, leaf <= 128, zero-mean charges U[-1,1) (full size):
    FP64 form against the oracle on 1000 sampled targets, mixed against FP64
    on all N within 1e-6 for phi and for F."""
    w = inputs.WORKLOADS["C3"]
    pos, q = inputs.workload("C3")
    t = inputs.targets(w.n, w.seed)
    ref = oracle_mod.fmm(pos, q, w.p, w.leaf_max, targets=t)
    phi, E, info = gpu_eval(pos, q, w.p, w.leaf_max, "fp64")
    assert info["levels"] == 6
    assert rel_l2(phi[t], ref["phi"]) < 1e-10
    assert rel_l2(E[t], ref["E"]) < 1e-10
    phm, Em, _ = gpu_eval(pos, q, w.p, w.leaf_max, "mixed")
    e_phi = rel_l2(phm, phi)
    e_F = rel_l2(q[:, None] * Em, q[:, None] * E)
    print("C3 mixed vs FP64 on all N: phi %.3e F %.3e" % (e_phi, e_F))
    assert e_phi < 1e-6
    assert e_F < 1e-6


def test_c4_sampled_fp32_inputs(oracle_mod):
    """N = 1e8 FP32 positions and charges, p = 8, leaf <= 128 (full size):
    FP64 form against the oracle (inputs widened exactly) on 1000 sampled
    targets; mixed against FP64 on all N."""
    w = inputs.WORKLOADS["C4"]
    pos, q = inputs.workload("C4")
    assert pos.dtype == np.float32
    t = inputs.targets(w.n, w.seed)
    # outputs come back in the caller's dtype: the FP64 check runs on the
    # exactly widened inputs, the mixed form on the FP32 inputs themselves
    pos64, q64 = pos.astype(np.float64), q.astype(np.float64)
    ref = oracle_mod.fmm(pos64, q64, w.p, w.leaf_max, targets=t)
    phi, E, info = gpu_eval(pos64, q64, w.p, w.leaf_max, "fp64")
    del pos64
    assert info["levels"] == 7
    assert rel_l2(phi[t], ref["phi"]) < 1e-10
    assert rel_l2(E[t], ref["E"]) < 1e-10
    phm, Em, _ = gpu_eval(pos, q, w.p, w.leaf_max, "mixed")
    assert rel_l2(phm, phi) < 1e-6
    assert rel_l2(q64[:, None] * Em, q64[:, None] * E) < 1e-6


def test_box_and_dtype_options(oracle_mod):
    rng = np.random.default_rng(30)
    lo = np.array([-2.0, 1.0, 0.5])
    size = 3.0
    pos = lo + size * rng.random((8000, 3))
    q = rng.uniform(-1, 1, 8000)
    ref = oracle_mod.fmm(pos, q, 5, 20, lo=lo, size=size)
    phi, E, _ = gpu_eval(pos, q, 5, 20, "fp64", box_lo=tuple(lo), box_size=size)
    assert rel_l2(phi, ref["phi"]) < 1e-10
    assert rel_l2(E, ref["E"]) < 1e-10
    pos32 = pos.astype(np.float32)
    q32 = q.astype(np.float32)
    ref32 = oracle_mod.fmm(pos32.astype(np.float64), q32.astype(np.float64), 5, 20, lo=lo, size=size)
    phi, E, _ = gpu_eval(pos32, q32, 5, 20, "mixed", box_lo=tuple(lo), box_size=size)
    assert rel_l2(phi, ref32["phi"]) < 2e-6
    assert rel_l2(E, ref32["E"]) < 2e-5


def test_force_output_and_newton(oracle_mod):
    pos, q = inputs.particles(20_000, 31)
    _, F, _ = gpu_eval(pos, q, 8, 32, "fp64", vec="force")
    _, E, _ = gpu_eval(pos, q, 8, 32, "fp64", vec="field")
    np.testing.assert_allclose(F, q[:, None] * E, rtol=1e-15, atol=0)
    assert np.linalg.norm(F.sum(0)) < 1e-4 * np.abs(F).sum()


def test_deterministic_and_rebuild():
    pos, q = inputs.particles(50_000, 32)
    a, Ea, _ = gpu_eval(pos, q, 6, 32, "mixed")
    b, Eb, _ = gpu_eval(pos, q, 6, 32, "mixed")
    assert np.array_equal(a, b) and np.array_equal(Ea, Eb)
    pos2, q2 = inputs.particles(20_000, 33)
    with fmm.Tree(dev(pos), p=6, leaf_max=32, precision="mixed") as t:
        t.rebuild(dev(pos2))
        c, Ec = t.evaluate(dev(q2))
    d, Ed, _ = gpu_eval(pos2, q2, 6, 32, "mixed")
    assert np.array_equal(c.cpu().numpy(), d) and np.array_equal(Ec.cpu().numpy(), Ed)


def test_concurrent_near_field_is_identical():
    """P2P on the library's side stream (overlap_near) gives the same bits as
    the serial order, forward and adjoint, across repeated calls."""
    pos, q = inputs.particles(60_000, 41)
    w = np.random.default_rng(42).standard_normal(60_000)
    out = {}
    for ov in (False, True):
        with fmm.Tree(dev(pos), p=6, leaf_max=32, precision="mixed", overlap_near=ov) as t:
            res = []
            for _ in range(3):
                phi, E = t.evaluate(dev(q))
                gq, gx = t.backward(dev(q), dev(w), E)
                res.append([x.cpu().numpy() for x in (phi, E, gq, gx)])
            torch.cuda.synchronize()
        for r in res[1:]:
            for a, b in zip(r, res[0]):
                np.testing.assert_array_equal(a, b)
        out[ov] = res[0]
    for a, b in zip(out[False], out[True]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_combine_in_p2p_and_in_l2p(oracle_mod, dtype, precision):
    """The forward chain ends its last kernel with the combine: P2P's in the
    serial order, L2P's after the join when P2P runs on the side stream.  Both
    give the same bits for every output kind and caller dtype, the force is
    q E, and the near-only and far-only parts (the latter through the combine
    kernel) add up to the whole."""
    pos, q = inputs.particles(30_000, 52, dtype=dtype)
    ref = oracle_mod.fmm(pos.astype(np.float64), q.astype(np.float64), 6, 32)
    out = {}
    for ov in (False, True):
        with fmm.Tree(dev(pos), p=6, leaf_max=32, precision=precision, overlap_near=ov) as t:
            for vec in ("field", "force", None):
                phi, v = t.evaluate(dev(q), vec=vec)
                out[ov, vec] = (phi.cpu().numpy(), None if v is None else v.cpu().numpy())
            near, En = t.evaluate(dev(q), part="near")
            far, Ef = t.evaluate(dev(q), part="far")
            torch.cuda.synchronize()
            parts = [x.cpu().numpy().astype(np.float64) for x in (near, En, far, Ef)]
    for vec in ("field", "force", None):
        for a, b in zip(out[False, vec], out[True, vec]):
            if a is not None:
                np.testing.assert_array_equal(a, b)
    phi, E = (x.astype(np.float64) for x in out[False, "field"])
    F = out[False, "force"][1].astype(np.float64)
    np.testing.assert_array_equal(out[False, None][0], out[False, "field"][0])
    eps = 1e-6 if dtype == "f32" else 1e-14
    np.testing.assert_allclose(F, q.astype(np.float64)[:, None] * E, rtol=eps, atol=eps * np.abs(F).max())
    assert rel_l2(parts[0] + parts[2], phi) < 10 * eps
    assert rel_l2(parts[1] + parts[3], E) < 10 * eps
    tol_phi, tol_e = (1e-10, 1e-10) if precision == "fp64" and dtype == "f64" else (2e-6, 2e-5)
    assert rel_l2(phi, ref["phi"]) < tol_phi
    assert rel_l2(E, ref["E"]) < tol_e


def test_leaves_split_into_chunks_at_level_7(oracle_mod):
    """Trees of 8^7 leaves and more run a target leaf as several chunks when
    that fills more lanes (here 73 particles a leaf on average, 84% of the
    leaves over 64): FP64 against the oracle at sampled targets, and the
    mixed form against FP64 within its budget."""
    rng = np.random.default_rng(5)
    n = 300_000
    pos = rng.random((n, 3)) * 0.125  # one corner: level 6 would hold ~590 a leaf
    q = rng.random(n)
    tg = rng.choice(n, 2000, replace=False)
    ref = oracle_mod.fmm(pos, q, 4, 128, targets=tg)
    phi64, E64, info = gpu_eval(pos, q, 4, 128, "fp64")
    assert info["levels"] == 7 == ref["level"]
    assert rel_l2(phi64[tg], ref["phi"]) < 1e-10
    assert rel_l2(E64[tg], ref["E"]) < 1e-10
    phim, Em, _ = gpu_eval(pos, q, 4, 128, "mixed")
    assert rel_l2(phim, phi64) < 1e-6
    assert rel_l2(Em, E64) < 1e-6


def test_domain_errors():
    pos, q = inputs.particles(1000, 34)
    for bad in (np.nan, 1.5, -0.25, np.inf):
        p2 = pos.copy()
        p2[17, 1] = bad
        with pytest.raises(fmm.FMMError) as e:
            fmm.Tree(dev(p2), p=4, leaf_max=16)
        assert e.value.status == fmm.FMM_EDOMAIN


def test_bf16_three_way_split_is_more_accurate():
    pos, q = inputs.particles(60_000, 35)
    ref, Er, _ = gpu_eval(pos, q, 10, 32, "fp64", part="far")
    a, Ea, _ = gpu_eval(pos, q, 10, 32, "mixed", part="far", bf16_splits=2, m2l_fp16=False)
    b, Eb, _ = gpu_eval(pos, q, 10, 32, "mixed", part="far", bf16_splits=3, m2l_fp16=False)
    assert rel_l2(b, ref) <= rel_l2(a, ref)
    assert rel_l2(a, ref) < 1e-6


@pytest.mark.parametrize("overlap", [False, True])
def test_profiled_stage_subset(overlap):
    """profile_stages: events only around the selected stages; their times
    are positive, the others are NaN."""
    pos, q = inputs.particles(60_000, 44)
    with fmm.Tree(dev(pos), p=6, leaf_max=32, precision="mixed", profile=True,
                  profile_stages=("M2L", "P2P"), overlap_near=overlap) as t:
        for _ in range(3):
            t.evaluate(dev(q))
        st = t.stage_times()
    assert st["M2L"] > 0 and st["P2P"] > 0
    assert all(np.isnan(v) for k, v in st.items() if k not in ("M2L", "P2P"))


# ------------------------------------------------------- orders above 10

@pytest.mark.parametrize("p", [11, 12, 13, 14, 15, 16])
def test_high_order_fp64_vs_oracle_and_mixed(oracle_mod, p):
    """Every order above the workloads' p = 10 that the library accepts: the
    FP64 form against the oracle (level 3, so that the oracle's Cartesian
    M2L of p(p+1)(p+2)/6 terms stays in seconds), and the mixed form in
    each M2L encoding it supports (binary16 at every p, 3 bf16 parts up to
    p = 13) against the FP64 form; the encodings it does not support (2 bf16
    parts above p = 10, 3 above 13) are rejected."""
    n, leaf = 4000, 32
    pos, q = inputs.particles(n, 100 + p)
    ref = oracle_mod.fmm(pos, q, p, leaf)
    phi, E, info = gpu_eval(pos, q, p, leaf, "fp64")
    assert info["levels"] == ref["level"] == 3
    assert rel_l2(phi, ref["phi"]) < 1e-10
    assert rel_l2(E, ref["E"]) < 1e-10
    phf, Ef, _ = gpu_eval(pos, q, p, leaf, "fp64", part="far")
    assert rel_l2(phf, ref["phi_far"]) < 1e-10
    assert rel_l2(Ef, ref["E_far"]) < 1e-10
    for name, kw in ENCODINGS.items():
        if (name == "bf16x3" and p > 13) or name == "bf16x2":
            with pytest.raises(fmm.FMMError) as e:
                gpu_eval(pos, q, p, leaf, "mixed", **kw)
            assert e.value.status == fmm.FMM_EUNSUPPORTED
            continue
        phm, Em, _ = gpu_eval(pos, q, p, leaf, "mixed", **kw)
        assert rel_l2(phm, phi) < 1e-6
        assert rel_l2(q[:, None] * Em, q[:, None] * E) < 1e-6


@pytest.mark.parametrize("p,enc", [(13, "bf16x3"), (16, "fp16x2"), (11, "fp16x2"), (4, "fp16x2")])
def test_high_order_mixed_at_level5(p, enc):
    """Mixed against FP64 on a level-5 tree (whole M2L tiles of 128
    targets, not only the K-split small levels), far part and whole."""
    pos, q = inputs.particles(300_000, 120 + p)
    phi, E, info = gpu_eval(pos, q, p, 32, "fp64")
    assert info["levels"] == 5
    phm, Em, _ = gpu_eval(pos, q, p, 32, "mixed", **ENCODINGS[enc])
    assert rel_l2(phm, phi) < 1e-6
    assert rel_l2(q[:, None] * Em, q[:, None] * E) < 1e-6
    phf, Ef, _ = gpu_eval(pos, q, p, 32, "fp64", part="far")
    phmf, Emf, _ = gpu_eval(pos, q, p, 32, "mixed", part="far", **ENCODINGS[enc])
    assert rel_l2(phmf, phf) < 1e-6
    assert rel_l2(Emf, Ef) < 1e-6


# --------------------------------------- graph replay, concurrent near field

def _modes_run(pos, q, w, p, leaf, precision, graph, overlap, reps=3):
    """Evaluate and backward `reps` times on one tree in the given launch
    mode (graph: replayed from the second call on); every call's outputs."""
    n = len(q)
    qd, wd = dev(q), dev(w)
    out = []
    with fmm.Tree(dev(pos), p=p, leaf_max=leaf, precision=precision, graph=graph,
                  overlap_near=overlap) as t:
        phi = torch.empty(n, dtype=torch.float64, device="cuda")
        E = torch.empty(n, 3, dtype=torch.float64, device="cuda")
        gq = torch.empty_like(phi)
        gx = torch.empty_like(E)
        for _ in range(reps):
            for x in (phi, E, gq, gx):
                x.fill_(float("nan"))
            t.evaluate(qd, phi=phi, out_vec=E)
            t.backward(qd, wd, E, out_q=gq, out_pos=gx)
            torch.cuda.synchronize()
            out.append([x.cpu().numpy() for x in (phi, E, gq, gx)])
    return out


@pytest.mark.parametrize("graph,overlap", [(False, False), (True, False), (False, True), (True, True)])
def test_launch_modes_fp64_match_oracle(oracle_mod, graph, overlap):
    """C1 (N = 1e4, p = 4) in the FP64 form with graph replay and/or the
    concurrent near field: every call's potential and field against the
    oracle FMM, and its gradients against the oracle's FMM gradient (which
    finite differences pin), within 1e-10."""
    wl = inputs.WORKLOADS["C1"]
    pos, q = inputs.workload("C1")
    w = inputs.weights(wl.n, wl.seed)
    ref = oracle_mod.fmm(pos, q, wl.p, wl.leaf_max)
    gq_o, gx_o, _ = oracle_mod.fmm_grad(pos, q, w, wl.p, wl.leaf_max)
    for phi, E, gq, gx in _modes_run(pos, q, w, wl.p, wl.leaf_max, "fp64", graph, overlap):
        assert rel_l2(phi, ref["phi"]) < 1e-10
        assert rel_l2(E, ref["E"]) < 1e-10
        assert rel_l2(gq, gq_o) < 1e-10
        assert rel_l2(gx, gx_o) < 1e-10


@pytest.mark.parametrize("graph,overlap", [(True, False), (False, True), (True, True)])
def test_launch_modes_c2_mixed_vs_fp64_and_oracle(oracle_mod, graph, overlap):
    """C2 (N = 1e6, p = 10, leaf <= 64): the FP64 form in the mode against
    the oracle FMM on 1000 sampled targets (1e-10), and the mixed form in the
    mode against the FP64 form on all N (1e-6, phi and F), every call."""
    wl = inputs.WORKLOADS["C2"]
    pos, q = inputs.workload("C2")
    w = inputs.weights(wl.n, wl.seed)
    t = inputs.targets(wl.n, wl.seed)
    ref = oracle_mod.fmm(pos, q, wl.p, wl.leaf_max, targets=t)
    f64 = _modes_run(pos, q, w, wl.p, wl.leaf_max, "fp64", graph, overlap, reps=2)
    for phi, E, _, _ in f64:
        assert rel_l2(phi[t], ref["phi"]) < 1e-10
        assert rel_l2(E[t], ref["E"]) < 1e-10
    phi, E, gq, gx = f64[0]
    for phm, Em, gqm, gxm in _modes_run(pos, q, w, wl.p, wl.leaf_max, "mixed", graph, overlap, reps=2):
        assert rel_l2(phm, phi) < 1e-6
        assert rel_l2(q[:, None] * Em, q[:, None] * E) < 1e-6


# ------------------------------------------------ rotation-based M2L (FP64)

@pytest.mark.parametrize("p", [2, 4, 10, 12, 16])
def test_rotation_m2l_fp64_vs_oracle(oracle_mod, p):
    """M2L by rotation (FP64 form): the same approximation as the dense
    operators, so the oracle FMM is matched to round-off, whole and far
    part."""
    n, leaf = 4000, 32
    pos, q = inputs.particles(n, 140 + p)
    ref = oracle_mod.fmm(pos, q, p, leaf)
    phi, E, info = gpu_eval(pos, q, p, leaf, "fp64", m2l_rotation=True)
    assert info["levels"] == ref["level"] == 3
    assert rel_l2(phi, ref["phi"]) < 1e-10
    assert rel_l2(E, ref["E"]) < 1e-10
    phf, Ef, _ = gpu_eval(pos, q, p, leaf, "fp64", part="far", m2l_rotation=True)
    assert rel_l2(phf, ref["phi_far"]) < 1e-10
    assert rel_l2(Ef, ref["E_far"]) < 1e-10


@pytest.mark.parametrize("p", [8, 13])
def test_rotation_m2l_matches_dense_forward_and_adjoint(p):
    """On a level-5 tree (every level 2..5, partial and whole target tiles):
    far field and adjoint gradients of the rotation form against the dense
    FP64 form."""
    pos, q = inputs.particles(300_000, 150 + p)
    w = np.random.default_rng(151).standard_normal(len(q))
    out = {}
    for rot in (False, True):
        with fmm.Tree(dev(pos), p=p, leaf_max=32, precision="fp64", m2l_rotation=rot) as t:
            assert t.info()["levels"] == 5
            phi, E = t.evaluate(dev(q), part="far")
            phi2, E2 = t.evaluate(dev(q))
            gq, gx = t.backward(dev(q), dev(w), E2)
            torch.cuda.synchronize()
            out[rot] = [x.cpu().numpy() for x in (phi, E, gq, gx)]
    for a, b in zip(out[True], out[False]):
        assert rel_l2(a, b) < 1e-12


def test_rotation_m2l_is_fp64_only():
    pos, q = inputs.particles(1000, 152)
    with pytest.raises(fmm.FMMError) as e:
        gpu_eval(pos, q, 8, 32, "mixed", m2l_rotation=True)
    assert e.value.status == fmm.FMM_EINVAL
