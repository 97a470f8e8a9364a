"""GPU parity of the adaptive octree (cfg.adaptive) against the oracle's
adaptive FMM, through the C ABI.

  boxes and particle order  bit-exact (levels, coordinates, ranges, parents,
                            leaf flags; the stable finest-level sort)
  U, V, W, X lists          equal as sets per box (their order is free)
  work counts               exact (pairs and evaluations implied by the lists)
  phi and E, FP64 form      relative L2 <= 1e-10 against the oracle (same lists
                            and truncation; the two differ by rounding only),
                            near and far parts separately as well
  phi and E, mixed form     relative L2 <= 1e-6 against the FP64 form on the
                            same tree (all N) and against the oracle
The inputs are Gaussian blobs (inputs.clustered), which put leaves on many
levels, plus uniform and degenerate cases."""
import ctypes

import numpy as np
import pytest

from conftest import rel_l2
from paper_1106_2176_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1106_2176_amd as fmm  # noqa: E402

TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_eval(t, q, part=None):
    phi, E = t.evaluate(dev(q), vec="field", part=part)
    torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64), E.cpu().numpy().astype(np.float64)


def _sets(lists):
    return [np.sort(np.asarray(x, dtype=np.int64)) for x in lists]


TREES = [  # (generator, n, leaf_max, max_level, seed)
    ("clustered", 20_000, 32, 8, 1),
    ("clustered", 50_000, 64, 7, 2),
    ("uniform", 30_000, 16, 8, 3),
    ("clustered", 3_000, 8, 5, 4),
    ("uniform", 700, 100, 8, 5),
]


def _input(kind, n, seed, dtype="f64"):
    if kind == "clustered":
        return inputs.clustered(n, seed, dtype=dtype)
    return inputs.particles(n, seed, dtype=dtype)


@pytest.mark.parametrize("kind,n,leaf,ml,seed", TREES)
def test_tree_and_lists_match_oracle(oracle_mod, kind, n, leaf, ml, seed):
    pos, _ = _input(kind, n, seed)
    if n > 100:
        pos[:4] = pos[4]  # duplicates keep input order
    ref = oracle_mod.adaptive_tree(pos, leaf, ml)
    print("adaptive tree", kind, n, leaf, ml, seed, flush=True)
    with fmm.Tree(dev(pos), p=4, leaf_max=leaf, max_level=ml, precision="fp64", adaptive=True) as t:
        got = t.export_adaptive()
        info = t.info()
        perm, lstart = t.export()
    np.testing.assert_array_equal(got["boxes"], ref["boxes"])
    np.testing.assert_array_equal(got["order"], ref["order"])
    assert got["depth"] == ref["depth"] == info["levels"]
    for name in "UVWX":
        for b, (g, r) in enumerate(zip(_sets(got[name]), _sets(ref[name]))):
            np.testing.assert_array_equal(g, r, err_msg="%s list of box %d" % (name, b))
    # leaves in particle order and the fullest one
    boxes = ref["boxes"]
    leaves = boxes[boxes[:, 7] == 1]
    leaves = leaves[np.argsort(leaves[:, 4])]
    np.testing.assert_array_equal(lstart[:-1].astype(np.int64), leaves[:, 4])
    assert lstart[-1] == n and info["n_leaves"] == len(leaves)
    assert info["max_leaf_count"] == int((leaves[:, 5] - leaves[:, 4]).max())
    np.testing.assert_array_equal(perm.astype(np.int64), ref["order"])
    # work counts implied by the lists
    cnt = boxes[:, 5] - boxes[:, 4]
    assert info["n_boxes"] == len(boxes)
    assert info["p2p_pairs"] == sum(int(cnt[b]) * int(cnt[ref["U"][b]].sum()) for b in range(len(boxes))) - n
    assert info["m2l_pairs"] == sum(len(v) for v in ref["V"])
    assert info["m2p_evals"] == sum(int(cnt[b]) * len(ref["W"][b]) for b in range(len(boxes)))
    assert info["p2l_evals"] == sum(int(cnt[ref["X"][b]].sum()) for b in range(len(boxes)))


@pytest.mark.parametrize("kind,n,leaf,ml,p,seed", [
    ("clustered", 20_000, 32, 8, 8, 11),
    ("clustered", 50_000, 64, 7, 6, 12),
    ("uniform", 30_000, 16, 8, 5, 13),
    ("clustered", 3_000, 8, 6, 16, 14),
    ("clustered", 8_000, 20, 8, 1, 15),
    ("clustered", 6_000, 24, 8, 11, 16),
])
def test_fmm_matches_oracle(oracle_mod, kind, n, leaf, ml, p, seed):
    pos, q = _input(kind, n, seed)
    q = q - 0.5  # charges of both signs
    ref = oracle_mod.fmm_adaptive(pos, q, p, leaf, ml)
    print("adaptive fmm", kind, n, leaf, ml, p, seed, flush=True)
    with fmm.Tree(dev(pos), p=p, leaf_max=leaf, max_level=ml, precision="fp64", adaptive=True) as t:
        phi, E = gpu_eval(t, q)
        pn, En = gpu_eval(t, q, part="near")
        pf, Ef = gpu_eval(t, q, part="far")
        info = t.info()
    assert info["levels"] == ref["depth"] and info["n_leaves"] == ref["nleaf"]
    assert rel_l2(phi, ref["phi"]) < TOL
    assert rel_l2(E, ref["E"]) < TOL
    assert rel_l2(pn, ref["phi_near"]) < TOL
    assert rel_l2(En, ref["E_near"]) < TOL
    assert rel_l2(pf, ref["phi_far"]) < TOL
    assert rel_l2(Ef, ref["E_far"]) < TOL


def test_float32_inputs_and_force(oracle_mod):
    pos, q = inputs.clustered(10_000, 21, dtype="f32")
    ref = oracle_mod.fmm_adaptive(pos.astype(np.float64), q.astype(np.float64), 6, 32, 8)
    with fmm.Tree(dev(pos), p=6, leaf_max=32, max_level=8, precision="fp64", adaptive=True) as t:
        phi, F = t.evaluate(dev(q), vec="force")
        torch.cuda.synchronize()
    # results are computed in FP64 and rounded once to FP32
    assert rel_l2(phi.cpu().numpy(), ref["phi"]) < 1e-6
    assert rel_l2(F.cpu().numpy(), ref["E"] * q.astype(np.float64)[:, None]) < 1e-6


@pytest.mark.parametrize("n,leaf,ml", [(1, 4, 8), (2, 4, 8), (200, 200, 8), (500, 100, 1), (400, 50, 0)])
def test_shallow_trees_equal_the_direct_sum(oracle_mod, n, leaf, ml):
    """Depth <= 1 (every box touches every other): the FMM is the direct sum."""
    pos, q = inputs.clustered(n, 31)
    phi_d, E_d = oracle_mod.direct(pos, q)
    with fmm.Tree(dev(pos), p=4, leaf_max=leaf, max_level=ml, precision="fp64", adaptive=True) as t:
        phi, E = gpu_eval(t, q)
        assert t.info()["levels"] <= 1
    if n == 1:
        assert phi[0] == 0 and np.all(E == 0)
        return
    assert rel_l2(phi, phi_d) < 1e-12
    assert rel_l2(E, E_d) < 1e-12


def test_coincident_points_beyond_the_cap(oracle_mod):
    """Many particles on one point: the box keeps splitting down to max_level
    and stays over leaf_max there; coincident pairs contribute nothing."""
    pos, q = inputs.clustered(4_000, 41)
    pos[:300] = pos[300]
    ref = oracle_mod.fmm_adaptive(pos, q, 6, 16, 6)
    with fmm.Tree(dev(pos), p=6, leaf_max=16, max_level=6, precision="fp64", adaptive=True) as t:
        phi, E = gpu_eval(t, q)
        info = t.info()
    assert info["levels"] == 6 and info["max_leaf_count"] >= 301
    assert rel_l2(phi, ref["phi"]) < TOL
    assert rel_l2(E, ref["E"]) < TOL


def test_rebuild_and_graph_replay(oracle_mod):
    """A rebuild in place for new positions gives a new tree (graph mode
    recaptures); replays equal eager calls."""
    pos1, q1 = inputs.clustered(12_000, 51)
    pos2, q2 = inputs.clustered(9_000, 52, blobs=3)
    ref2 = oracle_mod.fmm_adaptive(pos2, q2, 6, 32, fmm.ADAPTIVE_MAX_LEVEL)
    with fmm.Tree(dev(pos1), p=6, leaf_max=32, precision="fp64", adaptive=True) as eager, \
            fmm.Tree(dev(pos1), p=6, leaf_max=32, precision="fp64", adaptive=True, graph=True) as g:
        Q1 = dev(q1)
        phi_g = torch.empty(len(q1), dtype=torch.float64, device="cuda")
        E_g = torch.empty(len(q1), 3, dtype=torch.float64, device="cuda")
        phi_e, E_e = eager.evaluate(Q1)
        for _ in range(3):
            g.evaluate(Q1, phi=phi_g, out_vec=E_g)
            torch.cuda.synchronize()
            assert torch.equal(phi_g, phi_e) and torch.equal(E_g, E_e)
        g.rebuild(dev(pos2))
        Q2 = dev(q2)
        phi2 = torch.empty(len(q2), dtype=torch.float64, device="cuda")
        E2 = torch.empty(len(q2), 3, dtype=torch.float64, device="cuda")
        for _ in range(2):
            g.evaluate(Q2, phi=phi2, out_vec=E2)
            torch.cuda.synchronize()
            assert rel_l2(phi2.cpu().numpy(), ref2["phi"]) < TOL
            assert rel_l2(E2.cpu().numpy(), ref2["E"]) < TOL


def test_noalloc_matches_evaluate():
    pos, q = inputs.clustered(20_000, 61)
    with fmm.Tree(dev(pos), p=8, leaf_max=32, precision="fp64", adaptive=True) as t:
        Q = dev(q)
        outs = []
        L = fmm.lib()
        for fn in (L.fmm_evaluate, L.fmm_evaluate_noalloc):
            phi = torch.full((len(q),), float("nan"), dtype=torch.float64, device="cuda")
            vec = torch.full((len(q), 3), float("nan"), dtype=torch.float64, device="cuda")
            rc = fn(t._h, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                    ctypes.c_void_p(vec.data_ptr()), fmm.VEC_FIELD,
                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert rc == fmm.FMM_OK, L.fmm_last_error_message()
            torch.cuda.synchronize()
            outs.append((phi.cpu().numpy(), vec.cpu().numpy()))
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    np.testing.assert_array_equal(outs[1][1], outs[0][1])


@pytest.mark.parametrize("kind,n,leaf,ml,p,seed", [
    ("clustered", 20_000, 32, 8, 8, 81),
    ("clustered", 50_000, 64, 7, 10, 82),
    ("uniform", 30_000, 16, 8, 6, 83),
    ("clustered", 6_000, 24, 8, 13, 84),
    ("clustered", 3_000, 8, 6, 16, 85),
    ("clustered", 8_000, 20, 8, 1, 86),
])
def test_mixed_form_vs_fp64_and_oracle(oracle_mod, kind, n, leaf, ml, p, seed):
    """The mixed form (binary16 M2L; FP32 P2P pairs and P2M, L2P, P2L, M2P terms; the rest FP64) against the FP64 form on
    the same tree, all N, within the mixed form's 1e-6 budget, and against
    the oracle."""
    pos, q = _input(kind, n, seed)
    q = q - 0.5
    ref = oracle_mod.fmm_adaptive(pos, q, p, leaf, ml)
    print("adaptive mixed", kind, n, leaf, ml, p, seed, flush=True)
    out = {}
    for prec in ("fp64", "mixed"):
        with fmm.Tree(dev(pos), p=p, leaf_max=leaf, max_level=ml, precision=prec, adaptive=True) as t:
            out[prec] = gpu_eval(t, q)
            out[prec + "_far"] = gpu_eval(t, q, part="far")
    (p64, E64), (pm, Em) = out["fp64"], out["mixed"]
    e_phi, e_E = rel_l2(pm, p64), rel_l2(Em, E64)
    print("  mixed vs FP64: phi %.2e, E %.2e" % (e_phi, e_E))
    assert e_phi < 1e-6 and e_E < 1e-6
    assert rel_l2(pm, ref["phi"]) < 1e-6 and rel_l2(Em, ref["E"]) < 1e-6
    # the far field alone: the encoding's own error, against the far field's size
    assert rel_l2(out["mixed_far"][0], out["fp64_far"][0]) < 1e-6
    assert rel_l2(out["mixed_far"][1], out["fp64_far"][1]) < 1e-6


def test_mixed_noalloc_matches_evaluate():
    pos, q = inputs.clustered(20_000, 62)
    with fmm.Tree(dev(pos), p=8, leaf_max=32, precision="mixed", adaptive=True) as t:
        Q = dev(q)
        outs = []
        L = fmm.lib()
        for fn in (L.fmm_evaluate, L.fmm_evaluate_noalloc):
            phi = torch.full((len(q),), float("nan"), dtype=torch.float64, device="cuda")
            vec = torch.full((len(q), 3), float("nan"), dtype=torch.float64, device="cuda")
            rc = fn(t._h, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                    ctypes.c_void_p(vec.data_ptr()), fmm.VEC_FIELD,
                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert rc == fmm.FMM_OK, L.fmm_last_error_message()
            torch.cuda.synchronize()
            outs.append((phi.cpu().numpy(), vec.cpu().numpy()))
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    np.testing.assert_array_equal(outs[1][1], outs[0][1])


def test_unsupported_requests():
    pos, q = inputs.clustered(5_000, 71)
    P = dev(pos)
    with pytest.raises(fmm.FMMError) as e:
        fmm.Tree(P, precision="mixed", m2l_fp16=False, adaptive=True)
    assert e.value.status == fmm.FMM_EUNSUPPORTED
    with fmm.Tree(P, p=4, precision="fp64", adaptive=True) as t:
        Q = dev(q)
        # a rebuild keeps the tree kind
        cfg = fmm.make_config(p=4, precision="fp64")
        rc = fmm.lib().fmm_build_tree(ctypes.byref(cfg), len(q), fmm.FMM_F64, ctypes.c_void_p(P.data_ptr()),
                                      None, ctypes.byref(t._h))
        assert rc == fmm.FMM_EINVAL
        phi2, _ = t.evaluate(Q)  # the tree is untouched
        torch.cuda.synchronize()
        assert bool(torch.isfinite(phi2).all())


def test_million_blobs_sampled_against_the_direct_sum(oracle_mod):
    """The benchmark's adaptive workload (N = 1e6 Gaussian blobs, p = 8,
    leaf <= 64, max level 8) on 1000 sampled targets against the FP64 direct
    sum.  The bound is the truncation error the oracle's adaptive FMM shows
    on smaller inputs of the same distribution at p = 8 (phi about 3e-6,
    E about 5e-5 at N = 1e5), with a factor of 3 to 4 of room."""
    import bench
    a = bench.ADAPTIVE
    pos, q = inputs.clustered(a["n"], a["seed"], a["blobs"])
    t_idx = inputs.targets(a["n"], a["seed"])
    phi_d, E_d = oracle_mod.direct(pos, q, t_idx)
    with fmm.Tree(dev(pos), p=a["p"], leaf_max=a["leaf_max"], max_level=a["max_level"], precision="fp64",
                  adaptive=True) as t:
        phi, E = gpu_eval(t, q)
        info = t.info()
    print("1e6 blobs: depth %d, %d leaves, phi %.2e, E %.2e" % (
        info["levels"], info["n_leaves"], rel_l2(phi[t_idx], phi_d), rel_l2(E[t_idx], E_d)))
    assert info["levels"] == a["max_level"]
    assert rel_l2(phi[t_idx], phi_d) < 1e-5
    assert rel_l2(E[t_idx], E_d) < 2e-4


@pytest.mark.parametrize("kind,n,leaf,ml,p,seed", [
    ("clustered", 20_000, 32, 8, 8, 91),
    ("uniform", 20_000, 16, 8, 5, 92),
    ("clustered", 4_000, 16, 6, 12, 93),
])
def test_adjoint_fp64_matches_the_oracle(oracle_mod, kind, n, leaf, ml, p, seed):
    """Gradient of Loss = sum w phi on the adaptive tree (FP64 form).  The
    FMM operator A (q -> phi) is symmetric for fixed leaf assignments (V and
    U are symmetric, X and W are each other's transposes, and each
    translation of one direction is the transpose of the other's), so
    dL/dq = A w is the oracle's potential for the charges w, and
    dL/dx = -(w E_q + q E_w) with the oracle's fields for q and for w."""
    pos, q = _input(kind, n, seed)
    q = q - 0.5
    w = inputs.weights(n, seed)
    rq = oracle_mod.fmm_adaptive(pos, q, p, leaf, ml)
    rw = oracle_mod.fmm_adaptive(pos, w, p, leaf, ml)
    print("adaptive adjoint", kind, n, leaf, ml, p, seed, flush=True)
    with fmm.Tree(dev(pos), p=p, leaf_max=leaf, max_level=ml, precision="fp64", adaptive=True) as t:
        Q, W = dev(q), dev(w)
        _, E = t.evaluate(Q)
        gq, gx = t.backward(Q, W, E)
        torch.cuda.synchronize()
    gq, gx = gq.cpu().numpy(), gx.cpu().numpy()
    want_x = -(w[:, None] * rq["E"] + q[:, None] * rw["E"])
    print("  dL/dq %.2e, dL/dx %.2e" % (rel_l2(gq, rw["phi"]), rel_l2(gx, want_x)))
    assert rel_l2(gq, rw["phi"]) < TOL
    assert rel_l2(gx, want_x) < TOL


def test_adjoint_mixed_vs_fp64():
    """The mixed form's gradient against the FP64 form's on the same tree,
    with weights U[0,1) (no cancellation, so the 1e-6 budget applies as is)."""
    pos, q = inputs.clustered(30_000, 95)
    w = np.random.default_rng(96).random(len(q))
    out = {}
    for prec in ("fp64", "mixed"):
        with fmm.Tree(dev(pos), p=8, leaf_max=32, precision=prec, adaptive=True) as t:
            Q, W = dev(q), dev(w)
            _, E = t.evaluate(Q)
            gq, gx = t.backward(Q, W, E)
            torch.cuda.synchronize()
            out[prec] = (gq.cpu().numpy(), gx.cpu().numpy())
    e_q = rel_l2(out["mixed"][0], out["fp64"][0])
    e_x = rel_l2(out["mixed"][1], out["fp64"][1])
    print("adaptive adjoint mixed vs FP64: dL/dq %.2e, dL/dx %.2e" % (e_q, e_x))
    assert e_q < 1e-6 and e_x < 1e-6


def test_adjoint_graph_replay_matches_eager():
    pos, q = inputs.clustered(10_000, 97)
    w = inputs.weights(len(q), 97)
    with fmm.Tree(dev(pos), p=6, leaf_max=32, precision="fp64", adaptive=True) as eager, \
            fmm.Tree(dev(pos), p=6, leaf_max=32, precision="fp64", adaptive=True, graph=True) as g:
        Q, W = dev(q), dev(w)
        _, E = eager.evaluate(Q)
        gq_e, gx_e = eager.backward(Q, W, E)
        gq = torch.empty_like(Q)
        gx = torch.empty(len(q), 3, dtype=torch.float64, device="cuda")
        for _ in range(3):
            g.backward(Q, W, E, out_q=gq, out_pos=gx)
            torch.cuda.synchronize()
            assert torch.equal(gq, gq_e) and torch.equal(gx, gx_e)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_concurrent_near_field_is_identical(precision):
    """The near field on the library's side stream (overlap_near) gives the
    same bits as the serial chain, forward and adjoint, on repeated calls and
    under graph replay."""
    pos, q = inputs.clustered(15_000, 98)
    w = inputs.weights(len(q), 98)
    res = {}
    for name, kw in (("serial", {}), ("side", {"overlap_near": True}),
                     ("side_graph", {"overlap_near": True, "graph": True})):
        with fmm.Tree(dev(pos), p=6, leaf_max=32, precision=precision, adaptive=True, **kw) as t:
            Q, W = dev(q), dev(w)
            phi = torch.empty_like(Q)
            E = torch.empty(len(q), 3, dtype=torch.float64, device="cuda")
            gq = torch.empty_like(Q)
            gx = torch.empty_like(E)
            outs = []
            for _ in range(3):
                t.evaluate(Q, phi=phi, out_vec=E)
                t.backward(Q, W, E, out_q=gq, out_pos=gx)
                torch.cuda.synchronize()
                outs.append([x.cpu().numpy().copy() for x in (phi, E, gq, gx)])
            for o in outs[1:]:
                for a, b in zip(o, outs[0]):
                    np.testing.assert_array_equal(a, b)
            res[name] = outs[0]
    for name in ("side", "side_graph"):
        for a, b in zip(res[name], res["serial"]):
            np.testing.assert_array_equal(a, b)


def test_deep_tree_to_level_10(oracle_mod):
    """A blob narrower than a level-8 box: the tree refines to level 10 (the
    finest sort has 8^10 bins); boxes, lists and the FMM against the oracle."""
    pos, q = inputs.clustered(6_000, 99)
    c = pos[:2_500].mean(axis=0)
    pos[:2_500] = c + (pos[:2_500] - c) * 0.004  # a blob of width ~1e-4
    q = q - 0.5
    ref_t = oracle_mod.adaptive_tree(pos, 16, 10)
    ref = oracle_mod.fmm_adaptive(pos, q, 6, 16, 10)
    assert ref_t["depth"] == 10
    out = {}
    for prec in ("fp64", "mixed"):
        with fmm.Tree(dev(pos), p=6, leaf_max=16, max_level=10, precision=prec, adaptive=True) as t:
            if prec == "fp64":
                got = t.export_adaptive()
                np.testing.assert_array_equal(got["boxes"], ref_t["boxes"])
                for name in "UVWX":
                    for g, r in zip(_sets(got[name]), _sets(ref_t[name])):
                        np.testing.assert_array_equal(g, r)
            out[prec] = gpu_eval(t, q)
    assert rel_l2(out["fp64"][0], ref["phi"]) < TOL and rel_l2(out["fp64"][1], ref["E"]) < TOL
    assert rel_l2(out["mixed"][0], out["fp64"][0]) < 1e-6 and rel_l2(out["mixed"][1], out["fp64"][1]) < 1e-6
