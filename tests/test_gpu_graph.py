"""Graph mode (cfg.graph): the evaluate and backward chains replayed from a
captured HIP graph give the same bits as eager calls, replay after replay,
with eager work and synchronisations between replays, after in-place input
changes, and after rebuilds that keep or change the tree's shape."""
import numpy as np
import pytest

from paper_1106_2176_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1106_2176_amd as fmm  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def eager(pos, q, w, **kw):
    with fmm.Tree(dev(pos), **kw) as t:
        phi, E = t.evaluate(dev(q))
        gq, gx = t.backward(dev(q), dev(w), E)
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in (phi, E, gq, gx)]


def same(got, ref):
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision,overlap", [("mixed", False), ("mixed", True), ("fp64", False)])
def test_graph_replays_match_eager(precision, overlap):
    kw = dict(p=6, leaf_max=32, precision=precision, overlap_near=overlap)
    n = 50_000
    pos, q = inputs.particles(n, 61)
    _, q2 = inputs.particles(n, 62)
    w = np.random.default_rng(63).standard_normal(n)
    ref = eager(pos, q, w, **kw)
    ref2 = eager(pos, q2, w, **kw)
    qd, wd = dev(q), dev(w)
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    E = torch.empty(n, 3, dtype=torch.float64, device="cuda")
    gq = torch.empty_like(phi)
    gx = torch.empty_like(E)
    with fmm.Tree(dev(pos), graph=True, **kw) as t:
        for it in range(4):
            for x in (phi, E, gq, gx):
                x.fill_(float("nan"))
            t.evaluate(qd, phi=phi, out_vec=E)
            t.backward(qd, wd, E, out_q=gq, out_pos=gx)
            torch.cuda.synchronize()
            same([x.cpu().numpy() for x in (phi, E, gq, gx)], ref)
            # eager work of the program between replays
            (phi * 2.0 + E.sum(1)).sum().item()
        # charges changed in place: the graph reads the new values
        qd.copy_(dev(q2))
        t.evaluate(qd, phi=phi, out_vec=E)
        t.backward(qd, wd, E, out_q=gq, out_pos=gx)
        torch.cuda.synchronize()
        same([x.cpu().numpy() for x in (phi, E, gq, gx)], ref2)


def test_graph_after_rebuilds():
    kw = dict(p=5, leaf_max=32, precision="mixed")
    cases = [(40_000, 71), (40_000, 72), (9_000, 73), (40_000, 74)]  # same shape, new n, back
    with fmm.Tree(dev(inputs.particles(*cases[0])[0]), graph=True, **kw) as t:
        for n, seed in cases:
            pos, q = inputs.particles(n, seed)
            w = np.random.default_rng(seed).standard_normal(n)
            ref = eager(pos, q, w, **kw)
            t.rebuild(dev(pos))
            qd, wd = dev(q), dev(w)
            phi = torch.empty(n, dtype=torch.float64, device="cuda")
            E = torch.empty(n, 3, dtype=torch.float64, device="cuda")
            gq = torch.empty_like(phi)
            gx = torch.empty_like(E)
            for _ in range(2):
                t.evaluate(qd, phi=phi, out_vec=E)
                t.backward(qd, wd, E, out_q=gq, out_pos=gx)
                torch.cuda.synchronize()
                same([x.cpu().numpy() for x in (phi, E, gq, gx)], ref)


def test_graph_parts_and_kinds():
    """Near-only, far-only (whose near-field buffer is zeroed by a kernel, not
    by a memset node) and the force and potential-only kinds, each replayed."""
    n = 30_000
    pos, q = inputs.particles(n, 81)
    kw = dict(p=4, leaf_max=32, precision="mixed")
    for vec, part in (("field", "near"), ("field", "far"), ("force", None), (None, None)):
        with fmm.Tree(dev(pos), **kw) as t:
            r_phi, r_v = t.evaluate(dev(q), vec=vec, part=part)
            torch.cuda.synchronize()
            ref = [r_phi.cpu().numpy()] + ([] if r_v is None else [r_v.cpu().numpy()])
        with fmm.Tree(dev(pos), graph=True, **kw) as t:
            phi = torch.empty(n, dtype=torch.float64, device="cuda")
            v = torch.empty(n, 3, dtype=torch.float64, device="cuda") if vec else None
            qd = dev(q)
            for _ in range(3):
                phi.fill_(float("nan"))
                if v is not None:
                    v.fill_(float("nan"))
                t.evaluate(qd, vec=vec, phi=phi, out_vec=v, part=part)
                torch.cuda.synchronize()
                got = [phi.cpu().numpy()] + ([] if v is None else [v.cpu().numpy()])
                same(got, ref)
