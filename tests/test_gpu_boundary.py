"""The C-ABI ownership contract on the GPU: workspace memory through the
caller's allocator callbacks (torch's caching allocator in the Python
binding), FMM_ENOMEM from an allocator that fails, and the rejection of a
rebuild under settings the tree was not created with."""
import ctypes

import numpy as np
import pytest

from conftest import rel_l2
from paper_1106_2176_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1106_2176_amd as fmm  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _build(cfg, pos, handle):
    return fmm.lib().fmm_build_tree(ctypes.byref(cfg), pos.shape[0], fmm.FMM_F64,
                                    ctypes.c_void_p(pos.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    ctypes.byref(handle))


def test_failing_allocator_gives_enomem():
    pos, _ = inputs.particles(20_000, 90)
    P = dev(pos)
    calls = []

    def alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, stream, ctx):
        raise AssertionError("nothing was allocated, nothing may be freed")

    cbs = (fmm.ALLOC_FN(alloc), fmm.FREE_FN(free))
    cfg = fmm.make_config(p=6, leaf_max=32, allocator=cbs)
    h = ctypes.c_void_p(None)
    rc = _build(cfg, P, h)
    assert rc == fmm.FMM_ENOMEM
    assert not h.value
    assert calls and b"allocator returned NULL" in fmm.lib().fmm_last_error_message()
    with pytest.raises(fmm.FMMError) as e:
        fmm.Tree(P, p=6, leaf_max=32, allocator=cbs)
    assert e.value.status == fmm.FMM_ENOMEM


def test_counting_allocator_sees_every_buffer():
    """A caller allocator that forwards to torch: the tree's workspace is
    exactly what it handed out, and destroy gives all of it back."""
    pos, q = inputs.particles(50_000, 91)
    live = {}

    def alloc(nbytes, stream, ctx):
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0))
        live[ptr] = nbytes
        return ptr

    def free(ptr, stream, ctx):
        assert ptr in live
        del live[ptr]
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (fmm.ALLOC_FN(alloc), fmm.FREE_FN(free))
    with fmm.Tree(dev(pos), p=6, leaf_max=32, precision="mixed", allocator=cbs) as t:
        phi, E = t.evaluate(dev(q))
        torch.cuda.synchronize()
        info = t.info()
        assert sum(live.values()) == info["workspace_bytes"]
    torch.cuda.synchronize()
    assert not live


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_torch_allocator_same_bits_and_memory_returned(precision):
    pos, q = inputs.particles(80_000, 92)
    out = {}
    for al in ("library", "torch"):
        base = torch.cuda.memory_allocated()
        with fmm.Tree(dev(pos), p=7, leaf_max=32, precision=precision, allocator=al) as t:
            phi, E = t.evaluate(dev(q))
            gq, gx = t.backward(dev(q), dev(q), E)
            torch.cuda.synchronize()
            ws = t.info()["workspace_bytes"]
            held = torch.cuda.memory_allocated() - base
            out[al] = [x.cpu().numpy() for x in (phi, E, gq, gx)]
            del phi, E, gq, gx
        torch.cuda.synchronize()
        if al == "torch":
            # torch counts the tree's workspace (plus the outputs above)
            assert held >= ws
            assert torch.cuda.memory_allocated() <= base
    for a, b in zip(out["library"], out["torch"]):
        np.testing.assert_array_equal(a, b)


def test_rebuild_with_other_settings_is_rejected():
    """A rebuild whose p, precision, split count, dtype or allocator differs
    from the tree's returns FMM_EINVAL before any launch and leaves the tree
    usable as it was."""
    pos, q = inputs.particles(30_000, 93)
    pos2, _ = inputs.particles(30_000, 94)
    P, P2, Q = dev(pos), dev(pos2), dev(q)
    with fmm.Tree(P, p=6, leaf_max=32, precision="mixed") as t:
        ref_phi, ref_E = t.evaluate(Q)
        torch.cuda.synchronize()
        ref = (ref_phi.cpu().numpy(), ref_E.cpu().numpy())
        good = t.cfg
        bad = []
        for field, value in (("p", 7), ("precision", fmm.PREC_FP64), ("bf16_splits", 2),
                             ("m2l_fp16", 0)):
            c = fmm.make_config(p=6, leaf_max=32, precision="mixed")
            setattr(c, field, value)
            bad.append(c)
        bad.append(fmm.make_config(p=6, leaf_max=32, precision="mixed", allocator="library"))
        for c in bad:
            rc = _build(c, P2, t._h)
            assert rc == fmm.FMM_EINVAL, fmm.lib().fmm_last_error_message()
            assert b"rebuilt only" in fmm.lib().fmm_last_error_message()
        # another dtype
        P2f = P2.float()
        rc = fmm.lib().fmm_build_tree(ctypes.byref(good), P2.shape[0], fmm.FMM_F32,
                                      ctypes.c_void_p(P2f.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                      ctypes.byref(t._h))
        assert rc == fmm.FMM_EINVAL
        # the tree is untouched: same positions, same results
        phi, E = t.evaluate(Q)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(phi.cpu().numpy(), ref[0])
        np.testing.assert_array_equal(E.cpu().numpy(), ref[1])
        # a rebuild with the tree's own settings is accepted
        t.rebuild(P2)
        phi2, _ = t.evaluate(Q)
    with fmm.Tree(P2, p=6, leaf_max=32, precision="mixed") as t2:
        phi_ref2, _ = t2.evaluate(Q)
        torch.cuda.synchronize()
    assert rel_l2(phi2.cpu().numpy(), phi_ref2.cpu().numpy()) == 0.0
