"""fmm_evaluate_noalloc (buffers from the library's static scratch array)
against fmm_evaluate (buffers from the tree's workspace) through the C ABI:
bitwise equal outputs, on consecutive calls whose second input is smaller,
in both precision forms; a tree too large for the array is rejected before
any launch."""
import ctypes

import numpy as np
import pytest

from paper_1106_2176_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1106_2176_amd as fmm  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _both(t, q, flags):
    """(fmm_evaluate outputs, fmm_evaluate_noalloc outputs) on tree t."""
    L = fmm.lib()
    n = q.shape[0]
    outs = []
    for fn in (L.fmm_evaluate, L.fmm_evaluate_noalloc):
        phi = torch.full((n,), float("nan"), dtype=q.dtype, device="cuda")
        vec = torch.full((n, 3), float("nan"), dtype=q.dtype, device="cuda")
        rc = fn(t._h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                ctypes.c_void_p(vec.data_ptr()) if flags & 3 else None, flags, _stream())
        assert rc == fmm.FMM_OK, fmm.lib().fmm_last_error_message()
        torch.cuda.synchronize()
        outs.append((phi.cpu().numpy(), vec.cpu().numpy() if flags & 3 else None))
    return outs


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matches_evaluate_on_consecutive_calls(precision):
    # the second call's tree is smaller: what the first call left in the
    # array must not leak into it
    for n, p, leaf, seed in ((60_000, 8, 64, 201), (15_000, 6, 32, 202)):
        pos, q = inputs.particles(n, seed)
        with fmm.Tree(dev(pos), p=p, leaf_max=leaf, precision=precision) as t:
            assert t.info()["levels"] >= 3
            Q = dev(q)
            for flags in (fmm.VEC_FIELD, fmm.VEC_FORCE,
                          fmm.VEC_FIELD | fmm.PART_FAR_ONLY, fmm.VEC_NONE | fmm.PART_NEAR_ONLY):
                (phi_a, v_a), (phi_b, v_b) = _both(t, Q, flags)
                assert np.all(np.isfinite(phi_b))
                np.testing.assert_array_equal(phi_b, phi_a)
                if v_a is not None:
                    np.testing.assert_array_equal(v_b, v_a)


def test_noalloc_rejects_a_tree_beyond_the_scratch_size():
    pos, q = inputs.particles(1_000_000, 203)
    with fmm.Tree(dev(pos), p=10, leaf_max=64, precision="mixed") as t:
        Q = dev(q)
        phi = torch.full((len(q),), 7.0, dtype=torch.float64, device="cuda")
        rc = fmm.lib().fmm_evaluate_noalloc(t._h, ctypes.c_void_p(Q.data_ptr()),
                                            ctypes.c_void_p(phi.data_ptr()), None, fmm.VEC_NONE,
                                            _stream())
        assert rc == fmm.FMM_EINVAL
        assert b"FMM_NOALLOC_SCRATCH_BYTES" in fmm.lib().fmm_last_error_message()
        torch.cuda.synchronize()
        assert bool((phi == 7.0).all())  # nothing ran
