"""Adjoint (weighted-potential loss) on the GPU against the oracle.

Loss = sum_i w_i phi_i.  Pins:
  FP64 adjoint vs oracle FMM gradient   1e-10 (oracle gradient is itself
      pinned by finite differences of its own loss in test_oracle.py)
  dot-product test <w, A q> = <A^T w, q>  1e-12 relative (FP64)
  w = q (held fixed): dL/dq = A q = phi, dL/dx = -2 q E   1e-12 (FP64)
  mixed adjoint vs FP64 adjoint           1e-6 (each gradient's cancellation
      factor is printed beside its error)
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


def grads(pos, q, w, p, leaf, precision, **kw):
    with fmm.Tree(dev(pos), p=p, leaf_max=leaf, precision=precision, **kw) as t:
        phi, E = t.evaluate(dev(q))
        gq, gx = t.backward(dev(q), dev(w), E)
        torch.cuda.synchronize()
    return phi.cpu().numpy(), E.cpu().numpy(), gq.cpu().numpy(), gx.cpu().numpy()


@pytest.mark.parametrize("leaf", [64, 16])
def test_fd_sized_fp64_adjoint_matches_oracle(oracle_mod, leaf):
    n = 1000
    pos, q = inputs.particles(n, 5)
    w = inputs.weights(n, 5)
    gq_o, gx_o, a = oracle_mod.fmm_grad(pos, q, w, 8, leaf)
    _, _, gq, gx = grads(pos, q, w, 8, leaf, "fp64")
    assert a["level"] in (2, 3)
    assert rel_l2(gq, gq_o) < 1e-10
    assert rel_l2(gx, gx_o) < 1e-10


def test_dot_product_and_symmetric_cases():
    pos, q = inputs.particles(30_000, 40)
    w = inputs.weights(30_000, 40)
    phi_q, E_q, gq, gx = grads(pos, q, w, 8, 32, "fp64")
    # <w, A q> == <A^T w, q>
    lhs = float(w @ phi_q)
    rhs = float(gq @ q)
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(w) @ np.abs(phi_q))
    # w = q held fixed: dL/dq = A^T q = A q = phi (A symmetric), dL/dx = -2 q E
    _, _, gq2, gx2 = grads(pos, q, q, 8, 32, "fp64")
    assert rel_l2(gq2, phi_q) < 1e-12
    assert rel_l2(gx2, -2 * q[:, None] * E_q) < 1e-12


def test_c5_mixed_vs_fp64_and_direct(oracle_mod):
    """N = 1e6, p = 8, leaf <= 64: mixed adjoint against the FP64 adjoint and
    the analytic direct-sum gradient on sampled particles.

    Both gradients are held to the plain 1e-6 budget.  Rounding errors scale
    with the sums of the magnitudes of the terms, and the weights w are
    zero-mean, so each gradient's own cancellation factor is printed beside
    its error (they would justify a looser bar; none is needed):
      dL/dq = phi_w, the potential of w:
          kappa_q = ||phi_|w| || / ||dL/dq||            (about 510)
      dL/dx = -(w E_q + q E_w), componentwise:
          kappa_x = || |w| |E_|q|| + |q| |E_|w|| || / ||dL/dx||   (about 1.7)
    (phi_|w|, E_|w|: the FP64 FMM with charges |w|; E_|q| likewise)."""
    wl = inputs.WORKLOADS["C5"]
    pos, q = inputs.workload("C5")
    w = inputs.weights(wl.n, wl.seed)
    _, _, gq64, gx64 = grads(pos, q, w, wl.p, wl.leaf_max, "fp64")
    _, _, gqb, gxb = grads(pos, q, w, wl.p, wl.leaf_max, "mixed", m2l_fp16=False)
    print("C5 mixed (bf16 x3 M2L) vs FP64: dL/dq %.3e, dL/dx %.3e" % (rel_l2(gqb, gq64), rel_l2(gxb, gx64)))
    assert rel_l2(gqb, gq64) < 1e-6
    assert rel_l2(gxb, gx64) < 1e-6
    _, _, gqm, gxm = grads(pos, q, w, wl.p, wl.leaf_max, "mixed")
    phi_aw, E_aw, _, _ = grads(pos, np.abs(w), w, wl.p, wl.leaf_max, "fp64")
    _, E_aq, _, _ = grads(pos, np.abs(q), w, wl.p, wl.leaf_max, "fp64")
    kappa_q = max(1.0, np.linalg.norm(phi_aw) / np.linalg.norm(gq64))
    scale_x = np.abs(w)[:, None] * np.abs(E_aq) + np.abs(q)[:, None] * np.abs(E_aw)
    kappa_x = max(1.0, np.linalg.norm(scale_x) / np.linalg.norm(gx64))
    e_q, e_x = rel_l2(gqm, gq64), rel_l2(gxm, gx64)
    print("C5 mixed vs FP64: dL/dq %.3e (kappa_q %.1f), dL/dx %.3e (kappa_x %.2f)"
          % (e_q, kappa_q, e_x, kappa_x))
    assert e_q < 1e-6
    assert e_x < 1e-6
    t = inputs.targets(wl.n, wl.seed, 300)
    phw, Ew = oracle_mod.direct(pos, w, t)
    phq, Eq = oracle_mod.direct(pos, q, t)
    gx_d = -(w[t, None] * Eq + q[t, None] * Ew)
    # against the analytic gradient the error is the FMM truncation error of
    # p = 8, which the oracle FMM shows on the same samples
    ow = oracle_mod.fmm(pos, w, wl.p, wl.leaf_max, targets=t)
    oq = oracle_mod.fmm(pos, q, wl.p, wl.leaf_max, targets=t)
    eps_q = rel_l2(ow["phi"], phw)
    eps_x = rel_l2(-(w[t, None] * oq["E"] + q[t, None] * ow["E"]), gx_d)
    print("C5 vs direct-sum gradient: FP64 dL/dq %.3e dL/dx %.3e, mixed dL/dq %.3e dL/dx %.3e, "
          "oracle FMM %.3e %.3e" % (rel_l2(gq64[t], phw), rel_l2(gx64[t], gx_d), rel_l2(gqm[t], phw),
                                    rel_l2(gxm[t], gx_d), eps_q, eps_x))
    assert rel_l2(gq64[t], phw) < 1.01 * eps_q + 1e-12
    assert rel_l2(gx64[t], gx_d) < 1.01 * eps_x + 1e-12


def test_autograd_function():
    pos, q = inputs.particles(20_000, 41)
    w = inputs.weights(20_000, 41)
    P = dev(pos).requires_grad_(True)
    Q = dev(q).requires_grad_(True)
    phi = fmm.potential(P, Q, p=6, leaf_max=32, precision="fp64")
    loss = (dev(w) * phi).sum()
    loss.backward()
    _, _, gq, gx = grads(pos, q, w, 6, 32, "fp64")
    assert np.array_equal(Q.grad.cpu().numpy(), gq)
    assert np.array_equal(P.grad.cpu().numpy(), gx)
