"""CPU oracle for the Laplace FMM -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 reference written from the paper (Yokota & Barba,
arXiv:1106.2176): an O(N^2) direct sum and a Cartesian-Taylor FMM that follows
the paper's operator sequence (P2M, M2M, M2L, L2L, L2P, P2P; Fig. 1 and
Fig. 3).  Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg
may import it.  It shares no code with the GPU library.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        v = ctypes.c_void_p
        lib.oracle_direct.argtypes = [ctypes.c_int64, v, v, ctypes.c_int64, v, v, v]
        lib.oracle_fmm.argtypes = [ctypes.c_int64, v, v, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   v, ctypes.c_double, ctypes.c_int64, v, v, v, v, v, v]
        lib.oracle_select_level.argtypes = [ctypes.c_int64, v, ctypes.c_int, ctypes.c_int, v,
                                            ctypes.c_double, v, v]
        lib.oracle_tree.argtypes = [ctypes.c_int64, v, ctypes.c_int, v, ctypes.c_double, v, v, v]
        lib.oracle_taylor_coeffs.argtypes = [ctypes.c_int, v, v]
        lib.oracle_mindex.argtypes = [ctypes.c_int, v]
        lib.oracle_p2m.argtypes = [ctypes.c_int, ctypes.c_int64, v, v, v, v]
        lib.oracle_m2m.argtypes = [ctypes.c_int, v, v, v, v]
        lib.oracle_m2l.argtypes = [ctypes.c_int, v, v, v, v]
        lib.oracle_l2l.argtypes = [ctypes.c_int, v, v, v, v]
        lib.oracle_l2p.argtypes = [ctypes.c_int, v, v, ctypes.c_int64, v, v, v]
        lib.oracle_m_eval.argtypes = [ctypes.c_int, v, v, ctypes.c_int64, v, v]
        lib.oracle_num_threads.argtypes = []
        lib.oracle_adaptive_sizes.argtypes = [ctypes.c_int64, v, ctypes.c_int, ctypes.c_int, v,
                                              ctypes.c_double, v]
        lib.oracle_adaptive_lists.argtypes = [ctypes.c_int64, v, ctypes.c_int, ctypes.c_int, v,
                                              ctypes.c_double, v, v, v, v]
        lib.oracle_fmm_adaptive.argtypes = [ctypes.c_int64, v, v, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, v, ctypes.c_double, v, v, v, v, v]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(rc):
    if rc != 0:
        raise OracleError({1: "invalid argument", 2: "position outside the domain",
                           3: "out of memory"}.get(rc, "error %d" % rc))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def ncoef(p: int) -> int:
    """Cartesian coefficients with total degree < p."""
    return p * (p + 1) * (p + 2) // 6


def multi_indices(D: int) -> np.ndarray:
    """Multi-indices with |k| <= D in the oracle's order, shape [n, 3]."""
    n = (D + 1) * (D + 2) * (D + 3) // 6
    out = np.zeros((n, 3), dtype=np.int32)
    _check(_load().oracle_mindex(D, _ptr(out)))
    return out


def taylor_coeffs(D: int, x) -> np.ndarray:
    """t_k = D^k(1/|x|)/k! for |k| <= D (order of multi_indices(D))."""
    x = _f64(x, (3,))
    out = np.zeros((D + 1) * (D + 2) * (D + 3) // 6)
    _check(_load().oracle_taylor_coeffs(D, _ptr(x), _ptr(out)))
    return out


def direct(pos, q, targets=None):
    """Exact FP64 potential and field at targets (all particles if None)."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = pos.shape[0]
    if targets is None:
        nt, tptr = n, None
        t = None
    else:
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tptr = t.shape[0], _ptr(t)
    phi = np.zeros(nt)
    E = np.zeros((nt, 3))
    _check(_load().oracle_direct(n, _ptr(pos), _ptr(q), nt, tptr, _ptr(phi), _ptr(E)))
    return phi, E


def select_level(pos, leaf_max, max_level=10, lo=(0.0, 0.0, 0.0), size=1.0):
    pos = _f64(pos, (-1, 3))
    lo = _f64(lo, (3,))
    lev = ctypes.c_int(0)
    mx = ctypes.c_int64(0)
    _check(_load().oracle_select_level(pos.shape[0], _ptr(pos), leaf_max, max_level, _ptr(lo),
                                       size, ctypes.addressof(lev), ctypes.addressof(mx)))
    return lev.value, mx.value


def tree(pos, level, lo=(0.0, 0.0, 0.0), size=1.0):
    """Morton keys, leaf_start[8^level+1] and the stable sort permutation."""
    pos = _f64(pos, (-1, 3))
    lo = _f64(lo, (3,))
    n = pos.shape[0]
    keys = np.zeros(n, dtype=np.uint64)
    leaf_start = np.zeros(8 ** level + 1, dtype=np.int64)
    perm = np.zeros(n, dtype=np.int64)
    _check(_load().oracle_tree(n, _ptr(pos), level, _ptr(lo), size, _ptr(keys),
                               _ptr(leaf_start), _ptr(perm)))
    return keys, leaf_start, perm


def fmm(pos, q, p, leaf_max, max_level=10, lo=(0.0, 0.0, 0.0), size=1.0, targets=None):
    """FP64 FMM.  Returns dict with phi, E (total), near/far parts and level."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    lo = _f64(lo, (3,))
    n = pos.shape[0]
    if targets is None:
        nt, tptr = n, None
    else:
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tptr = t.shape[0], _ptr(t)
    pn = np.zeros(nt)
    en = np.zeros((nt, 3))
    pf = np.zeros(nt)
    ef = np.zeros((nt, 3))
    lev = ctypes.c_int(0)
    _check(_load().oracle_fmm(n, _ptr(pos), _ptr(q), p, leaf_max, max_level, _ptr(lo), size, nt,
                              tptr, _ptr(pn), _ptr(en), _ptr(pf), _ptr(ef),
                              ctypes.addressof(lev)))
    return {"phi": pn + pf, "E": en + ef, "phi_near": pn, "E_near": en, "phi_far": pf,
            "E_far": ef, "level": lev.value}


def p2m(p, pos, q, c):
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    c = _f64(c, (3,))
    M = np.zeros(ncoef(p))
    _check(_load().oracle_p2m(p, pos.shape[0], _ptr(pos), _ptr(q), _ptr(c), _ptr(M)))
    return M


def m2m(p, M, c1, c2):
    M = _f64(M)
    out = np.zeros(ncoef(p))
    _check(_load().oracle_m2m(p, _ptr(M), _ptr(_f64(c1, (3,))), _ptr(_f64(c2, (3,))), _ptr(out)))
    return out


def m2l(p, M, cs, ct):
    M = _f64(M)
    out = np.zeros(ncoef(p))
    _check(_load().oracle_m2l(p, _ptr(M), _ptr(_f64(cs, (3,))), _ptr(_f64(ct, (3,))), _ptr(out)))
    return out


def l2l(p, L, c1, c2):
    L = _f64(L)
    out = np.zeros(ncoef(p))
    _check(_load().oracle_l2l(p, _ptr(L), _ptr(_f64(c1, (3,))), _ptr(_f64(c2, (3,))), _ptr(out)))
    return out


def l2p(p, L, c, x):
    L = _f64(L)
    x = _f64(x, (-1, 3))
    phi = np.zeros(x.shape[0])
    E = np.zeros((x.shape[0], 3))
    _check(_load().oracle_l2p(p, _ptr(L), _ptr(_f64(c, (3,))), x.shape[0], _ptr(x), _ptr(phi),
                              _ptr(E)))
    return phi, E


def m_eval(p, M, c, x):
    M = _f64(M)
    x = _f64(x, (-1, 3))
    phi = np.zeros(x.shape[0])
    _check(_load().oracle_m_eval(p, _ptr(M), _ptr(_f64(c, (3,))), x.shape[0], _ptr(x), _ptr(phi)))
    return phi


def fmm_grad(pos, q, w, p, leaf_max, max_level=10, lo=(0.0, 0.0, 0.0), size=1.0):
    """Gradient of loss = sum_i w_i phi_i for the FP64 FMM.

    The FMM's far-field approximation of 1/|x_i - x_j| is the same double
    Taylor truncation for the pair (i, j) and for (j, i), so the FMM operator
    A (phi = A q) is symmetric: dL/dq = A w, the FMM potential of charges w.
    With E the exact gradient of the computed potential w.r.t. the target
    position, dL/dx_k = -(w_k E_q,k + q_k E_w,k).  (Pinned by central finite
    differences of this oracle's own loss in the tests.)
    """
    a = fmm(pos, q, p, leaf_max, max_level, lo, size)
    b = fmm(pos, w, p, leaf_max, max_level, lo, size)
    w = _f64(w)
    q = _f64(q)
    gq = b["phi"]
    gx = -(w[:, None] * a["E"] + q[:, None] * b["E"])
    return gq, gx, a


def direct_grad(pos, q, w):
    """Exact gradient of sum_i w_i phi_i for the direct sum."""
    phq, Eq = direct(pos, q)
    phw, Ew = direct(pos, w)
    w = _f64(w)
    q = _f64(q)
    return phw, -(w[:, None] * Eq + q[:, None] * Ew)


def adaptive_tree(pos, leaf_max, max_level=10, lo=(0.0, 0.0, 0.0), size=1.0):
    """The adaptive octree and its U/V/W/X lists.

    Returns a dict: boxes [nbox, 8] int64 (level, ix, iy, iz, start, end,
    parent, leaf; breadth-first, Morton order within a level, box 0 the
    root), order [n] (sorted position -> input index; every box is the range
    [start, end) of it), depth, and the lists U, V, W, X, each a Python list
    of nbox numpy arrays of box ids."""
    pos = _f64(pos, (-1, 3))
    lo = _f64(lo, (3,))
    n = pos.shape[0]
    sz = np.zeros(6, dtype=np.int64)
    L = _load()
    _check(L.oracle_adaptive_sizes(n, _ptr(pos), leaf_max, max_level, _ptr(lo), size, _ptr(sz)))
    nbox = int(sz[0])
    boxes = np.zeros((nbox, 8), dtype=np.int64)
    order = np.zeros(n, dtype=np.int64)
    starts = np.zeros(4 * (nbox + 1), dtype=np.int64)
    items = np.zeros(max(1, int(sz[1:5].sum())), dtype=np.int64)
    _check(L.oracle_adaptive_lists(n, _ptr(pos), leaf_max, max_level, _ptr(lo), size, _ptr(boxes),
                                   _ptr(order), _ptr(starts), _ptr(items)))
    out = {"boxes": boxes, "order": order, "depth": int(sz[5])}
    for w, name in enumerate("UVWX"):
        st = starts[w * (nbox + 1):(w + 1) * (nbox + 1)]
        out[name] = [items[st[b]:st[b + 1]].copy() for b in range(nbox)]
    return out


def fmm_adaptive(pos, q, p, leaf_max, max_level=10, lo=(0.0, 0.0, 0.0), size=1.0):
    """FP64 FMM on the adaptive octree (U/V/W/X lists).  Returns a dict with
    phi, E (total), the near (P2P) and far parts, and nbox, nleaf, depth."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    lo = _f64(lo, (3,))
    n = pos.shape[0]
    pn = np.zeros(n)
    en = np.zeros((n, 3))
    pf = np.zeros(n)
    ef = np.zeros((n, 3))
    info = np.zeros(3, dtype=np.int64)
    _check(_load().oracle_fmm_adaptive(n, _ptr(pos), _ptr(q), p, leaf_max, max_level, _ptr(lo), size,
                                       _ptr(pn), _ptr(en), _ptr(pf), _ptr(ef), _ptr(info)))
    return {"phi": pn + pf, "E": en + ef, "phi_near": pn, "E_near": en, "phi_far": pf,
            "E_far": ef, "nbox": int(info[0]), "nleaf": int(info[1]), "depth": int(info[2])}
