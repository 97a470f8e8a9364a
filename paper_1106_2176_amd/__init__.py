"""Laplace fast multipole method on AMD MI355X (gfx950).

Thin Python binding of ``libfmm.so`` (C ABI in ``include/fmm.h``): argument
marshalling only; every step of the evaluation runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.

Method: Yokota & Barba, "A Tuned and Scalable Fast Multipole Method as a
Preeminent Algorithm for Exascale Systems" (arXiv:1106.2176), Sec. 2.1
(problem and operators, Fig. 1 and Fig. 3), Sec. 3 (P2P and M2L as the hot
kernels), Sec. 5 (Morton-indexed uniform trees, sorted start/offset layout).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm.so")

FMM_ABI_VERSION = 1
FMM_OK, FMM_EINVAL, FMM_EDOMAIN, FMM_ENOMEM, FMM_EDEVICE, FMM_EUNSUPPORTED = range(6)
FMM_F32, FMM_F64 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
VEC_NONE, VEC_FIELD, VEC_FORCE = 0, 1, 2
PART_NEAR_ONLY, PART_FAR_ONLY = 4, 8
# default depth cap of the adaptive tree: the deepest, 10 (the build sorts
# the keys, so a deep cap costs little; on 10^7 particles in Gaussian blobs a
# cap of 8 leaves leaves far over leaf_max and takes 3x as long)
ADAPTIVE_MAX_LEVEL = 10
STAGES = ("gather", "P2M", "M2M", "pack", "M2L", "L2L", "L2P", "P2P", "combine")

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("p", ctypes.c_int32),
        ("leaf_max", ctypes.c_int32),
        ("max_level", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("bf16_splits", ctypes.c_int32),
        ("box_lo", ctypes.c_double * 3),
        ("box_size", ctypes.c_double),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
        ("profile", ctypes.c_int32),
        ("profile_stages", ctypes.c_uint32),
        ("overlap_near", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("m2l_fp16", ctypes.c_int32),
        ("m2l_rotation", ctypes.c_int32),
        ("adaptive", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1),
    ]


class TreeInfo(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("n_leaves", ctypes.c_int64),
        ("max_leaf_count", ctypes.c_int64),
        ("p2p_pairs", ctypes.c_int64),
        ("m2l_pairs", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
        ("n_boxes", ctypes.c_int64),
        ("m2p_evals", ctypes.c_int64),
        ("p2l_evals", ctypes.c_int64),
    ]


class FMMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (_STATUS.get(status, "error"), status, message))
        self.status = status


_STATUS = {1: "invalid argument", 2: "domain error", 3: "out of memory", 4: "device error",
           5: "unsupported"}

# name -> (restype, argtypes); mirrors include/fmm.h
_vp = ctypes.c_void_p
_SIGS = {
    "fmm_config_default": (None, [ctypes.POINTER(Config)]),
    "fmm_build_tree": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_int64, ctypes.c_int32, _vp, _vp,
                                      ctypes.POINTER(_vp)]),
    "fmm_evaluate": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp]),
    "fmm_evaluate_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp]),
    "fmm_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fmm_tree_info": (ctypes.c_int, [_vp, ctypes.POINTER(TreeInfo)]),
    "fmm_stage_times": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
    "fmm_stage_times_reset": (ctypes.c_int, [_vp]),
    "fmm_tree_export": (ctypes.c_int, [_vp, _vp, _vp]),
    "fmm_tree_export_adaptive": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fmm_tree_destroy": (None, [_vp]),
    "fmm_operator_host": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp]),
    "fmm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fmm_last_error_message": (ctypes.c_char_p, []),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """The loaded native library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfmm.so is not built (run __graft_entry__.build() or "
                               "python paper_1106_2176_amd/build_native.py); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != FMM_OK:
        msg = lib().fmm_last_error_message()
        raise FMMError(rc, msg.decode() if msg else "")


# Workspace memory through torch's caching allocator: the library asks for
# device memory with these callbacks (stream-ordered on the call's stream), so
# torch sees, reuses and can release it.  One pair for the whole process: a
# tree must be rebuilt with the allocator it was created with, which these
# fixed pointers guarantee.
_ALLOC_CB = None


def _torch_alloc(nbytes, stream, ctx):
    torch = _torch()
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  int(stream or 0))
    except Exception:  # out of memory (or no device): reported as FMM_ENOMEM
        return None


def _torch_free(ptr, stream, ctx):
    try:
        _torch().cuda.caching_allocator_delete(int(ptr))
    except Exception:  # interpreter shutdown: torch already torn down
        pass


def torch_allocator():
    """(alloc, free) ctypes callbacks backed by torch's caching allocator."""
    global _ALLOC_CB
    if _ALLOC_CB is None:
        _ALLOC_CB = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))
    return _ALLOC_CB


def make_config(p=8, leaf_max=64, precision="mixed", max_level=None, bf16_splits=3,
                box_lo=(0.0, 0.0, 0.0), box_size=1.0, profile=False, overlap_near=False,
                graph=False, profile_stages=None, allocator="torch", m2l_fp16=None,
                m2l_rotation=False, adaptive=False):
    """profile_stages: None (all) or an iterable of stage names (STAGES) whose
    boundaries get profiling events.  allocator: "torch" (workspace from
    torch's caching allocator), "library" (the library's own stream-ordered
    hipMallocAsync pool) or an (alloc, free) pair of ctypes callbacks.
    m2l_fp16: None (the library's default), True (the mixed M2L in two
    binary16 parts) or False (bf16_splits bf16 parts).  m2l_rotation: the
    FP64 form's M2L by rotation (O(p^3) per pair).  adaptive: the adaptive
    octree with U/V/W/X lists; max_level None selects 10 for the uniform
    tree and ADAPTIVE_MAX_LEVEL for the adaptive one."""
    c = Config()
    lib().fmm_config_default(ctypes.byref(c))
    c.p = int(p)
    c.leaf_max = int(leaf_max)
    if max_level is None:
        max_level = ADAPTIVE_MAX_LEVEL if adaptive else 10
    c.max_level = int(max_level)
    c.adaptive = 1 if adaptive else 0
    c.precision = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[precision] if isinstance(precision, str) \
        else int(precision)
    c.bf16_splits = int(bf16_splits)
    for a in range(3):
        c.box_lo[a] = float(box_lo[a])
    c.box_size = float(box_size)
    c.profile = 1 if profile else 0
    c.overlap_near = 1 if overlap_near else 0
    c.graph = 1 if graph else 0
    c.profile_stages = 0 if profile_stages is None else \
        sum(1 << STAGES.index(s) for s in profile_stages)
    if m2l_fp16 is not None:
        c.m2l_fp16 = 1 if m2l_fp16 else 0
    c.m2l_rotation = 1 if m2l_rotation else 0
    if allocator == "torch":
        c.alloc, c.free = torch_allocator()
    elif allocator != "library":
        c.alloc, c.free = allocator
    return c


def operator_host(p, kind, index):
    """Host FP64 translation operator (see fmm_operator_host), shape [p^2, p^2]."""
    out = np.zeros((p * p, p * p))
    _check(lib().fmm_operator_host(int(p), int(kind), int(index), out.ctypes.data_as(_vp)))
    return out


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return FMM_F64
    if t.dtype == torch.float32:
        return FMM_F32
    raise ValueError("positions/charges must be float32 or float64, got %s" % t.dtype)


def _check_tensor(t, name, shape, dtype):
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class Tree:
    """An octree built on the GPU; owns library memory until close().

    With allocator="torch" (the default) the tree's workspace is taken from
    torch's caching allocator on the stream current at the call that grows
    it, and given back to it by close(); as with any memory torch hands out
    for one stream, use the tree on streams ordered after that one.

    graph=True replays a HIP graph of the evaluate/backward chain; it is reused
    while the output tensors passed in (phi, out_vec, gradients) and the
    tree's memory stay the same, so pass preallocated outputs."""

    def __init__(self, pos, p=8, leaf_max=64, precision="mixed", max_level=None, bf16_splits=3,
                 box_lo=(0.0, 0.0, 0.0), box_size=1.0, profile=False, overlap_near=False,
                 graph=False, profile_stages=None, allocator="torch", m2l_fp16=None,
                 m2l_rotation=False, adaptive=False):
        self._h = ctypes.c_void_p(None)
        self.cfg = make_config(p, leaf_max, precision, max_level, bf16_splits, box_lo, box_size,
                               profile, overlap_near, graph, profile_stages, allocator, m2l_fp16,
                               m2l_rotation, adaptive)
        # the callback objects must outlive every call that can allocate or
        # free (the torch pair is held by the module)
        self._allocator = allocator
        self.rebuild(pos)

    def rebuild(self, pos):
        """Rebuild in place for new positions (same dtype), reusing memory."""
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("pos must have shape [n, 3]")
        self.dtype = pos.dtype
        self.n = int(pos.shape[0])
        _check_tensor(pos, "pos", (self.n, 3), pos.dtype)
        code = _dtype_code(pos)
        _check(lib().fmm_build_tree(ctypes.byref(self.cfg), self.n, code, _dptr(pos), _stream_ptr(),
                                    ctypes.byref(self._h)))
        return self

    def evaluate(self, q, vec="field", phi=None, out_vec=None, part=None):
        """phi [n] and the field E (vec='field'), force q E (vec='force') or None.
        part: None (near + far), 'near' or 'far' (one part only)."""
        torch = _torch()
        _check_tensor(q, "q", (self.n,), self.dtype)
        if phi is None:
            phi = torch.empty(self.n, dtype=self.dtype, device=q.device)
        flags = {None: VEC_NONE, "field": VEC_FIELD, "force": VEC_FORCE}[vec]
        if flags != VEC_NONE and out_vec is None:
            out_vec = torch.empty(self.n, 3, dtype=self.dtype, device=q.device)
        pf = {None: 0, "near": PART_NEAR_ONLY, "far": PART_FAR_ONLY}[part]
        _check(lib().fmm_evaluate(self._h, _dptr(q), _dptr(phi), _dptr(out_vec) if flags else None,
                                  flags | pf, _stream_ptr()))
        return phi, (out_vec if flags else None)

    def backward(self, q, w, field, grad_q=True, grad_pos=True, out_q=None, out_pos=None):
        """(dLoss/dq, dLoss/dpos) for Loss = sum w phi; out_q / out_pos are
        optional preallocated outputs."""
        torch = _torch()
        _check_tensor(q, "q", (self.n,), self.dtype)
        _check_tensor(w, "w", (self.n,), self.dtype)
        gq = gx = None
        if grad_q:
            gq = out_q if out_q is not None else torch.empty(self.n, dtype=self.dtype, device=q.device)
            _check_tensor(gq, "out_q", (self.n,), self.dtype)
        if grad_pos:
            gx = out_pos if out_pos is not None else \
                torch.empty(self.n, 3, dtype=self.dtype, device=q.device)
            _check_tensor(gx, "out_pos", (self.n, 3), self.dtype)
        if grad_pos:
            _check_tensor(field, "field", (self.n, 3), self.dtype)
        _check(lib().fmm_backward(self._h, _dptr(q), _dptr(w), _dptr(field) if field is not None else None,
                                  _dptr(gq), _dptr(gx), _stream_ptr()))
        return gq, gx

    def info(self):
        i = TreeInfo()
        _check(lib().fmm_tree_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in TreeInfo._fields_}

    def stage_times(self):
        """Mean stage times (ms) over the last min(calls, 32) profiled calls."""
        ms = (ctypes.c_double * len(STAGES))()
        _check(lib().fmm_stage_times(self._h, ms, len(STAGES)))
        return dict(zip(STAGES, list(ms)))

    def stage_times_reset(self):
        _check(lib().fmm_stage_times_reset(self._h))

    def export(self):
        """(perm [n], leaf_start [n_leaves + 1]) as numpy uint32 (synchronous);
        uniform tree: n_leaves = 8^L in Morton order; adaptive tree: its
        leaves in particle order."""
        nl = self.info()["n_leaves"]
        perm = np.zeros(self.n, dtype=np.uint32)
        start = np.zeros(nl + 1, dtype=np.uint32)
        _check(lib().fmm_tree_export(self._h, perm.ctypes.data_as(_vp), start.ctypes.data_as(_vp)))
        return perm, start

    def export_adaptive(self):
        """An adaptive tree's boxes and lists (synchronous): a dict with
        boxes [nbox, 8] int64 (level, ix, iy, iz, start, end, parent, leaf),
        order [n] (sorted position -> input index), depth, and U, V, W, X,
        each a list of nbox numpy arrays of box ids."""
        L = lib()
        sz = np.zeros(6, dtype=np.int64)
        _check(L.fmm_tree_export_adaptive(self._h, sz.ctypes.data_as(_vp), None, None, None, None))
        nbox = int(sz[0])
        boxes = np.zeros((nbox, 8), dtype=np.int32)
        perm = np.zeros(self.n, dtype=np.uint32)
        starts = np.zeros(4 * (nbox + 1), dtype=np.int64)
        items = np.zeros(max(1, int(sz[1:5].sum())), dtype=np.int32)
        _check(L.fmm_tree_export_adaptive(self._h, sz.ctypes.data_as(_vp), boxes.ctypes.data_as(_vp),
                                          perm.ctypes.data_as(_vp), starts.ctypes.data_as(_vp),
                                          items.ctypes.data_as(_vp)))
        out = {"boxes": boxes.astype(np.int64), "order": perm.astype(np.int64), "depth": int(sz[5])}
        at = 0
        for k, name in enumerate("UVWX"):
            st = starts[k * (nbox + 1):(k + 1) * (nbox + 1)] + at
            out[name] = [items[st[b]:st[b + 1]].astype(np.int64) for b in range(nbox)]
            at += int(sz[1 + k])
        return out

    def close(self):
        if self._h:
            lib().fmm_tree_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def evaluate(pos, q, p=8, leaf_max=64, precision="mixed", vec="field", **kw):
    """Build a tree and evaluate potentials (and field/force) in one call."""
    with Tree(pos, p=p, leaf_max=leaf_max, precision=precision, **kw) as t:
        return t.evaluate(q, vec=vec)


def _autograd_function():
    torch = _torch()

    class FMMPotential(torch.autograd.Function):
        """phi = FMM(pos, q); backward through the hand-written adjoint kernels.
        The tree is rebuilt in backward rather than stored."""

        @staticmethod
        def forward(ctx, pos, q, kw):
            with Tree(pos.detach(), **kw) as t:
                phi, E = t.evaluate(q.detach(), vec="field")
            ctx.save_for_backward(pos, q, E)
            ctx.kw = kw
            return phi

        @staticmethod
        def backward(ctx, w):
            pos, q, E = ctx.saved_tensors
            need_x, need_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            with Tree(pos.detach(), **ctx.kw) as t:
                gq, gx = t.backward(q.detach(), w.contiguous(), E, grad_q=need_q, grad_pos=need_x)
            return gx, gq, None

    return FMMPotential


_FMMPotential = None


def potential(pos, q, p=8, leaf_max=64, precision="mixed", **kw):
    """Differentiable potential phi(pos, q) (gradients w.r.t. pos and q)."""
    global _FMMPotential
    if _FMMPotential is None:
        _FMMPotential = _autograd_function()
    kw = dict(kw, p=p, leaf_max=leaf_max, precision=precision)
    return _FMMPotential.apply(pos, q, kw)
