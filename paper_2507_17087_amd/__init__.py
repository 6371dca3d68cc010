"""Python binding of libtaskmap (exact batched evaluation of index-task mappings
on MI355X).  Argument marshalling only: every step runs in the HIP library.

The functions carry the names of the C entry points declared in
include/taskmap.h.  Candidate arrays are numpy structured arrays with the
tm_candidate layout (TM_CANDIDATE_DTYPE, 328 bytes per record); device buffers are
torch tensors on the current HIP device; work is enqueued on torch's current
stream.  A missing or unloadable library raises TaskmapError: there is no fallback.
"""
import ctypes
import os

import numpy as np

from . import _ranker_api  # ctypes signatures of the ranker and search entry points

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtaskmap.so")

TM_OK, TM_EINVAL, TM_EOVERFLOW, TM_ECAPACITY, TM_ENOMEM, TM_EDEVICE, TM_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
TM_SPLIT, TM_MERGE, TM_SWAP, TM_BALANCE_SPLIT, TM_DECOMPOSE = 1, 2, 3, 4, 5
TM_BLOCK, TM_CYCLIC = 0, 1

_OP = np.dtype([("kind", "<i4"), ("a", "<i4"), ("b", "<i4"), ("nf", "<i4"), ("f", "<i4", (4,))])
TM_CANDIDATE_DTYPE = np.dtype([("lrank", "<i4"), ("nodes", "<i4"), ("gpus", "<i4"), ("nops", "<i4"),
                               ("extent", "<i8", (4,)), ("ops", _OP, (8,)), ("mrank", "<i4"),
                               ("pad0", "<i4"), ("proj_src", "i1", (8,)), ("proj_mode", "i1", (8,))])
TM_STENCIL_DTYPE = np.dtype([("lrank", "<i4"), ("elem_bytes", "<i4"), ("halo", "<i4", (4,))])
assert TM_CANDIDATE_DTYPE.itemsize == 328 and TM_STENCIL_DTYPE.itemsize == 24


class TaskmapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"taskmap error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libtaskmap.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TaskmapError(TM_ENOTSUP, f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "tm_abi_version": [], "tm_candidate_size": [],
            "tm_validate": [P, P, P],
            "tm_enumerate_factorizations": [I64, I32, P, I64, P],
            "tm_decompose_argmin": [I64, I32, P, P, P],
            "tm_decompose_argmin_transpose": [I64, I32, P, P, I32, P],
            "tm_greedy_grid": [I64, I32, P],
            "tm_workload_greedy": [I64, I32, P, P],
            "tm_chain_table": [P, P, I64, P, P],
            "tm_proc_map": [P, P, I64, P],
            "tm_eval_stencil_batch": [P, I64, P, P, P],
            "tm_eval_stencil_node_batch": [P, I64, P, P, P],
            "tm_eval_stencil_batch_noalloc": [P, I64, P, P, P],
            "tm_eval_redistribution_batch": [P, P, I64, I64, P, P],
            "tm_transpose_target": [P, I32, I32, P],
            "tm_eval_matmul_batch": [P, I64, P, P, P, P],
            "tm_select_best": [P, P, I64, P, P],
            "tm_plan_create": [I64, I64, P],
            "tm_plan_load": [P, P, I64, P, I64, P],
            "tm_plan_run": [P, P, P, P],
            "tm_plan_run_stage": [P, I32, P, P, P],
            "tm_plan_materialize": [P, P, I64, P, I64, P],
            "tm_plan_run_map": [P, P, P, P, I64, P],
            "tm_plan_autotune": [P, P, P, P, P],
            "tm_parse_index_task_map": [ctypes.c_char_p, ctypes.c_char_p, I32, P, I32, I32, P, P],
            "tm_plan_set_launch": [P, I64, I32, P],
            "tm_plan_info": [P, P, P, P],
            "tm_plan_class_tuples": [P, P, P],
            "tm_plan_destroy": [P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.tm_last_error.restype = ctypes.c_char_p
        L.tm_last_error.argtypes = []
        if L.tm_candidate_size() != TM_CANDIDATE_DTYPE.itemsize:
            raise TaskmapError(TM_EINVAL, "tm_candidate layout mismatch")
        _ranker_api.declare(L)
        _lib = L
    return _lib


def _check(rc):
    if rc != TM_OK:
        raise TaskmapError(rc, lib().tm_last_error().decode(errors="replace"))


def _cands(c):
    a = np.ascontiguousarray(c)
    if a.dtype.itemsize != TM_CANDIDATE_DTYPE.itemsize:
        raise TaskmapError(TM_EINVAL, "candidate records must have the tm_candidate layout")
    return a.reshape(-1) if a.ndim == 0 else a


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TaskmapError(TM_EINVAL, f"expected a contiguous CUDA {dtype} tensor")
    if numel is not None and t.numel() < numel:
        raise TaskmapError(TM_ECAPACITY, f"tensor holds {t.numel()} elements, {numel} needed")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- host calls

def tm_abi_version():
    return lib().tm_abi_version()


def tm_validate(c):
    """(code, final_shape or None) -- does not raise on invalid descriptors."""
    a = _cands(c)
    shape = np.zeros(8, np.int32)
    r = ctypes.c_int32(0)
    rc = lib().tm_validate(a.ctypes.data, shape.ctypes.data, ctypes.byref(r))
    return rc, (tuple(int(x) for x in shape[: r.value]) if rc == TM_OK else None)


def tm_enumerate_factorizations(P, k):
    cnt = ctypes.c_int64(0)
    rc = lib().tm_enumerate_factorizations(P, k, None, 0, ctypes.byref(cnt))
    if rc not in (TM_OK, TM_ECAPACITY):
        _check(rc)
    out = np.zeros((max(cnt.value, 1), k), np.int32)
    _check(lib().tm_enumerate_factorizations(P, k, out.ctypes.data, cnt.value, ctypes.byref(cnt)))
    return [tuple(int(x) for x in r) for r in out[: cnt.value]]


def tm_decompose_argmin(P, extent, halo=None):
    k = len(extent)
    ext = np.array(list(extent) + [1] * (4 - k), np.int64)
    h = np.array(list(halo if halo is not None else [1] * k) + [0] * (4 - k), np.int32)
    out = np.zeros(4, np.int32)
    _check(lib().tm_decompose_argmin(P, k, ext.ctypes.data, h.ctypes.data, out.ctypes.data))
    return tuple(int(x) for x in out[:k])


def tm_decompose_argmin_transpose(P, extent, halo=None, transpose=()):
    """decompose's argmin with all-to-all transposes along the dims in `transpose`."""
    k = len(extent)
    ext = np.array(list(extent) + [1] * (4 - k), np.int64)
    h = np.array(list(halo if halo is not None else [1] * k) + [0] * (4 - k), np.int32)
    mask = sum(1 << int(d) for d in set(transpose))
    out = np.zeros(4, np.int32)
    _check(lib().tm_decompose_argmin_transpose(P, k, ext.ctypes.data, h.ctypes.data, mask, out.ctypes.data))
    return tuple(int(x) for x in out[:k])


def tm_transpose_target(c, dim, into):
    """The pencil-transposed image of candidate c for an all-to-all transpose along
    launch dim `dim`, split along launch dim `into` (one TM_CANDIDATE_DTYPE record)."""
    a = _cands(c)
    if len(a) != 1:
        raise TaskmapError(TM_EINVAL, "one candidate expected")
    out = np.zeros((), dtype=TM_CANDIDATE_DTYPE)
    _check(lib().tm_transpose_target(a.ctypes.data, int(dim), int(into), out.ctypes.data))
    return out


def tm_greedy_grid(P, k):
    out = np.zeros(4, np.int32)
    _check(lib().tm_greedy_grid(P, k, out.ctypes.data))
    return tuple(int(x) for x in out[:k])


def tm_workload_greedy(P, extent):
    k = len(extent)
    ext = np.array(list(extent) + [1] * (4 - k), np.int64)
    out = np.zeros(4, np.int32)
    _check(lib().tm_workload_greedy(P, k, ext.ctypes.data, out.ctypes.data))
    return tuple(int(x) for x in out[:k])


# ---------------------------------------------------------------- device calls

def tm_parse_index_task_map(source, task, extent, nodes, gpus, halo=None):
    """One candidate record (TM_CANDIDATE_DTYPE) from the IndexTaskMap mapper of
    `task` in a mapping-language program."""
    k = len(extent)
    ext = np.array(list(extent) + [1] * (4 - k), np.int64)
    h = None if halo is None else np.array(list(halo) + [0] * (4 - k), np.int32)
    out = np.zeros((), dtype=TM_CANDIDATE_DTYPE)
    _check(lib().tm_parse_index_task_map(source.encode(), task.encode(), k, ext.ctypes.data, nodes, gpus,
                                         None if h is None else h.ctypes.data, out.ctypes.data))
    return out


def tm_chain_table(c, out=None):
    import torch
    a = _cands(c)
    cnt = ctypes.c_int64(0)
    rc = lib().tm_chain_table(a.ctypes.data, None, 0, ctypes.byref(cnt), _stream())
    if rc != TM_ECAPACITY:
        _check(rc)
    if out is None:
        out = torch.empty(cnt.value, dtype=torch.int32, device="cuda")
    _check(lib().tm_chain_table(a.ctypes.data, _dev_ptr(out, torch.int32, cnt.value), out.numel(),
                                ctypes.byref(cnt), _stream()))
    return out[: cnt.value]


def n_points(c):
    return int(np.prod([int(x) for x in c["extent"][: int(c["lrank"])]]))


def tm_proc_map(c, out=None):
    """int32 processor id of every launch point (C order), shaped like the domain."""
    import torch
    a = _cands(c)
    n = n_points(a[0])
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(lib().tm_proc_map(a.ctypes.data, _dev_ptr(out, torch.int32, n), n, _stream()))
    return out.view([int(x) for x in a[0]["extent"][: int(a[0]["lrank"])]])


def stencil(halo, elem_bytes=8):
    st = np.zeros((), dtype=TM_STENCIL_DTYPE)
    st["lrank"] = len(halo)
    st["elem_bytes"] = elem_bytes
    for d, h in enumerate(halo):
        st["halo"][d] = h
    return st


def _st(st):
    s = np.ascontiguousarray(st)
    if s.dtype.itemsize != TM_STENCIL_DTYPE.itemsize:
        raise TaskmapError(TM_EINVAL, "stencil must have the tm_stencil layout")
    return s


def tm_eval_stencil_batch(c, st, out=None):
    """int64 [n,4] device tensor: ghost_cells, inter_cells, bytes, inter_bytes."""
    import torch
    a = _cands(c)
    s = _st(st)
    n = len(a)
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int64, device="cuda")
    _check(lib().tm_eval_stencil_batch(a.ctypes.data, n, s.ctypes.data, _dev_ptr(out, torch.int64, 4 * n),
                                       _stream()))
    return out


def tm_eval_stencil_batch_noalloc(c, st, out):
    """tm_eval_stencil_batch through the entry point that allocates no device memory:
    `out` (int64 [n,4] device tensor) is required."""
    import torch
    a = _cands(c)
    s = _st(st)
    n = len(a)
    _check(lib().tm_eval_stencil_batch_noalloc(a.ctypes.data, n, s.ctypes.data, _dev_ptr(out, torch.int64, 4 * n),
                                               _stream()))
    return out


def tm_eval_stencil_node_batch(c, st, out=None):
    """int64 [n,4] device tensor: node-level exchange cells (twice), bytes (twice)."""
    import torch
    a = _cands(c)
    s = _st(st)
    n = len(a)
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int64, device="cuda")
    _check(lib().tm_eval_stencil_node_batch(a.ctypes.data, n, s.ctypes.data, _dev_ptr(out, torch.int64, 4 * n),
                                            _stream()))
    return out


def tm_eval_redistribution_batch(src, dst, elem_bytes=8, out=None):
    """int64 [n,4] device tensor per pair (src[i], dst[i]): moved cells, inter-node
    moved cells, bytes, inter-node bytes."""
    import torch
    a, b = _cands(src), _cands(dst)
    if len(a) != len(b):
        raise TaskmapError(TM_EINVAL, "src and dst differ in length")
    n = len(a)
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int64, device="cuda")
    _check(lib().tm_eval_redistribution_batch(a.ctypes.data, b.ctypes.data, n, int(elem_bytes),
                                              _dev_ptr(out, torch.int64, 4 * n), _stream()))
    return out


def tm_eval_matmul_batch(c, tile_bytes, per_proc=True):
    """(per_proc int64 [sum P, 3] or None, cost int64 [n, 7]) device tensors."""
    import torch
    a = _cands(c)
    n = len(a)
    mm = np.array([tile_bytes], np.int64)
    out = torch.empty((n, 7), dtype=torch.int64, device="cuda")
    pp = None
    if per_proc:
        P = int(sum(int(x["nodes"]) * int(x["gpus"]) for x in a))
        pp = torch.empty((max(P, 1), 3), dtype=torch.int64, device="cuda")
    _check(lib().tm_eval_matmul_batch(a.ctypes.data, n, mm.ctypes.data,
                                      _dev_ptr(pp, torch.int64) if pp is not None else None,
                                      _dev_ptr(out, torch.int64, 7 * n), _stream()))
    return pp, out


def tm_select_best(costs, seg):
    """Per segment [seg[s], seg[s+1]) of a [n,4] cost tensor: index (relative to the
    segment) of the minimum (bytes, inter_bytes, index)."""
    import torch
    sg = np.ascontiguousarray(seg, dtype=np.int64)
    nseg = len(sg) - 1
    best = torch.empty(max(nseg, 1), dtype=torch.int64, device="cuda")
    _check(lib().tm_select_best(_dev_ptr(costs, torch.int64), sg.ctypes.data, nseg,
                                _dev_ptr(best, torch.int64), _stream()))
    return best[:nseg]


class Plan:
    """tm_plan: batch evaluation replayed from hipGraphs (see taskmap.h)."""

    def __init__(self, max_cands=1, max_words=1):
        self._p = ctypes.c_void_p()
        _check(lib().tm_plan_create(max_cands, max_words, ctypes.byref(self._p)))
        self.n = 0

    def load(self, c, st, cells_per_item=0):
        a = _cands(c)
        self._keep = a
        _check(lib().tm_plan_load(self._p, a.ctypes.data, len(a), _st(st).ctypes.data, cells_per_item,
                                  _stream()))
        self.n = len(a)
        return self

    def run(self, out, best=None):
        import torch
        _check(lib().tm_plan_run(self._p, _dev_ptr(out, torch.int64, 4 * self.n),
                                 _dev_ptr(best, torch.int64, 1) if best is not None else None, _stream()))

    def run_stage(self, stage, out, best=None):
        import torch
        _check(lib().tm_plan_run_stage(self._p, stage, _dev_ptr(out, torch.int64, 4 * self.n),
                                       _dev_ptr(best, torch.int64, 1) if best is not None else None,
                                       _stream()))

    def run_map(self, out, best, pmap):
        """run(out, best), then the map of the selected candidate into pmap (int32
        device tensor), as one graph."""
        import torch
        _check(lib().tm_plan_run_map(self._p, _dev_ptr(out, torch.int64, 4 * self.n), _dev_ptr(best, torch.int64, 1),
                                     _dev_ptr(pmap, torch.int32), pmap.numel(), _stream()))

    def materialize(self, out, index=None, d_index=None):
        import torch
        _check(lib().tm_plan_materialize(self._p, _dev_ptr(d_index, torch.int64) if d_index is not None else None,
                                         -1 if index is None else index, _dev_ptr(out, torch.int32), out.numel(),
                                         _stream()))

    def autotune(self, out):
        import torch
        c = ctypes.c_int64(0)
        w = ctypes.c_int32(0)
        _check(lib().tm_plan_autotune(self._p, _dev_ptr(out, torch.int64, 4 * self.n), ctypes.byref(c),
                                      ctypes.byref(w), _stream()))
        return c.value, w.value

    def set_launch(self, cells_per_item=0, wg_per_cu=0):
        _check(lib().tm_plan_set_launch(self._p, int(cells_per_item), int(wg_per_cu), _stream()))

    def info(self):
        n, it, pts = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tm_plan_info(self._p, ctypes.byref(n), ctypes.byref(it), ctypes.byref(pts)))
        return n.value, it.value, pts.value

    def class_tuples(self):
        """Class tuples the counting kernel evaluates for the loaded batch (after a run)."""
        t = ctypes.c_int64()
        _check(lib().tm_plan_class_tuples(self._p, ctypes.byref(t), _stream()))
        return t.value

    def close(self):
        if self._p:
            lib().tm_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned ranker

def tm_ranker_param_count():
    return lib().tm_ranker_param_count()


def tm_ranker_features(plan):
    """fp32 [n, 64] features of the batch loaded in `plan` (device tensor)."""
    import torch
    out = torch.empty((max(plan.n, 1), lib().tm_ranker_feature_count()), dtype=torch.float32, device="cuda")
    _check(lib().tm_ranker_features(plan._p, _dev_ptr(out, torch.float32), _stream()))
    return out[: plan.n]


def tm_ranker_block_estimates(plan):
    """fp64 [n, 2] block-model estimates (ghost cells, inter-node ghost cells) of the
    batch loaded in `plan` (device tensor)."""
    import torch
    out = torch.empty((max(plan.n, 1), 2), dtype=torch.float64, device="cuda")
    _check(lib().tm_ranker_block_estimates(plan._p, _dev_ptr(out, torch.float64), _stream()))
    return out[: plan.n]


class Ranker:
    """tm_ranker: BF16-MFMA MLP surrogate of the exact cost (see taskmap.h)."""

    def __init__(self, seed=0, path=None):
        self._r = ctypes.c_void_p()
        if path is None:
            _check(lib().tm_ranker_create(seed, ctypes.byref(self._r)))
        else:
            _check(lib().tm_ranker_load(os.fsencode(path), ctypes.byref(self._r)))
        self.param_count = lib().tm_ranker_param_count()

    def get_params(self):
        import torch
        out = torch.empty(self.param_count, dtype=torch.float32, device="cuda")
        _check(lib().tm_ranker_get_params(self._r, _dev_ptr(out, torch.float32), _stream()))
        return out

    def set_params(self, p):
        import torch
        _check(lib().tm_ranker_set_params(self._r, _dev_ptr(p, torch.float32, self.param_count), _stream()))

    def scaling(self):
        a = (ctypes.c_float * 4)()
        _check(lib().tm_ranker_get_scaling(self._r, a))
        return tuple(a)

    def forward(self, feat):
        import torch
        n = feat.shape[0]
        out = torch.empty((max(n, 1), 2), dtype=torch.float32, device="cuda")
        _check(lib().tm_ranker_forward(self._r, _dev_ptr(feat, torch.float32), n, _dev_ptr(out, torch.float32),
                                       _stream()))
        return out[:n]

    def grad(self, feat, target):
        import torch
        g = torch.empty(self.param_count, dtype=torch.float32, device="cuda")
        _check(lib().tm_ranker_grad(self._r, _dev_ptr(feat, torch.float32), _dev_ptr(target, torch.float32),
                                    feat.shape[0], _dev_ptr(g, torch.float32), _stream()))
        return g

    def train(self, feat, costs, epochs=4, batch=4096, lr=2e-3, seed=1):
        import torch
        losses = (ctypes.c_float * max(epochs, 1))()
        _check(lib().tm_ranker_train(self._r, _dev_ptr(feat, torch.float32), _dev_ptr(costs, torch.int64),
                                     feat.shape[0], epochs, batch, lr, seed, losses, _stream()))
        return list(losses)[:epochs]

    def save(self, path):
        _check(lib().tm_ranker_save(self._r, os.fsencode(path)))

    def close(self):
        if self._r:
            lib().tm_ranker_destroy(self._r)
            self._r = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tm_search(plan, ranker, seg, topk=64, lam=0.05, margin=0.0, prefilter=0):
    """Per instance [seg[s], seg[s+1]) of the batch loaded in `plan`: (best index
    relative to the instance, its cost) as device tensors.  ranker None = exhaustive;
    prefilter > 0: the network keeps that many per instance and their block-model
    estimates choose the topk evaluated exactly; margin > 0 re-evaluates only the
    topk scoring within `margin` of the best."""
    import torch
    sg = np.ascontiguousarray(seg, dtype=np.int64)
    nseg = len(sg) - 1
    best = torch.empty(max(nseg, 1), dtype=torch.int64, device="cuda")
    cost = torch.empty((max(nseg, 1), 4), dtype=torch.int64, device="cuda")
    _check(lib().tm_search(plan._p, ranker._r if ranker is not None else None, sg.ctypes.data, nseg, prefilter, topk,
                           lam, margin, _dev_ptr(best, torch.int64), _dev_ptr(cost, torch.int64), _stream()))
    return best[:nseg], cost[:nseg]
