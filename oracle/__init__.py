"""CPU oracle for exact mapping evaluation -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product (the HIP library and its Python binding) never
calls it.  It shares no code with the HIP path: oracle.c restates every rule from
the paper on its own, and mlp.py is a float64 numpy model of the ranker.

Every function here is a thin ctypes wrapper over oracle.c; see that file's header
for what is computed and the readings taken where the paper is silent.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "liboracle.so")
_lib = None

OK, EINVAL, EOVERFLOW, ECAPACITY, ENOMEM = 0, -1, -2, -3, -4
CAND_BYTES = 328


def build():
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", _SO + ".tmp",
                           os.path.join(HERE, "oracle.c")])
    os.replace(_SO + ".tmp", _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        for name, args in [("or_validate", [P, P, P]), ("or_point_owner", [P, P, P, P]),
                           ("or_proc_map", [P, P, I64]), ("or_chain_table", [P, P, I64, P]),
                           ("or_stencil_cost", [P, P, P]), ("or_stencil_cost_batch", [P, I64, P, P]),
                           ("or_stencil_node_cost_batch", [P, I64, P, P]),
                           ("or_matmul_cost", [P, I64, P, P]),
                           ("or_redistribution_cost_batch", [P, P, I64, I64, P]),
                           ("or_enum_factorizations", [I64, I32, P, I64, P]),
                           ("or_decompose_argmin", [I64, I32, P, P, P]),
                           ("or_greedy_grid", [I64, I32, P]),
                           ("or_workload_greedy", [I64, I32, P, P]),
                           ("or_select_best", [P, I64, P])]:
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        assert L.or_sizeof_candidate() == CAND_BYTES
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _chk(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def _rec(c):
    a = np.ascontiguousarray(c)
    assert a.dtype.itemsize == CAND_BYTES
    return a


def validate(c):
    """(code, final_shape) for one candidate record."""
    a = _rec(c)
    shape = np.zeros(8, np.int32)
    r = ctypes.c_int32(0)
    rc = lib().or_validate(a.ctypes.data, shape.ctypes.data, ctypes.byref(r))
    return rc, tuple(int(x) for x in shape[: r.value]) if rc == OK else None


def point_owner(c, ip):
    """(node, gpu) of one launch point."""
    a = _rec(c)
    p = np.zeros(4, np.int64)
    p[: len(ip)] = ip
    nd, gp = ctypes.c_int32(), ctypes.c_int32()
    _chk(lib().or_point_owner(a.ctypes.data, p.ctypes.data, ctypes.byref(nd), ctypes.byref(gp)),
         "point_owner")
    return nd.value, gp.value


def n_points(c):
    return int(np.prod([int(x) for x in c["extent"][: int(c["lrank"])]]))


def proc_map(c):
    a = _rec(c)
    n = n_points(c)
    out = np.empty(n, np.int32)
    _chk(lib().or_proc_map(a.ctypes.data, out.ctypes.data, n), "proc_map")
    return out.reshape([int(x) for x in c["extent"][: int(c["lrank"])]])


def chain_table(c):
    a = _rec(c)
    cnt = ctypes.c_int64()
    lib().or_chain_table(a.ctypes.data, None, 0, ctypes.byref(cnt))
    out = np.empty(cnt.value, np.int32)
    _chk(lib().or_chain_table(a.ctypes.data, out.ctypes.data, cnt.value, ctypes.byref(cnt)),
         "chain_table")
    return out


def stencil_cost(c, st):
    """(ghost_cells, inter_cells, bytes, inter_bytes)."""
    a = _rec(c)
    s = np.ascontiguousarray(st)
    out = np.zeros(4, np.int64)
    _chk(lib().or_stencil_cost(a.ctypes.data, s.ctypes.data, out.ctypes.data), "stencil_cost")
    return tuple(int(x) for x in out)


def stencil_cost_batch(cands, st):
    a = _rec(cands)
    s = np.ascontiguousarray(st)
    out = np.zeros((len(a), 4), np.int64)
    _chk(lib().or_stencil_cost_batch(a.ctypes.data, len(a), s.ctypes.data, out.ctypes.data),
         "stencil_cost_batch")
    return out


def stencil_node_cost_batch(cands, st):
    """Node-level exchange volume per candidate: rows (cells, cells, bytes, bytes)."""
    a = _rec(cands)
    s = np.ascontiguousarray(st)
    out = np.zeros((len(a), 4), np.int64)
    _chk(lib().or_stencil_node_cost_batch(a.ctypes.data, len(a), s.ctypes.data, out.ctypes.data),
         "stencil_node_cost_batch")
    return out


def redistribution_cost_batch(src, dst, elem_bytes=8):
    """Per pair (src[i], dst[i]): (moved cells, inter-node moved cells, bytes, inter bytes)."""
    a, b = _rec(src), _rec(dst)
    assert len(a) == len(b)
    out = np.zeros((len(a), 4), np.int64)
    _chk(lib().or_redistribution_cost_batch(a.ctypes.data, b.ctypes.data, len(a), elem_bytes, out.ctypes.data),
         "redistribution_cost_batch")
    return out


def transpose_target(c, n, t):
    """The pencil-transposed image of mapping c for an all-to-all transpose along
    launch dim n (App. A.3), reading: the processors that share every final coordinate
    except the one taken from dim n (a pencil of d_n processors along n) split their
    joint data along launch dim t instead, d_n ways inside each block of t.  The final
    dim j_n projected from n is merged into the final dim j_t projected from t as its
    fast part (merge inverse b_p = a mod s_p, b_q = floor(a / s_p)), launch dim n is no
    longer projected, and the merged dim is a block projection of t.  Requires exactly
    one final dim projected from each of n and t, both block-projected, and room for
    two more operations."""
    r = np.array(_rec(c), copy=True).reshape(())
    mrank = int(r["mrank"])
    src = [int(x) for x in r["proj_src"][:mrank]]
    mode = [int(x) for x in r["proj_mode"][:mrank]]
    if n == t or src.count(n) != 1 or src.count(t) != 1:
        raise ValueError("need exactly one final dim projected from each of n and t")
    jn, jt = src.index(n), src.index(t)
    if mode[jn] != 0 or mode[jt] != 0:
        raise ValueError("both dims must be block-projected")
    ops = []
    if jn > jt:  # bring the dim of n in front of the dim of t
        ops.append((3, jt, jn))
        src[jn], src[jt] = src[jt], src[jn]
        mode[jn], mode[jt] = mode[jt], mode[jn]
        jn, jt = jt, jn
    ops.append((2, jn, jt))  # merge(p = jn, q = jt): the dim of n is the fast part
    nops = int(r["nops"])
    if nops + len(ops) > 8:
        raise ValueError("no room for the transpose operations")
    for i, (kind, a, b) in enumerate(ops):
        op = r["ops"][nops + i]
        op["kind"], op["a"], op["b"], op["nf"] = kind, a, b, 0
        op["f"][:] = 0
    r["nops"] = nops + len(ops)
    src[jn], mode[jn] = t, 0
    del src[jt], mode[jt]
    r["mrank"] = mrank - 1
    r["proj_src"][:] = 0
    r["proj_mode"][:] = 0
    r["proj_src"][: mrank - 1] = src
    r["proj_mode"][: mrank - 1] = mode
    return r


def matmul_cost(c, tile_bytes):
    """(per_proc int64[P,3], (tilesA, tilesB, tilesC, maxA, maxB, maxC, bytes))."""
    a = _rec(c)
    P = int(c["nodes"]) * int(c["gpus"])
    per = np.zeros((P, 3), np.int64)
    out = np.zeros(7, np.int64)
    _chk(lib().or_matmul_cost(a.ctypes.data, tile_bytes, per.ctypes.data, out.ctypes.data),
         "matmul_cost")
    return per, tuple(int(x) for x in out)


def enumerate_factorizations(P, k):
    cnt = ctypes.c_int64()
    lib().or_enum_factorizations(P, k, None, 0, ctypes.byref(cnt))
    out = np.zeros((cnt.value, k), np.int32)
    _chk(lib().or_enum_factorizations(P, k, out.ctypes.data, cnt.value, ctypes.byref(cnt)),
         "enumerate")
    return [tuple(int(x) for x in r) for r in out]


def decompose_argmin(P, extent, halo=None):
    k = len(extent)
    ext = np.array(list(extent) + [1] * (4 - k), np.int64)
    h = np.array(list(halo if halo is not None else [1] * k) + [0] * (4 - k), np.int32)
    out = np.zeros(4, np.int32)
    _chk(lib().or_decompose_argmin(P, k, ext.ctypes.data, h.ctypes.data, out.ctypes.data),
         "decompose_argmin")
    return tuple(int(x) for x in out[:k])


def greedy_grid(P, k):
    out = np.zeros(4, np.int32)
    _chk(lib().or_greedy_grid(P, k, out.ctypes.data), "greedy_grid")
    return tuple(int(x) for x in out[:k])


def workload_greedy(P, extent):
    k = len(extent)
    ext = np.array(list(extent) + [1] * (4 - k), np.int64)
    out = np.zeros(4, np.int32)
    _chk(lib().or_workload_greedy(P, k, ext.ctypes.data, out.ctypes.data), "workload_greedy")
    return tuple(int(x) for x in out[:k])


def select_best(costs):
    """Index of the minimum (bytes, inter_bytes, index) over rows of int64[n,4]."""
    a = np.ascontiguousarray(costs, dtype=np.int64)
    b = ctypes.c_int64()
    _chk(lib().or_select_best(a.ctypes.data, len(a), ctypes.byref(b)), "select_best")
    return b.value


def decompose_argmin_transpose(P, extent, halo, transpose):
    """decompose's argmin with all-to-all transposes (App. A.3), in exact rationals:
    V = sum_n h_n f_n prod_{m != n} l_m + sum_{n in T} (1 - 1/f_n) prod_m l_m over the
    ordered factorizations of P; the first minimum in lexicographic order."""
    from fractions import Fraction
    k = len(extent)
    total = 1
    for l in extent:
        total *= int(l)
    best, arg = None, None
    for f in enumerate_factorizations(P, k):
        v = Fraction(0)
        for n in range(k):
            area = 1
            for m in range(k):
                if m != n:
                    area *= int(extent[m])
            v += int(halo[n]) * int(f[n]) * area
        for n in transpose:
            v += (1 - Fraction(1, int(f[n]))) * total
        if best is None or v < best:
            best, arg = v, tuple(int(x) for x in f)
    return arg
