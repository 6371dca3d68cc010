"""CPU-side checks of the C ABI: the library loads, exports every declared entry
point, and its host calls agree with the oracle (no GPU needed for these)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import balance_split, decompose, merge, split, swap

tm = pytest.importorskip("paper_2507_17087_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = tm.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(L, n), n
    assert tm.tm_abi_version() == 1


def test_validate_matches_oracle_random_and_corrupted():
    rng = np.random.default_rng(0)
    cs = W.random_candidates(400, seed=99, ranks=(1, 2, 3, 4), octaves=(1, 6), nodes_max=40,
                             max_ops=5, cyclic_pct=20)
    bad = cs.copy()
    for c in bad:  # corrupt one field at random
        t = int(rng.integers(0, 7))
        if t == 0:
            c["ops"][int(rng.integers(0, 8))]["kind"] = int(rng.integers(0, 7))
        elif t == 1:
            c["ops"][int(rng.integers(0, max(int(c["nops"]), 1)))]["a"] += int(rng.integers(-2, 3))
        elif t == 2:
            c["ops"][int(rng.integers(0, max(int(c["nops"]), 1)))]["b"] += int(rng.integers(-2, 3))
        elif t == 3:
            c["mrank"] += int(rng.integers(-1, 2))
        elif t == 4:
            c["proj_src"][int(rng.integers(0, 8))] = int(rng.integers(-1, 5))
        elif t == 5:
            c["extent"][int(rng.integers(0, 4))] = int(rng.integers(-1, 3))
        else:
            c["nops"] = int(rng.integers(0, 9))
    nbad = 0
    for c in np.concatenate([cs, bad]):
        a, b = tm.tm_validate(c), oracle.validate(c)
        assert a[0] == b[0]
        if a[0] == 0:
            assert a[1] == b[1]
        else:
            nbad += 1
    assert nbad > 100


@pytest.mark.parametrize("P", [1, 6, 8, 12, 48, 64, 72, 97, 128, 360, 480, 512, 1 << 20, 720720])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_enumeration_matches_oracle(P, k):
    if P > 100000 and k > 3:
        pytest.skip("large")
    assert tm.tm_enumerate_factorizations(P, k) == oracle.enumerate_factorizations(P, k)


def test_argmin_and_greedy_match_oracle():
    rng = np.random.default_rng(1)
    for _ in range(300):
        k = int(rng.integers(1, 5))
        P = int(rng.integers(1, 600))
        ext = tuple(int(x) for x in rng.integers(1, 2000, size=k))
        halo = tuple(int(x) for x in rng.integers(0, 4, size=k))
        assert tm.tm_decompose_argmin(P, ext, halo) == oracle.decompose_argmin(P, ext, halo)
        assert tm.tm_greedy_grid(P, k) == oracle.greedy_grid(P, k)
        assert tm.tm_workload_greedy(P, ext) == oracle.workload_greedy(P, ext)


def test_error_codes_and_messages():
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_enumerate_factorizations(0, 2)
    assert e.value.code == tm.TM_EINVAL
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_greedy_grid(8, 5)
    assert e.value.code == tm.TM_EINVAL
    c = W.candidate((4, 4), 2, 4, [split(0, 3)])
    rc, _ = tm.tm_validate(c)
    assert rc == tm.TM_EINVAL
    assert b"split" in tm.lib().tm_last_error()
    cnt = ctypes.c_int64()
    rc = tm.lib().tm_enumerate_factorizations(128, 3, None, 0, ctypes.byref(cnt))
    assert rc == tm.TM_ECAPACITY and cnt.value == 36


def test_decompose_transpose_matches_oracle():
    """Host logic: the library's exact integer comparison against the oracle's
    rational arithmetic, random domains, halos and transpose sets."""
    import oracle
    rng = np.random.default_rng(8)
    for _ in range(60):
        k = int(rng.integers(1, 5))
        P = int(rng.choice([4, 8, 12, 30, 64, 96, 128, 360]))
        ext = tuple(int(x) for x in rng.integers(2, 900, size=k))  # at most 2^40 points
        h = tuple(int(x) for x in rng.integers(0, 5, size=k))
        T = [d for d in range(k) if rng.random() < 0.4]
        assert tm.tm_decompose_argmin_transpose(P, ext, h, T) == oracle.decompose_argmin_transpose(P, ext, h, T)
    with pytest.raises(tm.TaskmapError):
        tm.tm_decompose_argmin_transpose(8, (64, 64), (256, 1), [0])


def test_transpose_target_matches_oracle():
    """Host logic: the library's pencil-transposed image of a mapping equals the
    oracle's, record for record (ops, projections, rank), over random decompose
    chains with extra ops, and the same cases are rejected."""
    rng = np.random.default_rng(21)
    fields = ("lrank", "nodes", "gpus", "nops", "extent", "mrank", "proj_src", "proj_mode")
    checked = 0
    for _ in range(200):
        k = int(rng.integers(2, 5))
        P = int(rng.choice([2, 4, 6, 8, 12, 16]))
        g = int(rng.choice([g for g in (1, 2, 4) if P % g == 0]))
        F = oracle.enumerate_factorizations(P, k)[int(rng.integers(0, len(oracle.enumerate_factorizations(P, k))))]
        ext = tuple(int(x) for x in rng.integers(1, 40, size=k))
        tail = [] if rng.random() < 0.5 else [swap(0, 1)]
        proj = [(int(d), W.BLOCK if rng.random() < 0.8 else W.CYCLIC) for d in rng.permutation(k)]
        c = W.candidate(ext, P // g, g, [merge(0, 1), decompose(0, F)] + tail, proj)
        n, t = (int(x) for x in rng.choice(k, size=2, replace=False))
        try:
            want = oracle.transpose_target(c, n, t)
        except ValueError:
            with pytest.raises(tm.TaskmapError):
                tm.tm_transpose_target(c, n, t)
            continue
        got = tm.tm_transpose_target(c, n, t)
        for f in fields:
            assert np.array_equal(np.asarray(got[f]), np.asarray(want[f])), f
        for i in range(int(want["nops"])):
            for f in ("kind", "a", "b", "nf", "f"):
                assert np.array_equal(np.asarray(got["ops"][i][f]), np.asarray(want["ops"][i][f])), (i, f)
        checked += 1
    assert checked > 60
    c = W.candidate((8, 8), 1, 4, [merge(0, 1), decompose(0, (2, 2))])
    for n, t in ((0, 0), (0, 2), (-1, 0)):
        with pytest.raises(tm.TaskmapError):
            tm.tm_transpose_target(c, n, t)
    full = W.candidate((8, 8), 1, 4, [merge(0, 1), decompose(0, (2, 2))] + [swap(0, 1)] * 6)
    with pytest.raises(tm.TaskmapError):
        tm.tm_transpose_target(full, 0, 1)          # no room for merge
    assert int(tm.tm_transpose_target(W.candidate((8, 8), 1, 4, [merge(0, 1), decompose(0, (2, 2))] + [swap(0, 1)] * 5),
                                      0, 1)["nops"]) == 8


def test_row_limit_rejected_before_any_launch():
    """More than 2^30 rows (points / last extent) is TM_ENOTSUP from host-side
    validation, before any device memory is touched (a null output is never reached)."""
    st = W.stencil((1, 1), 8)
    rows_ok = W.candidate((1 << 30, 1), 1, 2, [merge(0, 1), decompose(0, (2, 1))])
    rows_bad = W.candidate(((1 << 30) + 1, 1), 1, 2, [merge(0, 1), decompose(0, (2, 1))])
    L = tm.lib()
    rc = L.tm_eval_stencil_batch(W.batch([rows_bad]).ctypes.data, 1, st.ctypes.data, None, None)
    assert rc == tm.TM_ENOTSUP and b"2^30 rows" in L.tm_last_error()
    rc = L.tm_eval_stencil_batch(W.batch([rows_ok]).ctypes.data, 1, st.ctypes.data, None, None)
    assert rc == tm.TM_EINVAL  # passes validation, then stops at the null output


def test_redistribution_validation_before_any_launch():
    """Host-side checks of tm_eval_redistribution_batch, all before device work: pairs
    on different machines or domains and a negative element size are TM_EINVAL, an
    empty batch is TM_OK; owner tables larger than the LDS budget together are
    accepted (they are read in place), so such a pair stops at the null output."""
    L = tm.lib()
    a = W.batch([W.candidate((8, 8), 1, 4, [merge(0, 1), decompose(0, (2, 2))])])
    other_machine = W.batch([W.candidate((8, 8), 2, 2, [merge(0, 1), decompose(0, (2, 2))])])
    other_domain = W.batch([W.candidate((8, 9), 1, 4, [merge(0, 1), decompose(0, (2, 2))])])
    for b in (other_machine, other_domain):
        assert L.tm_eval_redistribution_batch(a.ctypes.data, b.ctypes.data, 1, 8, None, None) == tm.TM_EINVAL
        assert b"pair 0" in L.tm_last_error()
    assert L.tm_eval_redistribution_batch(a.ctypes.data, a.ctypes.data, 1, -1, None, None) == tm.TM_EINVAL
    assert L.tm_eval_redistribution_batch(None, None, 0, 8, None, None) == tm.TM_OK
    big = W.batch([W.candidate((64, 512), 128, 128, [merge(0, 1), decompose(0, (128, 128))])])
    assert L.tm_eval_redistribution_batch(big.ctypes.data, big.ctypes.data, 1, 8, None, None) == tm.TM_EINVAL
    assert b"null output" in L.tm_last_error()
    # a valid pair passes validation and stops at the null output
    assert L.tm_eval_redistribution_batch(a.ctypes.data, a.ctypes.data, 1, 8, None, None) == tm.TM_EINVAL
    assert b"null output" in L.tm_last_error()

