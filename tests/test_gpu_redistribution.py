"""GPU parity of the redistribution evaluator (App. A.3 transposes as changes of
mapping): the HIP library against the CPU oracle, bit-exact, on seeded pairs; the
full-size 512^3 case against the divisible-case closed form."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import decompose, merge, swap

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available()
    import paper_2507_17087_amd as m
    m.lib()
    return m


def gpu_redist(tm, src, dst, elem_bytes=8):
    import torch
    out = tm.tm_eval_redistribution_batch(src, dst, elem_bytes)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _grid(extent, F, n, g, tail=(), proj=None):
    return W.candidate(extent, n, g, [merge(0, 1), decompose(0, F)] + list(tail), proj)


def _random_pairs(rng, count, max_last=300):
    """Transposes of random decompose chains (ragged extents, block and cyclic
    dims elsewhere), and pairs of unrelated chains on one domain and machine."""
    src, dst = [], []
    while len(src) < count:
        k = int(rng.integers(1, 4))
        P = int(rng.choice([1, 2, 4, 6, 8, 12, 16, 24, 32]))
        g = int(rng.choice([g for g in (1, 2, 4, 8) if P % g == 0]))
        facs = oracle.enumerate_factorizations(P, k)
        F = facs[int(rng.integers(0, len(facs)))]
        ext = [int(x) for x in rng.integers(1, 24, size=k)]
        ext[-1] = int(rng.integers(1, max_last))
        tail = [swap(0, 1)] if k > 1 and rng.random() < 0.3 else []
        modes = [W.BLOCK if rng.random() < 0.75 else W.CYCLIC for _ in range(k)]
        a = _grid(tuple(ext), F, P // g, g, tail, [(d, modes[d]) for d in range(k)])
        if k > 1 and rng.random() < 0.6:
            n, t = (int(x) for x in rng.choice(k, size=2, replace=False))
            try:
                b = oracle.transpose_target(a, n, t)
            except ValueError:
                continue
        else:
            F2 = facs[int(rng.integers(0, len(facs)))]
            b = _grid(tuple(ext), F2, P // g, g)
        src.append(a)
        dst.append(b)
    return W.batch(src), W.batch(dst)


@pytest.mark.parametrize("seed", [1, 2])
def test_redistribution_random_parity(tm, seed):
    say("redistribution random pairs seed", seed)
    src, dst = _random_pairs(np.random.default_rng(seed), 120)
    exp = oracle.redistribution_cost_batch(src, dst, 8)
    got = gpu_redist(tm, src, dst, 8)
    assert (got == exp).all()
    assert exp[:, 0].sum() > 0 and exp[:, 1].sum() > 0


def test_transpose_parity_and_library_target(tm):
    """The library's own transposed image evaluated on the GPU against the oracle's
    image evaluated on the CPU (several 512-cell chunks and a ragged tail per row)."""
    say("transpose targets, library vs oracle")
    rng = np.random.default_rng(5)
    src, lib_dst, or_dst = [], [], []
    for F in [(2, 4), (4, 2), (8, 1), (3, 5), (2, 3, 2)]:
        k = len(F)
        P = int(np.prod(F))
        for g in (1, P):
            ext = tuple(int(x) for x in rng.integers(5, 19, size=k - 1)) + (int(rng.integers(1100, 1700)),)
            a = _grid(ext, F, P // g, g)
            for n in range(k):
                t = (n + 1) % k
                src.append(a)
                lib_dst.append(tm.tm_transpose_target(a, n, t))
                or_dst.append(oracle.transpose_target(a, n, t))
    src, lib_dst, or_dst = W.batch(src), W.batch(lib_dst), W.batch(or_dst)
    exp = oracle.redistribution_cost_batch(src, or_dst, 4)
    got = gpu_redist(tm, src, lib_dst, 4)
    assert (got == exp).all()


def test_redistribution_edges(tm):
    import torch
    say("redistribution edges")
    # empty batch; identical mappings; 1-D; rows of one cell; a last dim longer than
    # the LDS budget (read from global memory)
    assert tm.tm_eval_redistribution_batch(W.batch([]), W.batch([])).numel() == 0
    cases = [(_grid((9, 7), (2, 2), 1, 4), _grid((9, 7), (2, 2), 1, 4)),
             (_grid((1000,), (6,), 2, 3), _grid((1000,), (6,), 2, 3, proj=[(0, W.CYCLIC)])),
             (_grid((33, 1), (4, 1), 2, 2), _grid((33, 1), (1, 4), 2, 2)),
             (_grid((3, 40000), (2, 4), 4, 2), _grid((3, 40000), (4, 2), 4, 2)),
             (_grid((1, 1), (1, 1), 1, 1), _grid((1, 1), (1, 1), 1, 1))]
    src, dst = W.batch([a for a, _ in cases]), W.batch([b for _, b in cases])
    exp = oracle.redistribution_cost_batch(src, dst, 8)
    got = gpu_redist(tm, src, dst, 8)
    assert (got == exp).all()
    assert tuple(got[0]) == (0, 0, 0, 0)
    # a pair on different machines or domains; negative element size
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_eval_redistribution_batch(W.batch([_grid((8, 8), (2, 2), 1, 4)]), W.batch([_grid((8, 8), (2, 2), 2, 2)]))
    assert e.value.code == tm.TM_EINVAL
    with pytest.raises(tm.TaskmapError):
        tm.tm_eval_redistribution_batch(W.batch([_grid((8, 8), (2, 2), 1, 4)]), W.batch([_grid((8, 9), (2, 2), 1, 4)]))
    with pytest.raises(tm.TaskmapError):
        tm.tm_eval_redistribution_batch(W.batch([cases[0][0]]), W.batch([cases[0][1]]), -1)
    # owner tables of 16,384 processors each (together over the LDS budget: read in
    # place), against a swapped spelling and a transposed grid
    big = _grid((64, 512), (128, 128), 128, 128)
    src = W.batch([big, big])
    dst = W.batch([_grid((64, 512), (128, 128), 128, 128, tail=[swap(0, 1), swap(0, 1)]),
                   _grid((64, 512), (64, 256), 128, 128)])
    assert (gpu_redist(tm, src, dst, 8) == oracle.redistribution_cost_batch(src, dst, 8)).all()
    torch.cuda.synchronize()


def test_transpose_full_size_closed_form(tm):
    """512^3 on 16 nodes x 8 GPUs: every divisible transpose of the 36 decompose
    candidates moves (f_n - 1) / f_n * 2^27 cells (App. A.3); with one GPU per node
    every moved cell changes node, on one node none does."""
    say("transpose 512^3 closed form")
    facs = oracle.enumerate_factorizations(128, 3)
    src, dst, want = [], [], []
    for F in facs:
        for n in range(3):
            t = (n + 1) % 3
            if (512 // F[t]) % F[n]:
                continue
            a = _grid((512, 512, 512), F, 16, 8)
            src.append(a)
            dst.append(oracle.transpose_target(a, n, t))
            want.append((F[n] - 1) * (1 << 27) // F[n])
    got = gpu_redist(tm, W.batch(src), W.batch(dst), 8)
    assert got[:, 0].tolist() == want
    assert (got[:, 2] == 8 * got[:, 0]).all() and (got[:, 1] <= got[:, 0]).all()
    for nodes, g in ((128, 1), (1, 128)):
        a = _grid((512, 512, 512), (4, 4, 8), nodes, g)
        r = gpu_redist(tm, W.batch([a]), W.batch([oracle.transpose_target(a, 2, 0)]), 8)[0]
        assert r[0] == 7 * (1 << 27) // 8
        assert r[1] == (r[0] if nodes == 128 else 0)
