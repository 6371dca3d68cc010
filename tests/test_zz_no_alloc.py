"""The stencil entry point that allocates no device memory,
tm_eval_stencil_batch_noalloc, against tm_eval_stencil_batch through the C ABI:
bit-equal results on consecutive calls of shrinking and growing batches (the
library's scratch array keeps the previous call's contents), a batch larger than
the scratch rejected with nothing launched, and the oracle on the small batch."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

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


def both(tm, cands, st):
    import torch
    n = len(cands)
    ref = tm.tm_eval_stencil_batch(cands, st)
    out = torch.full((n, 4), -3, dtype=torch.int64, device="cuda")
    tm.tm_eval_stencil_batch_noalloc(cands, st, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(tm):
    import torch
    say("no-alloc: mixed-rank random batch, then a smaller one")
    big = W.random_candidates(600, seed=21, ranks=(2, 3), octaves=(2, 7), nodes_max=32, max_ops=4, cyclic_pct=25)
    st = W.stencil((1, 2, 1), 8)
    got, ref = both(tm, big, st)
    assert (got == ref).all()
    small = W.c1_candidates(oracle.enumerate_factorizations(8, 2))[:7]
    st1 = W.c1_stencil()
    got, ref = both(tm, small, st1)
    assert (got == ref).all()
    assert (got == oracle.stencil_cost_batch(small, st1)).all()
    # a third call that grows again, after the smaller one
    got, ref = both(tm, big[:300], st)
    assert (got == ref).all()


def test_noalloc_rejects_a_batch_beyond_its_scratch(tm):
    import torch
    say("no-alloc: capacity")
    # 4,000 candidates of a 3000 x 3000 x 64 domain need over 100 MiB of tables
    fs = oracle.enumerate_factorizations(128, 3)
    cands = W.batch([W.candidate((3000, 3000, 64), 16, 8, [W.merge(0, 1), W.decompose(0, fs[i % len(fs)])])
                     for i in range(4000)])
    out = torch.full((len(cands), 4), -9, dtype=torch.int64, device="cuda")
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_eval_stencil_batch_noalloc(cands, W.c2_stencil(), out)
    assert e.value.code == tm.TM_ECAPACITY
    torch.cuda.synchronize()
    assert (out.cpu() == -9).all()
    # and the next call in range still works
    small = W.c1_candidates(oracle.enumerate_factorizations(8, 2))
    got, ref = both(tm, small, W.c1_stencil())
    assert (got == ref).all()
