"""GPU parity: the HIP library against the CPU oracle, element by element, on
seeded inputs.  Integer results must be bit-exact."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import balance_split, decompose, merge, split, swap

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


def gpu_costs(tm, cands, st):
    import torch
    out = tm.tm_eval_stencil_batch(cands, st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def by_rank(cands):
    for k, idx in W.split_by_rank(cands).items():
        yield k, idx, cands[idx]


# ---------------------------------------------------------------- c1: 64x64 on 2 x 4

def test_c1_costs_maps_tables(tm):
    import torch
    say("c1 16 candidates")
    c1 = W.c1_candidates(oracle.enumerate_factorizations(8, 2))
    st = W.c1_stencil()
    exp = oracle.stencil_cost_batch(c1, st)
    got = gpu_costs(tm, c1, st)
    assert (got == exp).all()
    for c in c1:
        assert (tm.tm_proc_map(c).cpu().numpy() == oracle.proc_map(c)).all()
        assert (tm.tm_chain_table(c).cpu().numpy() == oracle.chain_table(c)).all()
    best = tm.tm_select_best(torch.from_numpy(got).cuda(), [0, len(c1)]).cpu().numpy()
    assert best[0] == oracle.select_best(exp)


# ---------------------------------------------------------------- random chains, edges

@pytest.mark.parametrize("seed", [1, 2])
def test_random_small_parity(tm, seed):
    say("random small seed", seed)
    cs = W.random_candidates(240, seed=seed, ranks=(1, 2, 3), octaves=(0, 5), nodes_max=24,
                             max_ops=4, cyclic_pct=25)
    rng = np.random.default_rng(seed)
    for k, idx, sub in by_rank(cs):
        for h in [tuple(int(x) for x in rng.integers(0, 5, size=k)), (1,) * k]:
            st = W.stencil(h, 4)
            say("  rank", k, "halo", h, "n", len(sub))
            assert (gpu_costs(tm, sub, st) == oracle.stencil_cost_batch(sub, st)).all()
    for c in cs[:80]:
        assert (tm.tm_proc_map(c).cpu().numpy() == oracle.proc_map(c)).all()


def test_rank4_and_ragged(tm):
    say("rank 4 and ragged extents")
    cs = W.random_candidates(60, seed=7, ranks=(4,), octaves=(0, 3), nodes_max=12, max_ops=4,
                             cyclic_pct=30)
    for st in [W.stencil((1, 2, 1, 1), 8), W.stencil((2, 2, 2, 2), 8)]:
        assert (gpu_costs(tm, cs, st) == oracle.stencil_cost_batch(cs, st)).all()
    odd = [W.candidate((1, 1), 1, 1, [merge(0, 1), decompose(0, (1, 1))]),
           W.candidate((3, 1), 2, 3, [merge(0, 1), decompose(0, (3, 2))]),
           W.candidate((1, 70), 2, 3, [merge(0, 1), decompose(0, (2, 3))]),
           W.candidate((130, 67), 5, 7, [merge(0, 1), decompose(0, (5, 7)), swap(0, 1)]),
           W.candidate((9, 200), 64, 8, [merge(0, 1), decompose(0, (32, 16))]),
           W.candidate((200, 3), 6, 1, [merge(0, 1), balance_split(0, 5)])]
    odd = W.batch(odd)
    for h in [(0, 0), (1, 1), (4, 3), (2, 4)]:
        st = W.stencil(h, 8)
        assert (gpu_costs(tm, odd, st) == oracle.stencil_cost_batch(odd, st)).all()
    for c in odd:
        assert (tm.tm_proc_map(c).cpu().numpy() == oracle.proc_map(c)).all()
    one_d = W.batch([W.candidate((5000,), 7, 3, [merge(0, 1)]),
                     W.candidate((333,), 4, 4, [merge(0, 1)], proj=[(0, W.CYCLIC)])])
    st = W.stencil((3,), 8)
    assert (gpu_costs(tm, one_d, st) == oracle.stencil_cost_batch(one_d, st)).all()
    # rows too long for the last dim's offset lists to sit in LDS (read from global)
    long_rows = W.batch([W.candidate((3, 9001), 5, 4, [merge(0, 1), decompose(0, (2, 10))]),
                         W.candidate((4, 7000), 6, 2, [merge(0, 1), decompose(0, (3, 4))],
                                     proj=[(0, W.BLOCK), (1, W.CYCLIC)])])
    st = W.stencil((2, 4), 8)
    assert (gpu_costs(tm, long_rows, st) == oracle.stencil_cost_batch(long_rows, st)).all()


def test_long_rows_and_tall_outer_dims(tm):
    """Last dims too long for the LDS budget (coordinate table and offset lists read
    from global memory), outer dims with long tables (always global), block and
    cyclic projections, ragged blocks; costs and maps against the oracle."""
    say("long rows and tall outer dims")
    cands = W.batch([
        W.candidate((100_003,), 7, 4, [merge(0, 1)]),
        W.candidate((65_536,), 3, 2, [merge(0, 1)], proj=[(0, W.CYCLIC)]),
        W.candidate((3, 50_001), 5, 4, [merge(0, 1), decompose(0, (4, 5))]),
        W.candidate((2, 40_000), 6, 2, [merge(0, 1), decompose(0, (3, 4))], proj=[(0, W.BLOCK), (1, W.CYCLIC)]),
        W.candidate((2, 36_000), 4, 2, [merge(0, 1), decompose(0, (1, 8))]),
    ])
    for k, idx, sub in by_rank(cands):
        for h in ((1,) * k, (4,) * k, (2, 3)[:k] if k == 2 else (3,)):
            st = W.stencil(h, 8)
            say(f"  rank {k} halo {h}")
            assert (gpu_costs(tm, sub, st) == oracle.stencil_cost_batch(sub, st)).all()
    tall = W.batch([W.candidate((40_000, 5), 4, 4, [merge(0, 1), decompose(0, (8, 2))]),
                    W.candidate((20_011, 3, 7), 2, 4, [merge(0, 1), decompose(0, (4, 1, 2))],
                                proj=[(0, W.CYCLIC), (1, W.BLOCK), (2, W.BLOCK)])])
    for k, idx, sub in by_rank(tall):
        st = W.stencil((2,) * k, 8)
        say(f"  tall rank {k}")
        assert (gpu_costs(tm, sub, st) == oracle.stencil_cost_batch(sub, st)).all()
    for c in list(cands) + list(tall):
        assert (tm.tm_proc_map(c).cpu().numpy() == oracle.proc_map(c)).all()


def test_empty_batch_and_invalid_input(tm):
    import torch
    say("empty and invalid")
    out = torch.full((2, 4), -7, dtype=torch.int64, device="cuda")
    empty = np.zeros(0, dtype=W.CAND_DTYPE)
    tm.tm_eval_stencil_batch(empty, W.stencil((1, 1)), out)
    bad = W.batch([W.candidate((8, 8), 2, 2, [merge(0, 1), decompose(0, (2, 2))]),
                   W.candidate((8, 8), 2, 2, [split(0, 3)])])
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_eval_stencil_batch(bad, W.stencil((1, 1)), out)
    assert e.value.code == tm.TM_EINVAL
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_eval_stencil_batch(bad[:1], W.stencil((5, 1)), out)
    assert e.value.code == tm.TM_ENOTSUP
    with pytest.raises(tm.TaskmapError) as e:  # a stencil of lower rank than a candidate
        tm.tm_eval_stencil_batch(bad[:1], W.stencil((1,)), out)
    assert e.value.code == tm.TM_EINVAL
    torch.cuda.synchronize()
    assert (out.cpu() == -7).all()  # nothing was launched


# ---------------------------------------------------------------- c2: 512^3 on 16 x 8

def test_c2_scaled_all_candidates(tm):
    say("c2 at 64^3, 216 candidates")
    cands = W.c2_candidates(oracle.enumerate_factorizations(128, 3), extent=(64, 64, 64))
    st = W.c2_stencil()
    assert (gpu_costs(tm, cands, st) == oracle.stencil_cost_batch(cands, st)).all()


def test_c2_full_size_plan(tm):
    """The benchmark workload at full size (216 candidates of 512^3, halo 2) in the
    launch configurations the benchmark times: every total against the block closed
    form, 16 candidates covering all six chains against the oracle cell by cell, and
    the selected candidate's whole int32 map against the oracle's."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    say("c2 full 512^3 plan")
    fs = oracle.enumerate_factorizations(128, 3)
    cands = W.c2_candidates(fs)
    st = W.c2_stencil()
    plan = tm.Plan(len(cands), 1)
    plan.load(cands, st)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    plan.run(out, best)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    # every chain is a bijective block chain whose final dim j is projected from
    # launch dim j: its factors along the launch dims are the final shape, every
    # block is 512/f >= 4 >= h wide, and V = sum_m 2h (f_m - 1) prod_{j != m} l_j
    for i, c in enumerate(cands):
        rc, fsh = oracle.validate(c)
        assert rc == 0 and len(fsh) == 3
        assert got[i, 0] == sum(2 * 2 * (fm - 1) * 512 * 512 for fm in fsh), (i, fsh)
        assert got[i, 2] == 8 * got[i, 0] and got[i, 3] == 8 * got[i, 1]
    # 16 full-size candidates (all six chains) through the oracle, one per host thread
    picks = [(37 * i) % len(cands) for i in range(16)]
    assert sorted(set(p % 6 for p in picks)) == list(range(6))
    say("  oracle on 16 candidates of 134M points")
    with ThreadPoolExecutor(max_workers=16) as ex:
        exp = list(ex.map(lambda i: oracle.stencil_cost(cands[i], st), picks))
    for i, e in zip(picks, exp):
        assert tuple(got[i]) == e, (i, tuple(got[i]), e)
    b = int(best.cpu()[0])
    assert b == oracle.select_best(got)
    # the selected candidate's whole map
    m = torch.empty(512 ** 3, dtype=torch.int32, device="cuda")
    plan.materialize(m, d_index=best)
    torch.cuda.synchronize()
    say("  whole map of candidate", b)
    assert np.array_equal(m.cpu().numpy().reshape(512, 512, 512), oracle.proc_map(cands[b]))
    # the launch configurations the benchmark times: its autotuner's pick and a fixed
    # item size; identical costs and selection
    out2 = torch.empty_like(out)
    cpi, wg = plan.autotune(out2)
    say("  autotuned launch", cpi, wg)
    plan.run(out2, best)
    torch.cuda.synchronize()
    assert (out2.cpu().numpy() == got).all() and int(best.cpu()[0]) == b
    plan.set_launch(1 << 12, 0)
    plan.run(out2, best)
    torch.cuda.synchronize()
    assert (out2.cpu().numpy() == got).all() and int(best.cpu()[0]) == b
    plan.close()


# ---------------------------------------------------------------- c3: random batch

def test_c3_scaled_all(tm):
    say("c3 4096 candidates at scaled extents")
    cs = W.c3_candidates(4096, octaves=(1, 4), nodes_max=64)
    for k, idx, sub in by_rank(cs):
        st = W.c3_stencil(k)
        assert (gpu_costs(tm, sub, st) == oracle.stencil_cost_batch(sub, st)).all()


def test_c3_full_extents_subset(tm):
    """A seeded subset of 256 of the 4,096 random candidates at full extents (2.8e9
    points), launch ranks 2 and 3 mixed in one plan (one counting launch), against
    the oracle, one candidate per host thread."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    say("c3 full-extent subset of 256, one plan")
    cs = W.c3_candidates(4096)
    rng = np.random.default_rng(17087)
    sub = cs[np.sort(rng.choice(len(cs), size=256, replace=False))]
    assert set(int(k) for k in sub["lrank"]) == {2, 3}
    plan = tm.Plan(len(sub), 1)
    plan.load(sub, W.c3_stencil(3))  # a rank-2 candidate takes the first two halo widths
    out = torch.empty((len(sub), 4), dtype=torch.int64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    plan.run(out, best)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    with ThreadPoolExecutor(max_workers=16) as ex:
        exp = list(ex.map(lambda c: oracle.stencil_cost(c, W.c3_stencil(int(c["lrank"]))), sub))
    assert (got == np.array(exp)).all()
    assert int(best.cpu()[0]) == oracle.select_best(got)
    plan.close()


def test_mixed_rank_plan(tm):
    """Launch ranks 1 to 4 in one plan with per-dim halos: a candidate of rank k
    takes the stencil's first k halo widths; costs, selection and replays against
    the oracle per rank."""
    import torch
    say("mixed ranks 1..4 in one plan")
    cs = W.random_candidates(400, seed=11, ranks=(1, 2, 3, 4), octaves=(0, 4), nodes_max=16, max_ops=4,
                             cyclic_pct=25)
    halo = (2, 1, 3, 1)
    plan = tm.Plan(len(cs), 1)
    plan.load(cs, W.stencil(halo, 8))
    out = torch.empty((len(cs), 4), dtype=torch.int64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    exp = np.zeros((len(cs), 4), np.int64)
    for k, idx in W.split_by_rank(cs).items():
        exp[idx] = oracle.stencil_cost_batch(cs[idx], W.stencil(halo[:k], 8))
    for rep in range(3):
        out.fill_(-1)
        plan.run(out, best)
        torch.cuda.synchronize()
        assert (out.cpu().numpy() == exp).all(), rep
        assert int(best.cpu()[0]) == oracle.select_best(exp)
    # the single-shot call takes the same mixed batch
    assert (gpu_costs(tm, cs, W.stencil(halo, 8)) == exp).all()
    plan.close()


# ---------------------------------------------------------------- c4: matmul

def matmul_gpu(tm, cands, tile_bytes):
    import torch
    pp, out = tm.tm_eval_matmul_batch(cands, tile_bytes)
    torch.cuda.synchronize()
    return pp.cpu().numpy(), out.cpu().numpy()


def test_c4_scaled_all(tm):
    say("c4 at 32^3 tiles, 57 candidates")
    cands = W.c4_candidates(oracle.enumerate_factorizations(64, 3), extent=(32, 32, 32))
    pp, out = matmul_gpu(tm, cands, W.C4_TILE_BYTES)
    off = 0
    for i, c in enumerate(cands):
        P = int(c["nodes"]) * int(c["gpus"])
        per, tot = oracle.matmul_cost(c, W.C4_TILE_BYTES)
        assert (pp[off:off + P] == per).all()
        assert tuple(out[i]) == tot
        off += P


def test_c4_full_size(tm):
    say("c4 at 256^3 tiles")
    fs = oracle.enumerate_factorizations(64, 3)
    cands = W.c4_candidates(fs)
    pp, out = matmul_gpu(tm, cands, W.C4_TILE_BYTES)
    T = 256
    for i, f in enumerate(fs):
        nA = (T // f[0]) * (T // f[2])
        nB = (T // f[2]) * (T // f[1])
        nC = (T // f[0]) * (T // f[1])
        assert tuple(out[2 * i][:3]) == (64 * nA, 64 * nB, 64 * nC)
        assert tuple(out[2 * i][3:6]) == (nA, nB, nC)
    i881 = fs.index((8, 8, 1))
    assert tuple(out[-1][:6]) == tuple(out[2 * i881][:6])  # Cannon = (8,8,1) counts
    say("  oracle on one full candidate (16.7M tasks)")
    per, tot = oracle.matmul_cost(cands[-1], W.C4_TILE_BYTES)
    assert tuple(out[-1]) == tot
    assert (pp[-64:] == per).all()


def test_matmul_many_processors(tm):
    say("matmul P > 64")
    cs = W.batch([W.candidate((12, 10, 9), 40, 5, [merge(0, 1), decompose(0, (10, 5, 4))]),
                  W.candidate((7, 16, 5), 30, 8, [merge(0, 1), decompose(0, (6, 8, 5)), swap(0, 2)]),
                  W.candidate((9, 9, 9), 100, 10, [merge(0, 1), decompose(0, (10, 10, 10))],
                              proj=[(0, W.CYCLIC), (1, W.BLOCK), (2, W.CYCLIC)])])
    pp, out = matmul_gpu(tm, cs, 3)
    off = 0
    for i, c in enumerate(cs):
        P = int(c["nodes"]) * int(c["gpus"])
        per, tot = oracle.matmul_cost(c, 3)
        assert (pp[off:off + P] == per).all() and tuple(out[i]) == tot
        off += P


def test_matmul_random_chains(tm):
    say("matmul, random chains with cyclic projections")
    cs = np.concatenate([W.random_chain_instance((20, 24, 17), 6, 4, 48, seed=11, max_ops=4, cyclic_pct=30),
                         W.random_chain_instance((33, 9, 40), 8, 8, 24, seed=12, max_ops=5, cyclic_pct=50),
                         W.random_chain_instance((300, 6, 5), 3, 8, 8, seed=13, max_ops=3, cyclic_pct=100),
                         # 9000 classes along dim 0: the class blocks do not fit LDS (read in place)
                         W.batch([W.candidate((9000, 2, 3), 2, 4, [merge(0, 1), decompose(0, (8, 1, 1))],
                                              proj=[(0, W.CYCLIC), (1, W.BLOCK), (2, W.BLOCK)])])])
    pp, out = matmul_gpu(tm, cs, 5)
    off = 0
    for i, c in enumerate(cs):
        P = int(c["nodes"]) * int(c["gpus"])
        per, tot = oracle.matmul_cost(c, 5)
        assert (pp[off:off + P] == per).all(), i
        assert tuple(out[i]) == tot, i
        off += P


# ---------------------------------------------------------------- plans and graphs

def test_plan_graph_replay_deterministic(tm):
    import torch
    say("plan graph replay, layouts")
    cs = W.c3_candidates(1500, seed=3, ranks=(3,), octaves=(3, 6))
    st = W.c3_stencil(3)
    exp = oracle.stencil_cost_batch(cs[:300], st)
    ref = None
    for cpi in [0, 4096, 1 << 15, 1 << 20]:
        plan = tm.Plan(16, 16)  # grows on load
        plan.load(cs, st, cells_per_item=cpi)
        out = torch.empty((len(cs), 4), dtype=torch.int64, device="cuda")
        best = torch.empty(1, dtype=torch.int64, device="cuda")
        for rep in range(3):
            plan.run(out, best)
            torch.cuda.synchronize()
            got = out.cpu().numpy().copy()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            if ref is None:
                ref = got
                assert (got[:300] == exp).all()
            assert (got == ref).all()
        for stage in (0, 1, 2):
            plan.run_stage(stage, out, best)
        torch.cuda.synchronize()
        assert (out.cpu().numpy() == ref).all()
        assert int(best.cpu()[0]) == oracle.select_best(ref)
        plan.close()
    one = gpu_costs(tm, cs, st)
    assert (one == ref).all()


def test_plan_run_map_one_graph(tm):
    """The run and the winner's map in one graph equal a run followed by a separate
    map launch, on every replay (eager work between them), and again after the
    map buffer or the batch changes."""
    import torch
    say("plan run + map in one graph")
    st = W.c3_stencil(3)
    batches = [W.c3_candidates(600, seed=5, ranks=(3,), octaves=(3, 6)),
               W.c3_candidates(300, seed=6, ranks=(2, 3), octaves=(3, 7))]
    plan = tm.Plan(16, 16)
    for cs in batches:
        plan.load(cs, st)
        pts = [int(np.prod(c["extent"][: int(c["lrank"])].astype(np.int64))) for c in cs]
        npts = max(pts)
        out = torch.empty((len(cs), 4), dtype=torch.int64, device="cuda")
        best = torch.empty(1, dtype=torch.int64, device="cuda")
        plan.run(out, best)
        ref_map = torch.full((npts,), -7, dtype=torch.int32, device="cuda")
        plan.materialize(ref_map, d_index=best)
        torch.cuda.synchronize()
        ref_out, ref_best, ref_m = out.cpu().numpy().copy(), int(best.cpu()[0]), ref_map.cpu().numpy()
        assert ref_best == oracle.select_best(ref_out)
        npb = pts[ref_best]
        assert (ref_m[:npb] == oracle.proc_map(cs[ref_best]).ravel()).all()
        for m_rep in range(2):  # a second map buffer forces a new graph
            pmap = torch.full((npts,), -1, dtype=torch.int32, device="cuda")
            for rep in range(3):
                out.fill_(-1)
                plan.run_map(out, best, pmap)
                torch.cuda.synchronize()
                _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
                assert (out.cpu().numpy() == ref_out).all()
                assert int(best.cpu()[0]) == ref_best
                assert (pmap.cpu().numpy()[:npb] == ref_m[:npb]).all()
        with pytest.raises(RuntimeError):
            plan.run_map(out, best, torch.empty(npts - 1, dtype=torch.int32, device="cuda"))
    plan.close()


def test_plan_autotune_keeps_results(tm):
    import torch
    say("plan autotune")
    cands = W.c2_candidates(oracle.enumerate_factorizations(128, 3), extent=(128, 96, 64))
    st = W.c2_stencil()
    plan = tm.Plan(len(cands), 1)
    plan.load(cands, st)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    a = out.cpu().numpy().copy()
    cpi, wg = plan.autotune(out)
    say("  chose", cpi, wg)
    plan.run(out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == a).all()
    assert (a == oracle.stencil_cost_batch(cands, st)).all()
    # fixed launch configurations give the same counts
    for cpi, wg in ((1 << 12, 1), (1 << 15, 0), (0, 2)):
        say("  set_launch", cpi, wg)
        plan.set_launch(cpi, wg)
        out.fill_(-1)
        plan.run(out)
        torch.cuda.synchronize()
        assert (out.cpu().numpy() == a).all()
    plan.close()


def test_select_segments(tm):
    import torch
    say("segmented select")
    rng = np.random.default_rng(0)
    costs = np.zeros((1000, 4), np.int64)
    costs[:, 2] = rng.integers(0, 5, size=1000)
    costs[:, 3] = rng.integers(0, 3, size=1000)
    seg = [0, 10, 10, 300, 999, 1000]
    got = tm.tm_select_best(torch.from_numpy(costs).cuda(), seg).cpu().numpy()
    for s in range(len(seg) - 1):
        a, b = seg[s], seg[s + 1]
        assert got[s] == (oracle.select_best(costs[a:b]) if b > a else -1)


# ---------------------------------------------------------------- decompose vs Alg. A1 study

def test_study_full_size(tm):
    """Sec. 6.3's 180 2-D configurations at full size (up to 20,000 x 640,000 points):
    every candidate is a bijective block chain with blocks wider than the halo, so its
    total volume has the closed form sum_m 2 h (f_m - 1) prod_{j != m} l_j (both
    directions, Sec. 4.1's counting); single-node machines send nothing between nodes;
    the smallest configurations are checked against the oracle exactly."""
    import torch
    say("study: 2 x 180 configurations x 4 candidates at full size")
    cf = W.study_configs(long_last=True) + W.study_configs(long_last=False)
    fd = [oracle.decompose_argmin(g, ext, (1, 1)) for a, s_, g, ext, n, gp in cf]
    fg = [oracle.greedy_grid(g, 2) for a, s_, g, ext, n, gp in cf]
    cands = W.study_candidates(cf, fd, fg)
    st = W.stencil((1, 1), 8)
    plan = tm.Plan(len(cands), 1)
    plan.load(cands, st)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    plan.close()
    for i, (a, s_, g, (l0, l1), n, gp) in enumerate(cf):
        for j, f in enumerate((fd[i], fg[i])):
            assert f[0] <= l0 and f[1] <= l1
            cells = 2 * (f[0] - 1) * l1 + 2 * (f[1] - 1) * l0
            for o in range(2):
                row = got[4 * i + 2 * j + o]
                assert row[0] == cells and row[2] == 8 * cells, (cf[i], f, o)
                assert 0 <= row[1] <= row[0]
                if n == 1:
                    assert row[1] == 0
    small = [i for i, x in enumerate(cf) if x[3][0] * x[3][1] <= 2_100_000]
    assert len(small) >= 24
    idx = [4 * i + t for i in small for t in range(4)]
    assert (got[idx] == oracle.stencil_cost_batch(cands[idx], st)).all()


# ---------------------------------------------------------------- front end

def test_translated_mappers(tm):
    """Mappers written in the mapping language, translated by the front end, then
    evaluated on the GPU: costs and maps against the oracle."""
    from test_frontend_cpu import HIER, ROWS, TILES
    say("translated mappers")
    cases = []
    for src, task in ((TILES, "stencil_step"), (HIER, "cannon_tiles"), (ROWS, "any")):
        for ext, n, g in (((64, 64), 4, 4), ((96, 40), 6, 8), ((130, 67), 5, 2)):
            cases.append(tm.tm_parse_index_task_map(src, task, ext, n, g))
    cands = W.batch(cases)
    for h in ((1, 1), (2, 3)):
        st = W.stencil(h, 8)
        assert (gpu_costs(tm, cands, st) == oracle.stencil_cost_batch(cands, st)).all()
    for c in cands:
        assert (tm.tm_proc_map(c).cpu().numpy() == oracle.proc_map(c)).all()


# ---------------------------------------------------------------- node-level volume, two-level families

def node_costs(tm, cands, st):
    import torch
    out = tm.tm_eval_stencil_node_batch(cands, st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_node_level_parity(tm):
    say("node-level volume: random chains and two-level families")
    cs = W.random_candidates(600, seed=29, ranks=(2, 3), octaves=(1, 4), nodes_max=16, max_ops=4, cyclic_pct=25)
    for k, idx, sub in by_rank(cs):
        st = W.stencil((2,) * k, 8)
        assert (node_costs(tm, sub, st) == oracle.stencil_node_cost_batch(sub, st)).all()
    fam = W.two_level_candidates((32, 48, 40), 16, 8, oracle.enumerate_factorizations(16, 3),
                                 oracle.enumerate_factorizations(8, 3))
    st = W.c2_stencil()
    assert (node_costs(tm, fam, st) == oracle.stencil_node_cost_batch(fam, st)).all()
    assert (gpu_costs(tm, fam, st) == oracle.stencil_cost_batch(fam, st)).all()


def test_two_level_full_size(tm):
    """512^3 on 16 x 8, halo 2: all 15 x 10 node x GPU grids, both variants: the
    node-level volume of every candidate equals the node grid's surface-area count
    (blocks are at least 32 wide), and it never exceeds the per-processor
    inter-node volume."""
    say("two-level families at 512^3")
    fn_all = oracle.enumerate_factorizations(16, 3)
    fg_all = oracle.enumerate_factorizations(8, 3)
    fam = W.two_level_candidates((512, 512, 512), 16, 8, fn_all, fg_all)
    st = W.c2_stencil()
    node = node_costs(tm, fam, st)
    proc = gpu_costs(tm, fam, st)
    i = 0
    for fn in fn_all:
        for fg in fg_all:
            closed = sum(2 * 2 * (fn[m] - 1) * 512 * 512 for m in range(3))
            assert node[i][0] == closed and node[i + 1][0] == closed, (fn, fg)
            i += 2
    assert (node[:, 0] <= proc[:, 1]).all()


# ---------------------------------------------------------------- limits

def test_limits(tm):
    """Edges of the documented limits: a chain of the maximum 8 transformations, a
    final space of 32,760 processors (the largest owner table the LDS budget holds
    for these kernels) and one past it (TM_ENOTSUP, nothing launched), and a
    candidate of 2^32 points whose counts need 64 bits (closed form)."""
    import torch
    say("limits")
    eight = W.candidate((40, 36), 6, 4, [merge(0, 1), split(0, 4), swap(0, 1), merge(0, 1), split(0, 8),
                                         balance_split(1, 2), merge(1, 2), swap(0, 1)])
    assert tm.tm_validate(eight)[0] == 0
    big = W.candidate((300, 280), 4095, 8, [merge(0, 1), decompose(0, (182, 180))])
    cands = W.batch([eight])
    st = W.stencil((2, 3), 8)
    assert (gpu_costs(tm, cands, st) == oracle.stencil_cost_batch(cands, st)).all()
    assert (gpu_costs(tm, W.batch([big]), st) == oracle.stencil_cost_batch(W.batch([big]), st)).all()
    assert (tm.tm_proc_map(big).cpu().numpy() == oracle.proc_map(big)).all()
    too_big = W.candidate((300, 300), 4097, 8, [merge(0, 1), decompose(0, (241, 136))])
    out = torch.full((1, 4), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_eval_stencil_batch(W.batch([too_big]), st, out)
    assert e.value.code == tm.TM_ENOTSUP
    torch.cuda.synchronize()
    assert (out.cpu() == -5).all()
    # 2048 x 2048 x 1024 = 2^32 points, bijective blocks: V = sum_m 2 h (f_m - 1) prod_{j != m} l_j
    huge = W.candidate((2048, 2048, 1024), 16, 8, [merge(0, 1), decompose(0, (4, 8, 4))])
    st3 = W.stencil((2, 2, 2), 8)
    got = gpu_costs(tm, W.batch([huge]), st3)[0]
    ext, f = (2048, 2048, 1024), (4, 8, 4)
    cells = sum(2 * 2 * (f[m] - 1) * (ext[0] * ext[1] * ext[2] // ext[m]) for m in range(3))
    assert got[0] == cells and got[2] == 8 * cells and 0 < got[1] < got[0]


def test_class_structures(tm):
    """Candidates with many and few coordinate classes per dim, bit-exact against
    the oracle: blocks narrower and wider than the halo, one to 64 blocks along a
    dim, long last dims (512 to 1300 cells), cyclic last dims (a class per
    coordinate), launch rank 4, halos 1 to 4 per dim, and node-level counts for the
    same candidates."""
    say("class structures")
    P = 16
    cases = []
    for ext, F in [((24, 40, 512), (1, 1, 16)), ((24, 40, 512), (1, 2, 8)), ((24, 40, 512), (2, 2, 4)),
                   ((24, 40, 512), (16, 1, 1)), ((24, 40, 512), (4, 4, 1)), ((24, 40, 512), (1, 16, 1)),
                   ((9, 13, 509), (2, 1, 8)), ((6, 10, 1300), (2, 2, 4)), ((5, 7, 520), (1, 1, 16))]:
        for nodes, g in ((4, 4), (16, 1), (1, 16)):
            cases.append(W.candidate(ext, nodes, g, [merge(0, 1), decompose(0, F)]))
    cyc = W.candidate((24, 40, 512), 4, 4, [merge(0, 1), decompose(0, (2, 1, 8))],
                      proj=[(0, W.BLOCK), (1, W.BLOCK), (2, W.CYCLIC)])
    cases.append(cyc)
    wide = W.candidate((24, 40, 512), 8, 8, [merge(0, 1), decompose(0, (1, 1, 64))])
    cases.append(wide)
    cands = W.batch(cases)
    for halo in [(1, 1, 1), (2, 2, 2), (3, 1, 4), (4, 4, 2)]:
        st = W.stencil(halo, 8)
        exp = oracle.stencil_cost_batch(cands, st)
        assert (gpu_costs(tm, cands, st) == exp).all(), halo
    st = W.stencil((2, 3, 2), 8)
    exp = oracle.stencil_node_cost_batch(cands, st)
    import torch
    got = tm.tm_eval_stencil_node_batch(cands, st)
    torch.cuda.synchronize()
    assert (got.cpu().numpy() == exp).all()
    # launch rank 4: three outer dims (two in the slower prefix)
    r4 = W.batch([W.candidate((4, 6, 10, 300), 4, 4, [merge(0, 1), decompose(0, F)])
                  for F in [(2, 1, 2, 4), (1, 4, 1, 4), (4, 1, 1, 4), (1, 1, 1, 16)]])
    st4 = W.stencil((2, 1, 3, 2), 8)
    assert (gpu_costs(tm, r4, st4) == oracle.stencil_cost_batch(r4, st4)).all()


def test_cells_per_item_limit(tm):
    """Work items of more than 2^26 cells are rejected before anything runs (the
    counting kernel's 32-bit per-lane counts stay below 2^31 within one item); 2^26
    itself is accepted and gives the same costs."""
    import torch
    say("cells per item limit")
    cands = W.batch([W.candidate((64, 40, 96), 2, 4, [merge(0, 1), decompose(0, (2, 2, 2))])])
    st = W.stencil((2, 1, 2), 8)
    plan = tm.Plan(4, 1)
    with pytest.raises(tm.TaskmapError) as e:
        plan.load(cands, st, cells_per_item=(1 << 26) + 1)
    assert e.value.code == tm.TM_EINVAL
    plan.load(cands, st, cells_per_item=1 << 26)
    out = torch.empty((1, 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == oracle.stencil_cost_batch(cands, st)).all()
    with pytest.raises(tm.TaskmapError):
        plan.set_launch((1 << 26) + 1, 0)
    plan.close()
