"""GPU tests of the learned ranker and the ranked search: features, forward and
gradient element by element against the reference in the same bf16 arithmetic, one Adam step,
training progress, save/load, and search quality against exhaustive search."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp

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


def loaded_plan(tm, cands, st):
    p = tm.Plan(len(cands), 1)
    p.load(cands, st)
    return p


def exact_costs(tm, cands, st):
    import torch
    p = loaded_plan(tm, cands, st)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    p.run(out)
    torch.cuda.synchronize()
    return p, out


def test_features_parity(tm):
    import torch
    say("features")
    cs = np.concatenate([W.random_candidates(300, seed=41, ranks=(3,), octaves=(2, 9), nodes_max=64, max_ops=4,
                                             cyclic_pct=20),
                         W.c2_candidates(oracle.enumerate_factorizations(128, 3), extent=(96, 200, 64))])
    st = W.stencil((2, 1, 3), 8)
    p = loaded_plan(tm, cs, st)
    got = tm.tm_ranker_features(p).cpu().numpy()
    exp = np.stack([mlp.features(c, (2, 1, 3)) for c in cs])
    assert np.abs(got - exp).max() < 1e-5


def test_block_estimates_parity(tm):
    """The second stage's block-model estimates (owner keys of every processor-space
    coordinate, crossings, block boundaries) against the oracle's, candidate by
    candidate: block projections (the boundary-sum branch, halos wider than some
    blocks) and cyclic ones (the crossing-fraction branch)."""
    say("block-model estimates")
    cs = np.concatenate([W.random_candidates(300, seed=43, ranks=(3,), octaves=(2, 8), nodes_max=64, max_ops=4,
                                             cyclic_pct=20),
                         W.c2_candidates(oracle.enumerate_factorizations(128, 3), extent=(96, 200, 64))])
    st = W.stencil((2, 1, 3), 8)
    p = loaded_plan(tm, cs, st)
    got = tm.tm_ranker_block_estimates(p).cpu().numpy()
    exp = np.array([mlp.block_estimates(c, (2, 1, 3), oracle.chain_table) for c in cs])
    # every launch dim block-projected onto one final dim: sums of integer cell counts,
    # exact in fp64 in any order; otherwise the crossing fractions are fp32 ratios on
    # the GPU (within 2^-22 of the exact ratio: a rounded reciprocal, then a rounded
    # product), so the estimates agree to 1e-6 relative
    simple = np.array([int(c["mrank"]) == int(c["lrank"]) and
                       sorted(int(x) for x in c["proj_src"][:int(c["mrank"])]) == list(range(int(c["lrank"]))) and
                       all(int(x) == W.BLOCK for x in c["proj_mode"][:int(c["mrank"])]) for c in cs])
    say(f"  {int(simple.sum())} block-model candidates, {int((~simple).sum())} with crossing fractions")
    assert simple.sum() > 100 and (~simple).sum() > 20
    assert (got[simple] == exp[simple]).all()
    assert np.allclose(got[~simple], exp[~simple], rtol=1e-6, atol=0), np.abs(got - exp).max()


# Element-wise bar of the ranker kernels against the reference in the same bf16
# arithmetic: |got - ref| <= RTOL |ref| + ATOL max|ref| per tensor.  What remains
# between the two is the order of the fp32 sums (the reference sums in float64):
# it moves a stored bf16 activation or gradient by one bf16 step now and then, which
# an fp32 emulation of the kernels puts at <= 2.2e-4 of a tensor's largest value.
RTOL, ATOL = 1e-2, 1e-3


def _elementwise_ok(got, ref, what):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    lim = RTOL * np.abs(ref) + ATOL * max(np.abs(ref).max(), 1e-30)
    err = np.abs(got - ref)
    bad = int((err > lim).sum())
    say(f"  {what}: {ref.size} values, max err / max|ref| {err.max() / max(np.abs(ref).max(), 1e-30):.2e}, "
        f"over the bar: {bad}")
    return bad == 0


# 70,001 rows take the persistent inference kernel (weights held in registers), the
# smaller ones the per-tile kernel
@pytest.mark.parametrize("rows,seed", [(333, 3), (1000, 4), (64, 6), (70001, 8)])
def test_forward_parity(tm, rows, seed):
    import torch
    say(f"forward rows={rows} seed={seed}")
    r = tm.Ranker(seed=seed)
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(rows, mlp.F)).astype(np.float32)
    y = r.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    p = r.get_params().cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(p, X.astype(np.float64), "bf16")
    assert _elementwise_ok(y, ref, "outputs")


def _determined_rows(p, X, rows, margin=2e-5):
    """The first `rows` rows of X whose every hidden ReLU decision is determined:
    each pre-activation lies farther from zero than `margin` times the sum of the
    magnitudes of its terms, well above what the order of the fp32 sums (at most
    about 256 * 2^-24 of that sum) and a stored bf16 input one step off can move it.
    Elsewhere the kernel and the reference may take different decisions, both
    correct for their own sums, and one flipped mask changes a whole column of the
    weight gradient."""
    q = mlp.bf16_round
    w1, b1, w2, b2, w3, b3, _, _ = mlp.unpack(p)
    keep = np.ones(len(X), dtype=bool)
    h = q(X)
    for w, b in ((q(w1), b1), (q(w2), b2), (q(w3), b3)):
        z = h @ w + b
        mag = np.abs(h) @ np.abs(w) + np.abs(b)
        keep &= (np.abs(z) > margin * mag).all(axis=1)
        h = q(np.maximum(z, 0))
    idx = np.nonzero(keep)[0]
    assert len(idx) >= rows, (len(idx), rows)
    return X[idx[:rows]]


@pytest.mark.parametrize("rows,seed", [(1000, 5), (1537, 7)])
def test_gradient_parity(tm, rows, seed):
    import torch
    say(f"gradient rows={rows} seed={seed}")
    r = tm.Ranker(seed=seed)
    rng = np.random.default_rng(seed)
    p = r.get_params().cpu().numpy().astype(np.float64)
    X = rng.uniform(-1, 1, size=(4 * rows, mlp.F)).astype(np.float32)
    X = _determined_rows(p, X.astype(np.float64), rows).astype(np.float32)
    T = rng.normal(0, 1, size=(rows, mlp.O)).astype(np.float32)
    g = r.grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()).cpu().numpy().astype(np.float64)
    _, ref = mlp.loss_and_grad(p, X.astype(np.float64), T.astype(np.float64), "bf16")
    L = mlp.layout()
    ok = [_elementwise_ok(g[a:b], ref[a:b], k) for k, (a, b) in
          ((k, L[k]) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4"))]
    assert all(ok)


def test_one_adam_step(tm):
    import torch
    say("adam step")
    r = tm.Ranker(seed=9)
    p0 = r.get_params().cpu().numpy().astype(np.float64)
    cands = W.random_candidates(700, seed=9, ranks=(3,), octaves=(3, 5), nodes_max=16, max_ops=3)
    st = W.c3_stencil(3)
    plan, costs = exact_costs(tm, cands, st)
    feat = tm.tm_ranker_features(plan)
    twin = tm.Ranker(seed=9)
    r.train(feat, costs, epochs=1, batch=len(cands), lr=1e-3, seed=1)
    mu0, s0, mu1, s1 = r.scaling()
    c = costs.cpu().numpy().astype(np.float64)
    fb = feat.cpu().numpy()
    # residual targets over the base features (fp32, as trained): the descriptor
    # estimate for bytes, 0 for inter-node bytes
    b0 = (np.float32(32) * fb[:, 23]).astype(np.float64)
    b1 = (np.float32(32) * fb[:, 60]).astype(np.float64)
    T = np.stack([(np.log2(1 + c[:, 2]) - b0 - mu0) / s0, (np.log2(1 + c[:, 3]) - b1 - mu1) / s1],
                 1).astype(np.float32)
    # the scaling is the mean / standard deviation of those residuals
    assert abs(np.mean(np.log2(1 + c[:, 2]) - b0) - mu0) < 1e-4
    assert abs(np.std(np.log2(1 + c[:, 3]) - b1) - s1) < 1e-3 * max(1.0, s1)
    g = twin.grad(feat, torch.from_numpy(T).cuda()).cpu().numpy().astype(np.float64)
    exp, _, _ = mlp.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    got = r.get_params().cpu().numpy().astype(np.float64)
    assert np.abs(got - exp).max() < 1e-5


def search_instances(tm, count, seed, octaves, min_cands=1024, fact=None):
    fact = fact or tm.tm_enumerate_factorizations
    out = []
    first = 0
    while len(out) < count:
        for ext, n, g in W.random_instances(64, seed=seed, first=first, octaves=octaves):
            fs = fact(n * g, 3)
            if len(fs) * 32 >= min_cands:
                out.append((ext, n, g, fs))
                if len(out) == count:
                    break
        first += 64
    return out


def build_batch(instances):
    cands, seg = [], [0]
    for ext, n, g, fs in instances:
        c = W.instance_candidates(ext, n, g, fs)
        cands.append(c)
        seg.append(seg[-1] + len(c))
    return np.concatenate(cands), np.array(seg, np.int64)


@pytest.fixture(scope="module")
def trained(tm):
    import torch
    say("training set")
    inst = search_instances(tm, 48, seed=1, octaves=(3, 6))
    cands, _ = build_batch(inst)
    st = W.c3_stencil(3)
    plan, costs = exact_costs(tm, cands, st)
    feat = tm.tm_ranker_features(plan)
    r = tm.Ranker(seed=1)
    say(f"  training on {len(cands)} candidates")
    losses = r.train(feat, costs, epochs=20, batch=4096, lr=2e-3, seed=1)
    say("  losses", [round(x, 4) for x in losses])
    torch.cuda.synchronize()
    return r, losses


def test_training_reduces_loss(tm, trained):
    r, losses = trained
    assert losses[-1] < 0.5 * losses[0]


def test_save_load_roundtrip(tm, trained):
    import torch
    r, _ = trained
    X = torch.rand((200, 64), device="cuda") * 2 - 1
    a = r.forward(X).cpu().numpy()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ranker.bin")
        r.save(path)
        r2 = tm.Ranker(path=path)
        b = r2.forward(X).cpu().numpy()
        assert r2.scaling() == r.scaling()
    assert (a == b).all()


def test_search_matches_exhaustive_when_topk_covers(tm, trained):
    say("search, topk covers every instance")
    r, _ = trained
    inst = search_instances(tm, 3, seed=7, octaves=(3, 5), min_cands=0)
    cands, seg = build_batch(inst)
    plan = loaded_plan(tm, cands, W.c3_stencil(3))
    b_ex, c_ex = tm.tm_search(plan, None, seg)
    top = int(np.diff(seg).max())
    b_rk, c_rk = tm.tm_search(plan, r, seg, topk=top)
    assert (b_ex.cpu() == b_rk.cpu()).all() and (c_ex.cpu() == c_rk.cpu()).all()
    b_2, c_2 = tm.tm_search(plan, r, seg, topk=top, prefilter=top)
    assert (b_ex.cpu() == b_2.cpu()).all() and (c_ex.cpu() == c_2.cpu()).all()
    # the exhaustive search against the oracle on the smallest instance
    s = int(np.argmin(np.diff(seg)))
    sub = cands[seg[s]:seg[s + 1]]
    exp = oracle.stencil_cost_batch(sub, W.c3_stencil(3))
    e = oracle.select_best(exp)
    assert int(b_ex.cpu()[s]) == e and tuple(c_ex.cpu().numpy()[s]) == tuple(exp[e])


def _at_opt(ce, c):
    return (ce[:, 2] == c[:, 2]) & (ce[:, 3] == c[:, 3])


def _lex_le(a, b):
    """(bytes, inter-node bytes) of a <= those of b, row by row."""
    return (a[:, 2] < b[:, 2]) | ((a[:, 2] == b[:, 2]) & (a[:, 3] <= b[:, 3]))


@pytest.fixture(scope="module")
def held_out(tm):
    inst = search_instances(tm, 200, seed=2, octaves=(3, 6))
    cands, seg = build_batch(inst)
    plan = loaded_plan(tm, cands, W.c3_stencil(3))
    b_ex, c_ex = tm.tm_search(plan, None, seg)
    return inst, cands, seg, plan, c_ex.cpu().numpy()


PREFILTER, TOPK = 256, 32  # the search's default: the network keeps 256, the estimates choose 32


def test_ranked_search_quality(tm, trained, held_out):
    import torch
    say("ranked search quality")
    r, _ = trained
    inst, cands, seg, plan, ce = held_out
    b_rk, c_rk = tm.tm_search(plan, r, seg, topk=TOPK, prefilter=PREFILTER)
    torch.cuda.synchronize()
    cr = c_rk.cpu().numpy()
    ok = _at_opt(ce, cr)
    say(f"  {ok.sum()}/{len(ok)} instances at the exhaustive optimum; candidates {len(cands)}; "
        f"misses on total bytes {int((ce[:, 2] != cr[:, 2]).sum())}, on inter-node bytes only "
        f"{int(((ce[:, 2] == cr[:, 2]) & (ce[:, 3] != cr[:, 3])).sum())}")
    assert len(ok) >= 200 and ok.mean() >= 0.99
    # never better than the optimum
    assert _lex_le(ce, cr).all()


def _k_smallest(score, a, e, k):
    """Indices a..e-1 of the k smallest (score, index) pairs."""
    idx = np.arange(a, e)
    return idx[np.lexsort((idx, score[a:e]))[:k]]


@pytest.mark.parametrize("k", [3, 7, 20])
def test_topk_selection(tm, held_out, k):
    """The per-instance top-k below the instance's size, checked through the search:
    with an all-zero network and lambda = 0 a candidate's score is its descriptor
    ghost estimate plus the (zero) mean, the same fp32 value as 32 times feature 23,
    so the k smallest (score, index) pairs of each instance are known on the host;
    the search must return the cheapest of exactly those (ties in the estimate are
    common, so the index order of equal scores matters)."""
    import torch
    say(f"top-{k} selection")
    inst, cands, seg, plan, ce = held_out
    r = tm.Ranker(seed=4)
    r.set_params(torch.zeros(tm.tm_ranker_param_count(), dtype=torch.float32, device="cuda"))
    mu0 = np.float32(r.scaling()[0])
    feat = tm.tm_ranker_features(plan).cpu().numpy()
    score = np.float32(32) * feat[:, 23].astype(np.float32) + mu0
    b, c = tm.tm_search(plan, r, seg, topk=k, lam=0.0)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    allc, b, c = out.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    for s_ in range(len(seg) - 1):
        a, e = int(seg[s_]), int(seg[s_ + 1])
        assert e - a > k
        sel = _k_smallest(score, a, e, k)
        sub = allc[sel]
        best = sel[np.lexsort((sel, sub[:, 3], sub[:, 2]))[0]]
        assert b[s_] == best - a and tuple(c[s_]) == tuple(allc[best]), s_
    r.close()


@pytest.mark.parametrize("k", [1, 100, 4096])
def test_topk_selection_one_long_segment(tm, held_out, k):
    """The selection over one segment of every held-out candidate (several hundred
    thousand entries: many passes of the workgroup over its segment, long runs of
    equal scores): the search returns the cheapest of the k smallest (score, index)
    pairs, as known on the host."""
    import torch
    say(f"top-{k} selection over one long segment")
    inst, cands, seg, plan, ce = held_out
    r = tm.Ranker(seed=4)
    r.set_params(torch.zeros(tm.tm_ranker_param_count(), dtype=torch.float32, device="cuda"))
    mu0 = np.float32(r.scaling()[0])
    feat = tm.tm_ranker_features(plan).cpu().numpy()
    score = np.float32(32) * feat[:, 23].astype(np.float32) + mu0
    one = np.array([0, len(cands)], np.int64)
    b, c = tm.tm_search(plan, r, one, topk=k, lam=0.0)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    allc, b, c = out.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    say(f"  {len(cands)} entries, {len(np.unique(score))} distinct scores")
    sel = _k_smallest(score, 0, len(cands), k)
    sub = allc[sel]
    best = sel[np.lexsort((sel, sub[:, 3], sub[:, 2]))[0]]
    assert b[0] == best and tuple(c[0]) == tuple(allc[best])
    r.close()


@pytest.mark.parametrize("pre,k", [(40, 5), (300, 17)])
def test_two_stage_selection(tm, held_out, pre, k):
    """The two-stage search's selections, checked through its result: with an
    all-zero network and lambda = 0, the first stage keeps each instance's `pre`
    smallest (32 * feature 23 + mean, index) pairs, the second the k smallest
    (fp32 log2(1 + block-model ghost estimate), index) pairs among those; the
    search must return the cheapest of exactly those k."""
    import torch
    say(f"two-stage selection, prefilter {pre}, top-{k}")
    inst, cands, seg, plan, ce = held_out
    r = tm.Ranker(seed=4)
    r.set_params(torch.zeros(tm.tm_ranker_param_count(), dtype=torch.float32, device="cuda"))
    mu0 = np.float32(r.scaling()[0])
    feat = tm.tm_ranker_features(plan).cpu().numpy()
    s1 = np.float32(32) * feat[:, 23].astype(np.float32) + mu0
    est = tm.tm_ranker_block_estimates(plan).cpu().numpy()
    s2 = np.log2(1.0 + est[:, 0]).astype(np.float32)
    b, c = tm.tm_search(plan, r, seg, topk=k, lam=0.0, prefilter=pre)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    allc, b, c = out.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    for s_ in range(len(seg) - 1):
        a, e = int(seg[s_]), int(seg[s_ + 1])
        kept = _k_smallest(s1, a, e, pre)
        kept = np.sort(kept)
        sel = kept[np.lexsort((kept, s2[kept]))[:k]]
        sub = allc[sel]
        best = sel[np.lexsort((sel, sub[:, 3], sub[:, 2]))[0]]
        assert b[s_] == best - a and tuple(c[s_]) == tuple(allc[best]), s_
    r.close()


def test_network_gain(tm, trained, held_out):
    """What the trained network adds to the search, measured against the method
    without it -- ranking by the descriptor estimate alone (an all-zero network: the
    score is the estimate) -- as the share of held-out instances whose top-k holds
    the exhaustive optimum, k = 4 .. 256 (the network's cut is the first stage of
    the two-stage search); and what the search adds over the paper's own choice
    without any search, decompose's argmin factorization of the surface-area
    objective (Sec. 4.3) under the better of the two machine orders, evaluated
    exactly.  The descriptor estimate is exact for bijective block chains, so it
    ranks total bytes well; the network's inter-node head adds the node structure
    the estimate does not see."""
    import torch
    say("network gain")
    r, _ = trained
    inst, cands, seg, plan, ce = held_out
    r0 = tm.Ranker(seed=1)
    r0.set_params(torch.zeros(tm.tm_ranker_param_count(), dtype=torch.float32, device="cuda"))
    rates = {}
    for k in (4, 16, 64, 256):
        _, c_tr = tm.tm_search(plan, r, seg, topk=k)
        _, c_0 = tm.tm_search(plan, r0, seg, topk=k)
        torch.cuda.synchronize()
        rates[k] = (_at_opt(ce, c_tr.cpu().numpy()).mean(), _at_opt(ce, c_0.cpu().numpy()).mean())
    say("  optimum in the top-k (trained, estimate only): " +
        ", ".join(f"top-{k} {a:.3f} {b:.3f}" for k, (a, b) in rates.items()))
    for k, (a, b) in rates.items():
        assert a >= b - 0.02, (k, a, b)
    assert rates[64][0] > rates[64][1]
    _, c_rk = tm.tm_search(plan, r, seg, topk=TOPK, prefilter=PREFILTER)
    cr = c_rk.cpu().numpy()
    rate_tr = _at_opt(ce, cr).mean()
    assert rate_tr >= 0.99
    # decompose's pick, both machine orders, exact costs
    st = W.c3_stencil(3)
    base = []
    for ext, n, g, fs in inst:
        f = tm.tm_decompose_argmin(n * g, ext, (1, 1, 1))
        base.append(W.candidate(ext, n, g, [W.merge(0, 1), W.decompose(0, f)]))
        base.append(W.candidate(ext, n, g, [W.swap(0, 1), W.merge(0, 1), W.decompose(0, f)]))
    base = W.batch(base)
    cb = tm.tm_eval_stencil_batch(base, st).cpu().numpy()
    even, odd = cb[0::2], cb[1::2]
    cd = np.where(_lex_le(even, odd)[:, None], even, odd)
    assert _lex_le(ce, cd).all()  # the exhaustive optimum includes decompose's candidates
    better = ~_lex_le(cd, cr)
    worse = ~_lex_le(cr, cd)
    red_b = 1 - cr[:, 2].sum() / cd[:, 2].sum()
    red_i = 1 - cr[:, 3].sum() / max(1, cd[:, 3].sum())
    say(f"  ranked search vs decompose: better on {better.sum()}/{len(better)} instances, worse on "
        f"{worse.sum()}; total bytes -{100 * red_b:.1f} %, inter-node bytes -{100 * red_i:.1f} %")
    assert worse.mean() <= 1 - rate_tr + 1e-9
    assert better.sum() > 0
    r0.close()


def test_search_margin(tm, trained, held_out):
    """A score margin keeps, of the last stage's top-k, only candidates scoring within
    `margin` (log2 units) of the instance's best: a huge margin is plain top-k, 0.05
    keeps the quality bar with fewer exact evaluations, and nothing beats the
    optimum."""
    import torch
    say("search with a score margin")
    r, _ = trained
    inst, cands, seg, plan, ce = held_out
    _, c_k = tm.tm_search(plan, r, seg, topk=TOPK, prefilter=PREFILTER)
    _, c_m = tm.tm_search(plan, r, seg, topk=TOPK, prefilter=PREFILTER, margin=1e9)
    assert (c_k.cpu() == c_m.cpu()).all()
    _, c_5 = tm.tm_search(plan, r, seg, topk=TOPK, prefilter=PREFILTER, margin=0.05)
    torch.cuda.synchronize()
    c5 = c_5.cpu().numpy()
    rate = _at_opt(ce, c5).mean()
    say(f"  margin 0.05: {rate:.3f} of instances at the optimum")
    assert rate >= 0.98
    assert _lex_le(ce, c5).all()
    with pytest.raises(tm.TaskmapError):
        tm.tm_search(plan, r, seg, topk=64, margin=-1.0)
    with pytest.raises(tm.TaskmapError):
        tm.tm_search(plan, r, seg, topk=64, prefilter=32)  # below topk


def test_search_with_nonfinite_scores(tm, held_out):
    """A network whose parameters are all NaN scores every candidate +inf: the top-k
    then takes each instance's first k candidates by index, evaluates them exactly
    and returns the best of them, so no instance is left without a survivor."""
    import torch
    say("search with non-finite scores")
    inst, cands, seg, plan, ce = held_out
    r = tm.Ranker(seed=3)
    r.set_params(torch.full((tm.tm_ranker_param_count(),), float("nan"), dtype=torch.float32, device="cuda"))
    k = 4
    b, c = tm.tm_search(plan, r, seg, topk=k)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    allc, b, c = out.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    for s in range(len(seg) - 1):
        first = allc[seg[s]:seg[s] + k]
        e = int(np.lexsort((np.arange(len(first)), first[:, 3], first[:, 2]))[0])
        assert b[s] == e and tuple(c[s]) == tuple(first[e]), s
    r.close()
