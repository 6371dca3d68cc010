"""Pins for the ranker reference: finite differences for the gradient of the plain
network, hand-worked values of its bf16 arithmetic (where rounding happens and where
it does not), hand-worked feature vectors, and Adam's first step."""
import math

import numpy as np

import workloads as W
from oracle import mlp
from workloads import decompose, merge, swap


def small_params(seed=0):
    rng = np.random.default_rng(seed)
    L = mlp.layout()
    p = rng.normal(0, 0.08, size=L["count"])
    return p


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = small_params()
    X = rng.normal(0, 1, size=(6, mlp.F))
    T = rng.normal(0, 1, size=(6, mlp.O))
    _, g = mlp.loss_and_grad(p, X, T, arith="f64")
    L = mlp.layout()
    idx = np.concatenate([rng.integers(a, b, size=6) for a, b in
                          [L[k] for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")]])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp, _ = mlp.loss_and_grad(q, X, T, arith="f64")
        q[i] -= 2 * h
        lm, _ = mlp.loss_and_grad(q, X, T, arith="f64")
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8


def test_forward_of_identity_like_network():
    # a network that passes x0 through: y0 = relu(relu(relu(x0))) = x0 for x0 > 0
    L = mlp.layout()
    p = np.zeros(L["count"])
    p[L["w1"][0] + 0 * mlp.W + 0] = 1
    p[L["w2"][0] + 0 * mlp.W + 0] = 1
    p[L["w3"][0] + 0 * mlp.W + 0] = 1
    p[L["w4"][0] + 0 * mlp.O + 1] = 2
    p[L["b4"][0]] = 0.5
    X = np.zeros((3, mlp.F))
    X[:, 0] = [0.25, 1.5, -2]
    for arith in ("f64", "bf16"):
        y, _ = mlp.forward(p, X, arith)
        assert np.allclose(y[:, 0], 0.5) and np.allclose(y[:, 1], [0.5, 3.0, 0.0])


def _path_network(w=1.0, b1=0.0, b4=0.0):
    """Input 0 -> hidden unit 0 of every layer -> output 0, weights w, 1, 1, 1."""
    L = mlp.layout()
    p = np.zeros(L["count"])
    p[L["w1"][0]] = w
    p[L["b1"][0]] = b1
    p[L["w2"][0]] = 1
    p[L["w3"][0]] = 1
    p[L["w4"][0]] = 1
    p[L["b4"][0]] = b4
    return p


def test_bf16_arithmetic_rounds_activations_not_biases():
    """The defined arithmetic stores every hidden activation in bf16 (7 explicit
    mantissa bits: spacing 2^-7 just above 1) and keeps biases and outputs at full
    precision.  With x = 1 and bias 2^-9 + 2^-12 the first activation is
    1.00220703125, stored as 1.0; the output bias 2^-12 survives in the output."""
    p = _path_network(b1=2.0 ** -9 + 2.0 ** -12, b4=2.0 ** -12)
    X = np.zeros((1, mlp.F))
    X[0, 0] = 1.0
    y64, (_, h1_64, _, _) = mlp.forward(p, X, "f64")
    y16, (_, h1_16, _, _) = mlp.forward(p, X, "bf16")
    assert h1_64[0, 0] == 1 + 2.0 ** -9 + 2.0 ** -12 and h1_16[0, 0] == 1.0
    assert y64[0, 0] == 1 + 2.0 ** -9 + 2.0 ** -11 and y16[0, 0] == 1 + 2.0 ** -12
    # an activation exactly between two bf16 values goes to the even one:
    # 1 + 2^-8 lies between 1 and 1 + 2^-7 -> 1;  1 + 3 * 2^-8 -> 1 + 2^-6
    for b, exp in ((2.0 ** -8, 1.0), (3 * 2.0 ** -8, 1 + 2.0 ** -6)):
        _, (_, h1, _, _) = mlp.forward(_path_network(b1=b), X, "bf16")
        assert h1[0, 0] == exp
    # weights and inputs are bf16 too: w = 1 + 2^-9 and x = 1 + 2^-9 both read as 1
    y, _ = mlp.forward(_path_network(w=1 + 2.0 ** -9), X, "bf16")
    assert y[0, 0] == 1.0
    X2 = X.copy()
    X2[0, 0] = 1 + 2.0 ** -9
    y, _ = mlp.forward(_path_network(), X2, "bf16")
    assert y[0, 0] == 1.0


def test_bf16_arithmetic_rounds_hidden_gradients():
    """Backward: the output gradient dy = 2 (y - t) / (rows * outputs) stays at full
    precision (it weights W4's gradient directly); each hidden-layer gradient is
    stored in bf16.  One row, two outputs: dy = y - t.  With t0 = y0 - (1 + 2^-9) the
    output gradient is 1 + 2^-9, W4's gradient h3 * dy keeps it, the last hidden
    layer's gradient dy * w4 = 1 + 2^-9 is stored as 1.0 (so are b3's and W3's)."""
    p = _path_network()
    X = np.zeros((1, mlp.F))
    X[0, 0] = 1.0
    T = np.zeros((1, mlp.O))
    T[0, 0] = 1.0 - (1 + 2.0 ** -9)
    L = mlp.layout()
    _, g64 = mlp.loss_and_grad(p, X, T, "f64")
    _, g16 = mlp.loss_and_grad(p, X, T, "bf16")
    at = lambda g, k, i=0: g[L[k][0] + i]
    assert at(g64, "w4") == 1 + 2.0 ** -9 and at(g16, "w4") == 1 + 2.0 ** -9
    assert at(g64, "b4") == 1 + 2.0 ** -9 and at(g16, "b4") == 1 + 2.0 ** -9
    assert at(g64, "b3") == 1 + 2.0 ** -9 and at(g16, "b3") == 1.0
    assert at(g64, "w3") == 1 + 2.0 ** -9 and at(g16, "w3") == 1.0
    assert at(g16, "b1") == 1.0 and at(g16, "w1") == 1.0
    # units off the path get nothing: their activations are zero (ReLU mask)
    assert np.count_nonzero(g16) == np.count_nonzero(g64) == 8


def test_bf16_arithmetic_exact_when_representable():
    """With small-integer weights and inputs, sparse enough that every sum stays
    below 2^8, and a dyadic output gradient, nothing needs rounding: the bf16
    arithmetic gives exactly the plain network's outputs and gradient."""
    rng = np.random.default_rng(3)
    L = mlp.layout()
    p = np.zeros(L["count"])
    for k in ("w1", "w2", "w3", "w4"):
        a, b = L[k]
        m = rng.random(b - a) < 0.01
        p[a:b] = np.where(m, rng.integers(-1, 2, b - a), 0)
    for k in ("b1", "b2", "b3", "b4"):
        a, b = L[k]
        p[a:b] = rng.integers(0, 3, b - a)
    X = rng.integers(-2, 3, size=(8, mlp.F)).astype(np.float64)
    y64, acts = mlp.forward(p, X, "f64")
    assert max(np.abs(a).max() for a in acts[1:]) < 256 and np.abs(y64).max() < 256
    y16, _ = mlp.forward(p, X, "bf16")
    assert (y16 == y64).all()
    T = y64 - rng.integers(-3, 4, size=y64.shape)  # 2 (y - t) / 16: multiples of 1/8
    l64, g64 = mlp.loss_and_grad(p, X, T, "f64")
    l16, g16 = mlp.loss_and_grad(p, X, T, "bf16")
    assert l64 == l16 and (g64 == g16).all() and np.count_nonzero(g64) > 50


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    q, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # bias-corrected first step moves each parameter by lr * sign(g) (eps aside)
    assert np.allclose(q, p - 0.01 * np.sign(g), atol=1e-6)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 0.0], np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0  # tie to even
    assert r[2] == 1.0078125
    assert abs(r[3] - (-3.140625)) < 1e-12 and r[4] == 0.0


def test_features_hand_worked():
    # (64, 32) on 4 nodes x 2 GPUs, merge + decompose (4, 2) + swap(0,1), halo (1, 1)
    c = W.candidate((64, 32), 4, 2, [merge(0, 1), decompose(0, (4, 2)), swap(0, 1)])
    f = mlp.features(c, (1, 1))
    assert f[1] == 1 and f[0] == 0 and f[2] == 0
    assert math.isclose(f[4], 0.6) and math.isclose(f[5], 0.5)
    assert math.isclose(f[8], 2 / 6) and math.isclose(f[9], 1 / 3) and math.isclose(f[10], 3 / 9)
    assert math.isclose(f[11], 2 / 9) and math.isclose(f[12], 1 / 9)
    # after the swap the final shape is (2, 4): 2 blocks along dim 0, 4 along dim 1
    assert math.isclose(f[15], 1 / 9) and math.isclose(f[16], 2 / 9)
    assert math.isclose(f[19], (6 - 1) / 10) and math.isclose(f[20], (5 - 2) / 10)
    vf = 2 * (4 - 1) / 64 + 2 * (2 - 1) / 32
    # descriptor estimate: 1 block boundary along dim 0 (2 blocks), 3 along dim 1, 2h
    # cells of each cross-section at each: 2*1*32 + 2*3*64 = 448 ghost cells
    assert math.isclose(f[23], math.log2(1 + 448) / 32) and math.isclose(f[24], math.log2(1 + vf) / 4)
    assert math.isclose(f[25 + 1], 0.25) and math.isclose(f[25 + 4], 0.25) and math.isclose(f[25 + 2], 0.25)
    assert math.isclose(f[30], 2 / 5) and math.isclose(f[31], 1.0) and math.isclose(f[32], 3 / 5)
    assert f[39] == 0 and f[40] == 0 and math.isclose(f[41], 0 / 8)
    assert f[48] == 0 and f[53] == 2 / 8 and math.isclose(f[58], 1 / 3) and f[59] == 1
    assert f[60] == 0 and (f[61:64] == 0).all() and (f[36:39] == 0).all()  # no chain statistics
    # the block-model estimates from the chain table: final space (2, 4) after the
    # swap; decompose (4, 2) of merge(0,1) puts node = a mod 4 with a = F0-fastest
    # index, so along the final dim of size 4 (the old first factor) every step
    # changes node; along the other (size 2) a step adds 4 to a, which keeps a mod 4
    import oracle
    cells_t = (2 * (2 - 1) / 64 + 2 * (4 - 1) / 32) * 64 * 32   # = 448 ghost cells
    cells_i = (2 * (4 - 1) / 32) * 64 * 32                      # = 384 of them inter-node
    assert mlp.block_estimates(c, (1, 1), oracle.chain_table) == (cells_t, cells_i)
    # and both are exact here: the oracle's ghost count agrees
    gc, ic, _, _ = oracle.stencil_cost(c, W.stencil((1, 1), 8))
    assert (gc, ic) == (448, 384)


def test_features_hand_worked_cyclic():
    """The estimate's second branch (some launch dim not block-projected onto exactly
    one final dim).  (8, 6) on 2 nodes x 2 GPUs, merge(0,1) + decompose(0, (2, 2)),
    final dim 0 BLOCK from launch dim 0, final dim 1 CYCLIC from launch dim 1, halo
    (2, 1).  The chain gives node = a0, gpu = a1 (a = a0 + 2 a1; node = a mod 2),
    so proc = 2 a0 + a1.
      launch dim 0: block index x // 4, linear contribution 2 (x // 4) =
        [0,0,0,0,2,2,2,2]; cells with a differing value within 2 steps: x = 2..5,
        one distinct offset each -> 4, times 48 / 8 rows = 24 cells; along final
        dim 0 every step changes processor and node -> 24 total, 24 inter-node.
      launch dim 1: cyclic x mod 2 = [0,1,0,1,0,1]; every cell has one distinct
        offset -> 6, times 48 / 6 = 48 cells; along final dim 1 every step changes
        processor, never node -> 48 total, 0 inter-node.
    Estimate: 72 ghost cells, 24 inter-node; exact here (each cell's two foreign
    owners differ): the oracle's count agrees."""
    import oracle
    c = W.candidate((8, 6), 2, 2, [merge(0, 1), decompose(0, (2, 2))],
                    proj=[(0, W.BLOCK), (1, W.CYCLIC)])
    assert mlp.block_estimates(c, (2, 1), oracle.chain_table) == (72, 24)
    f = mlp.features(c, (2, 1))
    # the descriptor estimate counts 2h cells per coordinate boundary: 2*2*1*6 along
    # dim 0 and, cyclic, 2*1*5*8 along dim 1 = 104 (above the exact 72: under a
    # cyclic projection a cell's two neighbours along the dim share one owner)
    assert math.isclose(f[23], math.log2(1 + 104) / 32) and f[60] == 0
    assert f[49] == 0.0 and f[50] == 1.0  # the cyclic flag of final dim 1
    assert math.isclose(f[15], 1 / 9) and math.isclose(f[16], 1 / 9)  # 2 blocks per launch dim
    assert math.isclose(f[54], 2 / 4) and math.isclose(f[55], 1 / 4)
    gc, ic, _, _ = oracle.stencil_cost(c, W.stencil((2, 1), 8))
    assert (gc, ic) == (72, 24)


def test_block_estimate_exact_for_bijective_block_chains():
    """For a bijective block mapping (every processor owns one block), the ghost cells
    along a launch dim are, per cell, the blocks whose first or last cell lies within
    the halo; summed per block boundary that is min(h, b) + min(h, l - b) cells times
    the face area -- so the estimate equals the exact distinct-pair volume of the C
    oracle (Sec. 4.1's definition) for any block width, halos wider than blocks included.
    Inter-node cells are exact when no block is narrower than the halo."""
    import oracle
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(40):
        k = int(rng.integers(2, 4))
        ext = tuple(int(x) for x in rng.integers(3, 40, size=k))
        halo = tuple(int(x) for x in rng.integers(1, 5, size=k))
        n, g = int(rng.integers(1, 5)), int(rng.choice([1, 2, 4]))
        P = n * g
        fs = oracle.enumerate_factorizations(P, k)
        f = fs[int(rng.integers(0, len(fs)))]
        if any(f[d] > ext[d] for d in range(k)):
            continue  # empty blocks: not bijective
        base = [merge(0, 1)] if rng.integers(0, 2) else [swap(0, 1), merge(0, 1)]
        c = W.candidate(ext, n, g, base + [decompose(0, f)])
        cost = oracle.stencil_cost(c, W.stencil(halo, 8))
        est_t, est_i = mlp.block_estimates(c, halo, oracle.chain_table)
        assert math.isclose(est_t * 8, cost[2], rel_tol=1e-9, abs_tol=1e-6), (ext, halo, n, g, f)
        widths_ok = all(ext[d] // f[d] >= halo[d] for d in range(k))
        if widths_ok:
            assert math.isclose(est_i * 8, cost[3], rel_tol=1e-9, abs_tol=1e-6), (ext, halo, n, g, f)
        checked += 1
    assert checked >= 20


def test_descriptor_estimate_exact_for_bijective_wide_blocks():
    """For a bijective block mapping with one final dim per launch dim and blocks at
    least h wide, every cell within h of a block boundary has exactly one foreign
    owner across it, so the ghost cells are 2h per boundary per cross-section: the
    descriptor estimate equals the C oracle's exact volume (Sec. 4.1's definition)
    and the block-model estimate.  Swaps after decompose permute which factor blocks
    which launch dim; the estimate follows the final shape."""
    import oracle
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(60):
        k = int(rng.integers(2, 4))
        ext = tuple(int(x) for x in rng.integers(4, 48, size=k))
        halo = tuple(int(x) for x in rng.integers(0, 4, size=k))
        n, g = int(rng.integers(1, 5)), int(rng.choice([1, 2, 4]))
        fs = oracle.enumerate_factorizations(n * g, k)
        f = fs[int(rng.integers(0, len(fs)))]
        ops = ([merge(0, 1)] if rng.integers(0, 2) else [swap(0, 1), merge(0, 1)]) + [decompose(0, f)]
        if rng.integers(0, 2):
            ops.append(swap(0, k - 1))
        c = W.candidate(ext, n, g, ops)
        shape, _ = mlp.final_shape_and_blocks(c)
        if any(ext[d] // shape[d] < max(halo[d], 1) for d in range(k)):
            continue  # a block narrower than the halo, or empty
        cost = oracle.stencil_cost(c, W.stencil(halo, 8))
        est = mlp.descriptor_estimate(c, halo)
        assert est * 8 == cost[2], (ext, halo, n, g, f, ops)
        assert est == mlp.block_estimates(c, halo, oracle.chain_table)[0]
        checked += 1
    assert checked >= 25
