"""Pins for the float64 ranker reference: finite differences for the gradient,
a hand-worked feature vector, and Adam's first step."""
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
    _, g = mlp.loss_and_grad(p, X, T)
    L = mlp.layout()
    idx = np.concatenate([rng.integers(a, b, size=6) for a, b in
                          [L[k] for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")]])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp, _ = mlp.loss_and_grad(q, X, T)
        q[i] -= 2 * h
        lm, _ = mlp.loss_and_grad(q, X, T)
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
    y, _ = mlp.forward(p, X)
    assert np.allclose(y[:, 0], 0.5) and np.allclose(y[:, 1], [0.5, 3.0, 0.0])


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
    assert f[23] == 0 and math.isclose(f[24], math.log2(1 + vf) / 4)  # no chain table: no estimate
    assert math.isclose(f[25 + 1], 0.25) and math.isclose(f[25 + 4], 0.25) and math.isclose(f[25 + 2], 0.25)
    assert math.isclose(f[30], 2 / 5) and math.isclose(f[31], 1.0) and math.isclose(f[32], 3 / 5)
    assert f[39] == 0 and f[40] == 0 and math.isclose(f[41], 0 / 8)
    assert f[48] == 0 and f[53] == 2 / 8 and math.isclose(f[58], 1 / 3) and f[59] == 1
    assert f[60] == 0 and f[61] == 0  # no chain table given: no node crossings
    # with the chain table: final space (2, 4) after the swap; decompose (4, 2) of
    # merge(0,1) puts node = a mod 4 with a = F0-fastest index, so along the final
    # dim of size 4 (the old first factor) every step changes node; along the other
    # (size 2) a step adds 4 to a, which keeps a mod 4: no crossings
    import oracle
    g = mlp.features(c, (1, 1), oracle.chain_table)
    assert g[61] == 0.0 and g[62] == 1.0
    # every step along either final dim changes processor (a bijective chain)
    assert g[36] == 1.0 and g[37] == 1.0
    cells_t = (2 * (2 - 1) / 64 + 2 * (4 - 1) / 32) * 64 * 32   # = 448 ghost cells
    cells_i = (2 * (4 - 1) / 32) * 64 * 32                      # = 384 of them inter-node
    assert math.isclose(g[23], math.log2(1 + cells_t) / 32) and math.isclose(g[60], math.log2(1 + cells_i) / 32)
    # and the block model is exact here: the oracle's ghost count agrees
    gc, ic, _, _ = oracle.stencil_cost(c, W.stencil((1, 1), 8))
    assert (gc, ic) == (448, 384)


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
        feat = mlp.features(c, halo, oracle.chain_table)
        est_t = 2.0 ** (feat[23] * 32) - 1
        est_i = 2.0 ** (feat[60] * 32) - 1
        assert math.isclose(est_t * 8, cost[2], rel_tol=1e-9, abs_tol=1e-6), (ext, halo, n, g, f)
        widths_ok = all(ext[d] // f[d] >= halo[d] for d in range(k))
        if widths_ok:
            assert math.isclose(est_i * 8, cost[3], rel_tol=1e-9, abs_tol=1e-6), (ext, halo, n, g, f)
        checked += 1
    assert checked >= 20
