"""Reference of the learned ranker (sums in float64) -- TEST INFRASTRUCTURE ONLY.

Plain numpy, written independently of the HIP kernels: the feature encoding of a
candidate, the 64 -> 256 -> 256 -> 256 -> 2 ReLU network in its defined arithmetic
(bf16 weights and activations, sums at fp32 precision or better; see `_rounders`),
its mean-squared-error gradient by hand-written backpropagation through the same
arithmetic, and one Adam step.  Only the tests and the benchmark's CPU leg use it.

Parameter vector layout (flat): W1[64][256], b1[256], W2[256][256], b2[256],
W3[256][256], b3[256], W4[256][2], b4[2]; rows index inputs.

The ranker is not described by the paper (it is a learned pruning of decompose's
search space added by this library); its feature encoding below is a definition, so the
feature function is checked only against values worked out by hand in the tests
("parity unpinned" beyond those).
"""
import math

import numpy as np

F, W, O = 64, 256, 2
SPLIT, MERGE, SWAP, BALANCE_SPLIT, DECOMPOSE = 1, 2, 3, 4, 5


def layout():
    off, L = 0, {}
    for name, size in [("w1", F * W), ("b1", W), ("w2", W * W), ("b2", W), ("w3", W * W), ("b3", W),
                       ("w4", W * O), ("b4", O)]:
        L[name] = (off, off + size)
        off += size
    L["count"] = off
    return L


def unpack(p):
    L = layout()
    g = lambda k: np.asarray(p[L[k][0]:L[k][1]], dtype=np.float64)
    return (g("w1").reshape(F, W), g("b1"), g("w2").reshape(W, W), g("b2"), g("w3").reshape(W, W), g("b3"),
            g("w4").reshape(W, O), g("b4"))


def bf16_round(x):
    """Round to bfloat16 (nearest even) through float32, returned as float64: a value
    held in a float32 register and then stored as bf16 is rounded twice, and so is
    this one."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def _rounders(arith):
    """The arithmetic of the network.

    "bf16": the ranker's defined arithmetic -- bf16 inputs, bf16 weight matrices and
    bf16 hidden activations, every product summed at (at least) fp32 precision.  Here
    the sums are taken in float64 and each one is rounded to float32 and then to bf16
    where the definition stores a bf16 value: a hidden activation after bias and ReLU
    (forward), a hidden-layer gradient after the ReLU mask (backward).  Biases, the two
    outputs and the output gradient stay at full precision.
    "f64": every value float64 (the plain network; its gradient is pinned to finite
    differences).
    """
    if arith == "bf16":
        return bf16_round
    if arith == "f64":
        return _identity
    raise ValueError(arith)


def forward(p, X, arith="bf16"):
    """Outputs y [n][2] and the layer inputs (x, h1, h2, h3) as the network sees them."""
    q = _rounders(arith)
    w1, b1, w2, b2, w3, b3, w4, b4 = unpack(p)
    w1, w2, w3, w4 = q(w1), q(w2), q(w3), q(w4)
    x = q(X)
    h1 = q(np.maximum(x @ w1 + b1, 0))
    h2 = q(np.maximum(h1 @ w2 + b2, 0))
    h3 = q(np.maximum(h2 @ w3 + b3, 0))
    y = h3 @ w4 + b4
    return y, (x, h1, h2, h3)


def loss_and_grad(p, X, T, arith="bf16"):
    """Mean over rows and outputs of (y - t)^2, and its gradient (flat), by
    backpropagation through the same arithmetic as `forward`: each hidden-layer
    gradient is the next layer's gradient times the (rounded) transposed weights,
    masked where the forward activation was zero, and rounded like an activation."""
    q = _rounders(arith)
    w1, b1, w2, b2, w3, b3, w4, b4 = unpack(p)
    w2, w3, w4 = q(w2), q(w3), q(w4)
    y, (x, h1, h2, h3) = forward(p, X, arith)
    n = X.shape[0]
    d = y - T
    loss = float((d * d).sum() / (n * O))
    dy = 2.0 * d / (n * O)
    gw4 = h3.T @ dy
    gb4 = dy.sum(0)
    dh3 = q((dy @ w4.T) * (h3 > 0))
    gw3 = h2.T @ dh3
    gb3 = dh3.sum(0)
    dh2 = q((dh3 @ w3.T) * (h2 > 0))
    gw2 = h1.T @ dh2
    gb2 = dh2.sum(0)
    dh1 = q((dh2 @ w2.T) * (h1 > 0))
    gw1 = x.T @ dh1
    gb1 = dh1.sum(0)
    g = np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2, gw3.ravel(), gb3, gw4.ravel(), gb4])
    return loss, g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v


def final_shape_and_blocks(c):
    """Shapes after every op (forward rules) -> final shape, and the number of final
    coordinates projected from each launch dim."""
    s = [int(c["nodes"]), int(c["gpus"])]
    for t in range(int(c["nops"])):
        op = c["ops"][t]
        k, a, b = int(op["kind"]), int(op["a"]), int(op["b"])
        if k == SPLIT:
            s = s[:a] + [b, s[a] // b] + s[a + 1:]
        elif k == BALANCE_SPLIT:
            s = s[:a] + [b, -(-s[a] // b)] + s[a + 1:]
        elif k == MERGE:
            s = s[:a] + [s[a] * s[b]] + s[a + 1:b] + s[b + 1:]
        elif k == SWAP:
            s = list(s)
            s[a], s[b] = s[b], s[a]
        elif k == DECOMPOSE:
            f = [int(x) for x in op["f"][: int(op["nf"])]]
            s = s[:a] + f + s[a + 1:]
    blocks = [1.0] * 4
    for j, sz in enumerate(s):
        blocks[int(c["proj_src"][j])] *= sz
    return s, blocks


def descriptor_estimate(c, halo):
    """Ghost cells from the shapes alone, assuming every change of the final
    coordinates projected from a launch dim changes the processor (a bijective
    chain): along launch dim d the processor changes at l - 1 coordinate boundaries
    when a final dim of size > 1 is projected onto it cyclically, else at the
    interior block starts of its block-projected final dims (counted as the sum of
    their sizes less one each, at most l - 1); each boundary puts 2h cells of every
    cross-section (the product of the other extents) into the halo.  Exact for
    bijective chains with one final dim per launch dim and blocks at least h wide."""
    s, _ = final_shape_and_blocks(c)
    k = int(c["lrank"])
    cells = 0.0
    for d in range(k):
        l = int(c["extent"][d])
        nb, cyc = 0, False
        for j in range(len(s)):
            if int(c["proj_src"][j]) != d:
                continue
            if int(c["proj_mode"][j]) != 0:
                cyc = cyc or s[j] > 1
            else:
                nb += s[j] - 1
        nb = l - 1 if cyc else min(nb, l - 1)
        face = 1.0
        for e in range(k):
            if e != d:
                face *= float(c["extent"][e])
        cells += 2.0 * halo[d] * float(nb) * face
    return cells


def features(c, halo):
    """The 64 ranker features of one candidate (float64), from its descriptor alone."""
    f = np.zeros(F)
    k = int(c["lrank"])
    f[k - 1] = 1
    s, blocks = final_shape_and_blocks(c)
    F_ = [1, 1, 1, 1]
    nf = 0
    ops = c["ops"][: int(c["nops"])]
    for op in ops:
        if int(op["kind"]) == DECOMPOSE:
            nf = int(op["nf"])
            F_ = [int(x) for x in op["f"][:4]]
            break
    vf = 0.0
    for d in range(k):
        l = float(c["extent"][d])
        f[4 + d] = math.log2(l) / 10
        f[15 + d] = math.log2(blocks[d]) / 9
        f[19 + d] = (math.log2(l) - math.log2(blocks[d])) / 10
        if d < nf:
            vf += 2.0 * halo[d] * (F_[d] - 1.0) / l
        f[54 + d] = halo[d] / 4
    n, g = int(c["nodes"]), int(c["gpus"])
    f[8] = math.log2(n) / 6
    f[9] = math.log2(g) / 3
    f[10] = math.log2(n * g) / 9
    for m in range(min(nf, 4)):
        f[11 + m] = math.log2(F_[m]) / 9
    f[24] = math.log2(1 + vf) / 4
    for t, op in enumerate(ops):
        kd = int(op["kind"])
        if 1 <= kd <= 5:
            f[25 + kd - 1] += 0.25
        if t < 6:
            f[30 + t] = kd / 5
            if t < 3:
                f[39 + t] = int(op["a"]) / 8
            f[42 + t] = 0.0 if kd == DECOMPOSE else math.log2(1 + int(op["b"])) / 9
    f[48] = 1.0 if len(ops) and int(ops[0]["kind"]) == SWAP else 0.0
    for j in range(min(len(s), 4)):
        f[49 + j] = 1.0 if int(c["proj_mode"][j]) else 0.0
    f[53] = len(s) / 8
    f[58] = math.ceil(math.log2(g)) / 3 if g > 1 else 0.0
    f[59] = 1.0
    f[23] = math.log2(1 + descriptor_estimate(c, halo)) / 32
    return f


def block_estimates(c, halo, chain_table):
    """Block-model estimates of a candidate's ghost cells, total and inter-node (the
    second stage of a ranked search), from chain_table(c), the processor of every
    final-space coordinate."""
    k = int(c["lrank"])
    s, _ = final_shape_and_blocks(c)
    g = int(c["gpus"])
    # node / processor crossings: per final dim, the fractions of adjacent coordinate
    # pairs whose owners are on different nodes / are different processors (from the
    # oracle's own chain table); block-model estimates of ghost cells from them
    cross_n = [0.0] * len(s)
    cross_p = [0.0] * len(s)
    if int(np.prod(s)) <= 16384:
        proc = np.asarray(chain_table(c)).reshape(s)
        node = proc // g
        for j in range(len(s)):
            if s[j] > 1:
                a = np.arange(s[j] - 1)
                cross_n[j] = float((np.take(node, a, axis=j) != np.take(node, a + 1, axis=j)).mean())
                cross_p[j] = float((np.take(proc, a, axis=j) != np.take(proc, a + 1, axis=j)).mean())
    cn, cp = [0.0] * 4, [0.0] * 4
    for j in range(min(len(s), 8)):
        d = int(c["proj_src"][j])
        cn[d] = max(cn[d], cross_n[j])
        cp[d] = max(cp[d], cross_p[j])
    # block-model estimates of the ghost cells (total, inter-node).  When every launch
    # dim is block-projected onto exactly one final dim: at each block boundary b
    # along a launch dim the min(h, b) + min(h, l - b) cells within the halo, times
    # the face area (product of the other dims' block widths), count where the
    # owners (nodes) of the two adjacent blocks differ.  Otherwise: per launch dim,
    # the (cell, distinct foreign final coordinate) pairs along it, times the other
    # extents, times that dim's crossing fraction.
    pts = float(np.prod([int(x) for x in c["extent"][:k]]))
    est_t = est_i = 0.0
    proj = [(int(c["proj_src"][j]), int(c["proj_mode"][j])) for j in range(len(s))]
    simple = len(s) == k and sorted(p for p, _ in proj) == list(range(k)) and all(m == 0 for _, m in proj)
    have = int(np.prod(s)) <= 16384
    if have and simple:
        def width(a, S, l):
            return -(-(a + 1) * l // S) - (-(-a * l // S))
        for j in range(k):
            d = proj[j][0]
            l, S, h = int(c["extent"][d]), s[j], int(halo[d])
            if h == 0 or S == 1:
                continue
            # face area of every coordinate of the other final dims
            face = np.ones([s[jj] for jj in range(k) if jj != j])
            for ax, jj in enumerate([jj for jj in range(k) if jj != j]):
                ld = int(c["extent"][proj[jj][0]])
                wv = np.array([width(a, s[jj], ld) for a in range(s[jj])], dtype=np.float64)
                shp = [1] * face.ndim
                shp[ax] = s[jj]
                face = face * wv.reshape(shp)
            for aR in range(1, S):
                b = -(-aR * l // S)
                if b >= l or width(aR, S, l) == 0:
                    continue
                aL = (b - 1) * S // l
                pr, pl = np.take(proc, aR, axis=j), np.take(proc, aL, axis=j)
                w = min(h, b) + min(h, l - b)
                est_t += w * float(face[pr != pl].sum())
                est_i += w * float(face[pr // g != pl // g].sum())
    elif have:
        stride = [1] * len(s)
        for j in range(len(s) - 2, -1, -1):
            stride[j] = stride[j + 1] * s[j + 1]
        for d in range(k):
            l = int(c["extent"][d])
            h = int(halo[d])
            if h == 0 or l > 65536:
                continue
            x = np.arange(l, dtype=np.int64)
            val = np.zeros(l, dtype=np.int64)
            for j in range(len(s)):
                if proj[j][0] == d:
                    a = (x * s[j]) // l if proj[j][1] == 0 else x % s[j]
                    val += a * stride[j]
            nb = 0
            for xi in range(l):
                seen = set()
                for sft in range(1, h + 1):
                    for xx in (xi - sft, xi + sft):
                        if 0 <= xx < l and val[xx] != val[xi]:
                            seen.add(int(val[xx] - val[xi]))
                nb += len(seen)
            cells = nb * (pts / l)
            est_t += cells * cp[d]
            est_i += cells * cn[d]
    return est_t, est_i
