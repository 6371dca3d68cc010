"""Pins for the CPU oracle: values the paper prints, closed forms, invariants and
brute force on tiny inputs.  None of these re-types the oracle's own formulas; each
checks it against something that the paper or the mathematics fixes."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import balance_split, decompose, merge, split, swap

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def table(ops, n, g, extent=(4, 4)):
    c = W.candidate(extent, n, g, ops)
    return oracle.chain_table(c)


# ---------------------------------------------------------------- paper examples

def test_block2d_point_fig3():
    e = GOLD["block2d_point"]
    c = W.candidate(e["extent"], e["nodes"], e["gpus"], [])
    assert oracle.point_owner(c, e["point"]) == (e["node"], e["gpu"])


def test_split_index_formula_from_composition_example():
    # m'[x, y, a1] = m[x + y*d, a1] for m' = m.split(0, d)
    e = GOLD["split_then_merge"]
    n, g, d = e["nodes"], e["gpus"], e["d"]
    c = W.candidate((n // d, d, g), n, g, [split(0, d)],
                    proj=[(1, W.BLOCK), (0, W.BLOCK), (2, W.BLOCK)])
    # launch domain sized to the final space so that BLOCK projection is the identity
    x, y, a1 = e["split_index"]
    assert oracle.point_owner(c, (y, x, a1)) == (e["node"], e["gpu"])


def test_solomonik_shape():
    e = GOLD["solomonik_shape"]
    ops = [split(i, d) for i, d in e["splits"]]
    c = W.candidate((4, 4, 4), e["nodes"], e["gpus"], ops,
                    proj=[(0, W.BLOCK)] * 6)
    rc, shape = oracle.validate(c)
    assert rc == 0 and shape == tuple(e["shape"])


def test_factorization_counts_paper():
    e = GOLD["factorization_counts"]
    for P, k, cnt in e["cases"]:
        assert len(oracle.enumerate_factorizations(P, k)) == cnt
    assert sorted(oracle.enumerate_factorizations(6, 2)) == sorted(tuple(x) for x in e["six_2d"])


def test_greedy_grid_paper():
    e = GOLD["greedy_grid"]
    assert oracle.greedy_grid(e["P"], e["k"]) == tuple(e["grid"])


def test_greedy_grid_properties():
    """Alg. A1 (App. A.2) by what it guarantees: the factors multiply to P and come
    sorted descending; each prime (smallest first) goes to a smallest factor, so the
    largest factor is at most the smallest times the largest prime of P; a k-th power
    of a prime splits evenly.  Hand-worked: 8 -> (4, 2), 72 -> (12, 6) (primes 2, 2,
    2, 3, 3), 128 on three dims -> (8, 4, 4)."""
    def largest_prime(P):
        q, d = 1, 2
        while P > 1:
            while P % d == 0:
                q, P = d, P // d
            d += 1
        return q
    for P in range(1, 700):
        for k in range(1, 5):
            f = oracle.greedy_grid(P, k)
            assert len(f) == k and int(np.prod(f)) == P
            assert list(f) == sorted(f, reverse=True)
            assert f[0] <= f[-1] * largest_prime(P)
    for p in (2, 3, 5, 7):
        for k in range(1, 5):
            assert oracle.greedy_grid(p ** k, k) == (p,) * k
    assert oracle.greedy_grid(8, 2) == (4, 2)
    assert oracle.greedy_grid(72, 2) == (12, 6)
    assert oracle.greedy_grid(128, 3) == (8, 4, 4)


def ghost(extent, F, halo, n=None, g=1, tail=(), proj=None):
    P = int(np.prod(F))
    n = n if n is not None else P // g
    c = W.candidate(extent, n, g, [merge(0, 1), decompose(0, F)] + list(tail), proj)
    return oracle.stencil_cost(c, W.stencil(halo, 1))


def test_volumes_2d_paper():
    e = GOLD["volumes_2d"]
    for extent, grid, vol in e["cases"]:
        assert ghost(extent, grid, e["halo"])[0] == vol


def test_volume_3d_paper():
    e = GOLD["volume_3d"]
    assert ghost(e["extent"], e["factors"], (1, 1, 1))[0] == e["twoS"]


def test_decompose_argmin_paper():
    for extent, P, f in GOLD["decompose_argmin"]["cases"]:
        assert oracle.decompose_argmin(P, extent) == tuple(f)


def test_workload_greedy_paper():
    e = GOLD["workload_greedy"]
    assert oracle.workload_greedy(e["P"], e["extent"]) == tuple(e["factors"])
    # and the search finds the balanced optimum the greedy misses
    assert oracle.decompose_argmin(e["P"], e["extent"]) == (8, 9)


def test_block1d_x_translation():
    for n, g, Lx, Ly in GOLD["block1d_x"]["cases"]:
        c = W.candidate((Lx, Ly), n, g, [merge(0, 1), split(0, n * g)])
        pm = oracle.proc_map(c)
        for ix in range(Lx):
            a = ix * n * g // Lx
            for iy in range(Ly):
                assert pm[ix, iy] == (a % n) * g + a // n


# ---------------------------------------------------------------- identities

@pytest.mark.parametrize("n,g", [(2, 3), (4, 2), (6, 1), (1, 5), (3, 4)])
def test_split_then_merge_is_identity(n, g):
    ident = np.arange(n * g, dtype=np.int32)
    assert (table([], n, g) == ident).all()
    for d in range(1, n + 1):
        if n % d == 0:
            assert (table([split(0, d), merge(0, 1)], n, g) == ident).all()
    for d in range(1, g + 1):
        if g % d == 0:
            assert (table([split(1, d), merge(1, 2)], n, g) == ident).all()


@pytest.mark.parametrize("n,g", [(2, 3), (4, 2), (3, 4)])
def test_swap_involution_and_merge_split_roundtrip(n, g):
    ident = np.arange(n * g, dtype=np.int32)
    assert (table([swap(0, 1), swap(0, 1)], n, g) == ident).all()
    assert (table([swap(1, 0), swap(0, 1)], n, g) == ident).all()
    assert (table([merge(0, 1), split(0, n)], n, g) == ident).all()
    # swap alone is a genuine permutation (transpose) unless a side is 1
    t = table([swap(0, 1)], n, g)
    assert sorted(t) == list(ident)
    assert (t.reshape(g, n) == ident.reshape(n, g).T).all()


@pytest.mark.parametrize("P,F", [(8, (2, 4)), (12, (3, 2, 2)), (24, (2, 3, 4)), (16, (2, 2, 2, 2)),
                                 (6, (6, 1))])
def test_decompose_equals_split_chain(P, F):
    # decompose(i,F) == split(i, F0), split(i+1, F1), ... (Sec. 4.2)
    k = len(F)
    splits = [split(t, F[t]) for t in range(k - 1)]
    ext = (3,) * k
    a = W.candidate(ext, P, 1, [merge(0, 1), decompose(0, F)])
    b = W.candidate(ext, P, 1, [merge(0, 1)] + splits)
    assert (oracle.chain_table(a) == oracle.chain_table(b)).all()
    # and merging the factors back restores the 1-D space
    back = [merge(0, 1)] * (k - 1)
    c = W.candidate((3,), P, 1, [merge(0, 1), decompose(0, F)] + back)
    d = W.candidate((3,), P, 1, [merge(0, 1)])
    assert (oracle.chain_table(c) == oracle.chain_table(d)).all()


@pytest.mark.parametrize("s,d", [(8, 2), (8, 4), (12, 3), (6, 6), (5, 1)])
def test_balance_split_equals_split_when_divisible(s, d):
    a = W.candidate((4, 4), s, 1, [merge(0, 1), balance_split(0, d)])
    b = W.candidate((4, 4), s, 1, [merge(0, 1), split(0, d)])
    assert (oracle.chain_table(a) == oracle.chain_table(b)).all()


@pytest.mark.parametrize("s,d", [(8, 3), (7, 2), (10, 4), (5, 7), (13, 5), (3, 9)])
def test_balance_split_loads_differ_by_at_most_one(s, d):
    c = W.candidate((4, 4), s, 1, [merge(0, 1), balance_split(0, d)])
    rc, shape = oracle.validate(c)
    assert rc == 0 and shape == (d, -(-s // d))
    t = oracle.chain_table(c)
    loads = np.bincount(t, minlength=s)
    assert loads.sum() == d * (-(-s // d))
    assert loads.min() >= 1 and loads.max() - loads.min() <= 1  # surjective, balanced
    if (s, d) == (8, 3):
        assert list(loads) == [2, 1, 1, 1, 1, 1, 1, 1]


def test_bijective_chains_are_permutations():
    cs = W.random_candidates(300, seed=5, octaves=(2, 3), nodes_max=12, max_ops=4)
    for c in cs:
        kinds = c["ops"]["kind"][: c["nops"]]
        t = oracle.chain_table(c)
        P = int(c["nodes"]) * int(c["gpus"])
        assert t.min() >= 0 and t.max() < P
        if W.BALANCE_SPLIT not in kinds:
            assert len(t) == P and sorted(t) == list(range(P))
        else:
            assert len(set(t.tolist())) == P  # still reaches every processor


# ---------------------------------------------------------------- enumeration

def _prime_exponents(P):
    ex, p = [], 2
    while p * p <= P:
        e = 0
        while P % p == 0:
            P //= p
            e += 1
        if e:
            ex.append(e)
        p += 1
    if P > 1:
        ex.append(1)
    return ex


@pytest.mark.parametrize("P", [1, 2, 6, 8, 12, 16, 36, 48, 64, 72, 97, 128, 360, 480, 512])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_enumeration_count_formula_and_brute_force(P, k):
    fs = oracle.enumerate_factorizations(P, k)
    expect = math.prod(math.comb(a + k - 1, k - 1) for a in _prime_exponents(P))  # Sec. 4.3
    assert len(fs) == expect
    assert fs == sorted(fs) and len(set(fs)) == len(fs)  # lexicographic ascending, distinct
    if P <= 128:
        divs = [d for d in range(1, P + 1) if P % d == 0]
        brute = sorted(t for t in itertools.product(divs, repeat=k) if math.prod(t) == P)
        assert fs == brute


# ---------------------------------------------------------------- volumes: closed forms

@pytest.mark.parametrize("L,p,h", [(37, 5, 2), (64, 8, 1), (100, 7, 3), (9, 3, 3), (16, 1, 2), (50, 4, 6)])
def test_1d_halo_closed_form(L, p, h):
    # 2(p-1)h whenever the first and last blocks are at least h wide
    c = W.candidate((L,), p, 1, [merge(0, 1)])
    gc, ic, _, _ = oracle.stencil_cost(c, W.stencil((h,), 8))
    assert gc == 2 * (p - 1) * h and ic == gc  # one GPU per node: every cut is inter-node


def kd_closed_form(extent, F, halo):
    # V = sum_m 2 h_m (f_m - 1) prod_{j != m} l_j   (Sec. 4.2 / App. A.3, both directions)
    return sum(2 * h * (f - 1) * math.prod(extent) // l for l, f, h in zip(extent, F, halo))


def test_kd_closed_form_random():
    rng = np.random.default_rng(7)
    done = 0
    while done < 40:
        k = int(rng.integers(2, 4))
        F = tuple(int(x) for x in rng.integers(1, 5, size=k))
        halo = tuple(int(x) for x in rng.integers(1, 3, size=k))
        extent = tuple(int(f * rng.integers(max(h, 1), 6)) for f, h in zip(F, halo))
        if math.prod(extent) > 6000:
            continue
        # blocks f | l and width l/f >= h
        assert ghost(extent, F, halo)[0] == kd_closed_form(extent, F, halo)
        done += 1


def test_argmin_of_exact_volume_matches_decompose():
    """decompose's objective ranks factorizations exactly as the true ghost volume
    does when every block is at least h wide (Sec. 4.2 derivation)."""
    cases = [((12, 18), 6, (1, 1)), ((18, 12), 6, (1, 1)), ((8, 16, 4), 8, (1, 1, 1)),
             ((16, 16, 8), 16, (2, 1, 1)), ((24, 12), 12, (1, 2)), ((4, 8, 4), 16, (1, 1, 1))]
    for extent, P, halo in cases:
        fs = [f for f in oracle.enumerate_factorizations(P, len(extent))
              if all(l % f == 0 and l // f >= h for l, f, h in zip(extent, f, halo))]
        vols = {f: ghost(extent, f, halo)[0] for f in fs}
        best = min(vols.values())
        argmin = oracle.decompose_argmin(P, extent, halo)
        if argmin in vols:
            assert vols[argmin] == best


# ---------------------------------------------------------------- brute force (receiver side)

def receiver_volume(owner, halo, g):
    """Independent formulation: processor P needs every cell outside its own set that
    lies within the stencil of one of its cells.  Counts sum_P |need(P)| and the part
    whose owner sits on another node."""
    nd = owner.ndim
    procs = np.unique(owner)
    tot = inter = 0
    for P in procs:
        mine = owner == P
        reach = np.zeros_like(mine)
        for m in range(nd):
            for s in range(1, halo[m] + 1):
                for sgn in (1, -1):
                    shifted = np.zeros_like(mine)
                    src = [slice(None)] * nd
                    dst = [slice(None)] * nd
                    if sgn > 0:
                        src[m], dst[m] = slice(0, owner.shape[m] - s), slice(s, None)
                    else:
                        src[m], dst[m] = slice(s, None), slice(0, owner.shape[m] - s)
                    if owner.shape[m] > s:
                        shifted[tuple(dst)] = mine[tuple(src)]
                    reach |= shifted
        need = reach & ~mine
        tot += int(need.sum())
        inter += int((need & (owner // g != P // g)).sum())
    return tot, inter


def test_receiver_brute_force_random_chains():
    cs = W.random_candidates(120, seed=11, ranks=(1, 2, 3), octaves=(1, 3), nodes_max=6,
                             max_ops=4, cyclic_pct=25)
    rng = np.random.default_rng(3)
    for c in cs:
        k = int(c["lrank"])
        halo = tuple(int(x) for x in rng.integers(0, 4, size=k))
        owner = oracle.proc_map(c)
        got = oracle.stencil_cost(c, W.stencil(halo, 8))
        exp = receiver_volume(owner, halo, int(c["gpus"]))
        assert got[:2] == exp
        assert got[2:] == (8 * exp[0], 8 * exp[1])


def test_c1_by_receiver_brute_force():
    c1 = W.c1_candidates(oracle.enumerate_factorizations(8, 2))
    got = oracle.stencil_cost_batch(c1, W.c1_stencil())
    for c, row in zip(c1, got):
        exp = receiver_volume(oracle.proc_map(c), (1, 1), 4)
        assert tuple(row[:2]) == exp
    # identity-chain rows match the closed form
    for i, f in enumerate(oracle.enumerate_factorizations(8, 2)):
        assert got[4 * i, 0] == kd_closed_form((64, 64), f, (1, 1))


def test_cyclic_distinct_versus_pairs():
    # 4x4 cyclic on 2x2, h=1: every cell sends to one owner per axis -> 32 distinct
    c = W.candidate((4, 4), 2, 2, [], proj=[(0, W.CYCLIC), (1, W.CYCLIC)])
    assert oracle.stencil_cost(c, W.stencil((1, 1), 8))[0] == 32
    c = W.candidate((8,), 2, 1, [merge(0, 1)], proj=[(0, W.CYCLIC)])
    assert oracle.stencil_cost(c, W.stencil((1,), 8))[0] == 8


def test_single_node_and_single_gpu_special_cases():
    cs = W.random_candidates(60, seed=21, octaves=(2, 4), nodes_max=1, max_ops=3)
    for c in cs:
        assert oracle.stencil_cost(c, W.stencil((1,) * int(c["lrank"]), 8))[1] == 0
    cs = W.random_candidates(60, seed=22, octaves=(2, 4), nodes_max=9, gpus=(1,), max_ops=3)
    for c in cs:
        gc, ic, _, _ = oracle.stencil_cost(c, W.stencil((1,) * int(c["lrank"]), 8))
        assert gc == ic


def test_zero_halo_and_one_processor():
    c = W.candidate((7, 5), 3, 2, [merge(0, 1), decompose(0, (3, 2))])
    assert oracle.stencil_cost(c, W.stencil((0, 0), 8)) == (0, 0, 0, 0)
    c = W.candidate((7, 5), 1, 1, [merge(0, 1), decompose(0, (1, 1))])
    assert oracle.stencil_cost(c, W.stencil((2, 2), 8)) == (0, 0, 0, 0)


# ---------------------------------------------------------------- matmul

def matmul_brute(c):
    owner = oracle.proc_map(c)
    P = int(c["nodes"]) * int(c["gpus"])
    res = np.zeros((P, 3), np.int64)
    for p in range(P):
        m = owner == p
        res[p, 0] = m.any(axis=1).sum()  # (i,k) pairs
        res[p, 1] = m.any(axis=0).sum()  # (j,k) -> B[k,j]
        res[p, 2] = m.any(axis=2).sum()  # (i,j)
    return res


def test_matmul_brute_force_and_closed_form():
    for F in [(2, 2, 2), (4, 2, 1), (1, 1, 8), (2, 4, 1)]:
        T = (8, 8, 8)
        c = W.candidate(T, 8, 1, [merge(0, 1), decompose(0, F)])
        per, tot = oracle.matmul_cost(c, 10)
        assert (per == matmul_brute(c)).all()
        nA = (T[0] // F[0]) * (T[2] // F[2])
        nB = (T[2] // F[2]) * (T[1] // F[1])
        nC = (T[0] // F[0]) * (T[1] // F[1])
        assert (per[:, 0] == nA).all() and (per[:, 1] == nB).all() and (per[:, 2] == nC).all()
        # total tiles = prod(l) * sum f_m / l_m: decompose's objective
        assert sum(tot[:3]) == sum(math.prod(T) * f // l for f, l in zip(F, T))
        assert tot[6] == 10 * sum(tot[:3])
    cs = W.random_candidates(30, seed=31, ranks=(3,), octaves=(1, 2), nodes_max=6, max_ops=3,
                             cyclic_pct=30)
    for c in cs:
        per, _ = oracle.matmul_cost(c, 1)
        assert (per == matmul_brute(c)).all()


def test_cannon_hierarchical_matches_2d_grid_counts():
    # node block x GPU cyclic over an 8x8 processor grid touches as many tiles per
    # processor as the plain (8,8,1) block grid
    T = (32, 32, 32)
    can = W.cannon_candidate(T, 16, 4)
    blk = W.candidate(T, 16, 4, [merge(0, 1), decompose(0, (8, 8, 1))])
    pc, _ = oracle.matmul_cost(can, 1)
    pb, _ = oracle.matmul_cost(blk, 1)
    assert sorted(pc[:, 0]) == sorted(pb[:, 0]) and sorted(pc[:, 2]) == sorted(pb[:, 2])


# ---------------------------------------------------------------- selection and validation

def test_select_best_key_order():
    costs = np.array([[0, 0, 80, 8], [0, 0, 64, 40], [0, 0, 64, 16], [0, 0, 64, 16]], np.int64)
    assert oracle.select_best(costs) == 2


@pytest.mark.parametrize("ops,proj,code", [
    ([split(0, 3)], None, -1),                       # 3 does not divide 2 nodes
    ([merge(1, 0)], None, -1),                       # merge needs p < q
    ([merge(0, 2)], None, -1),                       # q out of range
    ([swap(0, 0)], None, -1),
    ([merge(0, 1), decompose(0, (3, 3))], None, -1),  # wrong product
    ([merge(0, 1), decompose(0, (8, 1))], [(2, 0), (0, 0)], -1),  # projection source out of range
    ([merge(0, 1), decompose(0, (8, 1))], [(0, 0)], -1),           # final rank mismatch
    ([merge(0, 1), decompose(0, (8, 1))], [(0, 2), (1, 0)], -1),   # bad projection mode
    ([split(0, 1)] * 7, [(0, 0)] * 8, -1),                        # rank above 8
    ([balance_split(0, 1 << 23), balance_split(2, 1 << 10)], None, -2),  # volume overflow
])
def test_validation_errors(ops, proj, code):
    c = W.candidate((4, 4), 2, 4, ops, proj)
    assert oracle.validate(c)[0] == code


def test_validation_extent_and_machine():
    c = W.candidate((4, 0), 2, 4, [])
    assert oracle.validate(c)[0] == -1
    c = W.candidate((4, 4), 0, 4, [])
    assert oracle.validate(c)[0] == -1


# ---------------------------------------------------------------- node-level exchange volume

def _node_level_brute(c, halo):
    """Independent formulation on the materialised map (numpy): per cell, the set of
    other nodes among its star neighbours' owners."""
    ext = tuple(int(x) for x in c["extent"][: int(c["lrank"])])
    node = (oracle.proc_map(c).reshape(ext) // int(c["gpus"])).astype(np.int64)
    k = len(ext)
    sets = [set() for _ in range(node.size)]
    flat_node = node.ravel()
    idx = np.arange(node.size).reshape(ext)
    for m in range(k):
        for s in range(1, halo[m] + 1):
            for sgn in (1, -1):
                src = [slice(None)] * k
                dst = [slice(None)] * k
                if sgn > 0:
                    src[m], dst[m] = slice(0, ext[m] - s), slice(s, None)
                else:
                    src[m], dst[m] = slice(s, None), slice(0, ext[m] - s)
                a = idx[tuple(src)].ravel()
                b = idx[tuple(dst)].ravel()
                for i, j in zip(a, b):
                    if flat_node[j] != flat_node[i]:
                        sets[i].add(int(flat_node[j]))
    return sum(len(x) for x in sets)


def test_node_level_matches_brute_force():
    rng = np.random.default_rng(11)
    cands = W.random_candidates(30, seed=23, ranks=(2,), octaves=(2, 4), nodes_max=6, gpus=(1, 2, 4), max_ops=3,
                                cyclic_pct=25)
    for c in cands:
        halo = tuple(int(x) for x in rng.integers(0, 3, size=2))
        got = oracle.stencil_node_cost_batch(W.batch([c]), W.stencil(halo, 8))[0]
        exp = _node_level_brute(c, halo)
        assert got[0] == exp and got[1] == exp and got[2] == 8 * exp


def test_node_level_closed_form_and_invariants():
    """Hierarchical blocks at least h wide: the node-level volume is the surface-area
    count of the node grid alone, sum_m 2 h (Fn_m - 1) prod_{j != m} l_j (Sec. 4.1's
    counting on the nodes); the GPU-cyclic variant has the same node partition and so
    the same value; de-duplicating per node never exceeds the per-processor
    inter-node count, and equals it with one GPU per node."""
    ext, n, g, h = (24, 36), 6, 4, (2, 1)
    fn_all = oracle.enumerate_factorizations(n, 2)
    fg_all = oracle.enumerate_factorizations(g, 2)
    cands = W.two_level_candidates(ext, n, g, fn_all, fg_all)
    st = W.stencil(h, 8)
    node = oracle.stencil_node_cost_batch(cands, st)
    proc = oracle.stencil_cost_batch(cands, st)
    i = 0
    for fn in fn_all:
        for fg in fg_all:
            closed = sum(2 * h[m] * (fn[m] - 1) * (ext[1 - m]) for m in range(2))
            assert node[i][0] == closed and node[i + 1][0] == closed, (fn, fg)
            i += 2
    assert (node[:, 0] <= proc[:, 1]).all()
    one = W.two_level_candidates(ext, 6, 1, fn_all, [(1, 1)])
    assert (oracle.stencil_node_cost_batch(one, st)[:, 0] == oracle.stencil_cost_batch(one, st)[:, 1]).all()


# ---------------------------------------------------------------- decompose with transposes (App. A.3)

def test_transpose_objective_hand_worked():
    """P = 8 on 64 x 64, halo 1, an all-to-all transpose along dim 0.  By hand from
    App. A.3's formula (area term + (1 - 1/f_0) * 4096):
      (1,8): 1*64 + 8*64 = 576,   + 0      = 576
      (2,4): 2*64 + 4*64 = 384,   + 2048   = 2432
      (4,2): 384,                 + 3072   = 3456
      (8,1): 576,                 + 3584   = 4160
    so the transposed dim stays whole: (1, 8); along dim 1 instead: (8, 1)."""
    assert oracle.decompose_argmin_transpose(8, (64, 64), (1, 1), [0]) == (1, 8)
    assert oracle.decompose_argmin_transpose(8, (64, 64), (1, 1), [1]) == (8, 1)
    # no transposes: plain decompose (ties to the lexicographically smallest)
    assert oracle.decompose_argmin_transpose(8, (64, 64), (1, 1), []) == (2, 4)
    assert oracle.decompose_argmin_transpose(8, (64, 64), (1, 1), []) == oracle.decompose_argmin(8, (64, 64), (1, 1))


def test_transpose_objective_without_transposes_is_decompose():
    rng = np.random.default_rng(4)
    for _ in range(40):
        k = int(rng.integers(1, 4))
        P = int(rng.choice([6, 8, 12, 16, 24, 36, 60]))
        ext = tuple(int(x) for x in rng.integers(4, 300, size=k))
        h = tuple(int(x) for x in rng.integers(0, 4, size=k))
        assert oracle.decompose_argmin_transpose(P, ext, h, []) == oracle.decompose_argmin(P, ext, h)


# ---------------------------------------------------------------- transposes as redistributions (App. A.3)

def _grid(extent, F, n, g, tail=()):
    return W.candidate(extent, n, g, [merge(0, 1), decompose(0, F)] + list(tail))


def _moved(a, b, elem_bytes=1):
    return tuple(int(x) for x in oracle.redistribution_cost_batch(W.batch([a]), W.batch([b]), elem_bytes)[0])


def test_transpose_redistribution_hand_worked():
    """4 x 4 on two processors, row blocks (F = (2, 1)); the transpose along dim 0 into
    dim 1 gives column blocks.  Cells whose row block differs from their column block
    move: rows 0-1 x cols 2-3 and rows 2-3 x cols 0-1 = 8 = (1 - 1/2) * 16.  On 3 x 3
    the blocks are uneven (rows {0,1},{2}; cols {0,1},{2}): 2 + 2 = 4 cells, where the
    divisible-case formula would give 4.5."""
    a = _grid((4, 4), (2, 1), 1, 2)
    b = oracle.transpose_target(a, 0, 1)
    assert oracle.validate(b)[1] == (2,)
    assert _moved(a, b) == (8, 0, 8, 0)               # one node: nothing crosses nodes
    a2 = _grid((4, 4), (2, 1), 2, 1)
    assert _moved(a2, oracle.transpose_target(a2, 0, 1), 8) == (8, 8, 64, 64)  # one GPU per node
    a3 = _grid((3, 3), (2, 1), 1, 2)
    assert _moved(a3, oracle.transpose_target(a3, 0, 1)) == (4, 0, 4, 0)
    pa = oracle.proc_map(a3)
    pb = oracle.proc_map(oracle.transpose_target(a3, 0, 1))
    assert pa.tolist() == [[0, 0, 0], [0, 0, 0], [1, 1, 1]]
    assert pb.tolist() == [[0, 0, 1], [0, 0, 1], [0, 0, 1]]


def test_transpose_target_is_the_pencil_split():
    """Divisible 2-D and 3-D grids: the transposed image gives the processor of block
    (i_0, .., i_{k-1}) the i_n-th of f_n equal slices of dim t inside its own block of
    t, dim n whole -- written out here from the block geometry, not from the chain."""
    rng = np.random.default_rng(11)
    for _ in range(30):
        k = int(rng.integers(2, 4))
        F = [int(x) for x in rng.choice([1, 2, 3, 4], size=k)]
        w = [int(x) for x in rng.integers(1, 4, size=k)]
        n, t = (int(x) for x in rng.choice(k, size=2, replace=False))
        w[t] *= F[n]                                   # slices of t divide evenly
        ext = tuple(F[d] * w[d] for d in range(k))
        P = int(np.prod(F))
        g = int(rng.choice([g for g in (1, 2, 3, 4) if P % g == 0]))
        a = _grid(ext, F, P // g, g)
        pa = oracle.proc_map(a)
        pb = oracle.proc_map(oracle.transpose_target(a, n, t))
        sl = w[t] // F[n]
        for ip in itertools.product(*[range(e) for e in ext]):
            blk = [ip[d] // w[d] for d in range(k)]
            blk[n] = (ip[t] % w[t]) // sl             # the slice of t picks the pencil member
            corner = tuple(blk[d] * w[d] for d in range(k))
            assert pb[ip] == pa[corner]


def test_transpose_volume_closed_form():
    """App. A.3: with f_n | l_n for every n, a transpose along n moves
    (1 - 1/f_n) * prod(w) * P = (f_n - 1) / f_n * prod(l) cells, whatever dim t
    absorbs the split (t's blocks divisible by f_n); inter-node cells are zero on one
    node and all of them with one GPU per node."""
    rng = np.random.default_rng(12)
    for _ in range(40):
        k = int(rng.integers(2, 4))
        F = [int(x) for x in rng.choice([1, 2, 3, 4, 6], size=k)]
        w = [int(x) for x in rng.integers(1, 4, size=k)]
        n, t = (int(x) for x in rng.choice(k, size=2, replace=False))
        w[t] *= F[n]
        ext = tuple(F[d] * w[d] for d in range(k))
        P = int(np.prod(F))
        total = int(np.prod(ext))
        for nodes, g in ((1, P), (P, 1)):
            a = _grid(ext, F, nodes, g)
            moved, inter, _, _ = _moved(a, oracle.transpose_target(a, n, t))
            assert moved * F[n] == (F[n] - 1) * total
            assert inter == (0 if nodes == 1 else moved)


def test_redistribution_invariants():
    rng = np.random.default_rng(13)
    for _ in range(20):
        F = [int(x) for x in rng.choice([1, 2, 3, 4], size=2)]
        ext = tuple(int(x) for x in rng.integers(3, 14, size=2))
        P = F[0] * F[1]
        g = int(rng.choice([g for g in (1, 2, 3, 4, 6) if P % g == 0]))
        a = _grid(ext, F, P // g, g)
        assert _moved(a, a) == (0, 0, 0, 0)
        # the same mapping written with a swap of the final dims moves nothing
        a_sw = W.candidate(ext, P // g, g, [merge(0, 1), decompose(0, F), swap(0, 1)],
                           proj=[(1, W.BLOCK), (0, W.BLOCK)])
        assert _moved(a, a_sw) == (0, 0, 0, 0)
        b = oracle.transpose_target(a, 0, 1)
        pa, pb = oracle.proc_map(a).ravel(), oracle.proc_map(b).ravel()
        m = _moved(a, b)
        assert m == _moved(b, a)
        assert m[0] == int((pa != pb).sum())
        assert m[1] == int((pa // g != pb // g).sum())


def test_transpose_argmin_matches_exact_volumes():
    """Without halos, decompose's objective with transposes (App. A.3) is the exact
    moved-cell count on divisible grids, so its argmin is the argmin of the exact
    counts (first in lexicographic order)."""
    for ext, P, T in (((12, 12), 6, [0]), ((12, 24), 6, [1]), ((8, 8, 8), 8, [0, 2]), ((6, 12, 4), 4, [2])):
        k = len(ext)
        best, arg = None, None
        for F in oracle.enumerate_factorizations(P, k):
            if any(ext[d] % F[d] for d in range(k)):
                continue
            a = _grid(ext, F, 1, P)
            tot = 0
            for n in T:
                tdim = (n + 1) % k
                if (ext[tdim] // F[tdim]) % F[n]:
                    break
                tot += _moved(a, oracle.transpose_target(a, n, tdim))[0]
            else:
                if best is None or tot < best:
                    best, arg = tot, tuple(F)
        assert arg == oracle.decompose_argmin_transpose(P, ext, (0,) * k, T)


def test_transpose_target_errors():
    a = _grid((8, 8), (2, 2), 1, 4)
    with pytest.raises(ValueError):
        oracle.transpose_target(a, 0, 0)
    cyc = W.candidate((8, 8), 1, 4, [merge(0, 1), decompose(0, (2, 2))], proj=[(0, W.CYCLIC), (1, W.BLOCK)])
    with pytest.raises(ValueError):
        oracle.transpose_target(cyc, 0, 1)
    bad = W.candidate((8, 8), 1, 4, [merge(0, 1), decompose(0, (2, 2))], proj=[(0, W.BLOCK), (0, W.BLOCK)])
    with pytest.raises(ValueError):
        oracle.transpose_target(bad, 0, 1)
