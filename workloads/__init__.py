"""Seeded synthetic workloads for the mapping evaluator (inputs only).

This module builds candidate descriptors; it evaluates nothing.  It is shared by
the tests, the benchmark and both sides of every parity check (the CPU oracle and
the HIP library), so it holds none of the evaluation arithmetic: no projection, no
inverse chain, no ghost or tile counting, no objective.  Lists of factorizations
are passed in by the caller (each side enumerates its own).

Workloads (shapes follow the paper's stencil and matmul studies, Sec. 4.1, 6.3 and
App. A.1; all data synthetic):
  c1  2-D 64x64 on 2 nodes x 4 GPUs, 4 factorizations x 4 chains, 5-point h=1
  c2  3-D 512^3 on 16 x 8, 36 factorizations x 6 chains, star h=2
  c3  random batch: ranks 2-3, extents log-uniform 32..1023, nodes 1..64,
      GPUs/node in {1,2,4,8}, 0-4 random transformations (gen.c)
  c4  matmul task space 256^3 on 16 x 4, 28 factorizations x 2 chains + Cannon
  c5  search instances: every factorization x a fixed menu of chains
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

SPLIT, MERGE, SWAP, BALANCE_SPLIT, DECOMPOSE = 1, 2, 3, 4, 5
BLOCK, CYCLIC = 0, 1

OP_DTYPE = np.dtype([("kind", "<i4"), ("a", "<i4"), ("b", "<i4"), ("nf", "<i4"),
                     ("f", "<i4", (4,))])
CAND_DTYPE = np.dtype([("lrank", "<i4"), ("nodes", "<i4"), ("gpus", "<i4"), ("nops", "<i4"),
                       ("extent", "<i8", (4,)), ("ops", OP_DTYPE, (8,)),
                       ("mrank", "<i4"), ("pad0", "<i4"),
                       ("proj_src", "i1", (8,)), ("proj_mode", "i1", (8,))])
STENCIL_DTYPE = np.dtype([("lrank", "<i4"), ("elem_bytes", "<i4"), ("halo", "<i4", (4,))])
assert CAND_DTYPE.itemsize == 328 and STENCIL_DTYPE.itemsize == 24


def split(i, d):
    return (SPLIT, i, d, ())


def merge(p, q):
    return (MERGE, p, q, ())


def swap(p, q):
    return (SWAP, p, q, ())


def balance_split(i, d):
    return (BALANCE_SPLIT, i, d, ())


def decompose(i, factors):
    return (DECOMPOSE, i, 0, tuple(int(x) for x in factors))


def _rank_after(ops):
    """Rank of the processor space after the ops (grammar bookkeeping only)."""
    r = 2
    for kind, _a, _b, f in ops:
        if kind in (SPLIT, BALANCE_SPLIT):
            r += 1
        elif kind == MERGE:
            r -= 1
        elif kind == DECOMPOSE:
            r += len(f) - 1
    return r


def candidate(extent, nodes, gpus, ops, proj=None):
    """One candidate record.  proj: list of (src_dim, mode) per final dim; default
    BLOCK with src_j = j over a final space of the launch rank."""
    rec = np.zeros((), dtype=CAND_DTYPE)
    rec["lrank"] = len(extent)
    for d, l in enumerate(extent):
        rec["extent"][d] = l
    rec["nodes"], rec["gpus"] = nodes, gpus
    if len(ops) > 8:
        raise ValueError("at most 8 ops")
    rec["nops"] = len(ops)
    for t, (kind, a, b, f) in enumerate(ops):
        rec["ops"][t]["kind"], rec["ops"][t]["a"], rec["ops"][t]["b"] = kind, a, b
        rec["ops"][t]["nf"] = len(f)
        for m, x in enumerate(f):
            rec["ops"][t]["f"][m] = x
    if proj is None:
        proj = [(j, BLOCK) for j in range(_rank_after(ops))]
    rec["mrank"] = len(proj)
    for j, (src, mode) in enumerate(proj):
        rec["proj_src"][j], rec["proj_mode"][j] = src, mode
    return rec


def batch(records):
    out = np.zeros(len(records), dtype=CAND_DTYPE)
    for i, r in enumerate(records):
        out[i] = r
    return out


def stencil(halo, elem_bytes=8):
    st = np.zeros((), dtype=STENCIL_DTYPE)
    st["lrank"] = len(halo)
    st["elem_bytes"] = elem_bytes
    for d, h in enumerate(halo):
        st["halo"][d] = h
    return st


# ---------------------------------------------------------------- named workloads

def c1_chains():
    """The four chain tails of the 64x64 workload, applied after merge(0,1) +
    decompose(0, F): identity, swap, re-split by 4, balance_split by 3."""
    return [[], [swap(0, 1)], [merge(0, 1), split(0, 4)], [merge(0, 1), balance_split(0, 3)]]


C1_FACTORIZATIONS = [(1, 8), (2, 4), (4, 2), (8, 1)]  # every ordered 2-factorization of 8


def c1_candidates(factorizations=C1_FACTORIZATIONS, extent=(64, 64), nodes=2, gpus=4):
    recs = []
    for f in factorizations:
        for tail in c1_chains():
            recs.append(candidate(extent, nodes, gpus, [merge(0, 1), decompose(0, f)] + tail))
    return batch(recs)


def c1_stencil():
    return stencil((1, 1), 8)


def c2_chains(f):
    """Six chain tails after merge(0,1) + decompose(0, F) on a 3-factorization."""
    return [[], [swap(0, 1)], [swap(1, 2)], [swap(0, 2)],
            [merge(0, 1), split(0, int(f[1]))], [merge(1, 2), split(1, int(f[2]))]]


def c2_candidates(factorizations, extent=(512, 512, 512), nodes=16, gpus=8):
    recs = []
    for f in factorizations:
        for tail in c2_chains(f):
            recs.append(candidate(extent, nodes, gpus, [merge(0, 1), decompose(0, f)] + tail))
    return batch(recs)


def c2_stencil():
    return stencil((2, 2, 2), 8)


C4_TILE_BYTES = 1024 * 1024 * 8  # one 1024x1024 fp64 tile


def c4_candidates(factorizations, extent=(256, 256, 256), nodes=16, gpus=4):
    """Every 3-factorization of 64 (block, with and without swap(0,1)), plus the
    hierarchical Cannon mapper of App. A.1: node grid from decompose of the node
    dim, GPU grid from decompose of the GPU dim, nodes blocked and GPUs cyclic,
    k unmapped."""
    recs = []
    for f in factorizations:
        recs.append(candidate(extent, nodes, gpus, [merge(0, 1), decompose(0, f)]))
        recs.append(candidate(extent, nodes, gpus, [merge(0, 1), decompose(0, f), swap(0, 1)]))
    recs.append(cannon_candidate(extent, nodes, gpus))
    return batch(recs)


def cannon_candidate(extent, nodes, gpus, node_grid=None, gpu_grid=None):
    node_grid = node_grid or _square_pair(nodes)
    gpu_grid = gpu_grid or _square_pair(gpus)
    ops = [decompose(0, node_grid), decompose(2, gpu_grid)]
    proj = [(0, BLOCK), (1, BLOCK), (0, CYCLIC), (1, CYCLIC)]
    return candidate(extent, nodes, gpus, ops, proj)


def _square_pair(v):
    a = int(round(v ** 0.5))
    while v % a:
        a -= 1
    return (max(a, v // a), min(a, v // a))


# ---------------------------------------------------------------- random batches

_gen = None


def _genlib():
    global _gen
    if _gen is None:
        so = os.path.join(HERE, "libtmgen.so")
        if not os.path.exists(so):
            build()
        _gen = ctypes.CDLL(so)
        _gen.gen_random_candidates.restype = ctypes.c_int
        _gen.gen_random_candidates.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64] + \
            [ctypes.c_int32] * 7 + [ctypes.c_void_p]
        _gen.gen_random_chains.restype = ctypes.c_int
        _gen.gen_random_chains.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p]
        assert _gen.gen_sizeof_candidate() == CAND_DTYPE.itemsize
    return _gen


def build():
    so = os.path.join(HERE, "libtmgen.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", so + ".tmp",
                           os.path.join(HERE, "gen.c")])
    os.replace(so + ".tmp", so)


C3_SEED = 17087


def random_candidates(n, seed=C3_SEED, first=0, ranks=(2, 3), octaves=(5, 9), nodes_max=64,
                      gpus=(1, 2, 4, 8), max_ops=4, cyclic_pct=0):
    """n random candidates (c3 recipe by default); candidate i depends only on
    (seed, first + i)."""
    out = np.zeros(n, dtype=CAND_DTYPE)
    kmask = sum(1 << k for k in ranks)
    gmask = sum(1 << (int(g).bit_length() - 1) for g in gpus)
    rc = _genlib().gen_random_candidates(seed, first, n, kmask, octaves[0], octaves[1], nodes_max,
                                         gmask, max_ops, cyclic_pct, out.ctypes.data)
    if rc != 0:
        raise ValueError("bad generator arguments")
    return out


def random_chain_instance(extent, nodes, gpus, n, seed, first=0, max_ops=4, cyclic_pct=25):
    """n random candidates of one search instance (launch domain `extent` on
    Machine(GPU) = (nodes, gpus)): each draws its factorization, 0..max_ops random
    transformations and its projections (cyclic with probability cyclic_pct per
    final dim) as the c3 recipe does; candidate i depends only on (seed, first + i)."""
    out = np.zeros(n, dtype=CAND_DTYPE)
    ext = np.array(list(extent) + [1] * (4 - len(extent)), dtype=np.int64)
    rc = _genlib().gen_random_chains(seed, first, n, len(extent), ext.ctypes.data, nodes, gpus, max_ops,
                                     cyclic_pct, out.ctypes.data)
    if rc != 0:
        raise ValueError("bad generator arguments")
    return out


def c3_candidates(n=4096, seed=C3_SEED, **kw):
    return random_candidates(n, seed=seed, **kw)


def c3_stencil(lrank):
    return stencil((1,) * lrank, 8)


def split_by_rank(cands):
    """c3 mixes ranks 2 and 3; the oracle's stencil fixes the rank, so its batches
    are evaluated per rank.  Returns {rank: index array}."""
    return {int(k): np.nonzero(cands["lrank"] == k)[0] for k in np.unique(cands["lrank"])}


# ---------------------------------------------------------------- search instances

def chain_menu(k):
    """A fixed menu of 32 chains (each a function of the factorization F) applied to
    Machine(GPU); each returns the full op list.  Node-major / GPU-major bases, the
    factor order permutations that swaps reach, re-splits and balance_splits."""
    menu = []
    bases = ([merge(0, 1)], [swap(0, 1), merge(0, 1)])
    tails = []
    if k == 2:
        tails = [lambda f: [], lambda f: [swap(0, 1)],
                 lambda f: [merge(0, 1), split(0, f[1])],
                 lambda f: [merge(0, 1), balance_split(0, np.maximum(1, f[0] - 1))],
                 lambda f: [merge(0, 1), balance_split(0, f[0] + 1)],
                 lambda f: [swap(0, 1), merge(0, 1), split(0, f[0])],
                 lambda f: [merge(0, 1), split(0, f[0] * f[1])],
                 lambda f: [merge(0, 1), split(0, 1)]]
    else:
        tails = [lambda f: [], lambda f: [swap(0, 1)], lambda f: [swap(1, 2)], lambda f: [swap(0, 2)],
                 lambda f: [swap(0, 1), swap(1, 2)], lambda f: [swap(1, 2), swap(0, 1)],
                 lambda f: [merge(0, 1), split(0, f[1])], lambda f: [merge(1, 2), split(1, f[2])],
                 lambda f: [merge(0, 1), balance_split(0, f[0] + 1)],
                 lambda f: [merge(1, 2), balance_split(1, f[1] + 1)],
                 lambda f: [merge(0, 2), split(0, f[2]), swap(1, 2)],
                 lambda f: [merge(0, 1), split(0, 1), swap(0, 2)],
                 lambda f: [swap(0, 2), swap(0, 1)],
                 lambda f: [merge(0, 1), balance_split(0, np.maximum(1, f[0] * f[1] - 1))],
                 lambda f: [merge(1, 2), split(1, f[2]), swap(0, 1)],
                 lambda f: [merge(0, 1), split(0, f[1]), swap(1, 2)]]
    for base in bases:
        for t in tails:
            menu.append((base, t))
    return menu


def instance_candidates(extent, nodes, gpus, factorizations, menu=None):
    """Every factorization x every menu chain, in that order."""
    k = len(extent)
    menu = menu or chain_menu(k)
    recs = []
    for f in factorizations:
        for base, tail in menu:
            recs.append(candidate(extent, nodes, gpus, base + [decompose(0, f)] + tail(tuple(f))))
    return batch(recs)


def random_instances(n, seed=2, first=0, octaves=(5, 9), nodes_max=64, gpus=(1, 2, 4, 8)):
    """Search instances (extent, nodes, gpus) with launch rank 3: the domain, the
    machine and the stencil of a random candidate; the chain is not used."""
    cs = random_candidates(n, seed=seed, first=first, ranks=(3,), octaves=octaves,
                           nodes_max=nodes_max, gpus=gpus, max_ops=0)
    return [(tuple(int(x) for x in c["extent"][:3]), int(c["nodes"]), int(c["gpus"])) for c in cs]


def _menu_templates(k):
    """The chain menu as (kind, a, b, factor-index or None) templates: the argument b
    of each op is either a constant or derived from F by the given function."""
    return chain_menu(k)


def instance_batch(instances, factorization_lists, menu=None):
    """Candidates of many search instances at once (vectorised over factorizations):
    returns (records, seg) with seg[s]..seg[s+1] the candidates of instance s, in the
    order of instance_candidates()."""
    out, seg = [], [0]
    for (extent, nodes, gpus), fs in zip(instances, factorization_lists):
        k = len(extent)
        fa = np.asarray(fs, dtype=np.int64).reshape(-1, k)
        menu_k = menu or chain_menu(k)
        m = len(fa)
        recs = np.zeros((m, len(menu_k)), dtype=CAND_DTYPE)
        recs["lrank"] = k
        recs["nodes"], recs["gpus"] = nodes, gpus
        for d, l in enumerate(extent):
            recs["extent"][:, :, d] = l
        cols = tuple(fa[:, j] for j in range(k))
        for mi, (base, tail) in enumerate(menu_k):
            ops = base + [(DECOMPOSE, 0, 0, None)] + tail(cols)
            r = recs[:, mi]
            r["nops"] = len(ops)
            rank = 2
            for t, (kind, a, b, f) in enumerate(ops):
                r["ops"][:, t]["kind"] = kind
                r["ops"][:, t]["a"] = a
                if kind == DECOMPOSE:
                    r["ops"][:, t]["nf"] = k
                    for j in range(k):
                        r["ops"][:, t]["f"][:, j] = fa[:, j]
                    rank += k - 1
                else:
                    r["ops"][:, t]["b"] = b
                    rank += 1 if kind in (SPLIT, BALANCE_SPLIT) else (-1 if kind == MERGE else 0)
            r["mrank"] = rank
            for j in range(rank):
                r["proj_src"][:, j] = j
        out.append(recs.reshape(-1))
        seg.append(seg[-1] + m * len(menu_k))
    return np.concatenate(out), np.array(seg, np.int64)


# ---------------------------------------------------------------- decompose vs Alg. A1 study
# Sec. 6.3 varies 2-D stencils over six aspect ratios 1:1 .. 1:32, five task-space sizes
# per node (1e6 .. 4e8 points) and 4 .. 128 GPUs in powers of two (4 per node, the
# paper's machines): 180 configurations.  Here each configuration's domain is
# (l0, l1) with l1 / l0 = the aspect ratio and l0 * l1 = size per node * nodes
# (rounded to integers), and two factorizations of the GPUs are compared: decompose's
# argmin of the surface-area objective and Alg. A1's even grid (its factors, sorted
# descending, assigned to dims 0, 1 in that order).

STUDY_ASPECTS = (1, 2, 4, 8, 16, 32)
STUDY_SIZES = (10**6, 10**7, 10**8, 2 * 10**8, 4 * 10**8)
STUDY_GPUS = (4, 8, 16, 32, 64, 128)
STUDY_GPUS_PER_NODE = 4


def study_configs(aspects=STUDY_ASPECTS, sizes=STUDY_SIZES, gpus=STUDY_GPUS, long_last=True):
    """[(aspect, size per node, GPUs, (l0, l1), nodes, GPUs per node)]; long_last: the
    longer dim is dim 1 (else dim 0) -- the paper does not say which, and Alg. A1's
    descending factors make the two orientations differ."""
    out = []
    for a in aspects:
        for s in sizes:
            for g in gpus:
                nodes = g // STUDY_GPUS_PER_NODE
                total = s * nodes
                short = max(1, int(round((total / a) ** 0.5)))
                long_ = max(1, int(round(total / short)))
                ext = (short, long_) if long_last else (long_, short)
                out.append((a, s, g, ext, nodes, STUDY_GPUS_PER_NODE))
    return out


def study_candidates(configs, f_decompose, f_greedy):
    """Four candidates per configuration, in this order: decompose's F and Alg. A1's F,
    each under the node-major machine order (swap(0,1) before the merge: consecutive
    processors share a node) and the GPU-major one (the merge alone)."""
    recs = []
    for (a, s, g, ext, n, gp), fd, fg in zip(configs, f_decompose, f_greedy):
        for f in (fd, fg):
            recs.append(candidate(ext, n, gp, [swap(0, 1), merge(0, 1), decompose(0, f)]))
            recs.append(candidate(ext, n, gp, [merge(0, 1), decompose(0, f)]))
    return batch(recs)


# ---------------------------------------------------------------- two-level decompositions
# App. A.1's hierarchical mappers: nodes tiled over the domain, then each node's GPUs
# over the node's tile.  Two variants per (node grid Fn, GPU grid Fg):
#   hierarchical block: swap(0,1), decompose the GPU dim by Fg, decompose the node
#     dim by Fn, then merge each GPU factor (fastest) with its node factor, so final
#     dim d has Fn_d * Fg_d coordinates gpu_d + Fg_d * node_d, projected BLOCK: every
#     node holds a contiguous block, cut into contiguous GPU sub-blocks;
#   node-block / GPU-cyclic: decompose the node dim by Fn and the GPU dim by Fg, node
#     dims BLOCK and GPU dims CYCLIC over the launch dims (the Cannon mapper's form).

def two_level_candidates(extent, nodes, gpus, node_grids, gpu_grids):
    """For every (Fn, Fg) pair: [hierarchical block, node-block / GPU-cyclic]."""
    k = len(extent)
    recs = []
    for fn in node_grids:
        for fg in gpu_grids:
            ops = [swap(0, 1), decompose(0, fg), decompose(k, fn)] + [merge(d, k) for d in range(k)]
            recs.append(candidate(extent, nodes, gpus, ops))
            proj = [(d, BLOCK) for d in range(k)] + [(d, CYCLIC) for d in range(k)]
            recs.append(candidate(extent, nodes, gpus, [decompose(0, fn), decompose(k, fg)], proj))
    return batch(recs)
