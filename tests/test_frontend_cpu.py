"""Front end: mapping-language mappers translated into candidates (host only).
Each mapper below is written for these tests in the language of the syntax figure
of Sec. 7 (none is one of the paper's listings): a block distribution, a two-level
node-block / GPU-cyclic distribution of the kind App. A.1 uses for the matmul
mappers, a merge+split row mapper and a swapped, halo-weighted decompose.  The
expected candidates are built by hand from the transformation primitives (Fig. 6)
and projections (Fig. 1, Fig. 3, App. A.1)."""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads import decompose, merge, split, swap


@pytest.fixture(scope="module")
def tm():
    import paper_2507_17087_amd as m
    m.lib()
    return m


def same(a, b):
    keys = ["lrank", "nodes", "gpus", "nops", "extent", "mrank"]
    for k in keys:
        assert np.array_equal(a[k], b[k]), k
    n = int(a["nops"])
    for t in range(n):
        for f in ("kind", "a", "b", "nf", "f"):
            assert np.array_equal(a["ops"][t][f], b["ops"][t][f]), (t, f)
    r = int(a["mrank"])
    assert np.array_equal(a["proj_src"][:r], b["proj_src"][:r])
    assert np.array_equal(a["proj_mode"][:r], b["proj_mode"][:r])


TILES = """
# a block distribution of a 2-D launch over the node x GPU grid: the point is
# scaled as a tuple, divided by the launch domain and unpacked into the index
gpus = Machine(GPU)

def tiles2d(Task t):
    scaled = t.ipoint * gpus.size
    return gpus[*(scaled / t.ispace)]

IndexTaskMap stencil_step tiles2d
Region * * GPU FBMEM
"""


def test_elementwise_block(tm):
    c = tm.tm_parse_index_task_map(TILES, "stencil_step", (60, 90), 3, 4)
    exp = W.candidate((60, 90), 3, 4, [], proj=[(0, W.BLOCK), (1, W.BLOCK)])
    same(c, exp)


HIER = """
# two levels: decompose tiles the nodes over the domain, then each node's GPUs
# over one node's share of it; a point takes its node by blocks and its GPU round
# robin, one coordinate at a time
def node_then_gpu(Tuple p, Tuple dom):
    nodes = Machine(GPU).decompose(0, dom)
    share = dom / nodes[:-1]
    two = nodes.decompose(2, share)
    n0 = p[0] * two[0] / dom[0]
    n1 = p[1] * two[1] / dom[1]
    return two[n0, n1, p[0] % two[2], p[1] % two[3]]

IndexTaskMap cannon_tiles node_then_gpu
"""


@pytest.mark.parametrize("ext,n,g", [((64, 64), 4, 4), ((96, 32), 6, 8), ((1000, 30), 12, 2)])
def test_hierarchical_block_cyclic(tm, ext, n, g):
    c = tm.tm_parse_index_task_map(HIER, "cannon_tiles", ext, n, g)
    fn = oracle.decompose_argmin(n, ext, (1, 1))
    per_node = tuple(ext[d] // fn[d] for d in range(2))
    fg = oracle.decompose_argmin(g, per_node, (1, 1))
    exp = W.candidate(ext, n, g, [decompose(0, fn), decompose(2, fg)],
                      proj=[(0, W.BLOCK), (1, W.BLOCK), (0, W.CYCLIC), (1, W.CYCLIC)])
    same(c, exp)


ROWS = """
m = Machine(GPU)
def rows(Tuple p, Tuple dom):
    flat = m.merge(0, 1).split(0, m.size[0] * m.size[1])
    return flat[p[0] * flat[0] / dom[0], 0]
IndexTaskMap * rows
"""


def test_merge_split_rows(tm):
    c = tm.tm_parse_index_task_map(ROWS, "anything", (100, 7), 2, 3)
    exp = W.candidate((100, 7), 2, 3, [merge(0, 1), split(0, 6)], proj=[(0, W.BLOCK), (0, W.BLOCK)])
    same(c, exp)


def test_swap_and_halo_weighted_decompose(tm):
    src = """
def f(Task t):
    s = t.ispace
    m = Machine(GPU).swap(0, 1).merge(0, 1).decompose(0, s)
    return m[t.ipoint[0] * m[0] / s[0], t.ipoint[1] * m[1] / s[1], t.ipoint[2] * m.size[2] // s[2]]
IndexTaskMap t3 f
"""
    ext, halo = (64, 32, 16), (1, 2, 3)
    c = tm.tm_parse_index_task_map(src, "t3", ext, 4, 8, halo)
    f = oracle.decompose_argmin(32, ext, halo)
    exp = W.candidate(ext, 4, 8, [swap(0, 1), merge(0, 1), decompose(0, f)])
    same(c, exp)
    rc, shape = tm.tm_validate(c)
    assert rc == 0 and len(shape) == 3 and int(np.prod(shape)) == 32


@pytest.mark.parametrize("src,where", [
    ("def f(Task t):\n    return Machine(GPU)[t.ipoint[0] + 1, 0]\nIndexTaskMap x f\n", "line 2"),
    ("def f(Task t):\n    m = Machine(GPU)\n    return m[t.ipoint[0] * 3 / 7, 0]\nIndexTaskMap x f\n", "line 3"),
    ("def f(Task t):\n    return q[0]\nIndexTaskMap x f\n", "unknown name"),
    ("def f(Task t):\n    m = Machine(GPU)\n    return m[*(t.ipoint * m.size / t.ispace), 0]\nIndexTaskMap x f\n",
     "coordinates"),
    ("def f(Task t):\n    m = Machine(CPU)\nIndexTaskMap x f\n", "Machine(GPU)"),
    ("def f(Task t):\n    m = Machine(GPU).split(0, 5)\n    return m[0, 0, 0]\nIndexTaskMap x f\n", "divide"),
    ("def g(Task t):\n    return 0\n", "no IndexTaskMap"),
])
def test_errors_name_the_place(tm, src, where):
    with pytest.raises(tm.TaskmapError) as e:
        tm.tm_parse_index_task_map(src, "x", (8, 8), 2, 2)
    assert e.value.code == tm.TM_EINVAL
    assert where in str(e.value)
