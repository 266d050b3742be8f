"""The mean-flow multigrid's hierarchy, built by the library's host code
(hb_precond_hierarchy, no GPU), against properties computed here from the
mesh alone: the aggregates of the finest level partition the nodes, are
connected in the node graph and hold at most four nodes (two passes of
pairwise matching) or a node with neighbours (greedy aggregation); the
level sizes shrink to at most coarse_max; no two neighbouring nodes share a
colour class; bad arguments are rejected."""
import numpy as np
import pytest

import paper_2411_14315_amd as hbl
from hbinputs.meshes import cube_mesh, cylinder_mesh


def adjacency(n, tets):
    nb = [set() for _ in range(n)]
    for t in tets:
        for a in t:
            nb[a].update(int(b) for b in t if b != a)
    return nb


def connected(nodes, nb):
    nodes = set(int(x) for x in nodes)
    seen, stack = set(), [next(iter(nodes))]
    while stack:
        v = stack.pop()
        if v in seen:
            continue
        seen.add(v)
        stack.extend(w for w in nb[v] if w in nodes and w not in seen)
    return seen == nodes


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(hbl.LIB_PATH):
        from paper_2411_14315_amd import build
        build.build(verbose=False)
    return hbl.load()


@pytest.mark.parametrize("mesh", ["cube", "pipe"])
@pytest.mark.parametrize("aggregation", [0, 1])
def test_hierarchy_properties(lib, mesh, aggregation):
    m = cube_mesh(5) if mesh == "cube" else cylinder_mesh(1.0, 6.0, 4, 16)
    n = m.n_nodes
    sizes, agg, colour = hbl.precond_hierarchy(n, m.tets, coarse_max=24,
                                               aggregation=aggregation)
    assert sizes[0] == n and len(sizes) >= 2
    assert all(b < a for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] <= 24 or sizes[-1] > 0.9 * sizes[-2]
    nb = adjacency(n, m.tets)
    # aggregates partition the finest level's nodes, each connected
    assert agg.min() == 0 and agg.max() == sizes[1] - 1
    groups = [np.flatnonzero(agg == a) for a in range(sizes[1])]
    assert all(len(g) > 0 for g in groups) and sum(len(g) for g in groups) == n
    assert all(connected(g, nb) for g in groups)
    if aggregation == 0:
        assert max(len(g) for g in groups) <= 4
    # colour classes: no edge inside a class
    for v in range(n):
        assert all(colour[w] != colour[v] for w in nb[v])
    assert colour.max() + 1 < 40


def test_single_level_and_errors(lib):
    m = cube_mesh(2)
    sizes, agg, colour = hbl.precond_hierarchy(m.n_nodes, m.tets, coarse_max=256)
    assert sizes == [m.n_nodes] and np.all(agg == -1)
    bad = m.tets.copy()
    bad[0, 0] = m.n_nodes
    with pytest.raises(hbl.HBError) as e:
        hbl.precond_hierarchy(m.n_nodes, bad)
    assert e.value.status == hbl.HB_ERR_ARG
    with pytest.raises(hbl.HBError):
        hbl.precond_hierarchy(m.n_nodes, m.tets, coarse_max=0)
    with pytest.raises(hbl.HBError):
        hbl.precond_hierarchy(m.n_nodes, m.tets, aggregation=2)
