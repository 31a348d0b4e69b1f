"""Pins for the connected-components oracle (Section 4 problem statement).

Checked against: a hand-worked golden example, brute-force transitive closure
on every graph with n <= 5 (and samples at n = 6, 7), the planted generator's
closed form (label = smallest id of each planted group), scipy's
connected_components partition, and the invariants (label[v] <= v,
label[label[v]] = label[v], both ends of every pair share a label, and the
number of classes matches).
"""

import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components as scipy_cc

import oracle
import workloads as W
from helpers import brute_components, check_cc_invariants, read_golden


def test_golden_worked_example():
    g = read_golden("cc_worked_example.txt")
    label = oracle.connected_components(g["src"], g["dst"], g["n"][0])
    assert label.tolist() == g["label"]


@pytest.mark.parametrize("n", range(1, 6))
def test_every_graph_brute_force(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[k] for k in range(len(pairs)) if mask >> k & 1]
        src = np.array([a for a, _ in edges], dtype=np.int32)
        dst = np.array([b for _, b in edges], dtype=np.int32)
        # alternate the orientation to exercise both directions
        if mask & 1:
            src, dst = dst, src
        label = oracle.connected_components(src, dst, n)
        assert label.tolist() == brute_components(n, edges)


@pytest.mark.parametrize("n", [6, 7])
def test_sampled_graphs_brute_force(n):
    rng = np.random.default_rng(n)
    for _ in range(300):
        m = int(rng.integers(0, 2 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        label = oracle.connected_components(src, dst, n)
        assert label.tolist() == brute_components(n, list(zip(src.tolist(), dst.tolist())))


def test_special_cases():
    assert oracle.connected_components([], [], 0).shape == (0,)
    assert oracle.connected_components([], [], 5).tolist() == [0, 1, 2, 3, 4]
    n = 1000
    path = np.arange(n - 1, dtype=np.int32)
    assert (oracle.connected_components(path[::-1], path[::-1] + 1, n) == 0).all()
    star_src = np.full(n - 1, n - 1, dtype=np.int32)
    star_dst = np.arange(n - 1, dtype=np.int32)
    assert (oracle.connected_components(star_src, star_dst, n) == 0).all()
    # self-loops and duplicates only
    assert oracle.connected_components([3, 3, 1], [3, 3, 1], 4).tolist() == [0, 1, 2, 3]


def test_out_of_range_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.connected_components([0], [5], 5)
    with pytest.raises(oracle.OracleError):
        oracle.connected_components([-1], [0], 5)


@pytest.mark.parametrize("n,m,groups,seed", [(5000, 12000, 40, 1), (1 << 16, 1 << 18, 1024, 2)])
def test_planted_closed_form(n, m, groups, seed):
    src, dst, group_of = W.planted_graph(n, m, groups, seed)
    label = oracle.connected_components(src, dst, n)
    # closed form: the smallest id of each planted group
    gmin = np.full(groups, n, dtype=np.int64)
    np.minimum.at(gmin, group_of.astype(np.int64), np.arange(n))
    assert np.array_equal(label, gmin[group_of].astype(np.int32))
    assert len(np.unique(label)) == groups
    check_cc_invariants(src, dst, label)


@pytest.mark.parametrize("family", ["lists", "trees1", "trees3", "trees20", "dense0.01",
                                    "dense0.1"])
def test_family_closed_form(family):
    # the paper's graph families carry their components by construction:
    # label = smallest id of the vertex's list / tree / component
    if family == "lists":
        src, dst, group_of = W.list_graph(30_000, 17, 6, with_groups=True)
    elif family.startswith("trees"):
        src, dst, group_of = W.random_tree_graph(30_000, int(family[5:]), 9, 7, with_groups=True)
    else:
        src, dst, group_of = W.component_density_graph(40_000, float(family[5:]), 13, 8)
    n = group_of.shape[0]
    groups = int(group_of.max()) + 1
    label = oracle.connected_components(src, dst, n)
    gmin = np.full(groups, n, dtype=np.int64)
    np.minimum.at(gmin, group_of.astype(np.int64), np.arange(n))
    assert np.array_equal(label, gmin[group_of].astype(np.int32))
    assert len(np.unique(label)) == groups
    check_cc_invariants(src, dst, label)


@pytest.mark.parametrize("n,m,seed", [(20000, 9000, 3), (1 << 17, 1 << 18, 4), (3000, 0, 5)])
def test_scipy_partition_cross_check(n, m, seed):
    src, dst = W.random_graph(n, m, seed)
    label = oracle.connected_components(src, dst, n)
    g = sp.coo_matrix((np.ones(m), (src, dst)), shape=(n, n))
    ncomp, lab = scipy_cc(g, directed=False)
    # min-canonicalise scipy's labels
    first = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(first, lab, np.arange(n))
    assert np.array_equal(label, first[lab].astype(np.int32))
    assert len(np.unique(label)) == ncomp
    check_cc_invariants(src, dst, label)


def test_batched_matches_single():
    graphs = []
    rng = np.random.default_rng(9)
    for g in range(25):
        n = int(rng.integers(0, 300))
        m = int(rng.integers(0, 3 * n + 1)) if n else 0
        s, d = W.random_graph(n, m, 100 + g)
        graphs.append((n, s, d))
    voff = np.zeros(len(graphs) + 1, np.int64)
    eoff = np.zeros(len(graphs) + 1, np.int64)
    voff[1:] = np.cumsum([g[0] for g in graphs])
    eoff[1:] = np.cumsum([len(g[1]) for g in graphs])
    src = np.concatenate([g[1] for g in graphs])
    dst = np.concatenate([g[2] for g in graphs])
    label = oracle.connected_components_batched(src, dst, voff, eoff)
    for i, (n, s, d) in enumerate(graphs):
        assert np.array_equal(label[voff[i]:voff[i + 1]], oracle.connected_components(s, d, n))


def test_invariants_catch_planted_mistakes():
    g = read_golden("cc_worked_example.txt")
    good = np.array(g["label"])
    check_cc_invariants(g["src"], g["dst"], good)
    for wrong in (good + 1, np.arange(10), np.where(good == 2, 5, good)):
        with pytest.raises(AssertionError):
            check_cc_invariants(g["src"], g["dst"], wrong)
