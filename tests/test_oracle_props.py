"""Property tests of the oracle on random small inputs (hypothesis).

Lists: for any permutation order and tail marker, the oracle's ranks equal
hop counting and satisfy the complete invariants; any corruption of a valid
list (a second tail, a branch, a cycle, an id out of range) is rejected
exactly when brute force finds no single list.  Graphs: the oracle's labels
equal the min-canonicalised scipy partition and satisfy the invariants.
Batched forms equal the per-instance calls.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components as scipy_cc

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import cpu_baseline  # noqa: E402
import oracle  # noqa: E402
from helpers import (brute_list_valid, brute_rank_from_head, check_cc_invariants,  # noqa: E402
                     check_rank_invariants)


def list_from_order(order, self_tail):
    n = len(order)
    succ = np.full(n, -1, np.int32)
    for k in range(n - 1):
        succ[order[k]] = order[k + 1]
    if n and self_tail:
        succ[order[-1]] = order[-1]
    return succ


@settings(max_examples=300, deadline=None)
@given(st.permutations(list(range(40))).flatmap(
    lambda p: st.tuples(st.just(p), st.integers(1, 40), st.booleans())))
def test_random_lists_match_hop_counting(args):
    perm, n, self_tail = args
    order = [v for v in perm if v < n]
    succ = list_from_order(order, self_tail)
    rank = oracle.list_rank(succ)
    assert rank.tolist() == brute_rank_from_head(succ.tolist())
    check_rank_invariants(succ, rank)


@settings(max_examples=300, deadline=None)
@given(st.integers(2, 12).flatmap(lambda n: st.tuples(
    st.permutations(list(range(n))), st.integers(0, n - 1), st.integers(-2, n + 1))))
def test_corrupted_lists_rejected_exactly_when_invalid(args):
    order, pos, val = args
    succ = list_from_order(order, False)
    succ[pos] = val
    st_, _ = oracle.list_rank_status(succ)
    valid = brute_list_valid(succ.tolist())
    assert (st_ == oracle.OK) == valid
    if valid:
        assert oracle.list_rank(succ).tolist() == brute_rank_from_head(succ.tolist())


@settings(max_examples=300, deadline=None)
@given(st.integers(1, 30).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=60))))
def test_random_graphs_match_scipy(args):
    n, edges = args
    src = np.array([a for a, _ in edges], np.int32)
    dst = np.array([b for _, b in edges], np.int32)
    label = oracle.connected_components(src, dst, n)
    g = sp.coo_matrix((np.ones(len(edges)), (src, dst)), shape=(n, n))
    k, comp = scipy_cc(g, directed=False)
    # min-canonicalise scipy's component numbering
    mins = {}
    for v in range(n):
        mins.setdefault(comp[v], v)
    assert label.tolist() == [mins[comp[v]] for v in range(n)]
    check_cc_invariants(src, dst, label)
    assert len(set(label.tolist())) == k


@settings(max_examples=100, deadline=None)
@given(st.lists(st.integers(0, 25), min_size=1, max_size=8), st.randoms(use_true_random=False))
def test_batched_lists_equal_single_calls(sizes, rnd):
    lists = []
    for n in sizes:
        order = list(range(n))
        rnd.shuffle(order)
        lists.append(list_from_order(order, rnd.random() < 0.5))
    off = np.zeros(len(lists) + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in lists])
    succ = np.concatenate(lists).astype(np.int32) if off[-1] else np.empty(0, np.int32)
    status, rank = oracle.list_rank_batched(succ, off)
    assert (status == oracle.OK).all()
    for i, s in enumerate(lists):
        assert rank[off[i]:off[i + 1]].tolist() == oracle.list_rank(s).tolist()


@settings(max_examples=200, deadline=None)
@given(st.permutations(list(range(30))).flatmap(
    lambda p: st.tuples(st.just(p), st.integers(1, 30), st.booleans(),
                        st.lists(st.integers(-2**31, 2**31 - 1), min_size=30, max_size=30))))
def test_weighted_ranks_step_by_the_weights(args):
    # rank[head] = 0 and rank[succ[i]] = rank[i] + weight[i] in 32-bit
    # two's complement, for any weights (the multi-threaded CPU baseline
    # agrees on unit weights)
    perm, n, self_tail, wl = args
    order = [v for v in perm if v < n]
    succ = list_from_order(order, self_tail)
    w = np.array(wl[:n], dtype=np.int64).astype(np.int32)
    rank = oracle.list_rank_weighted(succ, w).astype(np.int64)
    assert rank[order[0]] == 0
    for a, b in zip(order, order[1:]):
        assert (rank[b] - rank[a] - int(w[a])) % (1 << 32) == 0
    rc, cpu = cpu_baseline.ruling_set(succ, 4, 3)
    assert rc == cpu_baseline.OK and np.array_equal(cpu, oracle.list_rank(succ))
