"""Pins for the list-ranking oracle (list-ranking problem statement, Section 3).

The oracle is checked against things other than itself: a hand-worked golden
example, exhaustive brute force over tiny inputs (every permutation list for
n <= 8, every successor map for n <= 4), closed forms of the generators
(rank[order[k]] = k), the complete invariant characterisation, and planted
mistakes that each pin must catch.
"""

import itertools

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import (brute_list_valid, brute_rank_from_head, check_rank_invariants,
                     read_golden)


def test_golden_worked_example():
    g = read_golden("list_worked_example.txt")
    succ = np.array(g["succ"], dtype=np.int32)
    rank = oracle.list_rank(succ)
    assert rank.tolist() == g["rank_from_head"]
    assert ((g["n"][0] - 1) - rank).tolist() == g["rank_to_tail"]
    # the paper's own tail marker (succ[j] == j) gives the same ranks
    assert oracle.list_rank(W.to_self_loop_tails(succ)).tolist() == g["rank_from_head"]


@pytest.mark.parametrize("n", range(1, 9))
def test_every_permutation_list_brute_force(n):
    for order in itertools.permutations(range(n)):
        succ = [-1] * n
        for a, b in zip(order, order[1:]):
            succ[a] = b
        rank = oracle.list_rank(np.array(succ, dtype=np.int32)).tolist()
        assert rank == brute_rank_from_head(succ)
        # closed form: the k-th node of the walk has rank k
        assert [rank[v] for v in order] == list(range(n))


@pytest.mark.parametrize("n", range(1, 5))
def test_every_successor_map_validity(n):
    """All (n+2)^n maps into {-1, 0..n-1, n} (n is out of range): the oracle
    accepts exactly the single lists, and ranks them correctly."""
    for succ in itertools.product(range(-1, n + 1), repeat=n):
        succ = list(succ)
        rc, rank = oracle.list_rank_status(np.array(succ, dtype=np.int32))
        valid = brute_list_valid(succ)
        assert (rc == oracle.OK) == valid, succ
        if valid:
            assert rank.tolist() == brute_rank_from_head(succ)


def test_empty_and_tiny():
    assert oracle.list_rank(np.empty(0, np.int32)).shape == (0,)
    assert oracle.list_rank(np.array([-1], np.int32)).tolist() == [0]
    assert oracle.list_rank(np.array([0], np.int32)).tolist() == [0]
    assert oracle.list_rank(np.array([1, -1], np.int32)).tolist() == [0, 1]
    assert oracle.list_rank(np.array([-1, 0], np.int32)).tolist() == [1, 0]


@pytest.mark.parametrize("bad", [
    [-1, -1],              # two tails (two lists)
    [1, 0],                # a cycle, no tail
    [1, 2, 1, -1][:3],     # rho shape: 0 -> 1 -> 2 -> 1
    [2, 2, -1],            # two heads merging
    [1, 5, -1],            # out of range
    [1, -2, -1],           # negative non-marker
    [1, 2, -1, 4, 3],      # list plus detached 2-cycle
])
def test_malformed_rejected(bad):
    rc, _ = oracle.list_rank_status(np.array(bad, dtype=np.int32))
    assert rc == oracle.EBADLIST


@pytest.mark.parametrize("n,seed", [(1000, 1), (1 << 16, 2), ((1 << 20) + 3, 3)])
def test_random_closed_form(n, seed):
    succ, order = W.random_list_with_order(n, seed)
    rank = oracle.list_rank(succ)
    assert np.array_equal(rank[order], np.arange(n, dtype=np.int32))
    check_rank_invariants(succ, rank)


def test_sequential_closed_form():
    n = (1 << 18) + 7
    rank = oracle.list_rank(W.sequential_list(n))
    assert np.array_equal(rank, np.arange(n, dtype=np.int32))


@pytest.mark.parametrize("n,run", [(1 << 16, 4096), (50000, 4096), (4096 * 5 + 1, 4096)])
def test_blocked_closed_form(n, run):
    succ, order = W.blocked_list_with_order(n, run, 5)
    rank = oracle.list_rank(succ)
    assert np.array_equal(rank[order], np.arange(n, dtype=np.int32))
    # the j-th visited run, taken in ascending order inside, gets ranks run*j .. run*j+len-1
    runs = order.reshape(-1, run) if n % run == 0 else None
    if runs is not None:
        starts = runs[:, 0]
        assert (starts % run == 0).all()
        assert np.array_equal(rank[starts], np.arange(0, n, run, dtype=np.int32))


def test_batched_matches_single_and_flags_bad_lists():
    succ, off = W.batched_lists(40, 1, 12, 7)
    status, rank = oracle.list_rank_batched(succ, off)
    assert (status == 0).all()
    for i in range(40):
        seg = slice(off[i], off[i + 1])
        assert np.array_equal(rank[seg], oracle.list_rank(succ[seg]))
    bad = succ.copy()
    corrupt = [i for i in range(40) if off[i + 1] - off[i] >= 2][:2]
    seg = bad[off[corrupt[0]]:off[corrupt[0] + 1]]     # close the list into a cycle
    t = int(np.nonzero(seg == -1)[0][0])
    seg[t] = 0 if t != 0 else 1
    seg = bad[off[corrupt[1]]:off[corrupt[1] + 1]]     # second tail
    seg[int(np.nonzero(seg != -1)[0][0])] = -1
    status, _ = oracle.list_rank_batched(bad, off)
    for i in range(40):
        assert status[i] == (oracle.EBADLIST if i in corrupt else 0)


def _planted_oracle_mistakes():
    """Plausible mistakes, each of which some pin above must catch."""
    def off_by_one(succ):
        return oracle.list_rank(succ) + 1

    def to_tail(succ):
        r = oracle.list_rank(succ)
        return (len(succ) - 1) - r

    def skips_tail(succ):
        r = oracle.list_rank(succ).copy()
        r[np.asarray(succ) == -1] = 0
        return r
    return [off_by_one, to_tail, skips_tail]


@pytest.mark.parametrize("mistake", _planted_oracle_mistakes())
def test_pins_catch_planted_mistakes(mistake):
    g = read_golden("list_worked_example.txt")
    succ = np.array(g["succ"], dtype=np.int32)
    assert mistake(succ).tolist() != g["rank_from_head"]
    with pytest.raises(AssertionError):
        check_rank_invariants(succ, mistake(succ))


# ------------------------------------------------------------ weighted lists
# The weighted form ranks the splitter list of Section 3.2 (sublist lengths as
# weights): rank[x] = sum of the weights of the nodes before x.

def _weighted_brute(order, weight):
    """Exclusive prefix of the weights along `order`, by explicit summation."""
    rank = [0] * len(order)
    for k, v in enumerate(order):
        rank[v] = sum(int(weight[u]) for u in order[:k])
    return rank


def test_weighted_golden_worked_example():
    g = read_golden("list_weighted_worked_example.txt")
    succ = np.array(g["succ"], dtype=np.int32)
    w = np.array(g["weight"], dtype=np.int32)
    assert oracle.list_rank_weighted(succ, w).tolist() == g["weighted_rank"]
    # the paper's own tail marker gives the same ranks
    assert oracle.list_rank_weighted(W.to_self_loop_tails(succ), w).tolist() == g["weighted_rank"]


@pytest.mark.parametrize("n", range(1, 7))
def test_weighted_every_permutation_brute_force(n):
    rng = np.random.default_rng(n)
    for order in itertools.permutations(range(n)):
        succ = [-1] * n
        for a, b in zip(order, order[1:]):
            succ[a] = b
        w = rng.integers(-9, 10, n).astype(np.int32)
        got = oracle.list_rank_weighted(np.array(succ, dtype=np.int32), w).tolist()
        assert got == _weighted_brute(order, w)


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (1000, 3), (100_003, 4)])
def test_weighted_closed_form_and_unit_weights(n, seed):
    succ, order = W.random_list_with_order(n, seed)
    w = np.random.default_rng(seed).integers(-1000, 1000, n).astype(np.int32)
    want = np.empty(n, dtype=np.int64)
    want[order] = np.concatenate([[0], np.cumsum(w[order].astype(np.int64))[:-1]])
    assert np.array_equal(oracle.list_rank_weighted(succ, w), want.astype(np.int32))
    assert np.array_equal(oracle.list_rank_weighted(succ, np.ones(n, np.int32)),
                          oracle.list_rank(succ))
    # self-loop tail marker: same ranks
    assert np.array_equal(oracle.list_rank_weighted(W.to_self_loop_tails(succ), w),
                          want.astype(np.int32))


def test_weighted_wraps_and_rejects():
    big = np.int32(2**31 - 1)
    succ = np.array([1, 2, -1], dtype=np.int32)
    # sums wrap modulo 2^32: 2 * (2^31 - 1) = 2^32 - 2 -> -2
    assert oracle.list_rank_weighted(succ, np.array([big, big, 5], np.int32)).tolist() == [0, big, -2]
    with pytest.raises(ValueError):
        oracle.list_rank_weighted(succ, np.ones(2, np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.list_rank_weighted(np.array([1, 0, -1], np.int32), np.ones(3, np.int32))
