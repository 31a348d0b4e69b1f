"""The multi-threaded CPU ruling-set baseline (cpu_baseline/ruling_set.c),
which the benchmark times beside the GPU path, pinned against the oracle's
ranks."""

import numpy as np
import pytest

import cpu_baseline
import oracle
import workloads as W


@pytest.mark.parametrize("n", [1, 2, 3, 64, 1000, 65537, 300_007])
@pytest.mark.parametrize("spacing", [1, 4, 64, 100_000])
@pytest.mark.parametrize("threads", [1, 5, 16])
def test_matches_oracle(n, spacing, threads):
    succ = W.random_list(n, 61 + n % 13)
    rc, rank = cpu_baseline.ruling_set(succ, spacing, threads)
    assert rc == cpu_baseline.OK
    assert np.array_equal(rank, oracle.list_rank(succ))


@pytest.mark.parametrize("layout", ["sequential", "blocked", "self_loop_tail"])
def test_layouts(layout):
    n = 200_003
    if layout == "sequential":
        succ = W.sequential_list(n)
    elif layout == "blocked":
        succ = W.blocked_list(n, 4096, 62)
    else:
        succ = W.to_self_loop_tails(W.random_list(n, 63))
    rc, rank = cpu_baseline.ruling_set(succ, 16, 8)
    assert rc == cpu_baseline.OK and np.array_equal(rank, oracle.list_rank(succ))


@pytest.mark.parametrize("bad", ["two_tails", "no_tail", "out_of_range", "detached_cycle"])
def test_malformed_rejected(bad):
    n = 10_000
    succ, order = W.random_list_with_order(n, 64)
    succ = succ.copy()
    if bad == "two_tails":
        succ[order[n // 2]] = -1
    elif bad == "no_tail":
        succ[order[-1]] = order[0]
    elif bad == "out_of_range":
        succ[order[3]] = n + 5
    else:  # the list stops early; its last 100 nodes close into a cycle
        succ[order[n - 101]] = -1
        succ[order[-1]] = order[n - 100]
    rc, _ = cpu_baseline.ruling_set(succ, 64, 4)
    assert rc == cpu_baseline.EBADLIST
