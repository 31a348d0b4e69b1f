"""Pure-Python checkers used to pin the oracle.  Independent of oracle/ and of
the GPU library: brute force on tiny inputs and the complete invariants."""

import os

import numpy as np

from conftest import GOLDEN


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = [int(v) for v in vals]
    return out


def is_tail(succ, i):
    return succ[i] == -1 or succ[i] == i


def brute_list_valid(succ):
    """True iff succ is one linked list over all n nodes: some start node
    reaches a tail after visiting every node exactly once."""
    n = len(succ)
    if n == 0:
        return True
    for s in succ:
        if not (-1 <= s < n):
            return False
    for start in range(n):
        seen = set()
        cur = start
        while True:
            if cur in seen:
                break
            seen.add(cur)
            if is_tail(succ, cur):
                if len(seen) == n:
                    return True
                break
            cur = succ[cur]
    return False


def brute_rank_from_head(succ):
    """n - 1 - (number of hops from i to the tail), hop counting per node."""
    n = len(succ)
    out = []
    for i in range(n):
        d, cur = 0, i
        while not is_tail(succ, cur):
            cur = succ[cur]
            d += 1
        out.append(n - 1 - d)
    return out


def check_rank_invariants(succ, rank):
    """Complete characterisation: exactly one tail, rank is a permutation of
    0..n-1 and rank[succ[i]] = rank[i] + 1 for every non-tail i.  Together
    these exclude cycles, branching and several lists, and determine the
    ranks uniquely (the rank-0 node is then the head)."""
    succ = np.asarray(succ, dtype=np.int64)
    rank = np.asarray(rank, dtype=np.int64)
    n = succ.shape[0]
    if n == 0:
        return
    assert np.array_equal(np.sort(rank), np.arange(n)), "not a permutation"
    idx = np.arange(n)
    nt = ~((succ == -1) | (succ == idx))
    assert int((~nt).sum()) == 1, "not exactly one tail"
    assert np.array_equal(rank[succ[nt]], rank[nt] + 1), "successor rule broken"
    has_pred = np.zeros(n, dtype=bool)
    has_pred[succ[nt]] = True
    head = int(np.nonzero(rank == 0)[0][0])
    assert not has_pred[head], "rank-0 node has a predecessor"


def brute_components(n, edges):
    """Warshall transitive closure; label = smallest reachable id."""
    reach = [[i == j for j in range(n)] for i in range(n)]
    for a, b in edges:
        reach[a][b] = reach[b][a] = True
    for k in range(n):
        for i in range(n):
            if reach[i][k]:
                rk = reach[k]
                ri = reach[i]
                for j in range(n):
                    if rk[j]:
                        ri[j] = True
    return [min(j for j in range(n) if reach[i][j]) for i in range(n)]


def check_cc_invariants(src, dst, label):
    label = np.asarray(label, dtype=np.int64)
    n = label.shape[0]
    v = np.arange(n)
    assert (label <= v).all(), "label exceeds vertex id"
    assert (label >= 0).all()
    assert np.array_equal(label[label], label), "label is not its own label"
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    assert np.array_equal(label[src], label[dst]), "edge crosses components"
