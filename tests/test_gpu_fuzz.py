"""Seeded randomized parity sweep: many small inputs with random shapes,
layouts and parameters, each checked against the oracle element by element.

The cases are drawn from one seeded generator, so a failure names a
reproducible case (its index and parameters are in the assertion message).
"""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1002_4482_amd as pj
    pj.load()
    return pj


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _list(rng, n):
    kind = rng.integers(4)
    if kind == 0:
        return W.random_list(n, int(rng.integers(1 << 30)))
    if kind == 1:
        return W.sequential_list(n)
    if kind == 2:
        return W.blocked_list(n, int(rng.integers(1, 64)), int(rng.integers(1 << 30)))
    return W.to_self_loop_tails(W.random_list(n, int(rng.integers(1 << 30))))


def test_list_ranking_random_cases(pj):
    rng = np.random.default_rng(20240611)
    for case in range(400):
        n = int(rng.integers(1, 40_000)) if case % 4 else int(rng.integers(40_000, 300_000))
        succ = _list(rng, n)
        params = {}
        if rng.random() < 0.5:
            params["spacing"] = int(2 ** rng.integers(1, 9))
        if rng.random() < 0.3:
            params["spacing_up"] = int(2 ** rng.integers(1, 5))
        if rng.random() < 0.3:
            params["cutoff"] = int(rng.integers(64, 16385))
        if rng.random() < 0.3:
            params["max_walk"] = int(rng.integers(16, 2000))
        if rng.random() < 0.2:
            params["block"] = int(64 * rng.integers(1, 17))
        if rng.random() < 0.2:
            params["algo"] = "wyllie"
        to_tail = bool(rng.random() < 0.2)
        got = pj.list_rank(dev(succ), to_tail=to_tail, **params)
        torch.cuda.synchronize()
        want = oracle.list_rank(succ)
        if to_tail:
            want = n - 1 - want
        assert np.array_equal(got.cpu().numpy(), want), (case, n, params, to_tail)


def test_weighted_and_batched_random_cases(pj):
    rng = np.random.default_rng(20240612)
    for case in range(200):
        L = int(rng.integers(1, 300))
        succ, off = W.batched_lists(L, 0, float(rng.uniform(2, 13)), int(rng.integers(1 << 30)))
        w = rng.integers(-100, 100, succ.shape[0]).astype(np.int32)
        params = {}
        if rng.random() < 0.5:
            params["spacing"] = int(2 ** rng.integers(1, 8))
        if rng.random() < 0.3:
            params["cutoff"] = int(rng.integers(64, 16385))
        parts = [slice(off[i], off[i + 1]) for i in range(L)]
        if case % 2:
            want = np.concatenate([oracle.list_rank_weighted(succ[p], w[p]) for p in parts])
            got = pj.list_rank_weighted_batched(dev(succ), dev(w), dev(off), h_offsets=off,
                                                **params)
        else:
            want = np.concatenate([oracle.list_rank(succ[p]) for p in parts])
            got = pj.list_rank_batched(dev(succ), dev(off), h_offsets=off, **params)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want.astype(np.int32)), (case, L, params)


def test_components_random_cases(pj):
    rng = np.random.default_rng(20240613)
    for case in range(200):
        n = int(rng.integers(1, 200_000))
        kind = rng.integers(4)
        if kind == 0:
            m = int(rng.integers(0, 4 * n + 1))
            src, dst = W.random_graph(n, m, int(rng.integers(1 << 30)))
        elif kind == 1:
            src, dst = W.list_graph(n, int(rng.integers(1, min(n, 100) + 1)),
                                    int(rng.integers(1 << 30)))
        elif kind == 2:
            src, dst = W.random_tree_graph(n, int(rng.integers(1, 21)),
                                           int(rng.integers(1, min(n, 50) + 1)),
                                           int(rng.integers(1 << 30)))
        else:
            groups = int(rng.integers(1, min(n, 500) + 1))
            m = n - groups + int(rng.integers(0, 2 * n))
            src, dst, _ = W.planted_graph(n, m, groups, int(rng.integers(1 << 30)))
        if len(src) == 0:
            src = np.zeros(0, np.int32)
            dst = np.zeros(0, np.int32)
        got = pj.connected_components(dev(src), dev(dst), n)
        torch.cuda.synchronize()
        want = oracle.connected_components(src, dst, n)
        assert np.array_equal(got.cpu().numpy(), want), (case, n, int(kind), len(src))
