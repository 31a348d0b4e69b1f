"""GPU parity for list ranking: the HIP path through the C ABI against the CPU
oracle, element by element, bit-exact (integer work).

Sizes span the one-workgroup path, several walk levels, ragged tails and the
full 2^26-node benchmark list (checked there by the closed form
rank[order[k]] = k, which holds at any size, plus oracle-computed samples).
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


def run(pj, succ, **kw):
    out = pj.list_rank(dev(succ), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


SIZES = [1, 2, 3, 64, 1000, 8192, 8193, 65537, 300_007, (1 << 20) + 13]


@pytest.mark.parametrize("algo", ["ruling_set", "wyllie"])
@pytest.mark.parametrize("n", SIZES)
def test_random_list_matches_oracle(pj, algo, n):
    succ = W.random_list(n, W.SEED_BASE + n)
    got = run(pj, succ, algo=algo)
    assert np.array_equal(got, oracle.list_rank(succ))


@pytest.mark.parametrize("layout", ["sequential", "blocked", "reversed"])
@pytest.mark.parametrize("n", [5000, 123_457, 1 << 20])
def test_layouts_match_oracle(pj, layout, n):
    if layout == "sequential":
        succ = W.sequential_list(n)
    elif layout == "blocked":
        succ = W.blocked_list(n, 4096, 11)
    else:  # list runs from the highest id down to 0
        succ = np.arange(-1, n - 1, dtype=np.int32)
    want = oracle.list_rank(succ)
    for algo in ("ruling_set", "wyllie"):
        assert np.array_equal(run(pj, succ, algo=algo), want), algo


def test_paper_tail_convention_and_to_tail(pj):
    n = 200_003
    succ = W.random_list(n, 5)
    want = oracle.list_rank(succ)
    selfl = W.to_self_loop_tails(succ)
    for algo in ("ruling_set", "wyllie"):
        assert np.array_equal(run(pj, selfl, algo=algo), want)
        assert np.array_equal(run(pj, succ, algo=algo, to_tail=True), n - 1 - want)


@pytest.mark.parametrize("params", [
    dict(spacing=2), dict(spacing=4, spacing_up=2), dict(spacing=64, spacing_up=32),
    dict(spacing=1024), dict(max_walk=16), dict(cutoff=64), dict(seed=12345),
    dict(block=64), dict(block=512), dict(block=1024, spacing=128),
    dict(spacing=8, cutoff=256, max_walk=20, seed=7),
    dict(algo="wyllie", block=64), dict(algo="wyllie", block=1024),
])
def test_parameters_do_not_change_ranks(pj, params):
    n = 400_009
    succ = W.random_list(n, 99)
    assert np.array_equal(run(pj, succ, **params), oracle.list_rank(succ))


def test_adversarial_long_sublists(pj):
    # every splitter block's nodes visited consecutively after all others:
    # sequential order with a large spacing forces cut points
    n = 1 << 18
    succ = W.sequential_list(n)
    assert np.array_equal(run(pj, succ, spacing=65536, max_walk=16), np.arange(n))


@pytest.mark.parametrize("bad,why", [
    ("two_tails", "two lists"), ("cycle", "no tail"), ("detached_cycle", "list + cycle"),
    ("out_of_range", "bad id"), ("branch", "two heads"),
])
@pytest.mark.parametrize("algo", ["ruling_set", "wyllie"])
@pytest.mark.parametrize("n", [3000, 100_000])
def test_malformed_lists_are_reported(pj, bad, why, algo, n):
    succ = W.random_list(n, 3).copy()
    order = np.argsort(oracle.list_rank(succ))
    if bad == "two_tails":
        succ[order[n // 2]] = -1
    elif bad == "cycle":
        succ[order[-1]] = order[0]
    elif bad == "detached_cycle":
        succ[order[n // 2 - 1]] = -1
        succ[order[-1]] = order[n // 2]
    elif bad == "out_of_range":
        succ[order[7]] = n + 5
    elif bad == "branch":
        succ[order[10]] = order[20]
    assert oracle.list_rank_status(succ)[0] == oracle.EBADLIST
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pj.list_rank(dev(succ), algo=algo, validate=True, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == oracle.EBADLIST, why


def test_validate_accepts_good_lists(pj):
    for n in (1, 7, 9000, 300_000):
        succ = W.random_list(n, n)
        for algo in ("ruling_set", "wyllie"):
            status = torch.full((1,), 77, dtype=torch.int32, device="cuda")
            got = pj.list_rank(dev(succ), algo=algo, validate=True, status=status)
            torch.cuda.synchronize()
            assert int(status.item()) == 0
            assert np.array_equal(got.cpu().numpy(), oracle.list_rank(succ))


def test_empty_list_is_noop(pj):
    out = pj.list_rank(torch.empty(0, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert out.numel() == 0


def test_repeatable(pj):
    succ = dev(W.random_list(1 << 20, 1))
    a = pj.list_rank(succ)
    b = pj.list_rank(succ, seed=2, spacing=32)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_full_size_uniform_closed_form_and_samples(pj):
    """The 2^26-node uniform list at the benchmark's launch configuration."""
    n = 1 << 26
    succ, order = W.random_list_with_order(n, W.SEED_BASE + 2)
    d_succ = dev(succ)
    got = pj.list_rank(d_succ)
    torch.cuda.synchronize()
    d_order = dev(order).long()
    want = torch.arange(n, dtype=torch.int32, device="cuda")
    assert torch.equal(got[d_order], want)
    # sampled nodes against the oracle's ranks
    ref = oracle.list_rank(succ)
    idx = np.random.default_rng(0).integers(0, n, 100_000)
    assert np.array_equal(got.cpu().numpy()[idx], ref[idx])
    del d_succ, got, d_order, want
    torch.cuda.empty_cache()


@pytest.mark.parametrize("layout", ["sequential", "blocked"])
def test_full_size_other_layouts(pj, layout):
    n = 1 << 26
    if layout == "sequential":
        succ = W.sequential_list(n)
        order = None
    else:
        succ, order = W.blocked_list_with_order(n, 4096, W.SEED_BASE + 2)
    for algo in ("ruling_set", "wyllie"):
        got = pj.list_rank(dev(succ), algo=algo)
        torch.cuda.synchronize()
        if order is None:
            assert torch.equal(got, torch.arange(n, dtype=torch.int32, device="cuda")), algo
        else:
            assert torch.equal(got[dev(order).long()],
                               torch.arange(n, dtype=torch.int32, device="cuda")), algo
        del got
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ batched
def batched_case(L, lo, hi, seed):
    succ, off = W.batched_lists(L, lo, hi, seed)
    return succ, off


@pytest.mark.parametrize("L,lo,hi", [(1, 3, 4), (5, 0, 3), (100, 0, 10), (700, 6, 14),
                                     (64, 12, 17), (3000, 0, 6)])
@pytest.mark.parametrize("algo", ["ruling_set", "wyllie"])
def test_batched_matches_oracle(pj, L, lo, hi, algo):
    succ, off = batched_case(L, lo, hi, L * 31 + lo)
    status, want = oracle.list_rank_batched(succ, off)
    assert (status == 0).all()
    got = pj.list_rank_batched(dev(succ), dev(off), h_offsets=off, algo=algo)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    # without the host copy of the offsets
    got2 = pj.list_rank_batched(dev(succ), dev(off), algo=algo)
    torch.cuda.synchronize()
    assert np.array_equal(got2.cpu().numpy(), want)


def test_batched_with_empty_lists_and_statuses(pj):
    lists = [W.random_list(s, s) for s in (0, 5, 0, 0, 1, 20000, 3, 0)]
    succ, off = W.concat_lists(lists)
    bad = succ.copy()
    # list 5 (20000 nodes) gets a second tail
    a = off[5]
    seg = bad[a:off[6]]
    seg[np.nonzero(seg != -1)[0][0]] = -1
    for algo in ("ruling_set", "wyllie"):
        st = torch.full((8,), 9, dtype=torch.int32, device="cuda")
        got = pj.list_rank_batched(dev(succ), dev(off), h_offsets=off, algo=algo, status=st,
                                   validate=True)
        torch.cuda.synchronize()
        assert st.cpu().numpy().tolist() == [0] * 8
        assert np.array_equal(got.cpu().numpy(), oracle.list_rank_batched(succ, off)[1])
        st.fill_(9)
        pj.list_rank_batched(dev(bad), dev(off), h_offsets=off, algo=algo, status=st,
                             validate=True)
        torch.cuda.synchronize()
        assert st.cpu().numpy()[5] == oracle.EBADLIST


def test_batched_equals_per_list(pj):
    succ, off = batched_case(50, 4, 15, 77)
    d_succ = dev(succ)
    got = pj.list_rank_batched(d_succ, dev(off), h_offsets=off)
    for i in range(50):
        one = pj.list_rank(d_succ[off[i]:off[i + 1]].clone())
        torch.cuda.synchronize()
        assert torch.equal(one, got[off[i]:off[i + 1]])


# ----------------------------------------------------------- graph + tuning
def test_graph_replay_matches_eager_every_time(pj):
    """The captured batched graph, replayed several times with eager work and
    syncs in between, gives the eager result each time."""
    succ, off = batched_case(300, 3, 16, 5)
    d_succ, d_off = dev(succ), dev(off)
    want = oracle.list_rank_batched(succ, off)[1]
    eager = pj.list_rank_batched(d_succ, d_off, h_offsets=off)
    torch.cuda.synchronize()
    assert np.array_equal(eager.cpu().numpy(), want)
    out = torch.empty_like(d_succ)
    for rep in range(4):
        out.fill_(-7)
        pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        # unrelated eager work between replays
        pj.list_rank(d_succ[off[0]:off[1]].clone())
        torch.cuda.synchronize()
    # new contents, same buffers and sizes: the replay reads the new input
    succ2, _ = batched_case(300, 3, 16, 5)
    rng = np.random.default_rng(1)
    for i in range(300):
        seg = slice(off[i], off[i + 1])
        perm = rng.permutation(off[i + 1] - off[i]).astype(np.int32)
        s = np.empty_like(perm)
        if len(perm):
            s[perm[:-1]] = perm[1:]
            s[perm[-1]] = -1
        succ2[seg] = s
    d_succ.copy_(dev(succ2))
    pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.list_rank_batched(succ2, off)[1])
    pj.graph_cache_clear()


@pytest.mark.parametrize("algo", ["wyllie", "ruling_set"])
def test_graph_replay_after_list_sizes_change(pj, algo):
    """Same buffers, same L and the same node total, but the largest list
    grows past a power of two: Wyllie needs one more jump round than the
    captured graph ran, so the replay must not reuse it."""
    L = 4
    sizes1, sizes2 = [1000, 1000, 1000, 1000], [3980, 10, 5, 5]
    assert sum(sizes1) == sum(sizes2)
    total = sum(sizes1)

    def make(sizes, seed):
        lists = [W.random_list(s, seed + i) for i, s in enumerate(sizes)]
        return W.concat_lists(lists)

    succ1, off1 = make(sizes1, 300)
    succ2, off2 = make(sizes2, 400)
    d_succ = dev(succ1)
    d_off = dev(off1)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    pj.graph_cache_clear()
    h_off = off1.copy()
    for rep in range(2):
        out.fill_(-1)
        pj.list_rank_batched(d_succ, d_off, out, h_offsets=h_off, algo=algo, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.list_rank_batched(succ1, off1)[1]), rep
    # new sizes written into the same device buffers
    d_succ.copy_(dev(succ2))
    d_off.copy_(dev(off2))
    h_off[:] = off2
    st = torch.full((L,), 9, dtype=torch.int32, device="cuda")
    for rep in range(2):
        out.fill_(-1)
        pj.list_rank_batched(d_succ, d_off, out, h_offsets=h_off, algo=algo, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.list_rank_batched(succ2, off2)[1]), rep
    # with statuses (a different graph): a valid batch reports OK everywhere
    pj.list_rank_batched(d_succ, d_off, out, h_offsets=h_off, algo=algo, use_graph=True,
                         status=st)
    torch.cuda.synchronize()
    assert st.cpu().numpy().tolist() == [0] * L
    assert np.array_equal(out.cpu().numpy(), oracle.list_rank_batched(succ2, off2)[1])
    pj.graph_cache_clear()


def test_graph_replay_single_large_list(pj):
    n = 3_000_017
    succ = W.random_list(n, 12)
    off = np.array([0, n], dtype=np.int64)
    want = oracle.list_rank(succ)
    d_succ, d_off = dev(succ), dev(off)
    out = torch.empty_like(d_succ)
    for _ in range(3):
        out.zero_()
        pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)
    pj.graph_cache_clear()


def test_autotune_picks_parameters_and_keeps_results(pj, tmp_path):
    n = 1 << 20
    succ = W.random_list(n, 21)
    d_succ = dev(succ)
    pj.tune_clear()
    best, ms = pj.tune_list_rank(d_succ)
    assert best["spacing"] in (8, 16, 32, 64, 128, 256) and best["spacing_up"] in (4, 8, 16)
    assert best["cutoff"] in (2048, 4096, 8192, 16384) and best["block"] in (128, 256, 512, 1024)
    assert ms > 0
    assert pj.tune_lookup(n) == best
    got = pj.list_rank(d_succ)   # uses the tuned parameters
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank(succ))
    path = tmp_path / "tune.txt"
    pj.tune_save(path)
    pj.tune_clear()
    assert pj.tune_lookup(n) is None
    pj.tune_load(path)
    assert pj.tune_lookup(n) == best
    # batched tuning
    bs, boff = batched_case(200, 6, 14, 3)
    best_b, _ = pj.tune_list_rank(dev(bs), dev(boff), h_offsets=boff)
    assert pj.tune_lookup(int(boff[-1]), 200) == best_b
    got = pj.list_rank_batched(dev(bs), dev(boff), h_offsets=boff)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank_batched(bs, boff)[1])
    pj.tune_clear()


@pytest.mark.parametrize("local_frac", [0.0, 0.45, 0.55, 1.0])
def test_layout_locality_choice_keeps_ranks(pj, local_frac):
    """Lists of 2^22 nodes whose successors are local (the next id) for a
    given fraction of nodes: the walk picks its level-0 spacing on the device
    from that fraction, on both sides of the one-half threshold."""
    n = 1 << 22
    rng = np.random.default_rng(int(local_frac * 100) + 7)
    # runs of consecutive ids with geometric lengths (a run continues with
    # probability local_frac), laid out along the list in random order
    if local_frac >= 1.0:
        lengths = np.array([n])
    else:
        lengths = rng.geometric(1.0 - local_frac, size=n)
        lengths = lengths[:np.searchsorted(np.cumsum(lengths), n) + 1]
        lengths[-1] -= lengths.sum() - n
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    perm = rng.permutation(len(lengths))
    ls, st = lengths[perm], starts[perm]
    pos0 = np.concatenate([[0], np.cumsum(ls)[:-1]])
    order = np.repeat(st, ls) + (np.arange(n) - np.repeat(pos0, ls))
    succ = np.full(n, -1, np.int32)
    succ[order[:-1]] = order[1:]
    idx = np.nonzero(succ >= 0)[0]
    near = np.mean(np.abs(succ[idx].astype(np.int64) - idx) <= 64)
    assert abs(near - local_frac) < 0.02
    got = run(pj, succ)
    want = np.empty(n, np.int32)
    want[order] = np.arange(n, dtype=np.int32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("layout", ["uniform", "sequential"])
def test_wyllie_reports_rounds(pj, layout):
    # Wyllie runs the doubling bound ceil(log2 n) rounds and says so
    n = 300_007
    succ = W.random_list(n, 17) if layout == "uniform" else W.sequential_list(n)
    out, st = pj.list_rank(dev(succ), algo="wyllie", return_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.list_rank(succ))
    assert st["rounds"] == int(np.ceil(np.log2(n)))


@pytest.mark.parametrize("case", ["uniform", "sequential", "small", "wyllie", "batched",
                                  "batched_graph", "to_tail"])
def test_in_place(pj, case):
    # rank == succ: the ranks overwrite the successors (Section 3.2)
    if case.startswith("batched"):
        succ, off = W.batched_lists(37, 3, 14, 21)
        want = np.concatenate([oracle.list_rank(succ[off[i]:off[i + 1]]) for i in range(37)])
        d = dev(succ)
        kw = dict(use_graph=True) if case == "batched_graph" else {}
        for _ in range(2 if kw else 1):
            d.copy_(dev(succ))
            out = pj.list_rank_batched(d, dev(off), d, h_offsets=off, **kw)
        torch.cuda.synchronize()
        assert out.data_ptr() == d.data_ptr()
        assert np.array_equal(d.cpu().numpy(), want)
        pj.graph_cache_clear()
        return
    n = {"small": 3000, "sequential": 1 << 20}.get(case, 400_009)
    succ = W.sequential_list(n) if case == "sequential" else W.random_list(n, 23)
    want = oracle.list_rank(succ)
    d = dev(succ)
    kw = {"wyllie": dict(algo="wyllie"), "to_tail": dict(to_tail=True)}.get(case, {})
    out = pj.list_rank(d, d, **kw)
    torch.cuda.synchronize()
    assert out.data_ptr() == d.data_ptr()
    assert np.array_equal(d.cpu().numpy(), n - 1 - want if case == "to_tail" else want)


def test_in_place_rejects_validate_and_partial_overlap(pj):
    succ = W.random_list(5000, 29)
    d = dev(succ)
    with pytest.raises(Exception):
        pj.list_rank(d, d, validate=True)
    big = dev(np.concatenate([succ, np.zeros(16, np.int32)]))
    with pytest.raises(Exception):
        pj.list_rank(big[:5000], big[8:5008])
    # the input is untouched by the rejected calls
    assert np.array_equal(d.cpu().numpy(), succ)


# ------------------------------------------------------------ weighted lists

def _weights(n, seed, lo=-1000, hi=1000):
    return np.random.default_rng(seed).integers(lo, hi, n).astype(np.int32)


@pytest.mark.parametrize("n", SIZES)
def test_weighted_matches_oracle(pj, n):
    succ = W.random_list(n, 31 + n % 7)
    w = _weights(n, n)
    got = pj.list_rank_weighted(dev(succ), dev(w))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank_weighted(succ, w))


@pytest.mark.parametrize("params", [
    dict(), dict(spacing=2), dict(spacing=64, spacing_up=16), dict(max_walk=16),
    dict(cutoff=64), dict(block=1024, spacing=128), dict(seed=99),
])
@pytest.mark.parametrize("layout", ["uniform", "sequential", "blocked"])
def test_weighted_layouts_and_parameters(pj, params, layout):
    n = 300_007
    if layout == "uniform":
        succ = W.random_list(n, 41)
    elif layout == "sequential":
        succ = W.sequential_list(n)
    else:
        succ = W.blocked_list(n, 4096, 42)
    w = _weights(n, 43, 0, 50)
    got = pj.list_rank_weighted(dev(succ), dev(w), **params)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank_weighted(succ, w))


def test_weighted_unit_weights_and_in_place(pj):
    n = 1 << 20
    succ = W.random_list(n, 47)
    want = oracle.list_rank(succ)
    got = pj.list_rank_weighted(dev(succ), dev(np.ones(n, np.int32)))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    w = _weights(n, 48)
    d = dev(succ)
    out = pj.list_rank_weighted(d, dev(w), d)
    torch.cuda.synchronize()
    assert out.data_ptr() == d.data_ptr()
    assert np.array_equal(d.cpu().numpy(), oracle.list_rank_weighted(succ, w))


def test_weighted_closed_form_large(pj):
    # rank[order[k]] = exclusive prefix of the weights along the list order
    n = 1 << 24
    succ, order = W.random_list_with_order(n, 49)
    w = _weights(n, 50, 0, 100)
    got = pj.list_rank_weighted(dev(succ), dev(w))
    do = torch.from_numpy(order.astype(np.int64)).cuda()
    wo = dev(w)[do].to(torch.int64)
    want = torch.cumsum(wo, 0) - wo
    assert torch.equal(got[do].to(torch.int64), want)


@pytest.mark.parametrize("L,lo,hi", [(37, 3, 14), (500, 1, 10), (3, 16, 19)])
def test_weighted_batched(pj, L, lo, hi):
    succ, off = W.batched_lists(L, lo, hi, 51 + L)
    w = _weights(succ.shape[0], 52 + L)
    want = np.concatenate([oracle.list_rank_weighted(succ[off[i]:off[i + 1]],
                                                     w[off[i]:off[i + 1]]) for i in range(L)])
    got = pj.list_rank_weighted_batched(dev(succ), dev(w), dev(off), h_offsets=off)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    got2 = pj.list_rank_weighted_batched(dev(succ), dev(w), dev(off))
    torch.cuda.synchronize()
    assert np.array_equal(got2.cpu().numpy(), want)


def test_weighted_rejects_and_reports(pj):
    n = 5000
    succ = W.random_list(n, 53)
    w = _weights(n, 54)
    for kw in (dict(algo="wyllie"), dict(to_tail=True), dict(validate=True)):
        with pytest.raises(Exception):
            pj.list_rank_weighted(dev(succ), dev(w), **kw)
    dw = dev(w)
    with pytest.raises(Exception):
        pj.list_rank_weighted(dev(succ), dw, dw)
    # a valid list reports OK through the status (the coverage check compares
    # the weights the levels saw with the weights given)
    st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    got = pj.list_rank_weighted(dev(succ), dev(w), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == pj.PJ_OK
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank_weighted(succ, w))
    big = W.random_list(300_007, 55)
    wb = _weights(300_007, 56)
    st2 = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    pj.list_rank_weighted(dev(big), dev(wb), status=st2)
    torch.cuda.synchronize()
    assert int(st2.item()) == pj.PJ_OK
    # a detached cycle beside a shorter list: every node is no longer covered
    cyc, order = W.random_list_with_order(300_007, 57)
    cyc = cyc.copy()
    cyc[order[-1001]] = -1
    cyc[order[-1]] = order[-1000]
    pj.list_rank_weighted(dev(cyc), dev(wb), status=st2)
    torch.cuda.synchronize()
    assert int(st2.item()) == pj.PJ_EBADLIST
    # malformed list: the status names it
    bad = succ.copy()
    bad[int(np.nonzero(bad != -1)[0][0])] = -1  # a second tail: two lists
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    pj.list_rank_weighted(dev(bad), dev(w), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == pj.PJ_EBADLIST


def test_weighted_edge_cases(pj):
    # n = 1 and 2, all-zero weights, a batch with empty and one-node lists,
    # and cut points (max_walk 16) with large weights near the int32 range
    for succ, w in (([-1], [7]), ([1, -1], [3, 4]), ([-1, 0], [3, 4])):
        succ, w = np.array(succ, np.int32), np.array(w, np.int32)
        got = pj.list_rank_weighted(dev(succ), dev(w))
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), oracle.list_rank_weighted(succ, w))
    n = 200_003
    succ = W.random_list(n, 71)
    z = np.zeros(n, np.int32)
    assert (pj.list_rank_weighted(dev(succ), dev(z)).cpu().numpy() == 0).all()
    w = np.random.default_rng(72).integers(0, 10_000, n).astype(np.int32)  # total < 2^31
    got = pj.list_rank_weighted(dev(succ), dev(w), max_walk=16, spacing=4096, cutoff=64)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank_weighted(succ, w))
    sizes = [0, 1, 0, 5, 1, 0, 3000, 0]
    parts = [W.random_list(k, 73 + i) if k else np.empty(0, np.int32) for i, k in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = np.concatenate(parts).astype(np.int32)
    wc = np.random.default_rng(74).integers(-50, 50, cat.shape[0]).astype(np.int32)
    want = np.concatenate([oracle.list_rank_weighted(p, wc[off[i]:off[i + 1]])
                           for i, p in enumerate(parts)]).astype(np.int32)
    got = pj.list_rank_weighted_batched(dev(cat), dev(wc), dev(off), h_offsets=off)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)


def test_weighted_golden_worked_example(pj):
    from helpers import read_golden
    g = read_golden("list_weighted_worked_example.txt")
    succ = np.array(g["succ"], dtype=np.int32)
    w = np.array(g["weight"], dtype=np.int32)
    got = pj.list_rank_weighted(dev(succ), dev(w))
    torch.cuda.synchronize()
    assert got.cpu().numpy().tolist() == g["weighted_rank"]


# ------------------------------------------- chosen splitters, state layout
def _chosen(succ, kind, k, seed):
    """Splitter ids: `kind` "even" takes every k-th node in list order from a
    random phase; "random" takes n // k distinct nodes uniformly at random."""
    n = len(succ)
    order = np.argsort(oracle.list_rank(succ)).astype(np.int32)
    rng = np.random.default_rng(seed)
    if kind == "even":
        return order[int(rng.integers(0, k)) % n::k].copy()
    return rng.choice(n, max(1, n // k), replace=False).astype(np.int32)


@pytest.mark.parametrize("kind", ["even", "random"])
@pytest.mark.parametrize("n,k", [(20_000, 2), (20_000, 1000), (300_007, 16), (300_007, 64),
                                 ((1 << 20) + 13, 64), ((1 << 20) + 13, 4096)])
def test_chosen_splitters_match_oracle(pj, kind, n, k):
    succ = W.random_list(n, 900 + n % 97 + k)
    spl = _chosen(succ, kind, k, n + k)
    want = oracle.list_rank(succ)
    got, st = pj.list_rank(dev(succ), splitters=dev(spl), return_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    assert st["sublists0"] == len(spl) + 1 + st["cuts0"]
    if kind == "even" and k <= 1024:
        # every sublist holds k nodes (the piece before the first chosen
        # splitter starts at the head and holds fewer)
        assert st["cuts0"] == 0 and st["max_sublist0"] == k
    # in place, and with a status
    d = dev(succ)
    status = torch.full((1,), 9, dtype=torch.int32, device="cuda")
    pj.list_rank(d, d, splitters=dev(spl), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(d.cpu().numpy(), want)


def test_chosen_splitters_edge_cases(pj):
    n = 50_000
    succ, order = W.random_list_with_order(n, 77)
    want = oracle.list_rank(succ)
    cases = {
        "head_only": order[:1],
        "tail_only": order[-1:],
        "every_node": np.random.default_rng(1).permutation(n).astype(np.int32),
        "head_and_tail": order[[0, -1]],
        "one_in_the_middle": order[n // 2:n // 2 + 1],   # long walks: cut at max_walk
    }
    for name, spl in cases.items():
        got, st = pj.list_rank(dev(succ), splitters=dev(np.ascontiguousarray(spl)),
                               max_walk=64, return_stats=True)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), name
        assert st["max_sublist0"] <= 64, name
    # small inputs still take the splitters (no one-workgroup shortcut)
    for m in (1, 2, 3, 100):
        s = W.random_list(m, m)
        spl = np.arange(m, dtype=np.int32)[::2].copy()
        got = pj.list_rank(dev(s), splitters=dev(spl))
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), oracle.list_rank(s)), m


def test_chosen_splitters_rejected_and_reported(pj):
    n = 40_000
    succ = W.random_list(n, 5)
    status = torch.full((1,), 9, dtype=torch.int32, device="cuda")
    dup = np.array([5, 17, 5, 900], np.int32)
    pj.list_rank(dev(succ), splitters=dev(dup), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == pj.PJ_EINVAL
    out_of_range = np.array([3, n + 2], np.int32)
    pj.list_rank(dev(succ), splitters=dev(out_of_range), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == pj.PJ_EINVAL
    spl = dev(np.array([1, 2], np.int32))
    for kw in (dict(algo="wyllie"), dict(level0_state="separate")):
        with pytest.raises(Exception):
            pj.list_rank(dev(succ), splitters=spl, **kw)
    with pytest.raises(Exception):
        pj.list_rank_weighted(dev(succ), dev(np.ones(n, np.int32)), splitters=spl)
    off = np.array([0, n], np.int64)
    with pytest.raises(Exception):
        pj.list_rank_batched(dev(succ), dev(off), h_offsets=off, splitters=spl)
    # the input is a valid list: after the rejected calls a plain call is right
    got = pj.list_rank(dev(succ))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.list_rank(succ))


@pytest.mark.parametrize("layout", ["uniform", "sequential", "blocked"])
@pytest.mark.parametrize("n", [20_000, 300_007, (1 << 22) + 5])
def test_separate_state_matches_oracle(pj, layout, n):
    if layout == "uniform":
        succ = W.random_list(n, 61)
    elif layout == "sequential":
        succ = W.sequential_list(n)
    else:
        succ = W.blocked_list(n, 4096, 62)
    want = oracle.list_rank(succ)
    got = pj.list_rank(dev(succ), level0_state="separate")
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    d = dev(succ)
    pj.list_rank(d, d, level0_state="separate", to_tail=True)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), n - 1 - want)


def test_separate_state_batched_and_graph(pj):
    succ, off = W.batched_lists(300, 4, 16, 63)
    want = oracle.list_rank_batched(succ, off)[1]
    d_succ, d_off = dev(succ), dev(off)
    for use_graph in (False, True, True):
        out = pj.list_rank_batched(d_succ, d_off, h_offsets=off, level0_state="separate",
                                   use_graph=use_graph)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), use_graph
    # the same buffers with the packed state: a separate graph, same ranks
    out = pj.list_rank_batched(d_succ, d_off, h_offsets=off, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    pj.graph_cache_clear()
    with pytest.raises(Exception):
        pj.list_rank(d_succ, level0_state=7)
