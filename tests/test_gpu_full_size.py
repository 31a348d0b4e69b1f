"""GPU parity at the benchmark's full sizes, in the forms the benchmark times.

* The 4096-list batch (sizes floor(2^U), U ~ U[6, 20], about 4.3e8 nodes):
  eager, replayed hipGraph, autotuned parameters (eager and replayed) and one
  plain call per list.  Every form is checked on the device by the closed
  form of the generator (the k-th node of a list's order has rank k), and the
  eager form element by element against the oracle over every list.
* Wyllie pointer jumping on the 2^26-node uniform random list (26 jump
  rounds in place), checked by the closed form and oracle samples.
"""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L4096 = 4096


@pytest.fixture(scope="module")
def pj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1002_4482_amd as pj
    pj.load()
    return pj


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def batch4096(pj):
    """The benchmark's batch: device succ and offsets, the host offsets, and
    the closed form as device arrays (global position of the k-th node of each
    list, and k)."""
    succ, off, orders = W.batched_lists(L4096, 6, 20, W.SEED_BASE + 4, return_orders=True)
    print(f"batch of {L4096} lists, {int(off[-1])} nodes", flush=True)
    d_succ, d_off = dev(succ), dev(off)
    sizes = torch.from_numpy(np.diff(off)).cuda()
    base = torch.repeat_interleave(d_off[:-1], sizes)
    pos = dev(np.concatenate(orders)).long() + base
    k = (torch.arange(int(off[-1]), device="cuda") - base).int()
    del base, orders
    yield succ, off, d_succ, d_off, pos, k
    del d_succ, d_off, pos, k
    torch.cuda.empty_cache()


def closed_form_ok(rank, pos, k):
    return bool(torch.equal(rank[pos], k))


def test_batch4096_eager_matches_oracle(pj, batch4096):
    succ, off, d_succ, d_off, pos, k = batch4096
    out = torch.full_like(d_succ, -1)
    pj.list_rank_batched(d_succ, d_off, out, h_offsets=off)
    torch.cuda.synchronize()
    assert closed_form_ok(out, pos, k)
    status, want = oracle.list_rank_batched(succ, off)
    assert (status == 0).all()
    assert np.array_equal(out.cpu().numpy(), want)
    # without the host copy of the offsets (the library reads them back)
    out.fill_(-1)
    pj.list_rank_batched(d_succ, d_off, out)
    torch.cuda.synchronize()
    assert closed_form_ok(out, pos, k)


def test_batch4096_status_and_wyllie(pj, batch4096):
    succ, off, d_succ, d_off, pos, k = batch4096
    st = torch.full((L4096,), 9, dtype=torch.int32, device="cuda")
    out = torch.full_like(d_succ, -1)
    pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, status=st)
    torch.cuda.synchronize()
    assert int(st.abs().sum().item()) == 0
    assert closed_form_ok(out, pos, k)
    out.fill_(-1)
    pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, algo="wyllie")
    torch.cuda.synchronize()
    assert closed_form_ok(out, pos, k)


def test_batch4096_graph_replays(pj, batch4096):
    succ, off, d_succ, d_off, pos, k = batch4096
    pj.graph_cache_clear()
    out = torch.empty_like(d_succ)
    for rep in range(3):
        out.fill_(-1)
        pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, use_graph=True)
        torch.cuda.synchronize()
        assert closed_form_ok(out, pos, k), rep
        # eager work between replays
        pj.list_rank(d_succ[: int(off[1])].clone())
        torch.cuda.synchronize()
    pj.graph_cache_clear()


def test_batch4096_tuned_eager_and_graph(pj, batch4096):
    succ, off, d_succ, d_off, pos, k = batch4096
    pj.tune_clear()
    pj.graph_cache_clear()
    try:
        best, ms = pj.tune_list_rank(d_succ, d_off, h_offsets=off)
        assert ms > 0
        assert pj.tune_lookup(int(off[-1]), L4096) == best
        out = torch.empty_like(d_succ)
        out.fill_(-1)
        pj.list_rank_batched(d_succ, d_off, out, h_offsets=off)   # tuned parameters
        torch.cuda.synchronize()
        assert closed_form_ok(out, pos, k)
        for rep in range(2):
            out.fill_(-1)
            pj.list_rank_batched(d_succ, d_off, out, h_offsets=off, use_graph=True)
            torch.cuda.synchronize()
            assert closed_form_ok(out, pos, k), rep
    finally:
        pj.graph_cache_clear()
        pj.tune_clear()


def test_batch4096_one_call_per_list(pj, batch4096):
    succ, off, d_succ, d_off, pos, k = batch4096
    out = torch.full_like(d_succ, -1)
    for i in range(L4096):
        a, b = int(off[i]), int(off[i + 1])
        pj.list_rank(d_succ[a:b], out[a:b])
    torch.cuda.synchronize()
    assert closed_form_ok(out, pos, k)


def test_full_size_uniform_wyllie(pj):
    """Wyllie on the 2^26-node uniform list: 26 rounds of in-place jumps."""
    n = 1 << 26
    succ, order = W.random_list_with_order(n, W.SEED_BASE + 2)
    d_succ = dev(succ)
    got, st = pj.list_rank(d_succ, algo="wyllie", return_stats=True)
    torch.cuda.synchronize()
    assert st["rounds"] == 26
    d_order = dev(order).long()
    assert torch.equal(got[d_order], torch.arange(n, dtype=torch.int32, device="cuda"))
    # to-tail form, the paper's convention
    got2 = pj.list_rank(d_succ, algo="wyllie", to_tail=True)
    torch.cuda.synchronize()
    assert torch.equal(got2[d_order], torch.arange(n - 1, -1, -1, dtype=torch.int32,
                                                   device="cuda"))
    ref = oracle.list_rank(succ)
    idx = np.random.default_rng(1).integers(0, n, 100_000)
    assert np.array_equal(got.cpu().numpy()[idx], ref[idx])
    del d_succ, got, got2, d_order
    torch.cuda.empty_cache()
