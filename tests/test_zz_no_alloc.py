"""pj_list_rank_noalloc: the list ranking entry point that allocates nothing.

Called through the C ABI and checked against pj_list_rank_ex (the entry point
whose kernels it shares) and the oracle, on calls in a row that reuse the
library's fixed scratch with smaller inputs after larger ones.  The device
memory pool's high-water mark shows that the call takes nothing from it,
while pj_list_rank_ex does.
"""

import ctypes

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PJ_ESCRATCH = -10
POOL_USED_MEM_HIGH = 0x8  # hipMemPoolAttrUsedMemHigh


@pytest.fixture(scope="module")
def pj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1002_4482_amd as pj
    pj.load()
    return pj


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class Pool:
    """The default device memory pool the library's workspaces come from
    (the HIP runtime torch has loaded)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.pool = ctypes.c_void_p()
        rc = self.hip.hipDeviceGetDefaultMemPool(ctypes.byref(self.pool),
                                                 torch.cuda.current_device())
        assert rc == 0, rc

    def reset_high(self):
        zero = ctypes.c_uint64(0)
        assert self.hip.hipMemPoolSetAttribute(self.pool, POOL_USED_MEM_HIGH,
                                               ctypes.byref(zero)) == 0

    def used_high(self):
        v = ctypes.c_uint64(0)
        assert self.hip.hipMemPoolGetAttribute(self.pool, POOL_USED_MEM_HIGH,
                                               ctypes.byref(v)) == 0
        return v.value


def rank_both(pj, succ, **kw):
    """(noalloc ranks, pj_list_rank_ex ranks) of one list."""
    print(f"noalloc n={succ.shape[0]} {kw}", flush=True)
    d = dev(succ)
    got = torch.full_like(d, -7)
    pj.list_rank_noalloc(d, got, **kw)
    ref = pj.list_rank(d, **kw)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_two_calls_in_a_row_second_smaller(pj):
    """A multi-level solve, then a smaller one reusing the scratch: both equal
    the allocating entry point's ranks and the oracle's."""
    for n, seed in ((3_000_017, 11), (70_001, 12), (5_003, 13)):
        succ = W.random_list(n, seed)
        got, ref = rank_both(pj, succ)
        assert np.array_equal(got, ref), n
        assert np.array_equal(got, oracle.list_rank(succ)), n


def test_options_and_layouts(pj):
    n = 1_000_003
    succ = W.random_list(n, 21)
    want = oracle.list_rank(succ)
    for kw in (dict(algo="wyllie"), dict(algo="ruling_set", spacing=16), dict(to_tail=True),
               dict(level0_state="separate")):
        got, ref = rank_both(pj, succ, **kw)
        assert np.array_equal(got, ref), kw
        exp = (n - 1 - want) if kw.get("to_tail") else want
        assert np.array_equal(got, exp), kw
    seq = W.sequential_list(2_000_000)
    got, ref = rank_both(pj, seq)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, np.arange(2_000_000, dtype=np.int32))


def test_largest_default_input_and_refusal(pj):
    """2^24 nodes fit the 64 MiB scratch with the default options; 2^25 is
    refused before anything is enqueued."""
    n = 1 << 24
    succ, order = W.random_list_with_order(n, W.SEED_BASE + 5)
    d = dev(succ)
    got = torch.full_like(d, -7)
    pj.list_rank_noalloc(d, got)
    ref = pj.list_rank(d)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert torch.equal(got[dev(order).long()], torch.arange(n, dtype=torch.int32, device="cuda"))
    big = torch.zeros(1 << 25, dtype=torch.int32, device="cuda")
    with pytest.raises(pj.PjError) as e:
        pj.list_rank_noalloc(big, big)
    assert e.value.code == PJ_ESCRATCH


def test_in_place_status_and_malformed(pj):
    n = 400_009
    succ = W.random_list(n, 31)
    want = oracle.list_rank(succ)
    d = dev(succ)
    st = torch.full((1,), 9, dtype=torch.int32, device="cuda")
    pj.list_rank_noalloc(d, d, status=st)   # ranks over the successors
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(d.cpu().numpy(), want)
    # a branch: two nodes point at one successor
    bad = succ.copy()
    i = int(np.flatnonzero(bad >= 0)[0])
    j = int(np.flatnonzero(bad >= 0)[1])
    bad[j] = bad[i]
    db = dev(bad)
    out = torch.empty_like(db)
    pj.list_rank_noalloc(db, out, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == pj.PJ_EBADLIST
    # and a good call after the failed one
    got, ref = rank_both(pj, W.random_list(123_457, 32))
    assert np.array_equal(got, ref)


def test_no_pool_allocation(pj):
    pool = Pool()
    succ = dev(W.random_list(2_000_003, 41))
    out = torch.empty_like(succ)
    torch.cuda.synchronize()
    # the allocating entry point takes its workspace from the pool ...
    pool.reset_high()
    pj.list_rank(succ, out)
    torch.cuda.synchronize()
    assert pool.used_high() > 0
    # ... the no-allocation one takes nothing
    pool.reset_high()
    for _ in range(3):
        pj.list_rank_noalloc(succ, out)
    torch.cuda.synchronize()
    assert pool.used_high() == 0


def test_captured_in_a_graph_and_replayed(pj):
    """The caller the entry point is for: a HIP graph captured around it
    (torch.cuda.graph) and replayed several times, with eager work and new
    inputs between the replays; every replay equals the oracle."""
    n = 1_500_007
    lists = [W.random_list(n, 50 + i) for i in range(3)]
    d = dev(lists[0])
    out = torch.full_like(d, -7)
    pj.list_rank_noalloc(d, out)          # outside capture: plans and caches launch sizes
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pj.list_rank_noalloc(d, out)
    for i, succ in enumerate(lists):
        d.copy_(torch.from_numpy(succ))
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.list_rank(succ)), i
        # eager work between replays, on the same scratch
        other = dev(W.random_list(70_001, 60 + i))
        assert np.array_equal(pj.list_rank_noalloc(other).cpu().numpy(),
                              oracle.list_rank(other.cpu().numpy())), i


@pytest.mark.parametrize("n", [0, 1, 2, 3, 64, 16_385])
def test_small_and_degenerate_inputs(pj, n):
    """n = 0 is a no-op, one node has rank 0; the one-workgroup path (up to
    16 K nodes) and the first size above it, against the oracle."""
    succ = W.random_list(n, 70 + n) if n else np.zeros(0, dtype=np.int32)
    d = dev(succ)
    out = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")[:n]
    pj.list_rank_noalloc(d, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.list_rank(succ) if n else succ)
