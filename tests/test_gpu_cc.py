"""GPU parity for connected components: the HIP Shiloach-Vishkin path through
the C ABI against the union-find oracle, bit-exact on min-id labels."""

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


def run(pj, src, dst, n, **kw):
    out = pj.connected_components(dev(src), dev(dst), n, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,m", [(1, 0), (1, 3), (2, 1), (10, 0), (100, 50), (1000, 1000),
                                 (5000, 40000), (100_003, 70_001), (300_000, 1_000_003),
                                 (1 << 20, 1 << 22)])
def test_random_graph_matches_oracle(pj, n, m):
    src, dst = W.random_graph(n, m, n + m)
    assert np.array_equal(run(pj, src, dst, n), oracle.connected_components(src, dst, n))


@pytest.mark.parametrize("n,m,groups", [(4096, 8192, 64), (200_000, 600_000, 1024),
                                        (1 << 20, 1 << 22, 1024)])
def test_planted_matches_oracle(pj, n, m, groups):
    src, dst, _ = W.planted_graph(n, m, groups, 3)
    got = run(pj, src, dst, n)
    assert np.array_equal(got, oracle.connected_components(src, dst, n))
    assert len(np.unique(got)) == groups


@pytest.mark.parametrize("case", ["one_larger_end", "one_slice", "tiny_ids", "ragged"])
def test_slice_sorted_round_one_layouts(pj, case):
    """Round 1 sorts each chunk of 2048 pairs by the slice of its larger end,
    and the slice's workgroups take its runs of 8 chunks at a time: inputs
    that put every pair in one slice (runs of whole chunks, units far above
    2048 pairs), ids below one slice block, and a ragged last chunk."""
    rng = np.random.default_rng(77)
    if case == "one_larger_end":      # every pair's larger end is the same vertex
        n, m = 300_000, 50_000
        src = np.full(m, n - 1, dtype=np.int32)
        dst = rng.integers(0, n - 1, m).astype(np.int32)
    elif case == "one_slice":         # larger ends all inside one 1024-id block
        n, m = 1 << 20, 60_000
        src = rng.integers(5 * 1024, 6 * 1024, m).astype(np.int32)
        dst = rng.integers(0, 5 * 1024, m).astype(np.int32)
    elif case == "tiny_ids":          # n below one slice block: a single slice
        n, m = 20, 10_000
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
    else:                             # self-loops, duplicates and a ragged tail
        n, m = 77_777, 2048 * 37 + 5
        src = rng.integers(0, n, m).astype(np.int32)
        dst = src.copy()
        keep = rng.random(m) < 0.7
        dst[keep] = rng.integers(0, n, int(keep.sum()))
    want = oracle.connected_components(src, dst, n)
    assert np.array_equal(run(pj, src, dst, n), want), case
    # and in a batch between two other graphs
    a_s, a_d = W.random_graph(1000, 3000, 5)
    c_s, c_d = W.random_graph(5000, 1000, 6)
    voff = np.array([0, 1000, 1000 + n, 1000 + n + 5000], dtype=np.int64)
    eoff = np.array([0, 3000, 3000 + m, 3000 + m + 1000], dtype=np.int64)
    bs = np.concatenate([a_s, src, c_s]).astype(np.int32)
    bd = np.concatenate([a_d, dst, c_d]).astype(np.int32)
    got = pj.connected_components_batched(dev(bs), dev(bd), dev(voff), dev(eoff))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.connected_components_batched(bs, bd, voff, eoff))


@pytest.mark.parametrize("family", ["lists", "trees2", "trees7", "path_up", "path_down", "star",
                                    "self_loops", "dense0.001", "dense0.01"])
def test_graph_families(pj, family):
    n = 100_000
    if family.startswith("dense"):
        src, dst, group_of = W.component_density_graph(400_000, float(family[5:]), 16, 4)
        n = group_of.shape[0]
    elif family == "lists":
        src, dst = W.list_graph(n, 37, 1)
    elif family == "trees2":
        src, dst = W.random_tree_graph(n, 2, 11, 2)
    elif family == "trees7":
        src, dst = W.random_tree_graph(n, 7, 5, 3)
    elif family == "path_up":
        src = np.arange(n - 1, dtype=np.int32)
        dst = src + 1
    elif family == "path_down":
        dst = np.arange(n - 1, dtype=np.int32)
        src = dst + 1
        src, dst = src[::-1].copy(), dst[::-1].copy()
    elif family == "star":
        src = np.full(n - 1, n // 2, dtype=np.int32)
        dst = np.delete(np.arange(n, dtype=np.int32), n // 2)
    else:
        src = np.arange(n, dtype=np.int32)
        dst = src.copy()
    want = oracle.connected_components(src, dst, n)
    got, st = pj.connected_components(dev(src), dev(dst), n, return_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    # Shiloach-Vishkin bound the rounds that still change the forest by
    # floor(log_{3/2} n) + 2; the count reported here also includes the last
    # round, which changes nothing and ends the solve
    changing_rounds = st["rounds"] - 1
    assert changing_rounds <= int(np.floor(np.log(n) / np.log(1.5))) + 2


def test_unaligned_and_status(pj):
    n, m = 50_000, 120_001
    src, dst = W.random_graph(n, m, 8)
    # views starting one element in: not 16-byte aligned
    d_src = dev(np.concatenate([[0], src]).astype(np.int32))[1:]
    d_dst = dev(np.concatenate([[0], dst]).astype(np.int32))[1:]
    st = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    got = pj.connected_components(d_src, d_dst, n, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(got.cpu().numpy(), oracle.connected_components(src, dst, n))
    bad = dst.copy()
    bad[17] = n + 3
    pj.connected_components(dev(src), dev(bad), n, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == oracle.EINVAL


def test_full_size_uniform_and_planted(pj):
    n, m = 1 << 22, 1 << 25
    for kind in ("uniform", "planted"):
        if kind == "uniform":
            src, dst = W.random_graph(n, m, W.SEED_BASE + 3)
        else:
            src, dst, _ = W.planted_graph(n, m, 1024, W.SEED_BASE + 3)
        got = run(pj, src, dst, n)
        assert np.array_equal(got, oracle.connected_components(src, dst, n)), kind


def test_batched_matches_oracle(pj):
    rng = np.random.default_rng(4)
    graphs = []
    for g in range(300):
        n = int(np.floor(2 ** rng.uniform(0, 14)))
        m = int(n * rng.uniform(0, 8))
        s, d = W.random_graph(n, m, 1000 + g)
        graphs.append((n, s, d))
    graphs.insert(3, (0, np.empty(0, np.int32), np.empty(0, np.int32)))
    voff = np.zeros(len(graphs) + 1, np.int64)
    eoff = np.zeros(len(graphs) + 1, np.int64)
    voff[1:] = np.cumsum([g[0] for g in graphs])
    eoff[1:] = np.cumsum([len(g[1]) for g in graphs])
    src = np.concatenate([g[1] for g in graphs]).astype(np.int32)
    dst = np.concatenate([g[2] for g in graphs]).astype(np.int32)
    want = oracle.connected_components_batched(src, dst, voff, eoff)
    got = pj.connected_components_batched(dev(src), dev(dst), dev(voff), dev(eoff),
                                          h_vtx_off=voff, h_edge_off=eoff)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    got2 = pj.connected_components_batched(dev(src), dev(dst), dev(voff), dev(eoff))
    torch.cuda.synchronize()
    assert np.array_equal(got2.cpu().numpy(), want)


def _mid_graph(i):
    """Graphs of the serving mix whose parent arrays fit in one XCD's L2;
    solves of these shapes once returned wrong labels with status OK."""
    rng = np.random.default_rng(W.SEED_BASE + 5)
    for _ in range(24):
        rng.uniform(10, 24)
    out = None
    for k in range(i + 1):
        n = int(np.floor(2 ** rng.uniform(10, 22)))
        m = int(round(n * rng.uniform(2, 16) / 2))
        if k == i:
            out = (*W.random_graph(n, m, W.SEED_BASE + 5 + 100 + k), n)
    return out


def test_repeated_solves_are_always_correct(pj):
    src, dst, n = _mid_graph(5)          # 838956 vertices, 5151345 pairs
    want = oracle.connected_components(src, dst, n)
    d_src, d_dst = dev(src), dev(dst)
    for rep in range(24):
        got = pj.connected_components(d_src, d_dst, n)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), rep
    s8, d8, n8 = _mid_graph(8)           # 149341 vertices, two copies in one batch
    w8 = oracle.connected_components(s8, d8, n8)
    voff = np.array([0, n8, 2 * n8], np.int64)
    eoff = np.array([0, len(s8), 2 * len(s8)], np.int64)
    bs, bd = dev(np.concatenate([s8, s8])), dev(np.concatenate([d8, d8]))
    dvo, deo = dev(voff), dev(eoff)
    for rep in range(24):
        got = pj.connected_components_batched(bs, bd, dvo, deo, h_vtx_off=voff, h_edge_off=eoff)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert np.array_equal(got[:n8], w8) and np.array_equal(got[n8:], w8), rep


def test_batched_out_of_range_pairs_are_charged_to_their_graph(pj):
    # empty graphs between the others exercise the boundary walk of the pair
    # rewrite; graphs 5 and 200 get one pair out of their own range
    rng = np.random.default_rng(9)
    graphs = []
    for g in range(260):
        n = 0 if g % 37 == 3 else int(np.floor(2 ** rng.uniform(0, 12)))
        m = int(n * rng.uniform(0, 6))
        s, d = W.random_graph(n, m, 5000 + g)
        graphs.append((n, s.copy(), d.copy()))
    bad = [g for g in (5, 200) if graphs[g][0] > 0 and len(graphs[g][1]) > 0]
    for g in bad:
        graphs[g][2][len(graphs[g][2]) // 2] = graphs[g][0] + 3
    voff = np.zeros(len(graphs) + 1, np.int64)
    eoff = np.zeros(len(graphs) + 1, np.int64)
    voff[1:] = np.cumsum([g[0] for g in graphs])
    eoff[1:] = np.cumsum([len(g[1]) for g in graphs])
    src = np.concatenate([g[1] for g in graphs]).astype(np.int32)
    dst = np.concatenate([g[2] for g in graphs]).astype(np.int32)
    st = torch.full((len(graphs),), -9, dtype=torch.int32, device="cuda")
    got = pj.connected_components_batched(dev(src), dev(dst), dev(voff), dev(eoff),
                                          h_vtx_off=voff, h_edge_off=eoff, status=st)
    torch.cuda.synchronize()
    status = st.cpu().numpy()
    got = got.cpu().numpy()
    for g, (n, s, d) in enumerate(graphs):
        if g in bad:
            assert status[g] == pj.PJ_EINVAL, g
        else:
            assert status[g] == pj.PJ_OK, g
            assert np.array_equal(got[voff[g]:voff[g + 1]], oracle.connected_components(s, d, n)), g


# ------------------------------------------------------------ graph replay
def _batch_of_graphs(count, seed, max_exp=14):
    rng = np.random.default_rng(seed)
    graphs = []
    for g in range(count):
        n = int(np.floor(2 ** rng.uniform(0, max_exp)))
        m = int(n * rng.uniform(0, 8))
        s, d = W.random_graph(n, m, seed * 10_000 + g)
        graphs.append((n, s, d))
    voff = np.zeros(count + 1, np.int64)
    eoff = np.zeros(count + 1, np.int64)
    voff[1:] = np.cumsum([g[0] for g in graphs])
    eoff[1:] = np.cumsum([len(g[1]) for g in graphs])
    src = np.concatenate([g[1] for g in graphs]).astype(np.int32)
    dst = np.concatenate([g[2] for g in graphs]).astype(np.int32)
    return src, dst, voff, eoff


def test_batched_graph_replay_matches_eager_and_oracle(pj):
    src, dst, voff, eoff = _batch_of_graphs(300, 21)
    want = oracle.connected_components_batched(src, dst, voff, eoff)
    ds, dd, dv, de = dev(src), dev(dst), dev(voff), dev(eoff)
    eager = pj.connected_components_batched(ds, dd, dv, de, h_vtx_off=voff, h_edge_off=eoff)
    torch.cuda.synchronize()
    assert np.array_equal(eager.cpu().numpy(), want)
    lab = torch.empty_like(eager)
    st = torch.full((300,), 9, dtype=torch.int32, device="cuda")
    pj.graph_cache_clear()
    for rep in range(4):
        lab.fill_(-1)
        st.fill_(9)
        pj.connected_components_batched(ds, dd, dv, de, lab, h_vtx_off=voff, h_edge_off=eoff,
                                        use_graph=True, status=st)
        torch.cuda.synchronize()
        assert torch.equal(lab, eager), rep
        assert int(st.abs().sum().item()) == 0, rep
        # unrelated eager work between replays
        pj.connected_components(ds[:1000], dd[:1000], int(max(src[:1000].max(),
                                                             dst[:1000].max())) + 1)
        torch.cuda.synchronize()
    # new pair contents in the same buffers: the replay reads them
    src2, dst2, _, _ = _batch_of_graphs(300, 21)
    rng = np.random.default_rng(5)
    for g in range(300):
        a, b = eoff[g], eoff[g + 1]
        nv = voff[g + 1] - voff[g]
        if b > a:
            src2[a:b] = rng.integers(0, nv, b - a)
    ds.copy_(dev(src2))
    pj.connected_components_batched(ds, dd, dv, de, lab, h_vtx_off=voff, h_edge_off=eoff,
                                    use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(),
                          oracle.connected_components_batched(src2, dst2, voff, eoff))
    pj.graph_cache_clear()


def test_graph_replay_beyond_captured_rounds(pj):
    """A collection of long paths needs more rounds than the graph holds: the
    call finishes them without the graph."""
    n = 1 << 21
    src, dst = W.list_graph(n, 8, 33)
    want = oracle.connected_components(src, dst, n)
    ds, dd = dev(src), dev(dst)
    eager, st = pj.connected_components(ds, dd, n, return_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(eager.cpu().numpy(), want)
    assert st["rounds"] > 8
    lab = torch.empty_like(eager)
    for rep in range(3):
        lab.fill_(-1)
        pj.connected_components(ds, dd, n, lab, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(lab, eager), rep
    # a graph of the same shape that converges within the captured rounds
    s2, d2 = W.random_graph(n, len(src), 34)
    ds.copy_(dev(s2))
    dd.copy_(dev(d2))
    pj.connected_components(ds, dd, n, lab, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(), oracle.connected_components(s2, d2, n))
    pj.graph_cache_clear()


def test_graph_replay_reports_bad_pairs(pj):
    src, dst, voff, eoff = _batch_of_graphs(40, 23, max_exp=10)
    g = int(np.nonzero(np.diff(eoff) > 0)[0][3])
    bad = dst.copy()
    bad[eoff[g]] = voff[g + 1] - voff[g] + 7
    st = torch.full((40,), 9, dtype=torch.int32, device="cuda")
    ds, dd, dv, de = dev(src), dev(bad), dev(voff), dev(eoff)
    for rep in range(2):
        st.fill_(9)
        pj.connected_components_batched(ds, dd, dv, de, h_vtx_off=voff, h_edge_off=eoff,
                                        use_graph=True, status=st)
        torch.cuda.synchronize()
        got = st.cpu().numpy()
        assert got[g] == pj.PJ_EINVAL and (np.delete(got, g) == 0).all(), rep
    pj.graph_cache_clear()
