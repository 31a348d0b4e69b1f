"""Seeded input generators (numpy PCG64).  No list-ranking or CC arithmetic here.

Recipes
-------
Lists (list-ranking problem, Section 3):
  * random   -- node order is a uniform random permutation pi (numpy's
                Fisher-Yates shuffle): succ[pi[k]] = pi[k+1], succ[pi[n-1]] = -1.
  * sequential -- succ[i] = i + 1, tail n-1.
  * blocked  -- the index range is cut into runs of `run` consecutive nodes;
                the runs are visited in a random order and each run is walked
                in ascending index order.
Graphs (connected components, Section 4):
  * random   -- m pairs with endpoints iid uniform over [0, n).
  * planted  -- `groups` components of log-uniform size: raw sizes 2**(16u),
                u ~ U[0,1), normalised to sum n (each >= 1, the rounding
                remainder goes to the largest); vertex ids are dealt to groups
                by a random permutation; each group is first connected by a
                random recursive tree (member k attaches to a uniform earlier
                member), then the remaining pairs are spread over the groups by
                a multinomial draw proportional to group size, with uniform
                endpoints inside the group; finally the pair order is shuffled.
The paper's graph families (Section 4: collections of random lists, random
trees of degree k, random graphs made of connected components with edge
density d) are `list_graph`, `random_tree_graph` and
`component_density_graph`; `density_graph` is one G(n, m) graph of density d.
  * list_graph -- a random permutation of the vertices cut at `lists` - 1
                random places; consecutive vertices of a piece are joined.
  * random_tree_graph -- `trees` trees of near-equal size, each a complete
                k-ary tree (position p > 0 attaches to (p - 1) // k) whose
                positions carry random vertex ids.
  * component_density_graph -- `comps` components of c vertices, c chosen so
                that comps * d * c^2 / 2 is about m; each is a random recursive
                tree plus uniform pairs inside it, up to d * c * (c - 1) / 2
                pairs; vertex ids dealt by a random permutation, pair order
                shuffled.
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 10024482

__all__ = [
    "SEED_BASE",
    "random_list",
    "random_list_with_order",
    "sequential_list",
    "blocked_list",
    "blocked_list_with_order",
    "to_self_loop_tails",
    "batched_lists",
    "concat_lists",
    "random_graph",
    "planted_graph",
    "list_graph",
    "random_tree_graph",
    "density_graph",
    "component_density_graph",
    "serving_mix",
]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _succ_from_order(order: np.ndarray) -> np.ndarray:
    """Successor array of the list that visits `order[0], order[1], ...`."""
    n = order.shape[0]
    succ = np.empty(n, dtype=np.int32)
    if n == 0:
        return succ
    succ[order[:-1]] = order[1:]
    succ[order[-1]] = -1
    return succ


def random_list_with_order(n: int, seed: int):
    """Random list of n nodes; returns (succ, order) with order[k] = k-th node."""
    order = _rng(seed).permutation(n).astype(np.int32)
    return _succ_from_order(order), order


def random_list(n: int, seed: int) -> np.ndarray:
    return random_list_with_order(n, seed)[0]


def sequential_list(n: int) -> np.ndarray:
    succ = np.arange(1, n + 1, dtype=np.int64)
    if n:
        succ[-1] = -1
    return succ.astype(np.int32)


def blocked_list_with_order(n: int, run: int, seed: int):
    """Runs of `run` consecutive ids visited in random run order; (succ, order)."""
    if n == 0:
        return np.empty(0, np.int32), np.empty(0, np.int32)
    nruns = (n + run - 1) // run
    perm = _rng(seed).permutation(nruns).astype(np.int64)
    full = n // run
    if full == nruns:
        order = (perm[:, None] * run + np.arange(run, dtype=np.int64)[None, :]).ravel()
    else:
        parts = []
        last = nruns - 1
        for b in perm:
            lo = b * run
            hi = n if b == last else lo + run
            parts.append(np.arange(lo, hi, dtype=np.int64))
        order = np.concatenate(parts)
    order = order.astype(np.int32)
    return _succ_from_order(order), order


def blocked_list(n: int, run: int, seed: int) -> np.ndarray:
    return blocked_list_with_order(n, run, seed)[0]


def to_self_loop_tails(succ: np.ndarray) -> np.ndarray:
    """Rewrite tails from -1 to the paper's self-loop marker succ[j] == j."""
    out = succ.copy()
    tails = np.nonzero(out < 0)[0]
    out[tails] = tails.astype(np.int32)
    return out


def concat_lists(lists):
    """Concatenate per-list local successor arrays; returns (succ, offsets int64[L+1])."""
    sizes = np.array([len(s) for s in lists], dtype=np.int64)
    offsets = np.zeros(len(lists) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    succ = np.concatenate(lists).astype(np.int32) if lists else np.empty(0, np.int32)
    return succ, offsets


def batched_lists(L: int, lo_exp: float, hi_exp: float, seed: int, layout: str = "random",
                  return_orders: bool = False):
    """L independent lists with sizes floor(2**U), U ~ U[lo_exp, hi_exp].

    Successors are local to each list (ids 0..size-1).  Returns
    (succ int32[total], offsets int64[L+1]) and, if asked, the per-list node
    orders (order[k] = k-th node of the list, local id).
    """
    rng = _rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=L)).astype(np.int64)
    offsets = np.zeros(L + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    succ = np.empty(total, dtype=np.int32)
    orders = [] if return_orders else None
    for i in range(L):
        sz = int(sizes[i])
        if layout == "random":
            order = rng.permutation(sz).astype(np.int32)
        elif layout == "sequential":
            order = np.arange(sz, dtype=np.int32)
        else:
            raise ValueError(layout)
        seg = succ[offsets[i]:offsets[i + 1]]
        if sz:
            seg[order[:-1]] = order[1:]
            seg[order[-1]] = -1
        if return_orders:
            orders.append(order)
    if return_orders:
        return succ, offsets, orders
    return succ, offsets


def random_graph(n: int, m: int, seed: int):
    """m pairs with iid uniform endpoints over [0, n)."""
    rng = _rng(seed)
    src = rng.integers(0, n, size=m, dtype=np.int32) if n else np.empty(m, np.int32)
    dst = rng.integers(0, n, size=m, dtype=np.int32) if n else np.empty(m, np.int32)
    return src, dst


def planted_graph(n: int, m: int, groups: int, seed: int):
    """Graph with exactly `groups` components of log-uniform size.

    Returns (src, dst, group_of_vertex int32[n]).  Requires
    groups <= n and m >= n - groups.
    """
    if not (1 <= groups <= n) or m < n - groups:
        raise ValueError("need 1 <= groups <= n and m >= n - groups")
    rng = _rng(seed)
    raw = 2.0 ** (16.0 * rng.random(groups))
    sizes = np.maximum(1, np.floor(raw / raw.sum() * n)).astype(np.int64)
    diff = n - int(sizes.sum())
    big = int(np.argmax(sizes))
    sizes[big] += diff
    if sizes[big] < 1:  # pathological rounding when groups ~ n
        sizes = np.ones(groups, np.int64)
        sizes[0] += n - groups
    starts = np.zeros(groups, dtype=np.int64)
    np.cumsum(sizes[:-1], out=starts[1:])
    members = rng.permutation(n).astype(np.int32)  # group g owns members[starts[g]:starts[g]+sizes[g]]
    gid_by_pos = np.repeat(np.arange(groups, dtype=np.int64), sizes)
    group_of = np.empty(n, dtype=np.int32)
    group_of[members] = gid_by_pos.astype(np.int32)
    # random recursive tree inside each group
    pos = np.arange(n, dtype=np.int64)
    within = pos - starts[gid_by_pos]
    child = within > 0
    cpos = pos[child]
    cwithin = within[child]
    ppos = starts[gid_by_pos[child]] + np.floor(rng.random(cpos.shape[0]) * cwithin).astype(np.int64)
    tree_src = members[cpos]
    tree_dst = members[ppos]
    # remaining pairs, proportional to group size
    extra = m - (n - groups)
    counts = rng.multinomial(extra, sizes / n) if extra > 0 else np.zeros(groups, np.int64)
    eg = np.repeat(np.arange(groups, dtype=np.int64), counts)
    u = starts[eg] + np.floor(rng.random(extra) * sizes[eg]).astype(np.int64)
    v = starts[eg] + np.floor(rng.random(extra) * sizes[eg]).astype(np.int64)
    src = np.concatenate([tree_src, members[u]]).astype(np.int32)
    dst = np.concatenate([tree_dst, members[v]]).astype(np.int32)
    perm = rng.permutation(m)
    return src[perm], dst[perm], group_of


def list_graph(n: int, lists: int, seed: int, with_groups: bool = False):
    """Collection of `lists` random paths over a random split of n vertices.
    With `with_groups`, also returns the path index of every vertex."""
    rng = _rng(seed)
    order = rng.permutation(n).astype(np.int32)
    cuts = np.sort(rng.choice(np.arange(1, n), size=max(0, lists - 1), replace=False)) if n > 1 else []
    brk = np.zeros(n, dtype=bool)
    brk[np.asarray(cuts, dtype=np.int64)] = True
    keep = ~brk[1:]
    src, dst = order[:-1][keep].copy(), order[1:][keep].copy()
    if not with_groups:
        return src, dst
    group_of = np.empty(n, dtype=np.int32)
    group_of[order] = np.cumsum(brk).astype(np.int32)
    return src, dst, group_of


def random_tree_graph(n: int, k: int, trees: int, seed: int, with_groups: bool = False):
    """Collection of `trees` random k-ary trees (complete k-ary shape, random
    labels).  With `with_groups`, also returns the tree index of every vertex."""
    rng = _rng(seed)
    labels = rng.permutation(n).astype(np.int64)
    sizes = np.full(trees, n // trees, dtype=np.int64)
    sizes[: n % trees] += 1
    starts = np.zeros(trees, dtype=np.int64)
    np.cumsum(sizes[:-1], out=starts[1:])
    tid = np.repeat(np.arange(trees), sizes)
    pos = np.arange(n, dtype=np.int64) - starts[tid]
    child = pos > 0
    parent_pos = starts[tid[child]] + (pos[child] - 1) // k
    src, dst = labels[child].astype(np.int32), labels[parent_pos].astype(np.int32)
    if not with_groups:
        return src, dst
    group_of = np.empty(n, dtype=np.int32)
    group_of[labels] = tid.astype(np.int32)
    return src, dst, group_of


def component_density_graph(m: int, d: float, comps: int, seed: int):
    """`comps` connected components of equal size and edge density about d,
    about m pairs in all.  Returns (src, dst, group_of_vertex int32[n])."""
    if comps < 1 or not (0.0 < d <= 1.0) or m < 1:
        raise ValueError("need comps >= 1, 0 < d <= 1 and m >= 1")
    rng = _rng(seed)
    c = max(2, int(round(np.sqrt(2.0 * m / (comps * d)))))
    per = max(c - 1, int(round(d * c * (c - 1) / 2)))
    n = comps * c
    members = rng.permutation(n).astype(np.int32)  # component g owns members[g*c:(g+1)*c]
    group_of = np.empty(n, dtype=np.int32)
    group_of[members] = np.repeat(np.arange(comps, dtype=np.int32), c)
    base = np.repeat(np.arange(comps, dtype=np.int64) * c, c - 1)
    w = np.tile(np.arange(1, c, dtype=np.int64), comps)  # position inside the component
    parent = base + np.floor(rng.random(w.shape[0]) * w).astype(np.int64)
    tree_src, tree_dst = members[base + w], members[parent]
    extra = per - (c - 1)
    eb = np.repeat(np.arange(comps, dtype=np.int64) * c, extra)
    u = eb + rng.integers(0, c, size=eb.shape[0])
    v = eb + rng.integers(0, c, size=eb.shape[0])
    src = np.concatenate([tree_src, members[u]]).astype(np.int32)
    dst = np.concatenate([tree_dst, members[v]]).astype(np.int32)
    perm = rng.permutation(src.shape[0])
    return src[perm], dst[perm], group_of


def density_graph(n: int, d: float, seed: int):
    """G(n, m) with m = round(d * n * (n - 1) / 2) uniform pairs."""
    m = int(round(d * n * (n - 1) / 2))
    return random_graph(n, m, seed)


def serving_mix(num: int, seed: int, rate: float, lr_frac: float = 0.7,
                lr_exp=(10.0, 24.0), cc_exp=(10.0, 22.0), deg=(2.0, 16.0)):
    """Request specs for the serving loop: Poisson arrivals at `rate` per second.

    Each spec is a dict with kind ('lr' or 'cc'), n, m (0 for lists), a per-
    request input seed and the arrival time in seconds from the start.
    """
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=num) if rate > 0 else np.zeros(num)
    t = np.cumsum(gaps) - gaps[0] if num else gaps
    reqs = []
    for i in range(num):
        if rng.random() < lr_frac:
            n = int(np.floor(2.0 ** rng.uniform(*lr_exp)))
            reqs.append(dict(kind="lr", n=n, m=0, seed=int(seed * 7919 + i), t=float(t[i])))
        else:
            n = int(np.floor(2.0 ** rng.uniform(*cc_exp)))
            delta = rng.uniform(*deg)
            m = int(round(n * delta / 2))
            reqs.append(dict(kind="cc", n=n, m=m, seed=int(seed * 7919 + i), t=float(t[i])))
    return reqs
