"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only builds inputs: linked lists given as int32 successor arrays,
undirected graphs given as int32 edge-pair arrays, batches with int64 offset
tables, and request mixes for the serving loop.  It holds none of the
arithmetic of list ranking or connected components.  Everything is drawn from
numpy's PCG64 generator, seeded explicitly, so every input is reproducible on
any machine.

List inputs follow the list-ranking problem statement (Section 3): node i's
successor is succ[i]; the tail is marked with -1 (the paper's own marker,
succ[j] == j, is produced by `to_self_loop_tails`).  Graph inputs follow the
connected-components problem statement (Section 4): m unordered vertex pairs
over n vertices, self-loops and duplicates allowed.
"""

from .gen import (  # noqa: F401
    SEED_BASE,
    random_list,
    random_list_with_order,
    sequential_list,
    blocked_list,
    blocked_list_with_order,
    to_self_loop_tails,
    batched_lists,
    concat_lists,
    random_graph,
    planted_graph,
    list_graph,
    random_tree_graph,
    component_density_graph,
    density_graph,
    serving_mix,
)
