/*
 * ptrjump -- pointer jumping over int32 successor and parent arrays on one
 * AMD Instinct MI355X (gfx950): list ranking and connected components.
 *
 * Method: Dehne & Yogaratnam, "Exploring the Limits of GPUs With Parallel
 * Graph Algorithms".  List ranking follows the problem statement of Section 3,
 * solved either by Wyllie's pointer jumping (Section 3.1) or by the parallel
 * random-splitter (sparse ruling set) method of Reid-Miller (Section 3.2,
 * Algorithm "Parallel Random Splitter"), whose splitter list is itself ranked
 * recursively.  Connected components follow Section 4: a hook-and-shortcut
 * algorithm of the Shiloach-Vishkin family with the step split of the
 * paper's SV-GPU (shortcut and mark separated by a barrier, conditional and
 * stagnant-star hooking, shortcut, change flag), with labels canonicalised to
 * the smallest vertex id of each component.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller, unless the name
 *    starts with h_ (host pointer).  The library never frees them.
 *  - Calls are asynchronous on `stream` (NULL = the default stream); outputs
 *    are valid once the stream reaches the call.  The return value reports
 *    argument errors detected on the host before anything is enqueued, and HIP
 *    errors; 0 means enqueued.
 *  - Errors in the DATA (a successor array that is not one list per instance,
 *    a solve that does not converge) are found on the device.  They are
 *    written to opts->d_status when given (one int32 per instance); with
 *    opts->validate != 0 and no d_status, the call waits for the stream and
 *    returns the status itself.  Whatever the input, every kernel stays in
 *    bounds and terminates.
 *  - Ids are int32; counts are int64 but an instance (and a whole batch) must
 *    hold fewer than 2^31 nodes or vertices.
 *  - Temporary device memory is taken stream-ordered from the device's memory
 *    pool (hipMallocAsync / hipFreeAsync) unless the caller passes a workspace
 *    of at least *_workspace_bytes() bytes in opts->workspace.
 */
#ifndef PTRJUMP_H
#define PTRJUMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same type as HIP's hipStream_t. */
typedef struct ihipStream_t *pj_stream_t;

/* ----------------------------------------------------------- status codes */
#define PJ_OK 0
#define PJ_EINVAL (-1)    /* bad argument (null pointer, negative or too large size, aliasing) */
#define PJ_ENOMEM (-2)    /* device memory could not be obtained */
#define PJ_EHIP (-3)      /* a HIP runtime call failed (see pj_last_hip_error) */
#define PJ_EBADLIST (-4)  /* the successor array is not exactly one list over the instance */
#define PJ_ENOCONV (-5)   /* components did not converge within the round guard */
#define PJ_EBUDGET (-6)   /* serving: request larger than the whole HBM budget */
#define PJ_ENOTFOUND (-7) /* serving: unknown request id */
#define PJ_EBUSY (-8)     /* serving: request not finished yet (poll again) */
#define PJ_ESHUTDOWN (-9) /* serving: server is shutting down */
#define PJ_ESCRATCH (-10) /* pj_list_rank_noalloc: the input needs more than its fixed scratch */

/* ------------------------------------------------------------- algorithms */
#define PJ_ALGO_AUTO 0        /* tuned choice (ruling set for lists, SV for components) */
#define PJ_ALGO_WYLLIE 1      /* list ranking by pointer jumping, ceil(log2 n) device-wide rounds */
#define PJ_ALGO_RULING_SET 2  /* list ranking by random splitters with recursive splitter ranking */
#define PJ_ALGO_SV 3          /* components: Shiloach-Vishkin hook and shortcut */

/* Level-0 state layout of the ruling set (pj_opts.level0_state). */
#define PJ_STATE_AUTO 0      /* packed into the output array when the id space allows */
#define PJ_STATE_SEPARATE 1  /* a separate 8-byte (sublist, offset) array beside the output */

#define PJ_MAX_PHASES 16
#define PJ_MAX_LEVELS 8

/* Per-call options.  Zero-initialise (or call pj_opts_init) and set what you
 * need; every zero field means "library default / tuned value". */
typedef struct pj_opts {
    int32_t algo;             /* PJ_ALGO_* */
    int32_t block;            /* threads per workgroup of the sublist walks and of Wyllie's
                                 kernels, multiple of 64 in [64, 1024] (zero: 256) */
    int32_t spacing;          /* ruling set, first level: one splitter per `spacing`
                                 consecutive node ids (power of two, 2..65536);
                                 zero: n / 2^20 rounded down to a power of
                                 two, within 8..256 for one list and 8..64
                                 for a batch (a single list of >= 2^24 nodes
                                 keeps 8 when most successors are local) */
    int32_t spacing_up;       /* ruling set, recursion levels: same meaning
                                 (zero: 4) */
    int32_t cutoff;           /* ruling set: a level with at most this many nodes is ranked
                                 by one workgroup in LDS (64..16384) */
    int32_t max_walk;         /* ruling set: a sublist walk is cut after this many nodes,
                                 the cut node becoming a new splitter (>= 16) */
    uint64_t seed;            /* splitter hash seed (results do not depend on it) */
    int32_t validate;         /* 1: run the complete check of the output on the device */
    int32_t to_tail;          /* 1: list ranks count the distance to the tail (the paper's
                                 convention) instead of the distance from the head */
    int32_t rounds_per_check; /* components: rounds enqueued between host convergence checks */
    int32_t use_graph;        /* batched list ranking and components: replay a captured
                                 hipGraph (see pj_graph_cache_clear) */
    int32_t *d_status;        /* optional device int32[instances]: PJ_OK / PJ_EBADLIST / PJ_ENOCONV */
    void *workspace;          /* optional caller-owned device workspace */
    size_t workspace_bytes;
    const int64_t *h_offsets;      /* batched: host copy of the (vertex) offset table */
    const int64_t *h_edge_offsets; /* batched components: host copy of the edge offsets */
    struct pj_stats *stats;   /* optional: filled after the call (forces a stream sync) */
    int32_t level0_state;     /* ruling set: PJ_STATE_AUTO or PJ_STATE_SEPARATE.  Section 3.2
                                 weighs one packed word per node (one random line read and
                                 written per step) against narrower fields in separate
                                 arrays (a second random line per step); the separate form
                                 asks that question of this chip.  Results do not change. */
    int32_t reserved0;
    const int32_t *d_splitters; /* ruling set, one unweighted list: the level-0 splitters
                                   chosen by the caller (DEVICE int32[n_splitters], distinct
                                   node ids in [0, n)) instead of the hashed random ones, as in
                                   Section 3.2's comparison of random against evenly spaced
                                   splitters.  Needs the packed level-0 state, in place or
                                   not; the head is added as a splitter by the library.  Ids
                                   out of range or repeated are reported as PJ_EINVAL through
                                   d_status (the ranks are then unspecified).  Results do not
                                   change. */
    int64_t n_splitters;      /* entries of d_splitters, 1..n */
} pj_opts;

/* Diagnostics of one call, filled when opts->stats is set. */
typedef struct pj_stats {
    int32_t algo;                 /* algorithm actually run */
    int32_t levels;               /* ruling set: walk levels (recursion depth) */
    int32_t base_kind;            /* ruling set: 1 LDS workgroup, 2 device-wide pointer jumping */
    int32_t rounds;               /* components: Shiloach-Vishkin rounds run;
                                     Wyllie: pointer-jumping rounds, ceil(log2) of the
                                     longest list */
    int64_t level_nodes[PJ_MAX_LEVELS + 1]; /* nodes at each level (level 0 = input) */
    int32_t nphases;
    char phase_name[PJ_MAX_PHASES][24];
    float phase_ms[PJ_MAX_PHASES];  /* device time of each phase (HIP events) */
    int32_t status;               /* first data error found, or PJ_OK */
    int32_t max_sublist0;         /* ruling set: nodes of the longest level-0 sublist (a
                                     walk cut at max_walk nodes counts as separate pieces) */
    int64_t sublists0;            /* ruling set: level-0 sublists (splitters, list heads
                                     and cut points), i.e. the nodes of level 1 */
    int64_t cuts0;                /* ruling set: level-0 walks cut at max_walk nodes */
} pj_stats;

void pj_opts_init(pj_opts *opts);
const char *pj_strerror(int code);
/* Text of the last HIP error seen by the library on this thread. */
const char *pj_last_hip_error(void);
int pj_version(void);

/* ---------------------------------------------------------- list ranking */
/*
 * List ranking (Section 3 problem statement).  succ[i] is the successor of
 * node i in [0, n); the tail is marked by succ[i] == -1 or succ[i] == i.
 * Writes rank[i] = distance of node i from the head (rank[head] = 0), or with
 * opts->to_tail the distance to the tail, which is the paper's definition.
 * rank may be succ itself: the ranks then overwrite the successors in place
 * (Section 3.2 returns the ranks in the device successor array), and on an
 * error return the array's contents are unspecified; opts->validate needs
 * separate arrays (PJ_EINVAL in place).  Any other overlap of rank and succ
 * is PJ_EINVAL.  n == 0 is a no-op.
 */
int pj_list_rank(const int32_t *succ, int64_t n, int32_t *rank, pj_stream_t stream);
int pj_list_rank_ex(const int32_t *succ, int64_t n, int32_t *rank, const pj_opts *opts,
                    pj_stream_t stream);

/*
 * Batched list ranking: L independent lists concatenated, each ranked as in
 * the problem statement of Section 3 (the ruling set of Section 3.2 ranks
 * the whole batch as one forest, with a splitter at every list head, as its
 * recursion already does for the splitter list).  offsets is a
 * DEVICE int64[L+1] table (offsets[0] == 0, non-decreasing); list l occupies
 * [offsets[l], offsets[l+1]) and its successors are LOCAL ids in
 * [0, size_l) (tail -1 or self).  rank receives local ranks per list.  With
 * opts->h_offsets the host copy is used for planning and no device->host read
 * happens; otherwise offsets[L] is read back (the call then synchronises the
 * stream once).  d_status, when given, holds L entries.  In place (rank ==
 * succ) as for pj_list_rank_ex.
 */
int pj_list_rank_batched(const int32_t *succ, const int64_t *offsets, int64_t L, int32_t *rank,
                         pj_stream_t stream);
int pj_list_rank_batched_ex(const int32_t *succ, const int64_t *offsets, int64_t L,
                            int32_t *rank, const pj_opts *opts, pj_stream_t stream);

/* Bytes of workspace a call with these sizes needs (L = 1: enough for both the
 * plain call and a batched call holding one list). */
size_t pj_list_rank_workspace_bytes(int64_t total_nodes, int64_t L, const pj_opts *opts);

/*
 * List ranking that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and in-place
 * rule as pj_list_rank_ex; the workspace comes from one fixed device array
 * of pj_list_rank_noalloc_max_bytes() bytes (64 MiB) that the library holds
 * on every device it runs on until the process ends.  An input whose
 * workspace (pj_list_rank_workspace_bytes with the same options) exceeds
 * that size is refused with PJ_ESCRATCH before anything is enqueued: with
 * the default options that admits lists of up to about 2^24 nodes.
 * opts->workspace, opts->use_graph, opts->stats and validate without
 * d_status are PJ_EINVAL (they allocate or read back through host memory).
 * The call makes no hipMalloc, hipMallocAsync, hipFree or hipHostMalloc.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (on different streams, or from different threads without
 * ordering) race and give unspecified ranks; calls ordered on one stream are
 * safe.
 */
int pj_list_rank_noalloc(const int32_t *succ, int64_t n, int32_t *rank, const pj_opts *opts,
                         pj_stream_t stream);
size_t pj_list_rank_noalloc_max_bytes(void);

/*
 * Weighted list ranking: the problem the ruling set solves on its splitter
 * list (Section 3.2, where each splitter carries the length of its sublist).
 * weight is a DEVICE int32[n] array beside succ; rank[i] receives the sum of
 * the weights of the nodes before i in its list (exclusive prefix from the
 * head: rank[head] = 0, rank[succ[i]] = rank[i] + weight[i]).  Unit weights
 * give pj_list_rank's result.  Sums are int32: the total weight of a list
 * must fit, or the ranks are unspecified.  Always the ruling-set method;
 * opts->algo == PJ_ALGO_WYLLIE, opts->to_tail and opts->validate are
 * PJ_EINVAL (d_status still reports malformed lists), opts->use_graph is
 * ignored.  rank may be succ itself (in place); rank must not overlap
 * weight.  weight may be null only when there is nothing to rank.
 */
int pj_list_rank_weighted(const int32_t *succ, const int32_t *weight, int64_t n, int32_t *rank,
                          const pj_opts *opts, pj_stream_t stream);
/* The batched form (offsets and local ids as for pj_list_rank_batched_ex;
 * weight is laid out like succ). */
int pj_list_rank_weighted_batched(const int32_t *succ, const int32_t *weight,
                                  const int64_t *offsets, int64_t L, int32_t *rank,
                                  const pj_opts *opts, pj_stream_t stream);
/* Workspace bytes of the weighted calls (their level-0 state is not packed
 * into the output, so they need 8 more bytes per node). */
size_t pj_list_rank_weighted_workspace_bytes(int64_t total_nodes, int64_t L,
                                             const pj_opts *opts);

/*
 * Batched list ranking with opts->use_graph = 1 captures the call's whole
 * launch sequence once into a hipGraph (the cache owns the workspace) and
 * replays it with one hipGraphLaunch on later calls.  The cache key holds
 * the device, the succ / offsets / rank / d_status addresses, L, the node
 * total offsets[L], ceil(log2) of the largest list (Wyllie's round count),
 * every option field that selects a plan (algo, block, spacing, spacing_up,
 * cutoff, max_walk, seed, to_tail, validate, level0_state) and the
 * tune-cache generation.
 * A replay reads the current contents of succ and of the device offsets, so
 * the caller may change both between calls: any change the key does not
 * cover (list sizes with the same total and the same ceil(log2) of the
 * largest) leaves the captured plan valid.  Not used together with
 * opts->stats or with validate and no d_status.  The cache holds up to 8
 * graphs; pj_graph_cache_clear() frees them all (it synchronises the
 * device).
 */
void pj_graph_cache_clear(void);

/* ------------------------------------------------------------- autotuner */
/*
 * Times ruling-set parameters on this input by coordinate descent from the
 * defaults (first-level spacing 8..256, recursion spacing 4..16, LDS cutoff
 * 2048..16384, workgroup size of the sublist walks 128..1024, each swept with
 * the others at their best so far) and records the fastest in the tune
 * cache, keyed by (gfx arch, ceil(log2 nodes), ceil(log2 lists)).  Later
 * list-ranking calls whose spacing / spacing_up / cutoff / max_walk / block
 * are zero use the cached values for their size class; results never depend
 * on them.  offsets == NULL tunes the single-list call on n nodes; otherwise
 * offsets is the device table and h_offsets its host copy (required).  Writes
 * the chosen options to *best and their mean time to *best_ms (either may be
 * NULL).  Allocates a scratch output, runs ~60 solves and synchronises the
 * stream.
 */
int pj_tune_list_rank(const int32_t *succ, const int64_t *offsets, int64_t L,
                      const int64_t *h_offsets, int64_t n, pj_opts *best, float *best_ms,
                      pj_stream_t stream);
/* The tuned parameters for a size class, PJ_ENOTFOUND if none. */
int pj_tune_lookup(int64_t n, int64_t L, pj_opts *out);
/* Save / load the tune cache as text (one size class per line); the cache is
 * also loaded from the file named by $PJ_TUNE_CACHE on first use. */
int pj_tune_save(const char *path);
int pj_tune_load(const char *path);
void pj_tune_clear(void);

/* ---------------------------------------------------- connected components */
/*
 * Connected components (Section 4 problem statement).  src[e], dst[e] for
 * e in [0, m) are undirected vertex pairs in [0, n); self-loops and
 * duplicates are allowed.  Writes label[v] = smallest vertex id of v's
 * component.  label must not alias src or dst.
 */
int pj_connected_components(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                            int32_t *label, pj_stream_t stream);
int pj_connected_components_ex(const int32_t *src, const int32_t *dst, int64_t n, int64_t m,
                               int32_t *label, const pj_opts *opts, pj_stream_t stream);

/*
 * Batched components: G independent graphs, each solved as in the problem
 * statement of Section 4 (the batch is one disjoint union of the graphs,
 * solved by one Shiloach-Vishkin run).  vtx_off and edge_off are DEVICE
 * int64[G+1] tables; graph g owns vertices [vtx_off[g], vtx_off[g+1]) and
 * pairs [edge_off[g], edge_off[g+1]), with LOCAL vertex ids.  label receives
 * local labels (smallest local id of each component).
 */
int pj_connected_components_batched(const int32_t *src, const int32_t *dst,
                                    const int64_t *vtx_off, const int64_t *edge_off, int64_t G,
                                    int32_t *label, pj_stream_t stream);
int pj_connected_components_batched_ex(const int32_t *src, const int32_t *dst,
                                       const int64_t *vtx_off, const int64_t *edge_off,
                                       int64_t G, int32_t *label, const pj_opts *opts,
                                       pj_stream_t stream);

/*
 * Components with opts->use_graph = 1 (plain or batched, not with
 * opts->stats) capture the solve once into a hipGraph: the batched pair
 * rewrite and initialisation, the first 8 rounds (a round that follows one
 * without change returns at once on the device) and the canonicalisation,
 * which runs only if the solve converged within those rounds.  A call
 * launches the graph, reads the 8th round's change flag (one stream
 * synchronisation) and, only if it is raised, finishes the remaining rounds
 * and the canonicalisation without the graph, on the same state.  The cache
 * key holds the device, every array address, n, m and G (and whether the
 * status is read back); the arrays' contents may change between calls.  The
 * cache owns the workspace and holds up to 8 graphs; pj_graph_cache_clear()
 * frees them with the list-ranking graphs.
 */

/* Bytes of workspace a components call needs (G = 1: enough for both the plain
 * call and a batched call holding one graph). */
size_t pj_cc_workspace_bytes(int64_t n, int64_t m, int64_t G, const pj_opts *opts);

/* ----------------------------------------------------------------- serving */
/*
 * A request loop with continuous batching under an HBM budget.  Requests hold
 * HOST arrays (pinned memory keeps the copies asynchronous) that must stay
 * valid until the request is collected.  A scheduler thread admits waiting
 * requests in arrival order into a tick while the tick's exact device
 * footprint fits in the unused budget; each tick is one batched list ranking
 * plus one batched components solve, run by one of max_inflight worker
 * threads on its own stream, so ticks overlap on the device and requests that
 * arrive meanwhile join the next tick as memory and a worker free up.  A
 * large request (at least large_items list nodes, or graph vertices plus
 * pairs) is a tick of its own, and at most max_inflight - 1 such ticks run at
 * once, so small requests never queue behind a large solve.  Results are
 * identical to a solve of the request alone.
 */
typedef struct pj_server pj_server;

typedef struct pj_server_config {
    size_t hbm_budget;      /* device bytes all in-flight ticks may hold (0 = 16 GiB) */
    int32_t max_inflight;   /* ticks on the device at once, one worker and stream each (0 = 3);
                               more workers than the device's hardware queues (4 by
                               default) share queues and lose throughput */
    int32_t max_batch;      /* requests per tick (0 = 256) */
    int32_t device;         /* HIP device (-1 = the calling thread's current device) */
    int32_t reserved;
    pj_opts opts;           /* solve options; workspace, d_status, stats and d_splitters
                               are ignored */
    int64_t large_items;    /* size class boundary (0 = 2^22) */
} pj_server_config;

typedef struct pj_server_stats {
    int64_t submitted, completed, failed;
    int64_t ticks;           /* batched launches formed */
    int64_t inflight_peak;   /* most ticks running at once */
    int64_t budget_waits;    /* times the oldest request waited for memory */
    size_t bytes_peak;       /* most device bytes held by ticks at once */
    size_t bytes_in_use;
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency: submit to completion, completed requests */
    double wall_s;           /* first submit to last completion */
    double req_per_s;        /* completed requests per second of wall_s */
    double items_per_s;      /* list nodes + graph pairs per second of wall_s */
    int64_t large_ticks;     /* ticks formed for one large request */
} pj_server_stats;

int pj_server_create(const pj_server_config *cfg, pj_server **out);
/* Submit a request; PJ_EBUDGET if it alone exceeds the whole budget,
 * PJ_ESHUTDOWN after destroy began.  *id identifies it. */
int pj_server_submit_list_rank(pj_server *srv, const int32_t *h_succ, int64_t n, int32_t *h_rank,
                               uint64_t *id);
int pj_server_submit_cc(pj_server *srv, const int32_t *h_src, const int32_t *h_dst, int64_t n,
                        int64_t m, int32_t *h_label, uint64_t *id);
/* PJ_OK once finished (the request's result code goes to *status and its
 * latency to *latency_ms; the id is then forgotten), PJ_EBUSY while pending,
 * PJ_ENOTFOUND for an unknown id.  wait blocks up to timeout_us (< 0: forever). */
int pj_server_poll(pj_server *srv, uint64_t id, int32_t *status, double *latency_ms);
int pj_server_wait(pj_server *srv, uint64_t id, int32_t *status, double *latency_ms,
                   int64_t timeout_us);
/* Block until every submitted request has finished. */
int pj_server_drain(pj_server *srv);
int pj_server_get_stats(pj_server *srv, pj_server_stats *out);
/* Finish all submitted requests, stop the threads and free the server. */
int pj_server_destroy(pj_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* PTRJUMP_H */
