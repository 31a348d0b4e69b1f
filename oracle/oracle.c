/*
 * CPU oracle for list ranking and connected components.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or table with the GPU library.
 *
 * Each function is the plain definition of the result, written out
 * sequentially, not a fast method:
 *
 *   list ranking (Section 3, problem statement): the list is succ[0..n-1];
 *     the tail is the node whose successor is -1 or itself (the paper marks it
 *     with succ[j] == j).  The rank reported here is the distance from the head
 *     (rank[head] = 0, rank[succ[i]] = rank[i] + 1); the paper's "distance to
 *     the last element" is n - 1 minus this value.
 *
 *   weighted list ranking (the splitter list of Section 3.2, whose nodes
 *     carry their sublist lengths as weights): rank[x] = the sum of the weights
 *     of the nodes before x in list order (exclusive prefix from the head),
 *     in 32-bit two's complement (sums wrap modulo 2^32).  Unit weights give
 *     the unweighted rank.
 *
 *   connected components (Section 4, problem statement): an undirected graph
 *     given by m vertex pairs; label[v] is the smallest vertex id in v's
 *     component.  Computed with a sequential union-find (union by size, path
 *     halving), then a scan in ascending vertex order that records, for each
 *     root, the first (hence smallest) vertex that reaches it.
 *
 * Batched forms apply the single-instance definition to every instance of a
 * concatenation described by an int64 offset table; ids are local to each
 * instance.  Instances are spread over `nthreads` POSIX threads.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 out of memory, -4 the input is
 * not a single linked list over all n nodes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EBADLIST (-4)

/* ---------------------------------------------------------------- lists -- */

/* Rank from the head for one list of n nodes (local ids 0..n-1): the number
 * of nodes before each node, or with weights the sum of their weights. */
static int rank_one(const int32_t *succ, const int32_t *weight, int64_t n, int32_t *rank)
{
    if (n < 0 || n > INT32_MAX) return OR_EINVAL;
    if (n == 0) return OR_OK;
    if (!succ || !rank) return OR_EINVAL;

    /* 1. every successor is a node id or the tail marker; exactly one tail */
    int64_t tails = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = succ[i];
        if (s == -1 || s == (int32_t)i) { ++tails; continue; }
        if (s < 0 || s >= n) return OR_EBADLIST;
    }
    if (tails != 1) return OR_EBADLIST;

    /* 2. in-degrees: exactly one node without a predecessor, none with two */
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    if (!mark) return OR_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = succ[i];
        if (s == -1 || s == (int32_t)i) continue;
        if (mark[s]) { free(mark); return OR_EBADLIST; }
        mark[s] = 1;
    }
    int64_t head = -1, heads = 0;
    for (int64_t i = 0; i < n; ++i)
        if (!mark[i]) { ++heads; head = i; }
    if (heads != 1) { free(mark); return OR_EBADLIST; }

    /* 3. walk from the head: each node gets the count (or weight sum) of the
     *    nodes walked before it */
    memset(mark, 0, (size_t)n);
    int64_t r = 0, cur = head;
    uint32_t acc = 0;
    for (;;) {
        if (mark[cur]) { free(mark); return OR_EBADLIST; }
        mark[cur] = 1;
        ++r;
        rank[cur] = (int32_t)acc;
        acc += weight ? (uint32_t)weight[cur] : 1u;
        int32_t nx = succ[cur];
        if (nx == -1 || nx == (int32_t)cur) break;
        cur = nx;
    }
    free(mark);

    /* 4. the walk covered every node (otherwise a detached cycle exists) */
    return r == n ? OR_OK : OR_EBADLIST;
}

int oracle_list_rank(const int32_t *succ, int64_t n, int32_t *rank)
{
    return rank_one(succ, NULL, n, rank);
}

int oracle_list_rank_weighted(const int32_t *succ, const int32_t *weight, int64_t n,
                              int32_t *rank)
{
    if (n > 0 && !weight) return OR_EINVAL;
    return rank_one(succ, weight, n, rank);
}

/* ------------------------------------------------------------ components -- */

static int64_t uf_find(int32_t *parent, int64_t x)
{
    while (parent[x] != x) {            /* path halving */
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

int oracle_cc(const int32_t *src, const int32_t *dst, int64_t n, int64_t m, int32_t *label)
{
    if (n < 0 || m < 0 || n > INT32_MAX) return OR_EINVAL;
    if (n == 0) return m == 0 ? OR_OK : OR_EINVAL;
    if (!label || (m > 0 && (!src || !dst))) return OR_EINVAL;
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return OR_EINVAL;

    int32_t *parent = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *size = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!parent || !size) { free(parent); free(size); return OR_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) { parent[v] = (int32_t)v; size[v] = 1; }

    for (int64_t e = 0; e < m; ++e) {   /* union by size */
        int64_t a = uf_find(parent, src[e]);
        int64_t b = uf_find(parent, dst[e]);
        if (a == b) continue;
        if (size[a] < size[b]) { int64_t t = a; a = b; b = t; }
        parent[b] = (int32_t)a;
        size[a] += size[b];
    }

    /* smallest member of each set: first vertex seen in ascending order */
    int32_t *minv = size; /* reuse */
    for (int64_t v = 0; v < n; ++v) minv[v] = -1;
    for (int64_t v = 0; v < n; ++v) {
        int64_t r = uf_find(parent, v);
        if (minv[r] < 0) minv[r] = (int32_t)v;
        label[v] = minv[r];
    }
    free(parent);
    free(size);
    return OR_OK;
}

/* --------------------------------------------------------------- batched -- */

typedef struct {
    int kind; /* 0 list ranking, 1 components */
    const int32_t *a, *b;
    const int64_t *off, *eoff;
    int64_t count;
    int32_t *out;
    int32_t *status;
    int64_t next;          /* next instance to take (guarded by lock) */
    pthread_mutex_t lock;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *job = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t i = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (i >= job->count) break;
        int64_t v0 = job->off[i], v1 = job->off[i + 1];
        int rc;
        if (job->kind == 0) {
            rc = oracle_list_rank(job->a + v0, v1 - v0, job->out + v0);
        } else {
            int64_t e0 = job->eoff[i], e1 = job->eoff[i + 1];
            rc = oracle_cc(job->a + e0, job->b + e0, v1 - v0, e1 - e0, job->out + v0);
        }
        job->status[i] = rc;
    }
    return NULL;
}

static int run_batch(batch_job *job, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    pthread_mutex_init(&job->lock, NULL);
    job->next = 0;
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, batch_worker, job) == 0) ++started;
    if (started == 0) batch_worker(job);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&job->lock);
    int rc = OR_OK;
    for (int64_t i = 0; i < job->count; ++i)
        if (job->status[i] != OR_OK) { rc = job->status[i]; break; }
    return rc;
}

/* status[i] receives the code of instance i; the return value is the first
 * non-zero code, or 0. */
int oracle_list_rank_batched(const int32_t *succ, const int64_t *off, int64_t L,
                             int32_t *rank, int32_t *status, int nthreads)
{
    if (L < 0 || !off || !status) return OR_EINVAL;
    for (int64_t i = 0; i < L; ++i)
        if (off[i + 1] < off[i] || off[i + 1] - off[i] > INT32_MAX) return OR_EINVAL;
    batch_job job;
    memset(&job, 0, sizeof job);
    job.kind = 0; job.a = succ; job.off = off; job.count = L; job.out = rank; job.status = status;
    return run_batch(&job, nthreads);
}

int oracle_cc_batched(const int32_t *src, const int32_t *dst, const int64_t *voff,
                      const int64_t *eoff, int64_t G, int32_t *label, int32_t *status,
                      int nthreads)
{
    if (G < 0 || !voff || !eoff || !status) return OR_EINVAL;
    for (int64_t i = 0; i < G; ++i)
        if (voff[i + 1] < voff[i] || eoff[i + 1] < eoff[i] || voff[i + 1] - voff[i] > INT32_MAX)
            return OR_EINVAL;
    batch_job job;
    memset(&job, 0, sizeof job);
    job.kind = 1; job.a = src; job.b = dst; job.off = voff; job.eoff = eoff; job.count = G;
    job.out = label; job.status = status;
    return run_batch(&job, nthreads);
}
