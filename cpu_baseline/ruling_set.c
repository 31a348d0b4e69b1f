/*
 * Multi-threaded CPU list ranking by random splitters: the comparison
 * baseline for the paper's quad-core CPU runs (Section 3.2's sparse ruling
 * set, executed by POSIX threads on the host's cores).
 *
 * BENCHMARK INFRASTRUCTURE, and not a parity reference: the tests pin this
 * function against the CPU oracle's ranks.  It shares no code with the
 * oracle or the GPU library; neither includes, links or calls it.
 *
 * Steps, each a parallel pass over node ranges or a shared splitter counter:
 *   1. head = n(n-1)/2 - sum of the non-tail successors (every node but the
 *      head is exactly one node's successor); count the tails;
 *   2. splitters: the head, and every node whose hashed id falls in a 1/spacing
 *      slice; numbered by a prefix count over the thread ranges;
 *   3. threads take splitters from a shared counter and walk each sublist to
 *      the next splitter or the tail, storing (owner, offset) per node and
 *      (next splitter, length) per splitter;
 *   4. one thread ranks the splitter list from the head's splitter (an
 *      exclusive prefix of the lengths);
 *   5. rank[i] = splitter rank of owner[i] + offset[i].
 * Malformed input is caught where it is cheap: a tail count other than one,
 * an id out of range, a head outside the list, or splitter lengths that do
 * not add up to n (a cycle or a branch) return -4.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <stdatomic.h>

#define CB_OK 0
#define CB_EINVAL (-1)
#define CB_ENOMEM (-2)
#define CB_EBADLIST (-4)

typedef struct {
    const int32_t *succ;
    int64_t n;
    int spacing;
    int nthreads;
    uint8_t *split;        /* node is a splitter */
    int32_t *sid;          /* splitter id of a splitter node */
    int32_t *owner;        /* sublist of each node */
    int32_t *offset;       /* position of the node in its sublist */
    int32_t *nodes;        /* node of splitter s */
    int32_t *next;         /* next splitter, -1 after the last */
    int32_t *len;          /* nodes in the sublist of splitter s */
    int32_t *srank;        /* rank of splitter s */
    int32_t *rank;
    int64_t *chunk_sum;    /* per thread: sum of non-tail successors */
    int64_t *chunk_tails;
    int64_t *chunk_bad;
    int64_t *chunk_split;  /* per thread: splitters counted, then their first id */
    int64_t head;
    int64_t nsplit;
    atomic_long next_item;
    int pass;
} cb_job;

typedef struct { cb_job *job; int t; } cb_arg;

static uint64_t mix64(uint64_t z)  /* SplitMix64 finaliser */
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void range_of(const cb_job *j, int t, int64_t *lo, int64_t *hi)
{
    *lo = j->n * t / j->nthreads;
    *hi = j->n * (t + 1) / j->nthreads;
}

static void *cb_worker(void *p)
{
    cb_arg *a = (cb_arg *)p;
    cb_job *j = a->job;
    const int t = a->t;
    int64_t lo, hi;
    range_of(j, t, &lo, &hi);
    const int32_t *succ = j->succ;
    if (j->pass == 0) {            /* step 1 and the splitter count of step 2 */
        int64_t sum = 0, tails = 0, bad = 0, cnt = 0;
        for (int64_t i = lo; i < hi; ++i) {
            const int32_t s = succ[i];
            if (s == -1 || s == (int32_t)i) ++tails;
            else if (s < 0 || s >= j->n) ++bad;
            else sum += s;
            const uint8_t sp = (mix64((uint64_t)i + 0x9E3779B97F4A7C15ull) % (uint64_t)j->spacing) == 0;
            j->split[i] = sp;
            cnt += sp;
        }
        j->chunk_sum[t] = sum;
        j->chunk_tails[t] = tails;
        j->chunk_bad[t] = bad;
        j->chunk_split[t] = cnt;
    } else if (j->pass == 1) {     /* step 2: number the splitters */
        int64_t id = j->chunk_split[t];
        for (int64_t i = lo; i < hi; ++i)
            if (j->split[i]) {
                j->sid[i] = (int32_t)id;
                j->nodes[id] = (int32_t)i;
                ++id;
            }
    } else if (j->pass == 2) {     /* step 3: walk sublists */
        for (;;) {
            const long first = atomic_fetch_add(&j->next_item, 64);
            if (first >= j->nsplit) break;
            const long last = first + 64 < j->nsplit ? first + 64 : j->nsplit;
            for (long s = first; s < last; ++s) {
                int64_t x = j->nodes[s];
                int32_t k = 0;
                for (;;) {
                    j->owner[x] = (int32_t)s;
                    j->offset[x] = k++;
                    const int32_t y = succ[x];
                    if (y == -1 || y == (int32_t)x) { j->next[s] = -1; break; }
                    if (j->split[y]) { j->next[s] = j->sid[y]; break; }
                    if (k >= j->n) { j->next[s] = -2; break; }  /* a cycle without splitters */
                    x = y;
                }
                j->len[s] = k;
            }
        }
    } else {                       /* step 5 */
        for (int64_t i = lo; i < hi; ++i) j->rank[i] = j->srank[j->owner[i]] + j->offset[i];
    }
    return NULL;
}

static int run_pass(cb_job *j, int pass)
{
    pthread_t th[256];
    cb_arg args[256];
    j->pass = pass;
    int started = 0;
    for (int t = 1; t < j->nthreads; ++t) {
        args[t].job = j;
        args[t].t = t;
        if (pthread_create(&th[t], NULL, cb_worker, &args[t]) != 0) break;
        started = t;
    }
    args[0].job = j;
    args[0].t = 0;
    if (started == j->nthreads - 1) cb_worker(&args[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    return started == j->nthreads - 1 ? CB_OK : CB_ENOMEM;
}

int cpu_ruling_set_list_rank(const int32_t *succ, int64_t n, int32_t *rank, int spacing,
                             int nthreads)
{
    if (n < 0 || n >= INT32_MAX || spacing < 1 || nthreads < 1 || nthreads > 256) return CB_EINVAL;
    if (n == 0) return CB_OK;
    if (!succ || !rank) return CB_EINVAL;
    cb_job j;
    memset(&j, 0, sizeof j);
    j.succ = succ;
    j.n = n;
    j.spacing = spacing;
    j.nthreads = nthreads;
    j.rank = rank;
    int rc = CB_ENOMEM;
    j.split = (uint8_t *)malloc((size_t)n);
    j.sid = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    j.owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    j.offset = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    j.chunk_sum = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
    j.chunk_tails = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
    j.chunk_bad = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
    j.chunk_split = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
    if (!j.split || !j.sid || !j.owner || !j.offset || !j.chunk_sum || !j.chunk_tails ||
        !j.chunk_bad || !j.chunk_split)
        goto out;
    if ((rc = run_pass(&j, 0)) != CB_OK) goto out;
    int64_t sum = 0, tails = 0, bad = 0;
    for (int t = 0; t < nthreads; ++t) {
        sum += j.chunk_sum[t];
        tails += j.chunk_tails[t];
        bad += j.chunk_bad[t];
    }
    rc = CB_EBADLIST;
    if (tails != 1 || bad) goto out;
    {
        /* n(n-1)/2 fits in int64 for n < 2^31 */
        const int64_t head = n * (n - 1) / 2 - sum;
        if (head < 0 || head >= n) goto out;
        j.head = head;
        j.split[head] = 1;
    }
    /* recount with the head forced in, then number (the head's own range
     * gets one more if it was not already a splitter) */
    {
        int64_t lo, hi, total = 0;
        for (int t = 0; t < nthreads; ++t) {
            range_of(&j, t, &lo, &hi);
            int64_t cnt = 0;
            if (j.head >= lo && j.head < hi) {
                /* pass 0 counted the hashed splitters only */
                const uint8_t hashed =
                    (mix64((uint64_t)j.head + 0x9E3779B97F4A7C15ull) % (uint64_t)spacing) == 0;
                cnt = j.chunk_split[t] + (hashed ? 0 : 1);
            } else {
                cnt = j.chunk_split[t];
            }
            j.chunk_split[t] = total;
            total += cnt;
        }
        j.nsplit = total;
    }
    rc = CB_ENOMEM;
    j.nodes = (int32_t *)malloc(sizeof(int32_t) * (size_t)j.nsplit);
    j.next = (int32_t *)malloc(sizeof(int32_t) * (size_t)j.nsplit);
    j.len = (int32_t *)malloc(sizeof(int32_t) * (size_t)j.nsplit);
    j.srank = (int32_t *)malloc(sizeof(int32_t) * (size_t)j.nsplit);
    if (!j.nodes || !j.next || !j.len || !j.srank) goto out;
    if ((rc = run_pass(&j, 1)) != CB_OK) goto out;
    atomic_store(&j.next_item, 0);
    if ((rc = run_pass(&j, 2)) != CB_OK) goto out;
    /* step 4: the splitter list from the head's splitter */
    {
        rc = CB_EBADLIST;
        int64_t acc = 0, visited = 0;
        int32_t s = j.sid[j.head];
        while (s >= 0) {
            if (++visited > j.nsplit) goto out;  /* a cycle among splitters */
            j.srank[s] = (int32_t)acc;
            acc += j.len[s];
            s = j.next[s];
        }
        if (s == -2 || acc != n) goto out;  /* unreached or doubly owned nodes */
    }
    if ((rc = run_pass(&j, 3)) != CB_OK) goto out;
    rc = CB_OK;
out:
    free(j.split); free(j.sid); free(j.owner); free(j.offset);
    free(j.chunk_sum); free(j.chunk_tails); free(j.chunk_bad); free(j.chunk_split);
    free(j.nodes); free(j.next); free(j.len); free(j.srank);
    return rc;
}
