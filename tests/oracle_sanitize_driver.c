/*
 * Test driver: runs the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitize.py with gcc,
 * host code only).  Valid and malformed lists, graphs with self-loops,
 * duplicates and isolated vertices, and both batched forms on several
 * threads; the weighted ranking and the multi-threaded CPU baseline on the
 * same lists.  Exits non-zero on a wrong result; the sanitizers abort on a
 * memory or UB error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_list_rank(const int32_t *succ, int64_t n, int32_t *rank);
int oracle_list_rank_weighted(const int32_t *succ, const int32_t *weight, int64_t n,
                              int32_t *rank);
int cpu_ruling_set_list_rank(const int32_t *succ, int64_t n, int32_t *rank, int spacing,
                             int nthreads);
int oracle_cc(const int32_t *src, const int32_t *dst, int64_t n, int64_t m, int32_t *label);
int oracle_list_rank_batched(const int32_t *succ, const int64_t *off, int64_t L, int32_t *rank,
                             int32_t *status, int nthreads);
int oracle_cc_batched(const int32_t *src, const int32_t *dst, const int64_t *voff,
                      const int64_t *eoff, int64_t G, int32_t *label, int32_t *status,
                      int nthreads);

static uint64_t rng = 88172645463325252ull;
static uint32_t next_u32(void) {  /* xorshift64 */
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return (uint32_t)(rng >> 32);
}

static void random_order(int32_t *order, int32_t n) {
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
        int32_t j = (int32_t)(next_u32() % (uint32_t)(i + 1));
        int32_t t = order[i]; order[i] = order[j]; order[j] = t;
    }
}

static int check_list(int32_t n) {
    int32_t *order = malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *succ = malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *rank = malloc(sizeof(int32_t) * (n ? n : 1));
    random_order(order, n);
    for (int32_t k = 0; k + 1 < n; ++k) succ[order[k]] = order[k + 1];
    if (n) succ[order[n - 1]] = (n & 1) ? -1 : order[n - 1];
    int32_t *weight = malloc(sizeof(int32_t) * (n ? n : 1));
    int bad = oracle_list_rank(succ, n, rank) != 0;
    for (int32_t k = 0; k < n && !bad; ++k) bad = rank[order[k]] != k;
    /* weighted: the exclusive prefix of the weights along the order */
    for (int32_t i = 0; i < n; ++i) weight[i] = (int32_t)(next_u32() % 2001) - 1000;
    bad |= oracle_list_rank_weighted(succ, weight, n, rank) != 0;
    int64_t acc = 0;
    for (int32_t k = 0; k < n && !bad; ++k) {
        bad = rank[order[k]] != (int32_t)acc;
        acc += weight[order[k]];
    }
    /* the CPU baseline on 3 threads, one splitter per ~4 nodes */
    bad |= cpu_ruling_set_list_rank(succ, n, rank, 4, 3) != 0;
    for (int32_t k = 0; k < n && !bad; ++k) bad = rank[order[k]] != k;
    if (n > 2) {  /* a second tail, then a cycle: both rejected */
        int32_t keep = succ[order[n / 2]];
        succ[order[n / 2]] = -1;
        bad |= oracle_list_rank(succ, n, rank) != -4;
        bad |= cpu_ruling_set_list_rank(succ, n, rank, 4, 3) != -4;
        succ[order[n / 2]] = keep;
        succ[order[n - 1]] = order[0];
        bad |= oracle_list_rank(succ, n, rank) != -4;
        bad |= cpu_ruling_set_list_rank(succ, n, rank, 4, 3) != -4;
    }
    free(order); free(succ); free(rank); free(weight);
    return bad;
}

static int check_graph(int32_t n, int64_t m) {
    int32_t *src = malloc(sizeof(int32_t) * (m ? m : 1));
    int32_t *dst = malloc(sizeof(int32_t) * (m ? m : 1));
    int32_t *label = malloc(sizeof(int32_t) * (n ? n : 1));
    for (int64_t e = 0; e < m; ++e) {
        src[e] = (int32_t)(next_u32() % (uint32_t)n);
        dst[e] = (e % 7 == 0) ? src[e] : (int32_t)(next_u32() % (uint32_t)n);
    }
    int bad = oracle_cc(src, dst, n, m, label) != 0;
    for (int64_t e = 0; e < m && !bad; ++e) bad = label[src[e]] != label[dst[e]];
    for (int32_t v = 0; v < n && !bad; ++v) bad = label[v] > v || label[label[v]] != label[v];
    free(src); free(dst); free(label);
    return bad;
}

int main(void) {
    int bad = 0;
    const int32_t sizes[] = {0, 1, 2, 3, 17, 1000, 65537};
    for (int i = 0; i < 7; ++i) bad |= check_list(sizes[i]);
    bad |= check_graph(1, 3);
    bad |= check_graph(50, 0);
    bad |= check_graph(1000, 3000);
    bad |= check_graph(20000, 10000);
    /* batched lists: 64 lists of varied size, 4 threads */
    {
        const int64_t L = 64;
        int64_t off[65];
        off[0] = 0;
        for (int64_t l = 0; l < L; ++l) off[l + 1] = off[l] + (int64_t)(next_u32() % 300);
        int32_t *succ = malloc(sizeof(int32_t) * (off[L] ? off[L] : 1));
        int32_t *rank = malloc(sizeof(int32_t) * (off[L] ? off[L] : 1));
        int32_t status[64];
        int32_t *order = malloc(sizeof(int32_t) * 300);
        for (int64_t l = 0; l < L; ++l) {
            int32_t n = (int32_t)(off[l + 1] - off[l]);
            random_order(order, n);
            for (int32_t k = 0; k + 1 < n; ++k) succ[off[l] + order[k]] = order[k + 1];
            if (n) succ[off[l] + order[n - 1]] = -1;
        }
        bad |= oracle_list_rank_batched(succ, off, L, rank, status, 4) != 0;
        for (int64_t l = 0; l < L; ++l) bad |= status[l] != 0;
        free(succ); free(rank); free(order);
    }
    /* batched graphs: 16 graphs, 3 threads */
    {
        const int64_t G = 16;
        int64_t voff[17], eoff[17];
        voff[0] = eoff[0] = 0;
        for (int64_t g = 0; g < G; ++g) {
            voff[g + 1] = voff[g] + 1 + (int64_t)(next_u32() % 500);
            eoff[g + 1] = eoff[g] + (int64_t)(next_u32() % 800);
        }
        int32_t *src = malloc(sizeof(int32_t) * (eoff[G] ? eoff[G] : 1));
        int32_t *dst = malloc(sizeof(int32_t) * (eoff[G] ? eoff[G] : 1));
        int32_t *label = malloc(sizeof(int32_t) * voff[G]);
        int32_t status[16];
        for (int64_t g = 0; g < G; ++g) {
            uint32_t n = (uint32_t)(voff[g + 1] - voff[g]);
            for (int64_t e = eoff[g]; e < eoff[g + 1]; ++e) {
                src[e] = (int32_t)(next_u32() % n);
                dst[e] = (int32_t)(next_u32() % n);
            }
        }
        bad |= oracle_cc_batched(src, dst, voff, eoff, G, label, status, 3) != 0;
        for (int64_t g = 0; g < G && !bad; ++g)
            for (int64_t e = eoff[g]; e < eoff[g + 1] && !bad; ++e)
                bad = label[voff[g] + src[e]] != label[voff[g] + dst[e]];
        free(src); free(dst); free(label);
    }
    printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
