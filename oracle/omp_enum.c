/*
 * A multi-threaded CPU clique enumeration, for the benchmark's secondary CPU
 * line only (test and benchmark infrastructure, like the oracle beside it;
 * nothing in the library calls it).  It lists every h-clique once, from its
 * smallest-id member, with the members ascending, exactly as the oracle's
 * clique-degree function does (Definition 3), but hands the roots to OpenMP
 * threads (dynamic schedule), each with its own candidate buffers and its
 * own degree array, summed at the end.  Its output is checked against the
 * oracle's by tests/test_oracle.py.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OMP_HMAX 8

typedef struct {
    const int64_t *off;
    const int32_t *adj;
    int target;
    int32_t stack[OMP_HMAX];
    int32_t *buf[OMP_HMAX];
    uint64_t *deg;
    uint64_t mu;
} walker;

static int64_t intersect(const int32_t *a, int64_t na, const int32_t *b, int64_t nb, int32_t *out) {
    int64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { out[k++] = a[i]; i++; j++; }
    }
    return k;
}

static void walk(walker *w, int depth, const int32_t *cand, int64_t nc) {
    for (int64_t i = 0; i < nc; i++) {
        const int32_t x = cand[i];
        w->stack[depth] = x;
        if (depth + 1 == w->target) {
            for (int q = 0; q < w->target; q++) w->deg[w->stack[q]]++;
            w->mu++;
            continue;
        }
        int32_t *out = w->buf[depth + 1];
        const int64_t k = intersect(cand + i + 1, nc - i - 1, w->adj + w->off[x], w->off[x + 1] - w->off[x], out);
        if (k > 0) walk(w, depth + 1, out, k);
    }
}

/* deg[v] = h-cliques containing v, *mu = their number; adjacency rows sorted
 * ascending.  Returns the number of threads used, or -1 on bad arguments or
 * memory. */
int omp_clique_degrees(int32_t n, const int64_t *off, const int32_t *adj, int h, uint64_t *deg, uint64_t *mu) {
    if (h < 2 || h > OMP_HMAX || n < 0) return -1;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; v++)
        if (off[v + 1] - off[v] > maxd) maxd = (int32_t)(off[v + 1] - off[v]);
    const int nt = omp_get_max_threads();
    uint64_t *part = (uint64_t *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    uint64_t *mus = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    int bad = part == NULL || mus == NULL;
    if (!bad) {
#pragma omp parallel num_threads(nt) reduction(|| : bad)
        {
            const int t = omp_get_thread_num();
            walker w;
            memset(&w, 0, sizeof(w));
            w.off = off;
            w.adj = adj;
            w.target = h;
            w.deg = part + (size_t)t * (size_t)n;
            for (int i = 0; i < OMP_HMAX; i++) {
                w.buf[i] = (int32_t *)malloc((size_t)(maxd + 1) * sizeof(int32_t));
                if (!w.buf[i]) bad = 1;
            }
            /* every thread meets the loop (it ends in a barrier), one that
               lacks its buffers takes no root */
#pragma omp for schedule(dynamic, 64)
            for (int32_t v = 0; v < n; v++) {
                if (!bad) {
                    w.stack[0] = v;
                    const int32_t *row = adj + off[v];
                    const int64_t len = off[v + 1] - off[v];
                    int64_t s = 0;
                    while (s < len && row[s] < v) s++;
                    memcpy(w.buf[1], row + s, (size_t)(len - s) * sizeof(int32_t));
                    walk(&w, 1, w.buf[1], len - s);
                }
            }
            mus[t] = w.mu;
            for (int i = 0; i < OMP_HMAX; i++) free(w.buf[i]);
        }
    }
    if (!bad) {
        memset(deg, 0, (size_t)n * sizeof(uint64_t));
        uint64_t total = 0;
        for (int t = 0; t < nt; t++) {
            total += mus[t];
            const uint64_t *p = part + (size_t)t * (size_t)n;
            for (int32_t v = 0; v < n; v++) deg[v] += p[v];
        }
        *mu = total;
    }
    free(part);
    free(mus);
    return bad ? -1 : nt;
}
