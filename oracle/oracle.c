/*
 * CPU oracle for the k-clique-core densest-subgraph path (declarations and the
 * list of readings are in oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark.  It shares no code with the GPU library.
 *
 * Parity pins (all in tests/test_oracle_*.py): every function below is checked
 * against something other than itself -- the paper's worked examples, closed
 * forms on complete graphs, a dense matrix product for triangles, the
 * fixpoint definition of a core, exhaustive subset search, and agreement of
 * two independent exact routes.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define ORC_HMAX 8
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-4)

/* ------------------------------------------------------------------ */
/* Graph (Section 3, data model: undirected, unweighted, simple)        */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static orc_graph *graph_alloc(int32_t n, int64_t adj_len) {
    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    if (!g) return NULL;
    g->n = n;
    g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int32_t *)malloc((size_t)(adj_len > 0 ? adj_len : 1) * sizeof(int32_t));
    if (!g->off || !g->adj) { orc_graph_free(g); return NULL; }
    return g;
}

orc_graph *orc_graph_new(int32_t n, int64_t npairs, const int32_t *src, const int32_t *dst) {
    if (n < 0 || npairs < 0) return NULL;
    for (int64_t i = 0; i < npairs; i++)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return NULL;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return NULL;
    int64_t tot = 0;
    for (int64_t i = 0; i < npairs; i++)
        if (src[i] != dst[i]) { cnt[src[i]]++; cnt[dst[i]]++; tot += 2; }
    int64_t *pos = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *tmp = (int32_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
    if (!pos || !tmp) { free(cnt); free(pos); free(tmp); return NULL; }
    pos[0] = 0;
    for (int32_t v = 0; v < n; v++) pos[v + 1] = pos[v] + cnt[v];
    memcpy(cnt, pos, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < npairs; i++) {
        if (src[i] == dst[i]) continue;
        tmp[cnt[src[i]]++] = dst[i];
        tmp[cnt[dst[i]]++] = src[i];
    }
    /* sort each row, drop repeats */
    orc_graph *g = graph_alloc(n, tot);
    if (!g) { free(cnt); free(pos); free(tmp); return NULL; }
    int64_t w = 0;
    for (int32_t v = 0; v < n; v++) {
        int64_t a = pos[v], b = pos[v + 1];
        qsort(tmp + a, (size_t)(b - a), sizeof(int32_t), cmp_i32);
        g->off[v] = w;
        for (int64_t i = a; i < b; i++)
            if (i == a || tmp[i] != tmp[i - 1]) g->adj[w++] = tmp[i];
    }
    g->off[n] = w;
    g->m = w / 2;
    free(cnt); free(pos); free(tmp);
    return g;
}

void orc_graph_free(orc_graph *g) {
    if (!g) return;
    free(g->off);
    free(g->adj);
    free(g);
}

int32_t orc_graph_n(const orc_graph *g) { return g->n; }
int64_t orc_graph_m(const orc_graph *g) { return g->m; }

void orc_graph_adjacency(const orc_graph *g, int64_t *off, int32_t *adj) {
    memcpy(off, g->off, ((size_t)g->n + 1) * sizeof(int64_t));
    memcpy(adj, g->adj, (size_t)g->off[g->n] * sizeof(int32_t));
}

orc_graph *orc_graph_induced(const orc_graph *g, const uint8_t *mask, int32_t *map) {
    int32_t *newid = (int32_t *)malloc(((size_t)g->n + 1) * sizeof(int32_t));
    if (!newid) return NULL;
    int32_t k = 0;
    int64_t len = 0;
    for (int32_t v = 0; v < g->n; v++) {
        newid[v] = mask[v] ? k++ : -1;
        if (mask[v])
            for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
                if (mask[g->adj[e]]) len++;
    }
    orc_graph *s = graph_alloc(k, len);
    if (!s) { free(newid); return NULL; }
    int64_t w = 0;
    for (int32_t v = 0; v < g->n; v++) {
        if (!mask[v]) continue;
        map[newid[v]] = v;
        s->off[newid[v]] = w;
        for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
            if (mask[g->adj[e]]) s->adj[w++] = newid[g->adj[e]];  /* stays sorted */
    }
    s->off[k] = w;
    s->m = w / 2;
    free(newid);
    return s;
}

static int32_t max_degree(const orc_graph *g) {
    int64_t d = 0;
    for (int32_t v = 0; v < g->n; v++)
        if (g->off[v + 1] - g->off[v] > d) d = g->off[v + 1] - g->off[v];
    return (int32_t)d;
}

/* ------------------------------------------------------------------ */
/* Ordered clique listing (Definition 2).  Total order = vertex id.      */
/* A clique v1 < v2 < ... < vh is reached once: v_{i+1} is drawn from    */
/* the vertices adjacent to all of v1..vi that come after v_i.           */
/* ------------------------------------------------------------------ */

typedef void (*emit_fn)(void *ctx, const int32_t *members, int size);

typedef struct {
    const orc_graph *g;
    int32_t stack[ORC_HMAX];
    int32_t *buf[ORC_HMAX];
    emit_fn emit;
    void *ctx;
    int target;        /* clique size to list */
} lister;

static int lister_init(lister *L, const orc_graph *g, int target, emit_fn emit, void *ctx) {
    memset(L, 0, sizeof(*L));
    L->g = g;
    L->emit = emit;
    L->ctx = ctx;
    L->target = target;
    int32_t d = max_degree(g) + 1;
    for (int i = 0; i < ORC_HMAX; i++) {
        L->buf[i] = (int32_t *)malloc((size_t)d * sizeof(int32_t));
        if (!L->buf[i]) return ORC_ENOMEM;
    }
    return ORC_OK;
}

static void lister_free(lister *L) {
    for (int i = 0; i < ORC_HMAX; i++) free(L->buf[i]);
}

/* out = a ∩ b for sorted lists; returns the size. */
static int64_t intersect(const int32_t *a, int64_t na, const int32_t *b, int64_t nb, int32_t *out) {
    int64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { out[k++] = a[i]; i++; j++; }
    }
    return k;
}

/* stack[0..depth-1] is a clique; cand = sorted common neighbours of all of
 * them that may extend it (each later pick comes after the earlier ones). */
static void list_rec(lister *L, int depth, const int32_t *cand, int64_t nc) {
    const orc_graph *g = L->g;
    for (int64_t i = 0; i < nc; i++) {
        int32_t x = cand[i];
        L->stack[depth] = x;
        if (depth + 1 == L->target) {
            L->emit(L->ctx, L->stack, L->target);
            continue;
        }
        int32_t *out = L->buf[depth + 1];
        int64_t k = intersect(cand + i + 1, nc - i - 1, g->adj + g->off[x],
                              g->off[x + 1] - g->off[x], out);
        if (k > 0) list_rec(L, depth + 1, out, k);
    }
}

/* Every clique of size L->target in g, each once, members ascending. */
static void list_all(lister *L) {
    const orc_graph *g = L->g;
    for (int32_t v = 0; v < g->n; v++) {
        L->stack[0] = v;
        if (L->target == 1) { L->emit(L->ctx, L->stack, 1); continue; }
        /* neighbours after v */
        const int32_t *row = g->adj + g->off[v];
        int64_t len = g->off[v + 1] - g->off[v], s = 0;
        while (s < len && row[s] < v) s++;
        int32_t *out = L->buf[1];
        memcpy(out, row + s, (size_t)(len - s) * sizeof(int32_t));
        list_rec(L, 1, out, len - s);
    }
}

/* Every clique of size L->target that contains v, using only vertices with
 * alive[x] != 0 (alive may be NULL), each once; stack[0] = v. */
static void list_containing(lister *L, int32_t v, const uint8_t *alive) {
    const orc_graph *g = L->g;
    L->stack[0] = v;
    if (L->target == 1) { L->emit(L->ctx, L->stack, 1); return; }
    int32_t *out = L->buf[1];
    int64_t k = 0;
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
        if (!alive || alive[g->adj[e]]) out[k++] = g->adj[e];
    list_rec(L, 1, out, k);
}

/* ---- clique-degree (Definition 3) ---- */

typedef struct { uint64_t *deg; u128 mu; int overflow; } degctx;

static void emit_degree(void *c, const int32_t *mem, int size) {
    degctx *d = (degctx *)c;
    for (int i = 0; i < size; i++) {
        if (d->deg[mem[i]] == UINT64_MAX) d->overflow = 1;
        d->deg[mem[i]]++;
    }
    d->mu++;
}

int orc_clique_degrees(const orc_graph *g, int h, uint64_t *deg, uint64_t *mu) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    memset(deg, 0, (size_t)g->n * sizeof(uint64_t));
    degctx c = {deg, 0, 0};
    lister L;
    if (lister_init(&L, g, h, emit_degree, &c)) { lister_free(&L); return ORC_ENOMEM; }
    list_all(&L);
    lister_free(&L);
    if (c.overflow || c.mu > (u128)UINT64_MAX) return ORC_EOVERFLOW;
    *mu = (uint64_t)c.mu;
    return ORC_OK;
}

typedef struct { u128 count; } cntctx;
static void emit_count(void *c, const int32_t *mem, int size) {
    (void)mem; (void)size;
    ((cntctx *)c)->count++;
}

int orc_clique_degree_of(const orc_graph *g, int h, int32_t v, uint64_t *deg) {
    if (h < 2 || h > ORC_HMAX || v < 0 || v >= g->n) return ORC_EINVAL;
    cntctx c = {0};
    lister L;
    if (lister_init(&L, g, h, emit_count, &c)) { lister_free(&L); return ORC_ENOMEM; }
    list_containing(&L, v, NULL);
    lister_free(&L);
    if (c.count > (u128)UINT64_MAX) return ORC_EOVERFLOW;
    *deg = (uint64_t)c.count;
    return ORC_OK;
}

/* number of h-cliques of the subgraph induced by mask (mask may be NULL) */
static int count_cliques(const orc_graph *g, int h, const uint8_t *mask, u128 *mu) {
    if (!mask) {
        cntctx c = {0};
        lister L;
        if (lister_init(&L, g, h, emit_count, &c)) { lister_free(&L); return ORC_ENOMEM; }
        list_all(&L);
        lister_free(&L);
        *mu = c.count;
        return ORC_OK;
    }
    int32_t *map = (int32_t *)malloc(((size_t)g->n + 1) * sizeof(int32_t));
    orc_graph *s = orc_graph_induced(g, mask, map);
    free(map);
    if (!s) return ORC_ENOMEM;
    int rc = count_cliques(s, h, NULL, mu);
    orc_graph_free(s);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Indexed binary min-heap keyed by (value, id)                          */
/* ------------------------------------------------------------------ */

typedef struct { const uint64_t *key; int32_t *heap; int32_t *pos; int32_t size; } iheap;

static int hless(const iheap *H, int32_t a, int32_t b) {
    return H->key[a] < H->key[b] || (H->key[a] == H->key[b] && a < b);
}
static void hswap(iheap *H, int32_t i, int32_t j) {
    int32_t a = H->heap[i], b = H->heap[j];
    H->heap[i] = b; H->heap[j] = a;
    H->pos[b] = i; H->pos[a] = j;
}
static void hup(iheap *H, int32_t i) {
    while (i > 0) {
        int32_t p = (i - 1) / 2;
        if (!hless(H, H->heap[i], H->heap[p])) break;
        hswap(H, i, p);
        i = p;
    }
}
static void hdown(iheap *H, int32_t i) {
    for (;;) {
        int32_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < H->size && hless(H, H->heap[l], H->heap[s])) s = l;
        if (r < H->size && hless(H, H->heap[r], H->heap[s])) s = r;
        if (s == i) break;
        hswap(H, i, s);
        i = s;
    }
}
static int32_t hpop(iheap *H) {
    int32_t top = H->heap[0];
    hswap(H, 0, H->size - 1);
    H->size--;
    H->pos[top] = -1;
    if (H->size > 0) hdown(H, 0);
    return top;
}

/* ------------------------------------------------------------------ */
/* Alg. 3: (k, Psi)-core decomposition.                                  */
/* Pop the vertex of minimum current clique-degree, record it as its      */
/* core number, and for every clique containing it among the remaining    */
/* vertices decrease the clique-degree of each co-member whose degree is  */
/* larger than the popped one.                                           */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t *deg; iheap *H; int32_t v; } peelctx;

static void emit_peel(void *c, const int32_t *mem, int size) {
    peelctx *p = (peelctx *)c;
    for (int i = 0; i < size; i++) {
        int32_t u = mem[i];
        if (u == p->v) continue;
        if (p->deg[u] > p->deg[p->v]) {
            p->deg[u]--;
            hup(p->H, p->H->pos[u]);
        }
    }
}

int orc_core_decomposition(const orc_graph *g, int h, uint64_t *core, uint64_t *kmax) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    int32_t n = g->n;
    uint64_t *deg = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint8_t *alive = (uint8_t *)malloc((size_t)n + 1);
    int32_t *hp = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *pos = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!deg || !alive || !hp || !pos) { free(deg); free(alive); free(hp); free(pos); return ORC_ENOMEM; }
    uint64_t mu;
    int rc = orc_clique_degrees(g, h, deg, &mu);
    if (rc) { free(deg); free(alive); free(hp); free(pos); return rc; }
    iheap H = {deg, hp, pos, n};
    for (int32_t v = 0; v < n; v++) { hp[v] = v; pos[v] = v; alive[v] = 1; }
    for (int32_t i = n / 2 - 1; i >= 0; i--) hdown(&H, i);
    peelctx pc = {deg, &H, -1};
    lister L;
    if (lister_init(&L, g, h, emit_peel, &pc)) { lister_free(&L); free(deg); free(alive); free(hp); free(pos); return ORC_ENOMEM; }
    uint64_t km = 0;
    while (H.size > 0) {
        int32_t v = hpop(&H);
        core[v] = deg[v];
        if (deg[v] > km) km = deg[v];
        pc.v = v;
        list_containing(&L, v, alive);
        alive[v] = 0;
    }
    lister_free(&L);
    *kmax = km;
    free(deg); free(alive); free(hp); free(pos);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Level table: |R_k| and mu(R_k) for every distinct core value.          */
/* A clique lies in R_k iff the smallest core number among its members   */
/* is at least k.                                                        */
/* ------------------------------------------------------------------ */

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

typedef struct { const uint64_t *core; const uint64_t *levels; int64_t nl; u128 *cnt; } lvlctx;

static int64_t level_index(const uint64_t *levels, int64_t nl, uint64_t k) {
    /* largest i with levels[i] <= k */
    int64_t lo = 0, hi = nl - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (levels[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

static void emit_level(void *c, const int32_t *mem, int size) {
    lvlctx *l = (lvlctx *)c;
    uint64_t mn = UINT64_MAX;
    for (int i = 0; i < size; i++)
        if (l->core[mem[i]] < mn) mn = l->core[mem[i]];
    l->cnt[level_index(l->levels, l->nl, mn)]++;
}

int orc_level_table(const orc_graph *g, int h, const uint64_t *core,
                    uint64_t *levels, uint64_t *rsize, uint64_t *rmu, int64_t *nlevels) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    int32_t n = g->n;
    uint64_t *sorted = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!sorted) return ORC_ENOMEM;
    sorted[0] = 0;
    memcpy(sorted + 1, core, (size_t)n * sizeof(uint64_t));
    qsort(sorted, (size_t)n + 1, sizeof(uint64_t), cmp_u64);
    int64_t nl = 0;
    for (int64_t i = 0; i <= n; i++)
        if (i == 0 || sorted[i] != sorted[i - 1]) levels[nl++] = sorted[i];
    /* |R_k|: vertices with core >= levels[i] */
    for (int64_t i = 0; i < nl; i++) rsize[i] = 0;
    for (int32_t v = 0; v < n; v++) rsize[level_index(levels, nl, core[v])]++;
    for (int64_t i = nl - 2; i >= 0; i--) rsize[i] += rsize[i + 1];
    u128 *cnt = (u128 *)calloc((size_t)nl, sizeof(u128));
    if (!cnt) { free(sorted); return ORC_ENOMEM; }
    lvlctx c = {core, levels, nl, cnt};
    lister L;
    if (lister_init(&L, g, h, emit_level, &c)) { lister_free(&L); free(cnt); free(sorted); return ORC_ENOMEM; }
    list_all(&L);
    lister_free(&L);
    for (int64_t i = nl - 2; i >= 0; i--) cnt[i] += cnt[i + 1];
    int rc = ORC_OK;
    for (int64_t i = 0; i < nl; i++) {
        if (cnt[i] > (u128)UINT64_MAX) rc = ORC_EOVERFLOW;
        rmu[i] = (uint64_t)cnt[i];
    }
    *nlevels = nl;
    free(cnt);
    free(sorted);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Exact rationals                                                       */
/* ------------------------------------------------------------------ */

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}
static void reduce(uint64_t *num, uint64_t *den) {
    if (*num == 0) { *den = 1; return; }
    uint64_t g = gcd_u64(*num, *den);
    *num /= g; *den /= g;
}
/* a/b > c/d ? (b, d > 0) */
static int frac_gt(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
    return (u128)a * d > (u128)c * b;
}
static uint64_t frac_ceil(uint64_t a, uint64_t b) {
    return a / b + (a % b != 0);
}

/* ------------------------------------------------------------------ */
/* Alg. 5 (IncApp)                                                       */
/* ------------------------------------------------------------------ */

int orc_inc_app(const orc_graph *g, int h, uint8_t *member, uint64_t *kmax,
                uint64_t *num, uint64_t *den) {
    int32_t n = g->n;
    uint64_t *core = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!core) return ORC_ENOMEM;
    int rc = orc_core_decomposition(g, h, core, kmax);
    if (rc) { free(core); return rc; }
    uint64_t size = 0;
    for (int32_t v = 0; v < n; v++) {
        member[v] = (n > 0 && core[v] == *kmax && *kmax > 0) ? 1 : 0;
        size += member[v];
    }
    free(core);
    if (size == 0) { *num = 0; *den = 1; return ORC_OK; }
    u128 mu;
    rc = count_cliques(g, h, member, &mu);
    if (rc) return rc;
    if (mu > (u128)UINT64_MAX) return ORC_EOVERFLOW;
    *num = (uint64_t)mu;
    *den = size;
    reduce(num, den);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Alg. 6 (CoreApp)                                                      */
/* ------------------------------------------------------------------ */

/* C(x, r), saturating at UINT64_MAX */
static uint64_t binom_sat(uint64_t x, int r) {
    if ((uint64_t)r > x) return 0;
    u128 acc = 1;
    for (int i = 1; i <= r; i++) {
        acc = acc * (u128)(x - (uint64_t)r + (uint64_t)i) / (u128)i;
        if (acc > (u128)UINT64_MAX) return UINT64_MAX;
    }
    return (uint64_t)acc;
}

typedef struct { const uint64_t *gamma; } gctx;
static const uint64_t *g_sort_gamma;   /* qsort has no context argument */
static int cmp_gamma(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    uint64_t gx = g_sort_gamma[x], gy = g_sort_gamma[y];
    if (gx != gy) return gx > gy ? -1 : 1;
    return (x > y) - (x < y);
}

/* Delete-and-decrement peel on sub (a copy): repeatedly remove vertices of
 * current clique-degree < k; every clique through a removed vertex loses all
 * its other members' counts. */
typedef struct { uint64_t *deg; int32_t *queue; int64_t *qn; uint8_t *queued; uint64_t k; int32_t v; } delctx;

static void emit_delete(void *c, const int32_t *mem, int size) {
    delctx *d = (delctx *)c;
    for (int i = 0; i < size; i++) {
        int32_t u = mem[i];
        if (u == d->v) continue;
        d->deg[u]--;
        if (d->deg[u] < d->k && !d->queued[u]) { d->queued[u] = 1; d->queue[(*d->qn)++] = u; }
    }
}

static void peel_below(lister *L, delctx *dc, uint8_t *alive, int32_t n, uint64_t k, int64_t *alive_cnt) {
    dc->k = k;
    *dc->qn = 0;
    for (int32_t v = 0; v < n; v++)
        if (alive[v] && dc->deg[v] < k && !dc->queued[v]) { dc->queued[v] = 1; dc->queue[(*dc->qn)++] = v; }
    int64_t head = 0;
    while (head < *dc->qn) {
        int32_t v = dc->queue[head++];
        dc->v = v;
        list_containing(L, v, alive);
        alive[v] = 0;
        (*alive_cnt)--;
    }
}

int orc_core_app(const orc_graph *g, int h, int literal, int64_t w0,
                 uint8_t *member, uint64_t *kmax_out, uint64_t *num, uint64_t *den,
                 int64_t *iterations) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    int32_t n = g->n;
    memset(member, 0, (size_t)n);
    *kmax_out = 0; *num = 0; *den = 1; *iterations = 0;
    if (n == 0) return ORC_OK;
    /* gamma(v) = C(x_v, h-1), x_v = classic core number */
    uint64_t *x = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint64_t *gamma = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint8_t *inW = (uint8_t *)calloc((size_t)n, 1);
    int32_t *map = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!x || !gamma || !order || !inW || !map) { free(x); free(gamma); free(order); free(inW); free(map); return ORC_ENOMEM; }
    uint64_t xk;
    int rc = orc_core_decomposition(g, 2, x, &xk);
    if (rc) goto done;
    for (int32_t v = 0; v < n; v++) { gamma[v] = binom_sat(x[v], h - 1); order[v] = v; }
    g_sort_gamma = gamma;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_gamma);
    int64_t wsize = w0;
    if (wsize <= 0) {
        int64_t top = 0;
        while (top < n && gamma[order[top]] == gamma[order[0]]) top++;
        wsize = top > 64 ? top : 64;
    }
    if (wsize > n) wsize = n;
    uint64_t kmax = 0;
    uint8_t *best = member;   /* S*, as a mask over G */
    for (;;) {
        if (literal) {
            /* stop rule first, on the current W */
            if (wsize >= n) break;
            if (gamma[order[wsize]] < kmax) break;
            if (wsize == 0) break;  /* the printed loop would not terminate here */
        }
        (*iterations)++;
        memset(inW, 0, (size_t)n);
        for (int64_t i = 0; i < wsize; i++) inW[order[i]] = 1;
        orc_graph *s = orc_graph_induced(g, inW, map);
        if (!s) { rc = ORC_ENOMEM; goto done; }
        int32_t sn = s->n;
        uint64_t *deg = (uint64_t *)malloc(((size_t)sn + 1) * sizeof(uint64_t));
        uint8_t *alive = (uint8_t *)malloc((size_t)sn + 1);
        uint8_t *queued = (uint8_t *)calloc((size_t)sn + 1, 1);
        int32_t *queue = (int32_t *)malloc(((size_t)sn + 1) * sizeof(int32_t));
        int64_t qn = 0;
        uint64_t mu;
        rc = (!deg || !alive || !queued || !queue) ? ORC_ENOMEM : orc_clique_degrees(s, h, deg, &mu);
        if (rc) { free(deg); free(alive); free(queued); free(queue); orc_graph_free(s); goto done; }
        uint64_t kl = UINT64_MAX, ku = 0;
        for (int32_t v = 0; v < sn; v++) {
            if (deg[v] < kl) kl = deg[v];
            if (deg[v] > ku) ku = deg[v];
            alive[v] = 1;
        }
        int64_t alive_cnt = sn;
        delctx dc = {deg, queue, &qn, queued, 0, -1};
        lister L;
        if (lister_init(&L, s, h, emit_delete, &dc)) { lister_free(&L); rc = ORC_ENOMEM; free(deg); free(alive); free(queued); free(queue); orc_graph_free(s); goto done; }
        if (!literal) {
            uint64_t k = kl > kmax ? kl : kmax;
            while (k <= ku && alive_cnt > 0) {
                peel_below(&L, &dc, alive, sn, k, &alive_cnt);
                if (alive_cnt == 0) break;
                uint64_t mn = UINT64_MAX;
                for (int32_t v = 0; v < sn; v++) if (alive[v] && deg[v] < mn) mn = deg[v];
                kmax = mn;
                memset(best, 0, (size_t)n);
                for (int32_t v = 0; v < sn; v++) if (alive[v]) best[map[v]] = 1;
                if (mn == UINT64_MAX) break;
                k = mn + 1;
            }
        } else {
            uint64_t k = kl > kmax + 1 ? kl : kmax + 1;
            while (k <= ku && alive_cnt > 0) {
                peel_below(&L, &dc, alive, sn, k, &alive_cnt);
                if (alive_cnt > 0) {
                    if (k > kmax) {
                        kmax = k;
                        memset(best, 0, (size_t)n);
                        for (int32_t v = 0; v < sn; v++) if (alive[v]) best[map[v]] = 1;
                    }
                    k++;
                }
            }
        }
        lister_free(&L);
        free(deg); free(alive); free(queued); free(queue);
        orc_graph_free(s);
        if (literal) {
            int64_t next = 2 * alive_cnt;   /* 2|W| after the deletions */
            wsize = next > n ? n : next;
        } else {
            if (wsize >= n) break;
            if (gamma[order[wsize]] < kmax) break;
            wsize = 2 * wsize > n ? n : 2 * wsize;
        }
    }
    *kmax_out = kmax;
    {
        uint64_t size = 0;
        for (int32_t v = 0; v < n; v++) size += member[v];
        if (size > 0) {
            u128 mu;
            rc = count_cliques(g, h, member, &mu);
            if (rc) goto done;
            if (mu > (u128)UINT64_MAX) { rc = ORC_EOVERFLOW; goto done; }
            *num = (uint64_t)mu;
            *den = size;
            reduce(num, den);
        }
    }
done:
    free(x); free(gamma); free(order); free(inW); free(map);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Alg. 2 (PeelApp)                                                      */
/* S starts as G; a step removes vertices of minimum clique-degree in S   */
/* and every h-clique through them.  The answer is the densest of the     */
/* residual graphs seen before each step (G included), the first one      */
/* when several tie.  rounds = 0: one vertex per step, the smallest id     */
/* among the minima (Alg. 2 as printed).  rounds = 1: every vertex at the  */
/* minimum leaves in the same step.                                       */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t *deg; uint64_t destroyed; int32_t v; } papctx;

static void emit_remove(void *c, const int32_t *mem, int size) {
    papctx *p = (papctx *)c;
    for (int i = 0; i < size; i++)
        if (mem[i] != p->v) p->deg[mem[i]]--;
    p->destroyed++;
}

int orc_peel_app(const orc_graph *g, int h, int rounds, uint8_t *member,
                 uint64_t *num, uint64_t *den, int64_t *steps, int64_t *best_step) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    int32_t n = g->n;
    memset(member, 0, (size_t)n);
    *num = 0; *den = 1; *steps = 0; *best_step = -1;
    uint64_t *deg = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint8_t *alive = (uint8_t *)malloc((size_t)n + 1);
    int64_t *gone = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *F = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!deg || !alive || !gone || !F) { free(deg); free(alive); free(gone); free(F); return ORC_ENOMEM; }
    uint64_t mu;
    int rc = orc_clique_degrees(g, h, deg, &mu);
    if (rc) { free(deg); free(alive); free(gone); free(F); return rc; }
    papctx pc = {deg, 0, -1};
    lister L;
    if (lister_init(&L, g, h, emit_remove, &pc)) {
        lister_free(&L); free(deg); free(alive); free(gone); free(F); return ORC_ENOMEM;
    }
    for (int32_t v = 0; v < n; v++) { alive[v] = 1; gone[v] = -1; }
    uint64_t size = (uint64_t)n, bn = 0, bd = 1;
    int64_t t = 0;
    while (size > 0) {
        /* the residual graph S before this step: |S| = size, mu(S) = mu */
        if (frac_gt(mu, size, bn, bd)) { bn = mu; bd = size; *best_step = t; }
        uint64_t mn = UINT64_MAX;
        for (int32_t v = 0; v < n; v++)
            if (alive[v] && deg[v] < mn) mn = deg[v];
        int32_t nf = 0;
        for (int32_t v = 0; v < n; v++)
            if (alive[v] && deg[v] == mn) {
                F[nf++] = v;
                if (!rounds) break;
            }
        /* remove F one vertex after another: a clique with several members
         * in F is listed (and destroyed) once, from the first of them */
        for (int32_t i = 0; i < nf; i++) {
            pc.v = F[i];
            pc.destroyed = 0;
            list_containing(&L, F[i], alive);
            alive[F[i]] = 0;
            gone[F[i]] = t;
            mu -= pc.destroyed;
            size--;
        }
        t++;
    }
    lister_free(&L);
    *steps = t;
    if (*best_step >= 0 && bn > 0) {
        for (int32_t v = 0; v < n; v++) member[v] = gone[v] >= *best_step ? 1 : 0;
        *num = bn; *den = bd;
        reduce(num, den);
    } else {
        *best_step = -1;
    }
    free(deg); free(alive); free(gone); free(F);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Special patterns (the appendix on core decomposition for special        */
/* patterns).  An x-star (x >= 2) is a centre joined to x tails; a 4-loop  */
/* is a cycle on four vertices (the appendix's "diamond": two 2-paths from */
/* a vertex to the same 2-hop neighbour).  Instances are subgraphs, not    */
/* necessarily induced.  Degrees and cores come from listing instances.    */
/* ------------------------------------------------------------------ */

#define ORC_STAR 1
#define ORC_LOOP4 2

typedef void (*pemit_fn)(void *ctx, const int32_t *mem, int size);

/* every k-subset of cand[0..nc) after buf[0..np), emitted as buf[0..np+k) */
static void subsets_rec(const int32_t *cand, int nc, int k, int start, int32_t *buf, int np, int depth,
                        pemit_fn emit, void *ctx) {
    if (depth == k) { emit(ctx, buf, np + k); return; }
    for (int i = start; i <= nc - (k - depth); i++) {
        buf[np + depth] = cand[i];
        subsets_rec(cand, nc, k, i + 1, buf, np, depth + 1, emit, ctx);
    }
}

static int is_alive(const uint8_t *alive, int32_t v) { return !alive || alive[v]; }

/* x-stars containing v among alive vertices: v as the centre, or v as a
 * tail of an alive neighbour c; each instance once (its centre is unique) */
static void star_containing(const orc_graph *g, int x, int32_t v, const uint8_t *alive, int32_t *cand,
                            int32_t *buf, pemit_fn emit, void *ctx) {
    int nc = 0;
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
        if (is_alive(alive, g->adj[e])) cand[nc++] = g->adj[e];
    buf[0] = v;
    subsets_rec(cand, nc, x, 0, buf, 1, 0, emit, ctx);
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
        int32_t c = g->adj[e];
        if (!is_alive(alive, c)) continue;
        int n2 = 0;
        for (int64_t f = g->off[c]; f < g->off[c + 1]; f++)
            if (g->adj[f] != v && is_alive(alive, g->adj[f])) cand[n2++] = g->adj[f];
        buf[0] = c;
        buf[1] = v;
        subsets_rec(cand, n2, x - 1, 0, buf, 2, 0, emit, ctx);
    }
}

/* 4-loops containing v among alive vertices: v's two loop neighbours a < b
 * and the vertex w opposite v (a common neighbour of a and b); each once */
static void loop4_containing(const orc_graph *g, int32_t v, const uint8_t *alive, int32_t *cand, int32_t *tmp,
                             pemit_fn emit, void *ctx) {
    int nc = 0;
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
        if (is_alive(alive, g->adj[e])) cand[nc++] = g->adj[e];
    for (int i = 0; i < nc; i++)
        for (int j = i + 1; j < nc; j++) {
            int32_t a = cand[i], b = cand[j];
            int64_t k = intersect(g->adj + g->off[a], g->off[a + 1] - g->off[a], g->adj + g->off[b],
                                  g->off[b + 1] - g->off[b], tmp);
            for (int64_t t = 0; t < k; t++) {
                int32_t w = tmp[t];
                if (w == v || !is_alive(alive, w)) continue;
                int32_t mem[4] = {v, a, w, b};
                emit(ctx, mem, 4);
            }
        }
}

/* every instance of the pattern in g, each once */
static void pattern_all(const orc_graph *g, int pattern, int x, int32_t *cand, int32_t *tmp, int32_t *buf,
                        pemit_fn emit, void *ctx) {
    for (int32_t v = 0; v < g->n; v++) {
        if (pattern == ORC_STAR) {
            int nc = 0;
            for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) cand[nc++] = g->adj[e];
            buf[0] = v;
            subsets_rec(cand, nc, x, 0, buf, 1, 0, emit, ctx);      /* v as the centre */
        } else {
            /* loops whose smallest vertex is v: neighbours a < b above v, w above v */
            int nc = 0;
            for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
                if (g->adj[e] > v) cand[nc++] = g->adj[e];
            for (int i = 0; i < nc; i++)
                for (int j = i + 1; j < nc; j++) {
                    int32_t a = cand[i], b = cand[j];
                    int64_t k = intersect(g->adj + g->off[a], g->off[a + 1] - g->off[a], g->adj + g->off[b],
                                          g->off[b + 1] - g->off[b], tmp);
                    for (int64_t t = 0; t < k; t++)
                        if (tmp[t] > v) {
                            int32_t mem[4] = {v, a, tmp[t], b};
                            emit(ctx, mem, 4);
                        }
                }
        }
    }
}

static int pattern_args(const orc_graph *g, int pattern, int x) {
    if (pattern == ORC_STAR) return (x >= 2 && x <= 8) ? ORC_OK : ORC_EINVAL;
    if (pattern == ORC_LOOP4) return g ? ORC_OK : ORC_EINVAL;
    return ORC_EINVAL;
}

typedef struct { int32_t *cand, *tmp, *buf; } pbufs;

static int pbufs_init(pbufs *B, const orc_graph *g) {
    int32_t d = max_degree(g) + 2;
    B->cand = (int32_t *)malloc((size_t)d * sizeof(int32_t));
    B->tmp = (int32_t *)malloc((size_t)d * sizeof(int32_t));
    B->buf = (int32_t *)malloc((size_t)(ORC_HMAX + 2) * sizeof(int32_t));
    return (B->cand && B->tmp && B->buf) ? ORC_OK : ORC_ENOMEM;
}
static void pbufs_free(pbufs *B) { free(B->cand); free(B->tmp); free(B->buf); }

int orc_pattern_degrees(const orc_graph *g, int pattern, int x, uint64_t *deg, uint64_t *count) {
    int rc = pattern_args(g, pattern, x);
    if (rc) return rc;
    for (int32_t v = 0; v < g->n; v++) deg[v] = 0;
    degctx d = {deg, 0, 0};
    pbufs B;
    if (pbufs_init(&B, g)) { pbufs_free(&B); return ORC_ENOMEM; }
    pattern_all(g, pattern, x, B.cand, B.tmp, B.buf, emit_degree, &d);
    pbufs_free(&B);
    if (d.overflow || d.mu > (u128)UINT64_MAX) return ORC_EOVERFLOW;
    *count = (uint64_t)d.mu;
    return ORC_OK;
}

/* Alg. 3 with pattern instances in place of cliques: pop the vertex of
 * least pattern-degree, record it, and take one unit from every other
 * member (of larger degree) of every instance through it among the
 * remaining vertices. */
int orc_pattern_core(const orc_graph *g, int pattern, int x, uint64_t *core, uint64_t *kmax) {
    int32_t n = g->n;
    uint64_t cnt;
    uint64_t *deg = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint8_t *alive = (uint8_t *)malloc((size_t)n + 1);
    int32_t *hp = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *pos = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    pbufs B;
    int rc = (deg && alive && hp && pos) ? pbufs_init(&B, g) : ORC_ENOMEM;
    if (!rc) rc = orc_pattern_degrees(g, pattern, x, deg, &cnt);
    if (rc) { free(deg); free(alive); free(hp); free(pos); pbufs_free(&B); return rc; }
    iheap H = {deg, hp, pos, n};
    for (int32_t v = 0; v < n; v++) { hp[v] = v; pos[v] = v; alive[v] = 1; }
    for (int32_t i = n / 2 - 1; i >= 0; i--) hdown(&H, i);
    peelctx pc = {deg, &H, -1};
    uint64_t km = 0;
    while (H.size > 0) {
        int32_t v = hpop(&H);
        core[v] = deg[v];
        if (deg[v] > km) km = deg[v];
        pc.v = v;
        if (pattern == ORC_STAR) star_containing(g, x, v, alive, B.cand, B.buf, emit_peel, &pc);
        else loop4_containing(g, v, alive, B.cand, B.tmp, emit_peel, &pc);
        alive[v] = 0;
    }
    *kmax = km;
    free(deg); free(alive); free(hp); free(pos); pbufs_free(&B);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Pruning1 / Pruning2 (Section 6.1)                                     */
/* ------------------------------------------------------------------ */

/* components of the subgraph induced by mask; label[v] = -1 outside */
static int64_t components(const orc_graph *g, const uint8_t *mask, int32_t *label) {
    int32_t n = g->n;
    int32_t *queue = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) label[v] = -1;
    int64_t nc = 0;
    for (int32_t r = 0; r < n; r++) {
        if (!mask[r] || label[r] >= 0) continue;
        int64_t qh = 0, qt = 0;
        queue[qt++] = r;
        label[r] = (int32_t)nc;
        while (qh < qt) {
            int32_t v = queue[qh++];
            for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
                int32_t w = g->adj[e];
                if (mask[w] && label[w] < 0) { label[w] = (int32_t)nc; queue[qt++] = w; }
            }
        }
        nc++;
    }
    free(queue);
    return nc;
}

typedef struct { const int32_t *label; u128 *mu; } compctx;
static void emit_comp(void *c, const int32_t *mem, int size) {
    compctx *cc = (compctx *)c;
    for (int i = 0; i < size; i++) if (cc->label[mem[i]] < 0) return;
    cc->mu[cc->label[mem[0]]]++;
}

/* mu of every component (cliques whose members are all labelled) */
static int component_mu(const orc_graph *g, int h, const int32_t *label, int64_t nc, u128 *mu) {
    for (int64_t i = 0; i < nc; i++) mu[i] = 0;
    compctx c = {label, mu};
    lister L;
    if (lister_init(&L, g, h, emit_comp, &c)) { lister_free(&L); return ORC_ENOMEM; }
    list_all(&L);
    lister_free(&L);
    return ORC_OK;
}

int orc_locate(const orc_graph *g, int h, const uint64_t *core,
               uint64_t *rho1_num, uint64_t *rho1_den, uint64_t *k1,
               uint64_t *rho2_num, uint64_t *rho2_den, uint64_t *k2,
               int32_t *label, int64_t *ncomp) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    int32_t n = g->n;
    uint64_t *levels = (uint64_t *)malloc(((size_t)n + 2) * sizeof(uint64_t));
    uint64_t *rsize = (uint64_t *)malloc(((size_t)n + 2) * sizeof(uint64_t));
    uint64_t *rmu = (uint64_t *)malloc(((size_t)n + 2) * sizeof(uint64_t));
    uint8_t *mask = (uint8_t *)malloc((size_t)n + 1);
    if (!levels || !rsize || !rmu || !mask) { free(levels); free(rsize); free(rmu); free(mask); return ORC_ENOMEM; }
    int64_t nl;
    int rc = orc_level_table(g, h, core, levels, rsize, rmu, &nl);
    if (rc) goto out;
    /* rho' = max_k mu(R_k)/|R_k| */
    uint64_t a = 0, b = 1;
    for (int64_t i = 0; i < nl; i++)
        if (rsize[i] > 0 && frac_gt(rmu[i], rsize[i], a, b)) { a = rmu[i]; b = rsize[i]; }
    reduce(&a, &b);
    *rho1_num = a; *rho1_den = b;
    *k1 = frac_ceil(a, b);
    for (int32_t v = 0; v < n; v++) mask[v] = core[v] >= *k1;
    int64_t nc = components(g, mask, label);
    *ncomp = nc;
    u128 *mu = (u128 *)calloc((size_t)nc + 1, sizeof(u128));
    uint64_t *size = (uint64_t *)calloc((size_t)nc + 1, sizeof(uint64_t));
    if (!mu || !size) { free(mu); free(size); rc = ORC_ENOMEM; goto out; }
    for (int32_t v = 0; v < n; v++) if (label[v] >= 0) size[label[v]]++;
    rc = component_mu(g, h, label, nc, mu);
    uint64_t c = 0, d = 1;
    for (int64_t i = 0; i < nc; i++)
        if ((u128)mu[i] * d > (u128)c * size[i]) { c = (uint64_t)mu[i]; d = size[i]; }
    reduce(&c, &d);
    *rho2_num = c; *rho2_den = d;
    uint64_t kk = frac_ceil(c, d);
    *k2 = kk > *k1 ? kk : *k1;
    free(mu); free(size);
out:
    free(levels); free(rsize); free(rmu); free(mask);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Flow networks and Dinic's maximum flow (exact, 128-bit)               */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t nn, na, cap_na;
    int64_t *head, *nxt, *it;
    int64_t *to;
    i128 *cap;
    int64_t *level, *queue;
} flownet;

static int fn_init(flownet *F, int64_t nodes, int64_t arcs_hint) {
    memset(F, 0, sizeof(*F));
    F->nn = nodes;
    F->cap_na = arcs_hint > 16 ? arcs_hint : 16;
    F->head = (int64_t *)malloc((size_t)nodes * sizeof(int64_t));
    F->it = (int64_t *)malloc((size_t)nodes * sizeof(int64_t));
    F->level = (int64_t *)malloc((size_t)nodes * sizeof(int64_t));
    F->queue = (int64_t *)malloc((size_t)nodes * sizeof(int64_t));
    F->nxt = (int64_t *)malloc((size_t)F->cap_na * sizeof(int64_t));
    F->to = (int64_t *)malloc((size_t)F->cap_na * sizeof(int64_t));
    F->cap = (i128 *)malloc((size_t)F->cap_na * sizeof(i128));
    if (!F->head || !F->it || !F->level || !F->queue || !F->nxt || !F->to || !F->cap) return ORC_ENOMEM;
    for (int64_t i = 0; i < nodes; i++) F->head[i] = -1;
    return ORC_OK;
}

static void fn_free(flownet *F) {
    free(F->head); free(F->it); free(F->level); free(F->queue);
    free(F->nxt); free(F->to); free(F->cap);
}

static int fn_arc(flownet *F, int64_t u, int64_t v, i128 c) {
    if (F->na + 2 > F->cap_na) {
        int64_t nc = F->cap_na * 2;
        int64_t *nx = (int64_t *)realloc(F->nxt, (size_t)nc * sizeof(int64_t));
        if (nx) F->nxt = nx;
        int64_t *nt = (int64_t *)realloc(F->to, (size_t)nc * sizeof(int64_t));
        if (nt) F->to = nt;
        i128 *ncp = (i128 *)realloc(F->cap, (size_t)nc * sizeof(i128));
        if (ncp) F->cap = ncp;
        if (!nx || !nt || !ncp) return ORC_ENOMEM;
        F->cap_na = nc;
    }
    int64_t e = F->na;
    F->to[e] = v; F->cap[e] = c; F->nxt[e] = F->head[u]; F->head[u] = e;
    F->to[e + 1] = u; F->cap[e + 1] = 0; F->nxt[e + 1] = F->head[v]; F->head[v] = e + 1;
    F->na += 2;
    return ORC_OK;
}

static int fn_bfs(flownet *F, int64_t s, int64_t t) {
    for (int64_t i = 0; i < F->nn; i++) F->level[i] = -1;
    int64_t qh = 0, qt = 0;
    F->queue[qt++] = s;
    F->level[s] = 0;
    while (qh < qt) {
        int64_t v = F->queue[qh++];
        for (int64_t e = F->head[v]; e >= 0; e = F->nxt[e])
            if (F->cap[e] > 0 && F->level[F->to[e]] < 0) {
                F->level[F->to[e]] = F->level[v] + 1;
                F->queue[qt++] = F->to[e];
            }
    }
    return F->level[t] >= 0;
}

static i128 fn_dfs(flownet *F, int64_t v, int64_t t, i128 f) {
    if (v == t) return f;
    for (; F->it[v] >= 0; F->it[v] = F->nxt[F->it[v]]) {
        int64_t e = F->it[v], w = F->to[e];
        if (F->cap[e] > 0 && F->level[w] == F->level[v] + 1) {
            i128 d = fn_dfs(F, w, t, f < F->cap[e] ? f : F->cap[e]);
            if (d > 0) {
                F->cap[e] -= d;
                F->cap[e ^ 1] += d;
                return d;
            }
        }
    }
    return 0;
}

static void fn_maxflow(flownet *F, int64_t s, int64_t t) {
    const i128 big = ((i128)1) << 120;
    while (fn_bfs(F, s, t)) {
        for (int64_t i = 0; i < F->nn; i++) F->it[i] = F->head[i];
        while (fn_dfs(F, s, t, big) > 0) {}
    }
}

/* source side of the minimal minimum cut: residual reachability from s */
static void fn_source_side(flownet *F, int64_t s, uint8_t *side) {
    for (int64_t i = 0; i < F->nn; i++) side[i] = 0;
    int64_t qh = 0, qt = 0;
    F->queue[qt++] = s;
    side[s] = 1;
    while (qh < qt) {
        int64_t v = F->queue[qh++];
        for (int64_t e = F->head[v]; e >= 0; e = F->nxt[e])
            if (F->cap[e] > 0 && !side[F->to[e]]) { side[F->to[e]] = 1; F->queue[qt++] = F->to[e]; }
    }
}

/* (h-1)-cliques of a graph, in the order the ordered lister produces
 * (lexicographic in the sorted member tuples) */
typedef struct { int32_t *tuples; int64_t n, cap; int r; int fail; } tupctx;
static void emit_tuple(void *c, const int32_t *mem, int size) {
    tupctx *t = (tupctx *)c;
    if (t->n + 1 > t->cap) {
        int64_t nc = t->cap ? t->cap * 2 : 1024;
        int32_t *p = (int32_t *)realloc(t->tuples, (size_t)nc * (size_t)t->r * sizeof(int32_t));
        if (!p) { t->fail = 1; return; }
        t->tuples = p; t->cap = nc;
    }
    memcpy(t->tuples + t->n * t->r, mem, (size_t)size * sizeof(int32_t));
    t->n++;
}

static int tuple_cmp(const int32_t *a, const int32_t *b, int r) {
    for (int i = 0; i < r; i++) if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

static int64_t tuple_find(const tupctx *t, const int32_t *key) {
    int64_t lo = 0, hi = t->n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = tuple_cmp(t->tuples + mid * t->r, key, t->r);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

typedef struct { flownet *F; const tupctx *lam; int64_t base; i128 unit; int h; int fail; } netctx;
/* for every h-clique K and member v: arc v -> (K \ {v}) of capacity `unit` */
static void emit_net(void *c, const int32_t *mem, int size) {
    netctx *nc = (netctx *)c;
    int32_t key[ORC_HMAX];
    for (int drop = 0; drop < size; drop++) {
        int r = 0;
        for (int i = 0; i < size; i++) if (i != drop) key[r++] = mem[i];
        int64_t id = tuple_find(nc->lam, key);
        if (id < 0) { nc->fail = 1; return; }
        if (fn_arc(nc->F, 2 + mem[drop], nc->base + id, nc->unit)) nc->fail = 1;
    }
}

/* Strict test on graph s for alpha = a/b: is there a subgraph of density
 * > alpha?  Alg. 1's network scaled by b (h >= 3), or Goldberg's network
 * scaled by b (h = 2).  side_v[v] = 1 for v on the source side.  forced
 * (may be NULL): vertices whose source arc is infinite, so that every cut of
 * finite capacity keeps them on the source side (then *found only says the
 * side is non-empty; the caller compares densities). */
static int denser_than_forced(const orc_graph *s, int h, uint64_t a, uint64_t b, const uint8_t *forced,
                              uint8_t *side_v, int *found) {
    int32_t n = s->n;
    *found = 0;
    for (int32_t v = 0; v < n; v++) side_v[v] = 0;
    if (n == 0) return ORC_OK;
    flownet F;
    int rc;
    uint8_t *side = NULL;
    tupctx lam = {NULL, 0, 0, h - 1, 0};
    if (h == 2) {
        int64_t nodes = 2 + (int64_t)n;
        rc = fn_init(&F, nodes, 2 * (int64_t)n + 2 * s->off[n] + 8);
        if (rc) { fn_free(&F); return rc; }
        i128 M = (i128)s->m;
        /* infinity: more than the sum of every finite capacity */
        i128 inf = 1;
        for (int32_t v = 0; v < n; v++)
            inf += 2 * (i128)b * M + 2 * (i128)a + (i128)b * (i128)(s->off[v + 1] - s->off[v]);
        for (int32_t v = 0; v < n; v++) {
            i128 dv = (i128)(s->off[v + 1] - s->off[v]);
            rc |= fn_arc(&F, 0, 2 + v, forced && forced[v] ? inf : (i128)b * M);
            rc |= fn_arc(&F, 2 + v, 1, (i128)b * M + 2 * (i128)a - (i128)b * dv);
            for (int64_t e = s->off[v]; e < s->off[v + 1]; e++)
                rc |= fn_arc(&F, 2 + v, 2 + s->adj[e], (i128)b);
        }
    } else {
        uint64_t *deg = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
        uint64_t mu;
        rc = deg ? orc_clique_degrees(s, h, deg, &mu) : ORC_ENOMEM;
        if (rc) { free(deg); return rc; }
        lister L;
        if (lister_init(&L, s, h - 1, emit_tuple, &lam)) { lister_free(&L); free(deg); return ORC_ENOMEM; }
        list_all(&L);
        lister_free(&L);
        if (lam.fail) { free(deg); free(lam.tuples); return ORC_ENOMEM; }
        int64_t base = 2 + (int64_t)n;
        int64_t nodes = base + lam.n;
        rc = fn_init(&F, nodes, 2 * (2 * (int64_t)n + (int64_t)h * (int64_t)mu + (int64_t)(h - 1) * lam.n) + 8);
        if (rc) { fn_free(&F); free(deg); free(lam.tuples); return rc; }
        /* infinity: more than the sum of every finite capacity */
        u128 fin = 0;
        for (int32_t v = 0; v < n; v++) fin += (u128)b * deg[v] + (u128)h * a;
        fin += (u128)b * (u128)h * (u128)mu;
        if (fin >= ((u128)1) << 118) { fn_free(&F); free(deg); free(lam.tuples); return ORC_EOVERFLOW; }
        i128 inf = (i128)fin + 1;
        for (int32_t v = 0; v < n; v++) {
            rc |= fn_arc(&F, 0, 2 + v, forced && forced[v] ? inf : (i128)b * (i128)deg[v]);
            rc |= fn_arc(&F, 2 + v, 1, (i128)h * (i128)a);
        }
        for (int64_t i = 0; i < lam.n; i++)
            for (int j = 0; j < h - 1; j++)
                rc |= fn_arc(&F, base + i, 2 + lam.tuples[i * (h - 1) + j], inf);
        netctx nc = {&F, &lam, base, (i128)b, h, 0};
        if (lister_init(&L, s, h, emit_net, &nc)) { lister_free(&L); fn_free(&F); free(deg); free(lam.tuples); return ORC_ENOMEM; }
        list_all(&L);
        lister_free(&L);
        if (nc.fail) rc = ORC_ENOMEM;
        free(deg);
    }
    if (!rc) {
        fn_maxflow(&F, 0, 1);
        side = (uint8_t *)malloc((size_t)F.nn);
        if (!side) rc = ORC_ENOMEM;
        else {
            fn_source_side(&F, 0, side);
            for (int32_t v = 0; v < n; v++) {
                side_v[v] = side[2 + v];
                if (side_v[v]) *found = 1;
            }
        }
    }
    free(side);
    free(lam.tuples);
    fn_free(&F);
    return rc;
}

static int denser_than(const orc_graph *s, int h, uint64_t a, uint64_t b, uint8_t *side_v, int *found) {
    return denser_than_forced(s, h, a, b, NULL, side_v, found);
}

int orc_denser_than(const orc_graph *g, int h, uint64_t a, uint64_t b, uint8_t *member) {
    if (h < 2 || h > ORC_HMAX || b == 0) return ORC_EINVAL;
    int found;
    int rc = denser_than(g, h, a, b, member, &found);
    return rc ? rc : found;
}

/* strict test on G[mask]; result mask over G */
static int denser_than_in(const orc_graph *g, int h, const uint8_t *mask, uint64_t a, uint64_t b,
                          uint8_t *result, int *found, int64_t *calls) {
    int32_t n = g->n;
    int32_t *map = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!map) return ORC_ENOMEM;
    orc_graph *s = orc_graph_induced(g, mask, map);
    if (!s) { free(map); return ORC_ENOMEM; }
    uint8_t *sv = (uint8_t *)malloc((size_t)s->n + 1);
    int rc = sv ? denser_than(s, h, a, b, sv, found) : ORC_ENOMEM;
    (*calls)++;
    if (!rc) {
        memset(result, 0, (size_t)n);
        for (int32_t v = 0; v < s->n; v++) if (sv[v]) result[map[v]] = 1;
    }
    free(sv);
    orc_graph_free(s);
    free(map);
    return rc;
}

static int density_of(const orc_graph *g, int h, const uint8_t *mask, uint64_t *num, uint64_t *den) {
    uint64_t size = 0;
    for (int32_t v = 0; v < g->n; v++) size += mask[v] ? 1 : 0;
    if (size == 0) { *num = 0; *den = 1; return ORC_OK; }
    u128 mu;
    int rc = count_cliques(g, h, mask, &mu);
    if (rc) return rc;
    if (mu > (u128)UINT64_MAX) return ORC_EOVERFLOW;
    *num = (uint64_t)mu;
    *den = size;
    reduce(num, den);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Densest subgraph containing a query set Q (Section 6.3, the variant of  */
/* the problem).  Start from Q itself; while the minimum cut of the network */
/* with Q forced to the source side yields a set of density > l (its       */
/* source side maximises mu(S) - l|S| over S containing Q), move to it.    */
/* Densities strictly increase, so this ends, at the largest density of a  */
/* set containing Q.                                                       */
/* ------------------------------------------------------------------ */

int orc_exact_query(const orc_graph *g, int h, int32_t nq, const int32_t *q, uint8_t *member,
                    uint64_t *num, uint64_t *den, int64_t *flow_calls) {
    if (h < 2 || h > ORC_HMAX || nq < 1) return ORC_EINVAL;
    int32_t n = g->n;
    for (int32_t i = 0; i < nq; i++)
        if (q[i] < 0 || q[i] >= n) return ORC_EINVAL;
    uint8_t *forced = (uint8_t *)calloc((size_t)n + 1, 1);
    uint8_t *side = (uint8_t *)malloc((size_t)n + 1);
    if (!forced || !side) { free(forced); free(side); return ORC_ENOMEM; }
    for (int32_t i = 0; i < nq; i++) forced[q[i]] = 1;
    memcpy(member, forced, (size_t)n);
    int rc = density_of(g, h, member, num, den);
    *flow_calls = 0;
    while (!rc) {
        int found;
        rc = denser_than_forced(g, h, *num, *den, forced, side, &found);
        (*flow_calls)++;
        if (rc) break;
        uint64_t sn, sd;
        rc = density_of(g, h, side, &sn, &sd);
        if (rc || !frac_gt(sn, sd, *num, *den)) break;
        memcpy(member, side, (size_t)n);
        *num = sn;
        *den = sd;
    }
    free(forced);
    free(side);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Alg. 1 (Exact) and Alg. 4 (CoreExact)                                 */
/* alpha = p / Q on an integer grid; the search ends when p_u - p_l = 1, */
/* i.e. u - l = 1/Q with Q = s^2 < s(s-1)... strictly below the gap      */
/* 1/(s(s-1)) between distinct densities (Lemma 12), s = vertex count.   */
/* ------------------------------------------------------------------ */

static int exact_whole(const orc_graph *g, int h, uint8_t *member, uint64_t *num, uint64_t *den, int64_t *calls) {
    int32_t n = g->n;
    uint64_t *deg = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint8_t *all = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *cur = (uint8_t *)malloc((size_t)n + 1);
    if (!deg || !all || !cur) { free(deg); free(all); free(cur); return ORC_ENOMEM; }
    uint64_t mu;
    int rc = orc_clique_degrees(g, h, deg, &mu);
    memset(member, 0, (size_t)n);
    *num = 0; *den = 1;
    if (rc || mu == 0 || n < 2) goto out;
    uint64_t maxdeg = 0;
    for (int32_t v = 0; v < n; v++) { all[v] = 1; if (deg[v] > maxdeg) maxdeg = deg[v]; }
    u128 Q = (u128)n * (u128)n;
    u128 pl = 0, pu = (u128)maxdeg * Q;
    if (pu >> 63) { rc = ORC_EOVERFLOW; goto out; }
    while (pu - pl > 1) {
        u128 p = pl + (pu - pl) / 2;
        int found;
        rc = denser_than_in(g, h, all, (uint64_t)p, (uint64_t)Q, cur, &found, calls);
        if (rc) goto out;
        if (found) { pl = p; memcpy(member, cur, (size_t)n); }
        else pu = p;
    }
    rc = density_of(g, h, member, num, den);
out:
    free(deg); free(all); free(cur);
    return rc;
}

typedef struct { int64_t id; uint64_t mu, size; } compinfo;
static int cmp_comp(const void *a, const void *b) {
    const compinfo *x = (const compinfo *)a, *y = (const compinfo *)b;
    u128 l = (u128)x->mu * y->size, r = (u128)y->mu * x->size;
    if (l != r) return l > r ? -1 : 1;   /* denser first */
    return (x->id > y->id) - (x->id < y->id);
}

static int core_exact(const orc_graph *g, int h, uint8_t *member, uint64_t *num, uint64_t *den, int64_t *calls) {
    int32_t n = g->n;
    memset(member, 0, (size_t)n);
    *num = 0; *den = 1;
    uint64_t *core = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    int32_t *label1 = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *label2 = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    uint8_t *mask = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *cur = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *U = (uint8_t *)malloc((size_t)n + 1);
    compinfo *ci = NULL;
    u128 *cmu = NULL;
    int rc = ORC_OK;
    if (!core || !label1 || !label2 || !mask || !cur || !U) { rc = ORC_ENOMEM; goto out; }
    uint64_t kmax;
    rc = orc_core_decomposition(g, h, core, &kmax);
    if (rc) goto out;
    if (kmax == 0 || n < 2) goto out;            /* no clique at all */
    uint64_t r1n, r1d, k1, r2n, r2d, k2;
    int64_t nc1;
    rc = orc_locate(g, h, core, &r1n, &r1d, &k1, &r2n, &r2d, &k2, label1, &nc1);
    if (rc) goto out;
    /* D <- a component of R_{k'} attaining rho'' */
    {
        u128 *mu1 = (u128 *)calloc((size_t)nc1 + 1, sizeof(u128));
        uint64_t *sz1 = (uint64_t *)calloc((size_t)nc1 + 1, sizeof(uint64_t));
        if (!mu1 || !sz1) { free(mu1); free(sz1); rc = ORC_ENOMEM; goto out; }
        for (int32_t v = 0; v < n; v++) if (label1[v] >= 0) sz1[label1[v]]++;
        rc = component_mu(g, h, label1, nc1, mu1);
        int64_t best = -1;
        for (int64_t i = 0; i < nc1 && !rc; i++)
            if (sz1[i] > 0 && (u128)mu1[i] * r2d == (u128)r2n * sz1[i] && mu1[i] > 0) { best = i; break; }
        for (int32_t v = 0; v < n; v++) member[v] = (best >= 0 && label1[v] == best);
        free(mu1); free(sz1);
        if (rc) goto out;
    }
    uint64_t dn = r2n, dd = r2d;     /* density of D */
    /* components of R_{k''} (Alg. 4, line 3) in descending density */
    for (int32_t v = 0; v < n; v++) mask[v] = core[v] >= k2;
    int64_t nc = components(g, mask, label2);
    ci = (compinfo *)calloc((size_t)nc + 1, sizeof(compinfo));
    cmu = (u128 *)calloc((size_t)nc + 1, sizeof(u128));
    if (!ci || !cmu) { rc = ORC_ENOMEM; goto out; }
    rc = component_mu(g, h, label2, nc, cmu);
    if (rc) goto out;
    for (int64_t i = 0; i < nc; i++) { ci[i].id = i; ci[i].mu = (uint64_t)cmu[i]; ci[i].size = 0; }
    for (int32_t v = 0; v < n; v++) if (label2[v] >= 0) ci[label2[v]].size++;
    qsort(ci, (size_t)nc, sizeof(compinfo), cmp_comp);
    uint64_t la = dn, lb = dd;          /* l as a rational */
    for (int64_t c = 0; c < nc; c++) {
        /* C, shrunk to the ceil(l)-core when l > k'' */
        uint64_t cl = frac_ceil(la, lb);
        uint64_t floor_k = cl > k2 ? cl : k2;
        uint64_t s0 = 0, kC = 0;
        for (int32_t v = 0; v < n; v++) {
            mask[v] = label2[v] == ci[c].id && core[v] >= floor_k;
            if (mask[v]) { s0++; if (core[v] > kC) kC = core[v]; }
        }
        if (s0 < 2) continue;
        int found;
        rc = denser_than_in(g, h, mask, la, lb, U, &found, calls);
        if (rc) goto out;
        if (!found) continue;                    /* cannot beat l */
        u128 Q = (u128)s0 * (u128)s0;
        u128 pl = (u128)la * Q / lb;             /* floor(l Q): p_l/Q <= l */
        u128 pu = (u128)kC * Q;                  /* Lemma 5 on C */
        if (pu >> 63) { rc = ORC_EOVERFLOW; goto out; }
        uint64_t pruned = floor_k;
        while (pu - pl > 1) {
            u128 p = pl + (pu - pl) / 2;
            rc = denser_than_in(g, h, mask, (uint64_t)p, (uint64_t)Q, cur, &found, calls);
            if (rc) goto out;
            if (!found) { pu = p; continue; }
            pl = p;
            memcpy(U, cur, (size_t)n);
            /* every vertex of the found set has clique-degree > alpha inside
             * it, so the search can stay inside the ceil(alpha)-core */
            uint64_t ca = (uint64_t)((p + Q - 1) / Q);
            if (ca > pruned) {
                pruned = ca;
                for (int32_t v = 0; v < n; v++) if (mask[v] && core[v] < pruned) mask[v] = 0;
            }
        }
        uint64_t un, ud;
        rc = density_of(g, h, U, &un, &ud);
        if (rc) goto out;
        if (frac_gt(un, ud, dn, dd)) {
            memcpy(member, U, (size_t)n);
            dn = un; dd = ud;
        }
        la = dn; lb = dd;
    }
    *num = dn; *den = dd;
    reduce(num, den);
out:
    free(core); free(label1); free(label2); free(mask); free(cur); free(U); free(ci); free(cmu);
    return rc;
}

int orc_exact(const orc_graph *g, int h, int route, uint8_t *member,
              uint64_t *num, uint64_t *den, int64_t *flow_calls) {
    if (h < 2 || h > ORC_HMAX) return ORC_EINVAL;
    *flow_calls = 0;
    if (route == 0) return exact_whole(g, h, member, num, den, flow_calls);
    return core_exact(g, h, member, num, den, flow_calls);
}
