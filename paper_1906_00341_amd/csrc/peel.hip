// K4: round-synchronous (k, Psi)-core peel (Definition 6, Algorithm 3).
//
// Algorithm 3 removes one minimum-clique-degree vertex at a time.  Here a
// round removes every alive vertex whose current clique-degree is <= k at
// once (the frontier F); core numbers are unique, so the result is the same.
// Each alive clique with a member in F is destroyed exactly once: it is
// listed from the frontier member with the smallest rank (the owner rule),
// and each surviving member loses one unit of clique-degree.  A survivor
// whose degree drops from > k to <= k joins the next frontier with core k.
// When no frontier is left, k jumps to the smallest alive degree (a new
// level; no level in between can remove anything).
//
// In the min-degree mode (PeelApp, Algorithm 2) every round is a level of
// its own: the frontier is the alive vertices at the graph's smallest
// clique-degree, survivors only lose degree (they never join the next
// frontier), core[] receives each vertex's removal round, and the level
// table holds |S| and mu(S) of the residual graph before every round.
//
// With triangle lists (h = 3) a round walks the stored triangles {v, a, b}
// of every frontier vertex v instead of intersecting neighbourhoods; the
// owner rule picks the same destroyer, and each neighbour's losses are summed
// over its run of pairs before they reach its degree.  A row is cut into
// items of TL_CHUNK pairs, so a hub's triangles spread over many waves.
//
// For an x-star pattern (the appendix on special patterns) a round works from
// the closed form deg(w) = C(y_w, x) + sum over neighbours u of C(y_u - 1,
// x - 1), y the residual degrees: after the frontier F leaves, a survivor w
// loses C(y_w, x) - C(y'_w, x), C(y_f - 1, x - 1) for every neighbour f in
// F, and C(y_u - 1, x - 1) - C(y'_u - 1, x - 1) for every surviving
// neighbour u whose degree fell (primes: after the round).  k_star_front
// walks the frontier's edges (degree drops, the middle term), k_star_touch
// the rows of the survivors whose degree fell (the other two).
//
// For the 4-loop pattern (a cycle on four vertices; the appendix's diamond,
// two 2-paths from a vertex to the same vertex) a round takes one workgroup
// per frontier vertex v: its 2-hop neighbours w are counted in a hash of
// the workgroup's own (the common neighbours through which v reaches w),
// each group of c 2-paths holds C(c, 2) loops, and under the owner rule v
// destroys them: w loses C(c, 2), every middle vertex c - 1.
//
// A batch of graphs is peeled as one disjoint union in which every graph
// keeps its own level k (GraphState): cliques never cross graphs, so each
// graph's peel is exactly its own, and one round advances all of them.
//
// State lives on the device (PeelCtl, GraphState).  One round is a fixed
// sequence of grid-wide kernels (level-min, level-build, process, finish)
// that read the state themselves, so the host enqueues many rounds without
// waiting.  For h = 3 a large frontier vertex is split into items of CHUNK
// neighbours plus one item per neighbour with a long out-list, so that even a
// round that removes a single hub keeps thousands of waves busy; its
// neighbourhood hash sits in global memory, shared by those items.
#include <hip/hip_ext.h>

#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "engine.hpp"
#include "graph.hpp"

namespace dsd {

struct PeelCtl {
    int64_t n_alive;   // alive vertices over all graphs (the host polls it)
    int32_t round;
    int32_t cur;       // frontier buffer in use
    int32_t nF[2];     // frontier sizes (all graphs)
    int32_t nB[2];     // chunk items of large frontier vertices (h = 3)
    int32_t nlist[2];  // alive-list sizes
    int32_t lcur;      // alive list in use
    int32_t nsel[2];   // graphs that open a level in the round using buffer 0 / 1
    int32_t nitems[8]; // (v, w) work items per class (h >= 4)
    int64_t htop[2];   // slots handed out in the global neighbourhood hashes (h = 3)
    int64_t nW;        // wide (v, w) items of this round (h = 3)
    int32_t nT[2];     // row items of the frontier (triangle lists)
    int32_t pending;   // tail mode: a round has been started and not yet finished
    int32_t nTouch;    // x-star pattern: survivors whose degree fell this round
    int32_t nBig[2];   // h >= 4 root mode: single-workgroup items of the frontier
    u64 work[4];       // main kernel's pairs, neighbours and (h >= 4) row entries, counting kernel's bitmap
                       // words, over the whole peel (when counted)
};

// one graph of the batch (a single graph is a batch of one)
struct GraphState {
    u64 k;             // current level
    u64 kcand;         // smallest alive degree, gathered when a level opens
    u64 mu_alive;      // cliques among the graph's alive vertices
    u64 destroyed;     // cliques destroyed in this round
    u64 destroyed_m;   // root mode: per-member counts of this round's cliques (each clique h - 1 times)
    int64_t n_alive;
    int64_t lv_base;   // first entry of the graph's level table
    int32_t nF[2];     // the graph's frontier sizes
    int32_t nlevels;
    int32_t sel;       // this round opens a new level (fixed for the whole round)
};

struct PeelBufs {
    PeelCtl *ctl;
    GraphState *gs;
    const int32_t *gid;  // [n] graph of every vertex (nullptr: one graph)
    int32_t G;
    const int64_t *row_ptr;
    const int32_t *col;
    const int64_t *dag_off;
    int32_t *stamp;    // ALIVE, removal round, or -1 (not taking part)
    u64 *deg;          // current clique-degree
    u64 *core;
    int32_t *F;        // [2][n] frontiers
    int64_t *B;        // [2][bcap] (v << 32 | chunk) for frontier vertices of degree > SMALL_DEG
    int64_t bcap;
    int32_t *lists;    // [2][n] alive lists
    u64 *lv_k, *lv_size, *lv_mu;  // level tables
    int32_t *item_v, *item_w;     // [5][cap] work items (h >= 4)
    int64_t item_cap;
    int32_t *hkey;     // [2][hcap] global hashes of N(v) for large frontier vertices (h = 3)
    uint32_t *hval;
    int64_t hcap;
    int64_t *hbase;    // [n] first slot of v's hash in its round's half
    int64_t *W;        // [wcap] wide items (v << 32 | w): w with a long out-list (h = 3)
    int64_t wcap;
    int32_t n;
    int32_t h;
    const int64_t *tvoff; // triangle lists (nullptr: none): row starts, (a, b) pairs
    const int32_t *tpairs;
    int64_t *T;          // [2][tcap] row items (v << 32 | chunk) of frontier vertices
    int64_t tcap;
    int32_t pattern;     // 0: cliques; 1: x-stars with px tails; 2: 4-loops
    int32_t px;
    int32_t *ydeg;       // x-star: residual degree, now and at the start of the round
    int32_t *yold;
    int32_t *tround;     // x-star: round in which the vertex's degree last fell
    int32_t *touch;      // x-star: this round's survivors whose degree fell
    int32_t *lkey;       // 4-loop: [blocks][lsize] hash of a frontier vertex's 2-hop neighbours
    uint32_t *lval;
    int64_t lsize;
    int32_t count_work;  // the main kernel adds up its pairs and neighbours
    int32_t minpeel;     // min-degree mode: every round removes the minimum-degree vertices
    const u64 *eset;     // h >= 4: open-addressing set of the edges among the peel's vertices
    int32_t eset_bits;   // (2^eset_bits slots, keys (lo << 32 | hi) in rank space)
    int32_t rootmode;    // h >= 4: the frontier vertices' own cliques (k_root_edges / k_root_count)
    int64_t *Big;        // [2][bigcap] root mode: (v << 32 | chunk) single-workgroup items
    int64_t bigcap;
    u64 *rbits;          // [2][rcap] root mode: bitmap rows of the sliced vertices' neighbourhoods
    int64_t rcap;
    int64_t *rbase;      // [n] first word of v's region in its round's half
};

constexpr int SMALL_DEG = 64;           // h = 3: larger frontier vertices are split into chunks
constexpr int CHUNK = 32;               // neighbours per chunk item (one wave)
constexpr int SLOTS_PER_CHUNK = 64;     // global hash slots per chunk (load factor <= 1/2)
constexpr int WIDE_OUT = 32;            // neighbours w with |N+(w)| >= this get a wave of their own
constexpr int SMALL_HASH_BITS = 7;      // per-wave hash for degree <= SMALL_DEG
constexpr int TL_CHUNK = 128;           // pairs per row item (two per lane), triangle lists
constexpr int CHUNK4 = 64;              // h >= 4: neighbours per chunk item of a frontier vertex (one wave)
constexpr int ROOT_CAP = 2048;          // h >= 4, root mode: members of C_v one workgroup holds
constexpr int ROOT_HB = 12;             // its hash: 2^12 >= 2 * ROOT_CAP slots
constexpr int ROOT_SW = ROOT_CAP * 32;  // words of one workgroup's bitmap rows in global memory
constexpr int ROOT_SLICE = ROOT_SW + 32; // and their mask words
constexpr int ROOT_WAVE_MAX = 64;       // rows up to this long: one wave per frontier vertex
constexpr int ROOT_SL = 64;             // members of C_v per item of a sliced vertex (a slice)
constexpr int ROOT_SLICED_H4 = 4096;    // h = 4: rows up to this long are sliced (64-word bitmap rows)
constexpr int ROOT_SUB = ROOT_SL / WAVES_PER_BLOCK;  // workgroups per slice: one wave per member

// words per bitmap row of a vertex whose row holds d entries (|C_v| <= d)
__device__ __forceinline__ int root_words(int64_t d) {
    return d <= 256 ? 4 : d <= 768 ? 12 : d <= 1280 ? 20 : d <= 2048 ? 32 : 64;
}
// the longest row a sliced vertex may have: at h = 4 the counting keeps no
// per-lane word arrays, so its rows may take 64 words
__device__ __forceinline__ int64_t root_sliced_max(int h) { return h == 4 ? ROOT_SLICED_H4 : ROOT_CAP; }
// words of a sliced vertex's region: one bitmap row per entry of v's row
// (d * W; bit j > i of row i: entries i and j are adjacent; only the words
// from i / 64 up are written), then the mask of the entries that take part
// in v's cliques (W)
__device__ __forceinline__ int64_t root_region(int64_t d) {
    const int W = root_words(d);
    return d * W + W;
}
constexpr u64 ESET_EMPTY = ~0ull;

// Edge membership for the h >= 4 peel: one probe sequence in a table of
// 64-bit keys instead of a binary search in a (possibly long) row.
__device__ __forceinline__ u64 eset_key(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((u64)lo << 32) | hi;
}
__device__ __forceinline__ u64 eset_slot(u64 key, int bits) { return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits); }
__device__ __forceinline__ bool eset_has(const u64 *t, int bits, int32_t a, int32_t b) {
    const u64 key = eset_key(a, b), mask = (1ull << bits) - 1ull;
    for (u64 i = eset_slot(key, bits);; i = (i + 1) & mask) {
        const u64 k = t[i];
        if (k == key) return true;
        if (k == ESET_EMPTY) return false;
    }
}

__device__ __forceinline__ int32_t graph_of(const PeelBufs &b, int32_t v) { return b.gid ? b.gid[v] : 0; }

// the level of graph g in the current round: a round that opens a level
// records it only when it finishes, so until then it is max(k, smallest
// alive degree)
__device__ __forceinline__ u64 level_of(const PeelBufs &b, int32_t g) {
    const GraphState &s = b.gs[g];
    if (!s.sel) return s.k;
    if (b.minpeel) return s.kcand;
    return s.k > s.kcand ? s.k : s.kcand;
}

// the alive list is copied (compacted) by level-build once more than an
// eighth of it are removed vertices; n_alive and the list length do not
// change between level-build and the end of the round, so every reader of
// this test agrees
__device__ __forceinline__ bool list_compacts(const PeelCtl *c) {
    const int32_t cnt = c->nlist[c->lcur];
    return (int64_t)(cnt - c->n_alive) * 8 > (int64_t)cnt;
}

// all lanes of the wave must call this together
__device__ __forceinline__ void wave_push(bool pred, int32_t val, int32_t *arr, int32_t *counter) {
    u64 m = __ballot(pred);
    if (!m) return;
    int leader = __builtin_ctzll(m);
    int32_t base = 0;
    if (lane() == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, WAVE);
    if (pred) arr[base + __popcll(m & lanemask_lt())] = val;
}

// all threads of the block call this together; one atomic per block
__device__ __forceinline__ void block_push(bool pred, int32_t val, int32_t *arr, int32_t *counter) {
    __shared__ int32_t sOff[WAVES_PER_BLOCK];
    __shared__ int32_t sBase;
    const u64 m = __ballot(pred);
    const int wv = threadIdx.x / WAVE;
    if (lane() == 0) sOff[wv] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t tot = 0;
        for (int i = 0; i < WAVES_PER_BLOCK; i++) {
            int32_t t = sOff[i];
            sOff[i] = tot;
            tot += t;
        }
        sBase = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    if (pred) arr[sBase + sOff[wv] + __popcll(m & lanemask_lt())] = val;
    __syncthreads();
}

// Per-graph counter increments: the lanes of a wave usually belong to one
// graph (the alive list runs in id order), so the wave adds once; otherwise
// every lane adds for itself.  All lanes call together; g < 0: nothing to
// add.  The counter of graph g is at base[g * stride].
template <typename T>
__device__ __forceinline__ void wave_add_by_graph(int32_t g, T *base, size_t stride) {
    const u64 act = __ballot(g >= 0);
    if (!act) return;
    const int first = __builtin_ctzll(act);
    const int32_t g0 = __shfl(g, first, WAVE);
    if (__ballot(g >= 0 && g != g0) == 0) {
        if (lane() == first) atomicAdd(base + (size_t)g0 * stride, (T)__popcll(act));
    } else if (g >= 0) {
        atomicAdd(base + (size_t)g * stride, (T)1);
    }
}

// chunk items of a large frontier vertex, and the slots of its neighbourhood
// hash (h = 3)
__device__ __forceinline__ void push_chunks(const PeelBufs &b, int32_t x, int which) {
    if (b.rootmode) {
        // root mode: a short row is one wave item (T); a row of at most
        // root_sliced_max entries gets bitmap rows in its half of the arena
        // and one item per ROOT_SL-member slice (B); a longer row, or one the
        // arena has no room for, a single-workgroup item per ROOT_CAP
        // neighbours (Big)
        const int64_t d = b.row_ptr[x + 1] - b.row_ptr[x];
        if (d == 0) return;
        if (d <= ROOT_WAVE_MAX) {
            const int32_t pos = atomicAdd(&b.ctl->nT[which], 1);
            b.T[(size_t)which * b.tcap + pos] = (int64_t)x << 32;
            return;
        }
        if (d <= root_sliced_max(b.h)) {
            const int64_t words = root_region(d);
            const int64_t off = (int64_t)atomicAdd((unsigned long long *)&b.ctl->htop[which], (unsigned long long)words);
            if (off + words <= b.rcap) {
                b.rbase[x] = off;
                const int32_t nsl = (int32_t)((d + ROOT_SL - 1) / ROOT_SL);
                const int32_t base = atomicAdd(&b.ctl->nB[which], nsl);
                int64_t *Bw = b.B + (size_t)which * b.bcap;
                for (int32_t c = 0; c < nsl; c++) Bw[base + c] = ((int64_t)x << 32) | c;
                return;
            }
        }
        const int32_t nc = (int32_t)((d + ROOT_CAP - 1) / ROOT_CAP);
        const int32_t base = atomicAdd(&b.ctl->nBig[which], nc);
        int64_t *Gw = b.Big + (size_t)which * b.bigcap;
        for (int32_t c = 0; c < nc; c++) Gw[base + c] = ((int64_t)x << 32) | c;
        return;
    }
    if (b.h >= 4) {
        // h >= 4: one item per CHUNK4 neighbours; k_peel_items expands them
        const int64_t d = b.row_ptr[x + 1] - b.row_ptr[x];
        if (d == 0) return;
        const int32_t nc = (int32_t)((d + CHUNK4 - 1) / CHUNK4);
        const int32_t base = atomicAdd(&b.ctl->nB[which], nc);
        int64_t *Bw = b.B + (size_t)which * b.bcap;
        for (int32_t c = 0; c < nc; c++) Bw[base + c] = ((int64_t)x << 32) | c;
        return;
    }
    if (b.h != 3) return;
    int64_t d = b.row_ptr[x + 1] - b.row_ptr[x];
    if (d <= SMALL_DEG) return;
    int32_t nc = (int32_t)((d + CHUNK - 1) / CHUNK);
    int32_t base = atomicAdd(&b.ctl->nB[which], nc);
    b.hbase[x] = (int64_t)atomicAdd((unsigned long long *)&b.ctl->htop[which],
                                    (unsigned long long)nc * SLOTS_PER_CHUNK);
    int64_t *Bw = b.B + (size_t)which * b.bcap;
    for (int32_t c = 0; c < nc; c++) Bw[base + c] = ((int64_t)x << 32) | c;
}

// Row items (triangle lists) of the vertices that join frontier `which`
// (pred), written where they join it: TL_CHUNK pairs of a row each, since a
// hub's row holds thousands of them.  The whole wave calls this; one scan
// over the lanes and one atomic give the joining vertices their ranges of
// items, which the wave then writes vertex by vertex.
__device__ __forceinline__ void wave_push_items(const PeelBufs &b, bool pred, int32_t v, int which) {
    const u64 m = __ballot(pred);
    if (!m) return;
    int32_t nc = 0;
    if (pred) nc = (int32_t)((b.tvoff[v + 1] - b.tvoff[v] + TL_CHUNK - 1) / TL_CHUNK);
    const int32_t inc = wave_incl_scan(nc);
    const int32_t tot = __shfl(inc, WAVE - 1, WAVE);
    if (tot == 0) return;
    int32_t base = 0;
    if (lane() == 0) base = atomicAdd(&b.ctl->nT[which], tot);
    base = __shfl(base, 0, WAVE) + inc - nc;
    int64_t *Tw = b.T + (size_t)which * b.tcap;
    for (u64 mm = m; mm; mm &= mm - 1) {
        const int j = __builtin_ctzll(mm);
        const int32_t vj = __shfl(v, j, WAVE), ncj = __shfl(nc, j, WAVE), bj = __shfl(base, j, WAVE);
        for (int32_t c = lane(); c < ncj; c += WAVE) Tw[bj + c] = ((int64_t)vj << 32) | c;
    }
}

// a frontier vertex's work items for the round's process kernels (with
// triangle lists they are written by wave_push_items where the vertex joins
// the frontier)
__device__ __forceinline__ void push_work(const PeelBufs &b, int32_t x, int which) {
    if (!b.tpairs) push_chunks(b, x, which);
}

// a survivor x loses c cliques; if that takes it to the level of its graph it
// joins the next frontier with that core number
__device__ __forceinline__ void dec_deg(const PeelBufs &b, int32_t x, u64 c, int32_t r) {
    if (b.minpeel) {                      // the next round takes the new minimum itself
        atomic_sub_u64(&b.deg[x], c);
        return;
    }
    const int32_t g = graph_of(b, x);
    const u64 k = level_of(b, g);
    const u64 old = atomic_sub_u64(&b.deg[x], c);
    const bool cross = old > k && old - c <= k;
    // the lanes that cross together take their frontier slots with one atomic
    const int nx = b.ctl->cur ^ 1;
    constexpr size_t GS_STRIDE = sizeof(GraphState) / sizeof(int32_t);
    wave_push(cross, x, b.F + (size_t)nx * b.n, &b.ctl->nF[nx]);
    wave_add_by_graph<int32_t>(cross ? g : -1, &b.gs[0].nF[nx], GS_STRIDE);
    if (cross) {
        b.stamp[x] = r + 1;
        b.core[x] = k;
        push_work(b, x, nx);
    }
}

// two survivors per lane lose cliques (c = 0: none): both atomics are in
// flight before either result is needed, and the whole wave calls this
__device__ __forceinline__ void dec_deg2(const PeelBufs &b, int32_t x1, u64 c1, int32_t x2, u64 c2, int32_t r) {
    if (b.minpeel) {
        if (c1) atomic_sub_u64(&b.deg[x1], c1);
        if (c2) atomic_sub_u64(&b.deg[x2], c2);
        return;
    }
    const int32_t g1 = c1 ? graph_of(b, x1) : -1, g2 = c2 ? graph_of(b, x2) : -1;
    const u64 k1 = c1 ? level_of(b, g1) : 0, k2 = c2 ? level_of(b, g2) : 0;
    u64 o1 = 0, o2 = 0;
    if (c1) o1 = atomic_sub_u64(&b.deg[x1], c1);
    if (c2) o2 = atomic_sub_u64(&b.deg[x2], c2);
    const bool cr1 = c1 && o1 > k1 && o1 - c1 <= k1;
    const bool cr2 = c2 && o2 > k2 && o2 - c2 <= k2;
    const int nx = b.ctl->cur ^ 1;
    constexpr size_t GS_STRIDE = sizeof(GraphState) / sizeof(int32_t);
    wave_push(cr1, x1, b.F + (size_t)nx * b.n, &b.ctl->nF[nx]);
    wave_add_by_graph<int32_t>(cr1 ? g1 : -1, &b.gs[0].nF[nx], GS_STRIDE);
    wave_push(cr2, x2, b.F + (size_t)nx * b.n, &b.ctl->nF[nx]);
    wave_add_by_graph<int32_t>(cr2 ? g2 : -1, &b.gs[0].nF[nx], GS_STRIDE);
    if (b.tpairs) {
        wave_push_items(b, cr1, x1, nx);
        wave_push_items(b, cr2, x2, nx);
    }
    if (cr1) {
        b.stamp[x1] = r + 1;
        b.core[x1] = k1;
        push_work(b, x1, nx);
    }
    if (cr2) {
        b.stamp[x2] = r + 1;
        b.core[x2] = k2;
        push_work(b, x2, nx);
    }
}

// cliques destroyed through frontier vertex v
__device__ __forceinline__ void add_destroyed(const PeelBufs &b, int32_t v, u64 t) {
    if (t) atomicAdd(&b.gs[graph_of(b, v)].destroyed, t);
}

// Cliques destroyed, summed by one lane over the frontier vertices or items
// it handles in a row: one atomic per run of one graph's vertices instead of
// one per vertex (a large round's frontier would otherwise queue on the one
// counter of its graph).
struct DestroyedTally {
    int32_t g = -1;
    u64 t = 0;
    __device__ __forceinline__ void add(const PeelBufs &b, int32_t v, u64 c) {
        const int32_t gv = graph_of(b, v);
        if (gv != g) {
            flush(b);
            g = gv;
        }
        t += c;
    }
    __device__ __forceinline__ void flush(const PeelBufs &b) {
        if (t) atomicAdd(&b.gs[g].destroyed, t);
        t = 0;
    }
};

// the main kernel's counted work: lane 0 of every wave holds its wave's
// tally; one atomic per block.  All threads of the block call together.
__device__ __forceinline__ void add_work(const PeelBufs &b, u64 pairs, u64 nbrs) {
    __shared__ u64 sP[WAVES_PER_BLOCK], sN[WAVES_PER_BLOCK];
    const int wv = threadIdx.x / WAVE;
    if (lane() == 0) {
        sP[wv] = pairs;
        sN[wv] = nbrs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 p = 0, q = 0;
        for (int i = 0; i < WAVES_PER_BLOCK; i++) {
            p += sP[i];
            q += sN[i];
        }
        if (p) atomicAdd(&b.ctl->work[0], p);
        if (q) atomicAdd(&b.ctl->work[1], q);
    }
}

// a clique through frontier vertex v may use x iff x was alive at the start
// of the round and is not a frontier vertex of smaller rank (owner rule)
__device__ __forceinline__ bool allowed(int32_t st, int32_t r, int32_t x, int32_t v) {
    return st > r || (st == r && x > v);
}

// ---------------------------------------------------------------- level selection

// smallest alive degree of every graph that opens a level
__global__ __launch_bounds__(BLOCK) void k_level_min(PeelBufs b) {
    PeelCtl *c = b.ctl;
    if (c->nsel[c->cur] == 0) return;
    const int32_t *list = b.lists + (size_t)c->lcur * b.n;
    const int32_t cnt = c->nlist[c->lcur];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    if (b.G == 1) {
        u64 m = ~0ull;
        for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < cnt; i += stride) {
            int32_t v = list[i];
            if (b.stamp[v] == ALIVE) {
                u64 d = b.deg[v];
                m = d < m ? d : m;
            }
        }
        __shared__ u64 sMin[WAVES_PER_BLOCK];
        m = wave_min(m);
        if (lane() == 0) sMin[threadIdx.x / WAVE] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < WAVES_PER_BLOCK; i++) m = sMin[i] < m ? sMin[i] : m;
            if (m != ~0ull) atomicMin(&b.gs[0].kcand, m);
        }
        return;
    }
    for (int64_t base = blockIdx.x * (int64_t)BLOCK; base < cnt; base += stride) {
        const int64_t i = base + threadIdx.x;
        int32_t g = -1;
        u64 d = ~0ull;
        if (i < cnt) {
            const int32_t v = list[i];
            if (b.stamp[v] == ALIVE) {
                const int32_t gv = b.gid[v];
                if (b.gs[gv].sel) {
                    g = gv;
                    d = b.deg[v];
                }
            }
        }
        const u64 act = __ballot(g >= 0);
        if (!act) continue;
        const int first = __builtin_ctzll(act);
        const int32_t g0 = __shfl(g, first, WAVE);
        if (__ballot(g >= 0 && g != g0) == 0) {
            const u64 m = wave_min(d);
            if (lane() == first) atomicMin(&b.gs[g0].kcand, m);
        } else if (g >= 0) {
            atomicMin(&b.gs[g].kcand, d);
        }
    }
}

// frontier of every graph that opens a level: its alive vertices of degree <= k
__global__ __launch_bounds__(BLOCK) void k_level_build(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nsel[cur] == 0) return;
    const int32_t r = c->round, lc = c->lcur;
    const int32_t *in = b.lists + (size_t)lc * b.n;
    int32_t *out = b.lists + (size_t)(lc ^ 1) * b.n;
    int32_t *F = b.F + (size_t)cur * b.n;
    const int32_t cnt = c->nlist[lc];
    const bool compact = list_compacts(c);
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    constexpr size_t GS_STRIDE = sizeof(GraphState) / sizeof(int32_t);
    for (int64_t base = blockIdx.x * (int64_t)BLOCK; base < cnt; base += stride) {
        const int64_t i = base + threadIdx.x;
        int32_t v = -1, g = 0;
        bool alive = false, take = false;
        if (i < cnt) {
            v = in[i];
            alive = b.stamp[v] == ALIVE;
            if (alive) {
                g = graph_of(b, v);
                if (b.gs[g].sel) {
                    const u64 k = level_of(b, g);
                    take = b.deg[v] <= k;
                    if (take) {
                        b.stamp[v] = r;
                        b.core[v] = b.minpeel ? (u64)r : k;
                        push_work(b, v, cur);
                    }
                }
            }
        }
        wave_push(take, v, F, &c->nF[cur]);
        wave_add_by_graph<int32_t>(take ? g : -1, &b.gs[0].nF[cur], GS_STRIDE);
        if (b.tpairs) wave_push_items(b, take, v, cur);
        if (compact) block_push(alive && !take, v, out, &c->nlist[lc ^ 1]);
    }
}

// End of a round, per graph: a graph that opened a level records it; its
// frontier is retired; it opens a level next round if nothing is pending.
__device__ __forceinline__ void finish_graph(const PeelBufs &b, int32_t g) {
    PeelCtl *c = b.ctl;
    GraphState &s = b.gs[g];
    const int32_t cur = c->cur, nx = cur ^ 1;
    if (!s.sel && s.nF[cur] == 0) return;          // finished graph: nothing happened
    if (s.sel) {
        const u64 k = level_of(b, g);
        if (s.nF[cur] > 0) {
            const int64_t L = s.lv_base + s.nlevels;
            b.lv_k[L] = k;
            b.lv_size[L] = (u64)s.n_alive;
            b.lv_mu[L] = s.mu_alive;
            s.nlevels += 1;
        }
        s.k = k;
        s.kcand = ~0ull;
    }
    if (s.nF[cur] == s.n_alive)
        s.mu_alive = 0;                             // every alive vertex left: no clique remains
    else
        s.mu_alive -= s.destroyed + (s.destroyed_m ? s.destroyed_m / (u64)(b.h - 1) : 0ull);
    s.n_alive -= s.nF[cur];
    s.destroyed = 0;
    s.destroyed_m = 0;
    s.nF[cur] = 0;
    s.sel = (s.nF[nx] == 0 && s.n_alive > 0) ? 1 : 0;
    if (s.sel) atomicAdd(&c->nsel[nx], 1);
}

// End of a round, global part (after every graph's part).
__device__ __forceinline__ void finish_global(PeelCtl *c) {
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0 && c->nsel[cur] == 0) return;   // nothing happened
    if (c->nsel[cur] > 0 && list_compacts(c)) {
        c->nlist[c->lcur] = 0;
        c->lcur ^= 1;
    }
    c->n_alive -= c->nF[cur];
    c->nsel[cur] = 0;
    c->nF[cur] = 0;
    c->nB[cur] = 0;
    c->nT[cur] = 0;
    c->nTouch = 0;
    c->htop[cur] = 0;
    c->nW = 0;
    c->nBig[cur] = 0;
    for (int i = 0; i < 8; i++) c->nitems[i] = 0;
    c->cur = cur ^ 1;
    c->round += 1;
}

// ---------------------------------------------------------------- tail mode
//
// Once few vertices are left, the round's control work fits one workgroup:
// k_tail_level ends the previous round (what k_finish_* do), then selects
// the level and builds the frontier (what k_level_min and k_level_build do),
// so a round is this kernel plus the process kernels.  k_tail_finish ends
// the last round before the host reads the alive count.

constexpr int TAIL_BLOCK = 1024;
constexpr int TAIL_WAVES = TAIL_BLOCK / WAVE;

// end of the pending round; all threads of the (single) block call it
__device__ __forceinline__ void tail_finish_block(const PeelBufs &b) {
    PeelCtl *c = b.ctl;
    if (c->pending) {
        for (int32_t g = threadIdx.x; g < b.G; g += blockDim.x) finish_graph(b, g);
        __syncthreads();
        if (threadIdx.x == 0) {
            finish_global(c);
            c->pending = 0;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(TAIL_BLOCK) void k_tail_finish(PeelBufs b) { tail_finish_block(b); }

// the frontier decision for one alive-list entry (v, its stamp and degree)
__device__ __forceinline__ bool tail_take(const PeelBufs &b, int32_t v, int32_t st, u64 d, int32_t r, int32_t cur,
                                          int32_t *g_out) {
    *g_out = 0;
    if (st != ALIVE) return false;
    const int32_t g = graph_of(b, v);
    *g_out = g;
    if (!b.gs[g].sel) return false;
    const u64 k = level_of(b, g);
    if (d > k) return false;
    b.stamp[v] = r;
    b.core[v] = b.minpeel ? (u64)r : k;
    push_work(b, v, cur);
    return true;
}

__global__ __launch_bounds__(TAIL_BLOCK) void k_tail_level(PeelBufs b) {
    // each thread keeps its first TAIL_REG alive-list entries in registers, so
    // the level's minimum and its frontier need one round of loads
    constexpr int TAIL_REG = 16;
    __shared__ u64 sMin[TAIL_WAVES];
    PeelCtl *c = b.ctl;
    tail_finish_block(b);
    const int32_t cur = c->cur;
    if (c->nsel[cur] > 0) {
        const int32_t lc = c->lcur, cnt = c->nlist[lc], r = c->round;
        const int32_t *in = b.lists + (size_t)lc * b.n;
        int32_t rv[TAIL_REG], rs[TAIL_REG];
        u64 rd[TAIL_REG];
#pragma unroll
        for (int j = 0; j < TAIL_REG; j++) {
            const int32_t i = j * TAIL_BLOCK + threadIdx.x;
            rv[j] = i < cnt ? in[i] : -1;
        }
#pragma unroll
        for (int j = 0; j < TAIL_REG; j++) {
            rs[j] = rv[j] >= 0 ? b.stamp[rv[j]] : -1;
            rd[j] = rv[j] >= 0 ? b.deg[rv[j]] : ~0ull;
        }
        // smallest alive degree of every graph that opens a level
        if (b.G == 1) {
            u64 m = ~0ull;
#pragma unroll
            for (int j = 0; j < TAIL_REG; j++)
                if (rs[j] == ALIVE && rd[j] < m) m = rd[j];
            for (int32_t i = TAIL_REG * TAIL_BLOCK + threadIdx.x; i < cnt; i += TAIL_BLOCK) {
                const int32_t v = in[i];
                if (b.stamp[v] == ALIVE) {
                    const u64 d = b.deg[v];
                    m = d < m ? d : m;
                }
            }
            m = wave_min(m);
            if (lane() == 0) sMin[threadIdx.x / WAVE] = m;
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int i = 1; i < TAIL_WAVES; i++) m = sMin[i] < m ? sMin[i] : m;
                if (m < b.gs[0].kcand) b.gs[0].kcand = m;
            }
        } else {
#pragma unroll
            for (int j = 0; j < TAIL_REG; j++)
                if (rs[j] == ALIVE && b.gs[b.gid[rv[j]]].sel) atomicMin(&b.gs[b.gid[rv[j]]].kcand, rd[j]);
            for (int32_t i = TAIL_REG * TAIL_BLOCK + threadIdx.x; i < cnt; i += TAIL_BLOCK) {
                const int32_t v = in[i];
                if (b.stamp[v] == ALIVE) {
                    const int32_t g = b.gid[v];
                    if (b.gs[g].sel) atomicMin(&b.gs[g].kcand, b.deg[v]);
                }
            }
        }
        __syncthreads();
        // the level's frontier: alive vertices of degree <= k
        int32_t *out = b.lists + (size_t)(lc ^ 1) * b.n;
        int32_t *F = b.F + (size_t)cur * b.n;
        const bool compact = list_compacts(c);
        constexpr size_t GS_STRIDE = sizeof(GraphState) / sizeof(int32_t);
#pragma unroll
        for (int j = 0; j < TAIL_REG; j++) {
            int32_t g = 0;
            const bool take = rv[j] >= 0 && tail_take(b, rv[j], rs[j], rd[j], r, cur, &g);
            wave_push(take, rv[j], F, &c->nF[cur]);
            wave_add_by_graph<int32_t>(take ? g : -1, &b.gs[0].nF[cur], GS_STRIDE);
            if (b.tpairs) wave_push_items(b, take, rv[j], cur);
            if (compact) wave_push(rs[j] == ALIVE && !take, rv[j], out, &c->nlist[lc ^ 1]);
        }
        for (int32_t base = TAIL_REG * TAIL_BLOCK; base < cnt; base += TAIL_BLOCK) {
            const int32_t i = base + threadIdx.x;
            int32_t v = -1, st = -1, g = 0;
            bool take = false;
            if (i < cnt) {
                v = in[i];
                st = b.stamp[v];
                take = tail_take(b, v, st, b.deg[v], r, cur, &g);
            }
            wave_push(take, v, F, &c->nF[cur]);
            wave_add_by_graph<int32_t>(take ? g : -1, &b.gs[0].nF[cur], GS_STRIDE);
            if (b.tpairs) wave_push_items(b, take, v, cur);
            if (compact) wave_push(st == ALIVE && !take, v, out, &c->nlist[lc ^ 1]);
        }
    }
    if (threadIdx.x == 0) c->pending = 1;
}

__global__ void k_finish_one(PeelBufs b) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        finish_graph(b, 0);
        finish_global(b.ctl);
    }
}

__global__ void k_finish_graphs(PeelBufs b) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < b.G) finish_graph(b, g);
}

__global__ void k_finish_global(PeelBufs b) {
    if (blockIdx.x == 0 && threadIdx.x == 0) finish_global(b.ctl);
}

// ---------------------------------------------------------------- h = 2

// A large h = 2 round from the other side: every alive vertex x counts its
// frontier neighbours and takes them off its own degree (one writer per
// degree, no atomics); a frontier vertex counts its frontier neighbours of
// larger rank, so every removed edge is counted once.  Worth it once the
// frontier is a sizeable share of the alive vertices, whose rows (the
// compacted adjacency) are then read in place of the frontier's.
constexpr int64_t H2_PULL_MIN = 16384, H2_PULL_SHARE = 16;

__device__ __forceinline__ void process_h2_pull(const PeelBufs &b, int32_t r) {
    PeelCtl *c = b.ctl;
    const int32_t lc = c->lcur, cnt = c->nlist[lc];
    const int32_t *list = b.lists + (size_t)lc * b.n;
    const int nx = c->cur ^ 1;
    const u64 k = level_of(b, 0);
    const int wv = threadIdx.x / WAVE;
    constexpr size_t GS_STRIDE = sizeof(GraphState) / sizeof(int32_t);
    DestroyedTally tally;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < cnt; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t x = list[i];
        const int32_t sx = b.stamp[x];
        if (sx < r) continue;   // removed in an earlier round (or not taking part)
        uint32_t n_in = 0;
        for (int64_t e = b.row_ptr[x] + lane(); e < b.row_ptr[x + 1]; e += WAVE) {
            const int32_t y = b.col[e];
            if (b.stamp[y] == r && (sx != r || y > x)) n_in++;
        }
        n_in = wave_sum(n_in);
        if (lane() == 0) tally.add(b, x, n_in);
        bool cross = false;
        if (sx > r && n_in && lane() == 0) {
            const u64 old = b.deg[x];
            b.deg[x] = old - n_in;
            cross = old > k && old - n_in <= k;
        }
        wave_push(cross, x, b.F + (size_t)nx * b.n, &c->nF[nx]);
        wave_add_by_graph<int32_t>(cross ? 0 : -1, &b.gs[0].nF[nx], GS_STRIDE);
        if (cross) {
            b.stamp[x] = r + 1;
            b.core[x] = k;
        }
    }
    if (lane() == 0) tally.flush(b);
}

__global__ __launch_bounds__(BLOCK) void k_process_h2(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    if (b.G == 1 && !b.minpeel && b.pattern == 0 && nF >= H2_PULL_MIN && (int64_t)nF * H2_PULL_SHARE >= c->n_alive) {
        process_h2_pull(b, r);
        return;
    }
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE;
    u64 wp = 0, wn = 0;   // counted work (lane 0's tally is the wave's)
    DestroyedTally tally;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nF; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[i];
        u64 destroyed = 0;
        for (int64_t e = b.row_ptr[v] + lane(); e < b.row_ptr[v + 1]; e += WAVE) {
            int32_t w = b.col[e];
            int32_t st = b.stamp[w];
            if (st == r) {
                destroyed += (v < w) ? 1 : 0;       // both ends leave: count the edge once
            } else if (st > r) {
                destroyed += 1;
                dec_deg(b, w, 1, r);
            }
        }
        destroyed = wave_sum(destroyed);
        if (lane() == 0) tally.add(b, v, destroyed);
        if (b.count_work) wp += (u64)(b.row_ptr[v + 1] - b.row_ptr[v]), wn += 1;
    }
    if (lane() == 0) tally.flush(b);
    if (b.count_work) add_work(b, wp, wn);
}

// ---------------------------------------------------------------- h = 3

// Hash over the allowed neighbourhood of frontier vertex v.  The value of a
// slot counts the cliques through v found so far that contain that
// neighbour; the counts go to dec_deg once per neighbour (flush), so the pair
// loop itself never waits on a global atomic.  size: any number of slots >=
// 2 (a power of two in LDS, chunk-sized in global memory); at most half of
// them are ever filled.
struct NbHash {
    int32_t *keys;
    uint32_t *vals;
    uint32_t size;
    __device__ __forceinline__ uint32_t start(int32_t x) const {
        return (uint32_t)(((u64)((uint32_t)x * 2654435761u) * size) >> 32);
    }
    __device__ __forceinline__ uint32_t next(uint32_t slot) const { return slot + 1 == size ? 0 : slot + 1; }
    __device__ __forceinline__ int find(int32_t x) const {
        uint32_t slot = start(x);
        while (true) {
            int32_t key = keys[slot];
            if (key == x) return (int)slot;
            if (key == HASH_EMPTY) return -1;
            slot = next(slot);
        }
    }
    __device__ __forceinline__ void put(int32_t x) const {
        uint32_t slot = start(x);
        while (true) {
            int32_t prev = atomicCAS(&keys[slot], HASH_EMPTY, x);
            if (prev == HASH_EMPTY || prev == x) return;
            slot = next(slot);
        }
    }
};

// insert the allowed neighbours N(v)[rv0, rv1) (threads t, t + step, ...)
__device__ __forceinline__ void hash_fill(const PeelBufs &b, const NbHash &hs, int32_t v, int64_t rv0, int64_t rv1,
                                          int32_t r, int t, int step) {
    for (int64_t e = rv0 + t; e < rv1; e += step) {
        int32_t x = b.col[e];
        if (allowed(b.stamp[x], r, x, v)) hs.put(x);
    }
}

// apply the pending counts of slots [s0, s1) (threads t, t + step, ...) and empty them
__device__ __forceinline__ void hash_flush(const PeelBufs &b, const NbHash &hs, int32_t r, uint32_t s0, uint32_t s1,
                                           int t, int step) {
    for (uint32_t i = s0 + t; i < s1; i += step) {
        int32_t key = hs.keys[i];
        if (key == HASH_EMPTY) continue;
        uint32_t c = hs.vals[i];
        if (c && b.stamp[key] > r) dec_deg(b, key, c, r);
        hs.keys[i] = HASH_EMPTY;
        hs.vals[i] = 0;
    }
}

// One wave handles the neighbours N(v)[lo, hi) of frontier vertex v: for each
// allowed neighbour w it probes N+(w) against the hash of v's allowed
// neighbourhood, so every triangle {v, w, x} with w before x is seen once.
// Neighbours w whose out-list holds wide_out or more entries are skipped (a
// wide item of their own covers them).  sPre/sSt/sW/sCnt: this wave's
// 64-entry LDS scratch.
__device__ __forceinline__ u64 h3_wave_range(const PeelBufs &b, int32_t v, int64_t lo, int64_t hi, int32_t r,
                                            const NbHash &hs, int32_t *sPre, int64_t *sSt, int32_t *sW,
                                            uint32_t *sCnt, int32_t wide_out, u64 *pairs = nullptr,
                                            u64 *nbrs = nullptr) {
    const int L = lane();
    u64 destroyed = 0;
    for (int64_t base = lo; base < hi; base += WAVE) {
        int32_t w = -1, len = 0, wslot = -1;
        int64_t st0 = 0;
        if (base + L < hi) {
            w = b.col[base + L];
            if (allowed(b.stamp[w], r, w, v)) {
                st0 = b.dag_off[w];
                len = (int32_t)(b.row_ptr[w + 1] - st0);
                if (len >= wide_out) len = 0;
                wslot = hs.find(w);
            }
        }
        int32_t inc = wave_incl_scan(len);
        sPre[L] = inc;
        sSt[L] = st0;
        sW[L] = wslot;
        sCnt[L] = 0;
        const int32_t total = __shfl(inc, WAVE - 1, WAVE);
        if (pairs) {
            *pairs += (u64)total;
            *nbrs += (u64)__popcll(__ballot(len > 0));
        }
        __builtin_amdgcn_wave_barrier();
        for (int32_t pb = 0; pb < total; pb += WAVE) {
            int32_t p = pb + L;
            if (p < total) {
                int i = upper_bound_i32(sPre, WAVE, p);
                int32_t off = p - (i ? sPre[i - 1] : 0);
                int32_t x = b.col[sSt[i] + off];
                int slot = hs.find(x);
                if (slot >= 0) {                      // triangle {v, w, x}, owned by v
                    destroyed++;
                    atomicAdd(&sCnt[i], 1u);
                    atomicAdd(&hs.vals[slot], 1u);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t cw = sCnt[L];
        if (cw) atomicAdd(&hs.vals[sW[L]], cw);
        __builtin_amdgcn_wave_barrier();
    }
    return destroyed;
}

// Larger frontier vertices (degree > SMALL_DEG) are cut into chunks of CHUNK
// neighbours, one wave each, so that the pairs of a hub spread over the whole
// chip.  Their neighbourhood hashes live in global memory (SLOTS_PER_CHUNK
// slots per chunk): fill inserts the allowed neighbours (and queues a wide
// item for each neighbour with a long out-list), probe counts the triangles,
// flush hands each neighbour's count to dec_deg once and empties the slots
// for later rounds.

__device__ __forceinline__ NbHash big_hash(const PeelBufs &b, int32_t cur, int32_t v, int64_t d) {
    const int64_t nc = (d + CHUNK - 1) / CHUNK;
    const size_t off = (size_t)cur * b.hcap + b.hbase[v];
    return NbHash{b.hkey + off, b.hval + off, (uint32_t)(nc * SLOTS_PER_CHUNK)};
}

__global__ __launch_bounds__(BLOCK) void k_h3_fill(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0) return;
    const int32_t r = c->round, nB = c->nB[cur];
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const int wv = threadIdx.x / WAVE;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nB; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int64_t item = Bc[it];
        const int32_t v = (int32_t)(item >> 32), ch = (int32_t)(item & 0xffffffff);
        const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
        const int64_t e = rv0 + (int64_t)ch * CHUNK + lane();
        bool wide = false;
        int32_t x = -1;
        if (e < rv1 && lane() < CHUNK) {
            x = b.col[e];
            if (allowed(b.stamp[x], r, x, v)) {
                big_hash(b, cur, v, rv1 - rv0).put(x);
                wide = b.row_ptr[x + 1] - b.dag_off[x] >= WIDE_OUT;
            }
        }
        const u64 m = __ballot(wide);
        if (m) {
            const int leader = __builtin_ctzll(m);
            int64_t base = 0;
            if (lane() == leader) base = (int64_t)atomicAdd((unsigned long long *)&c->nW, (unsigned long long)__popcll(m));
            base = __shfl(base, leader, WAVE);
            if (wide) b.W[base + __popcll(m & lanemask_lt())] = ((int64_t)v << 32) | (uint32_t)x;
        }
    }
}

// The round's triangle work, one wave per item: chunk items and wide items
// of the large frontier vertices (their hashes filled by k_h3_fill), then
// every small frontier vertex (degree <= SMALL_DEG) whole, with a per-wave
// LDS hash that the wave fills, probes and flushes itself.
__global__ __launch_bounds__(BLOCK) void k_h3_probe(PeelBufs b) {
    __shared__ int32_t sKey[WAVES_PER_BLOCK][1 << SMALL_HASH_BITS];
    __shared__ uint32_t sVal[WAVES_PER_BLOCK][1 << SMALL_HASH_BITS];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    __shared__ uint32_t sCnt[WAVES_PER_BLOCK][WAVE];
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round, nB = c->nB[cur];
    const int64_t nW = c->nW;
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE, L = lane();
    const NbHash small{sKey[wv], sVal[wv], 1u << SMALL_HASH_BITS};
    for (int i = L; i < (1 << SMALL_HASH_BITS); i += WAVE) {
        small.keys[i] = HASH_EMPTY;
        small.vals[i] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    u64 wp = 0, wn = 0;   // counted work (wave-uniform)
    DestroyedTally tally;
    const int64_t total = (int64_t)nB + nW + nF;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < total; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        int32_t v;
        u64 destroyed;
        if (it >= (int64_t)nB + nW) {
            // a small frontier vertex, whole
            v = F[it - nB - nW];
            const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
            if (rv1 - rv0 > SMALL_DEG) continue;                 // its chunk items cover it
            hash_fill(b, small, v, rv0, rv1, r, L, WAVE);
            __builtin_amdgcn_wave_barrier();
            destroyed = h3_wave_range(b, v, rv0, rv1, r, small, sPre[wv], sSt[wv], sW[wv], sCnt[wv], 0x7fffffff,
                                      &wp, &wn);
            __builtin_amdgcn_wave_barrier();
            hash_flush(b, small, r, 0, small.size, L, WAVE);
            __builtin_amdgcn_wave_barrier();
            destroyed = wave_sum(destroyed);
        } else if (it < nB) {
            // chunk item: the neighbours with short out-lists, their pairs flattened over the wave
            const int64_t item = Bc[it];
            v = (int32_t)(item >> 32);
            const int32_t ch = (int32_t)(item & 0xffffffff);
            const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
            const int64_t lo = rv0 + (int64_t)ch * CHUNK, hi = min(rv1, lo + CHUNK);
            const NbHash hs = big_hash(b, cur, v, rv1 - rv0);
            destroyed = h3_wave_range(b, v, lo, hi, r, hs, sPre[wv], sSt[wv], sW[wv], sCnt[wv], WIDE_OUT, &wp, &wn);
            destroyed = wave_sum(destroyed);
        } else {
            // wide item (v, w): the lanes walk N+(w)
            const int64_t item = b.W[it - nB];
            v = (int32_t)(item >> 32);
            const int32_t w = (int32_t)(item & 0xffffffff);
            const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
            const NbHash hs = big_hash(b, cur, v, rv1 - rv0);
            uint32_t cw = 0;
            wp += (u64)(b.row_ptr[w + 1] - b.dag_off[w]);
            wn += 1;
            for (int64_t e = b.dag_off[w] + lane(); e < b.row_ptr[w + 1]; e += WAVE) {
                const int slot = hs.find(b.col[e]);
                if (slot >= 0) {                          // triangle {v, w, x}, owned by v
                    cw++;
                    atomicAdd(&hs.vals[slot], 1u);
                }
            }
            cw = wave_sum(cw);
            if (lane() == 0 && cw) {
                const int ws = hs.find(w);                // present: fill inserted every allowed neighbour
                if (ws >= 0) atomicAdd(&hs.vals[ws], cw);
            }
            destroyed = cw;
        }
        if (lane() == 0) tally.add(b, v, destroyed);
    }
    if (lane() == 0) tally.flush(b);
    if (b.count_work) add_work(b, wp, wn);
}

__global__ __launch_bounds__(BLOCK) void k_h3_flush(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0) return;
    const int32_t r = c->round, nB = c->nB[cur];
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const int wv = threadIdx.x / WAVE;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nB; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int64_t item = Bc[it];
        const int32_t v = (int32_t)(item >> 32), ch = (int32_t)(item & 0xffffffff);
        const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
        const NbHash hs = big_hash(b, cur, v, rv1 - rv0);
        const uint32_t s0 = (uint32_t)ch * SLOTS_PER_CHUNK;
        hash_flush(b, hs, r, s0, min(s0 + SLOTS_PER_CHUNK, hs.size), lane(), WAVE);
    }
}

// ---------------------------------------------------------------- h = 3, triangle lists

// One wave per row item: TL_CHUNK pairs (a, b) of a frontier vertex v, each
// a triangle {v, a, b}.  v destroys the triangle iff a and b may share a
// clique with v this round (alive, or frontier vertices of larger rank: the
// owner rule makes v the triangle's frontier member of smallest rank).  The
// pairs of one neighbour a are contiguous, so its losses are summed over its
// run of lanes and applied once; b loses each triangle on its own.  Each
// triangle sits once in v's row.  Counted work: pairs walked (pairs) and
// items (nbrs).
__global__ __launch_bounds__(BLOCK) void k_tl_process(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0) return;
    const int32_t r = c->round, nT = c->nT[cur];
    const int64_t *Tc = b.T + (size_t)cur * b.tcap;
    const int wv = threadIdx.x / WAVE, L = lane();
    u64 wp = 0, wn = 0;
    DestroyedTally tally;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nT; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int64_t item = Tc[it];
        const int32_t v = (int32_t)(item >> 32), ch = (int32_t)(item & 0xffffffff);
        const int64_t lo = b.tvoff[v] + (int64_t)ch * TL_CHUNK;
        const int64_t hi = min(b.tvoff[v + 1], lo + TL_CHUNK);
        u64 destroyed = 0;
        for (int64_t base = lo; base < hi; base += WAVE) {
            const int64_t e = base + L;
            const bool valid = e < hi;
            int32_t a = -1, x = -1, sa = -1, sx = -1;
            bool ok = false;
            if (valid) {
                const int2 pr = *(const int2 *)&b.tpairs[2 * e];
                a = pr.x;
                x = pr.y;
                sa = b.stamp[a];
                sx = b.stamp[x];
                ok = allowed(sa, r, a, v) && allowed(sx, r, x, v);
            }
            destroyed += ok ? 1 : 0;
            // runs of equal a over the valid lanes
            const int32_t pa = __shfl_up(a, 1, WAVE);
            const bool head = valid && (L == 0 || pa != a);
            const u64 hm = __ballot(head), om = __ballot(ok);
            const u64 le = lanemask_lt() | (1ull << L);
            const u64 nxt = hm & ~le;
            const int end = nxt ? __builtin_ctzll(nxt) : WAVE;
            const u64 upto = end == WAVE ? ~0ull : ((1ull << end) - 1);
            const uint32_t cnt = head ? (uint32_t)__popcll(om & upto & ~lanemask_lt()) : 0u;
            dec_deg2(b, a, sa > r ? cnt : 0u, x, (ok && sx > r) ? 1u : 0u, r);
        }
        destroyed = wave_sum(destroyed);
        if (L == 0) tally.add(b, v, destroyed);
        wp += (u64)(hi - lo);
        wn += 1;
    }
    if (L == 0) tally.flush(b);
    if (b.count_work) add_work(b, wp, wn);
}

// ---------------------------------------------------------------- x-star pattern

// C(n, k) for k <= 8 (the terms of a residual graph never exceed the
// degrees the enumeration accepted without overflow)
__device__ __forceinline__ u64 binom_small(int64_t n, int k) {
    if (n < k || n < 0) return 0;
    unsigned __int128 acc = 1;
    for (int i = 1; i <= k; i++) acc = acc * (unsigned __int128)(n - k + i) / (unsigned __int128)i;
    return (u64)acc;
}

// one wave per frontier vertex f: its surviving neighbours lose a unit of
// degree and the stars centred at f that use them as tails
__global__ __launch_bounds__(BLOCK) void k_star_front(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE;
    u64 wp = 0, wn = 0;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nF; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t f = F[i];
        const u64 tail = binom_small((int64_t)b.yold[f] - 1, b.px - 1);
        for (int64_t e = b.row_ptr[f] + lane(); e < b.row_ptr[f + 1]; e += WAVE) {
            const int32_t u = b.col[e];
            if (b.stamp[u] <= r) continue;
            atomicSub(&b.ydeg[u], 1);
            if (atomicExch(&b.tround[u], r) != r) b.touch[atomicAdd(&c->nTouch, 1)] = u;
            if (tail) dec_deg(b, u, tail, r);
        }
        wp += (u64)(b.row_ptr[f + 1] - b.row_ptr[f]);
        wn += 1;
    }
    if (b.count_work) add_work(b, wp, wn);
}

// one wave per survivor u whose degree fell: its own centre term, and the
// stars centred at u whose other tails remain
__global__ __launch_bounds__(BLOCK) void k_star_touch(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t nt = c->nTouch;
    const int32_t r = c->round;
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nt; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t u = b.touch[i];
        const int32_t yo = b.yold[u], yn = b.ydeg[u];
        const u64 own = binom_small(yo, b.px) - binom_small(yn, b.px);
        const u64 two = binom_small((int64_t)yo - 1, b.px - 1) - binom_small((int64_t)yn - 1, b.px - 1);
        if (lane() == 0 && own) dec_deg(b, u, own, r);
        if (two)
            for (int64_t e = b.row_ptr[u] + lane(); e < b.row_ptr[u + 1]; e += WAVE) {
                const int32_t w = b.col[e];
                if (b.stamp[w] > r) dec_deg(b, w, two, r);
            }
        __builtin_amdgcn_wave_barrier();
        if (lane() == 0) b.yold[u] = yn;
    }
}

// ---------------------------------------------------------------- 4-loop pattern

constexpr int LOOP_EMPTY = -1;

__device__ __forceinline__ uint32_t loop_slot(int32_t w, uint32_t mask) {
    return (uint32_t)(((u64)((uint32_t)w * 2654435761u) * (mask + 1ull)) >> 32) & mask;
}

// add one 2-path to w's count (the table is never more than half full)
__device__ __forceinline__ void loop_add(int32_t *keys, uint32_t *vals, uint32_t mask, int32_t w) {
    uint32_t slot = loop_slot(w, mask);
    while (true) {
        const int32_t k = keys[slot];
        if (k == w) break;
        if (k == LOOP_EMPTY) {
            const int32_t prev = atomicCAS(&keys[slot], LOOP_EMPTY, w);
            if (prev == LOOP_EMPTY || prev == w) break;
            continue;          // another thread took the slot: look at it again
        }
        slot = (slot + 1) & mask;
    }
    atomicAdd(&vals[slot], 1u);
}

__device__ __forceinline__ uint32_t loop_get(const int32_t *keys, const uint32_t *vals, uint32_t mask, int32_t w) {
    uint32_t slot = loop_slot(w, mask);
    while (true) {
        const int32_t k = keys[slot];
        if (k == w) return vals[slot];
        if (k == LOOP_EMPTY) return 0;
        slot = (slot + 1) & mask;
    }
}

// The 2-paths v - a - w of one workgroup, flattened over its threads 256
// middles a at a time: fn(i, a, w) for every neighbour a of v (i its index in
// the chunk, from sA) with keep_a(a), and every neighbour w != v of a with
// keep_w(w).  after_chunk(n) runs once the chunk's pairs are done (all
// threads, n middles in sA).
template <class KA, class KW, class FN, class AC>
__device__ __forceinline__ void loop_two_paths(const int64_t *row_ptr, const int32_t *col, int32_t v, KA keep_a,
                                               KW keep_w, FN fn, AC after_chunk, int32_t *sA, int64_t *sSt,
                                               int32_t *sPre, int32_t *wtmp) {
    const int64_t r0 = row_ptr[v], r1 = row_ptr[v + 1];
    for (int64_t base = r0; base < r1; base += BLOCK) {
        const int64_t e = base + threadIdx.x;
        int32_t a = -1, len = 0;
        int64_t st0 = 0;
        if (e < r1) {
            a = col[e];
            if (keep_a(a)) {
                st0 = row_ptr[a];
                len = (int32_t)(row_ptr[a + 1] - st0);
            }
        }
        sA[threadIdx.x] = a;
        sSt[threadIdx.x] = st0;
        sPre[threadIdx.x] = len;
        __syncthreads();
        const int cnt = (int)min((int64_t)BLOCK, r1 - base);
        const int32_t total = block_incl_scan_lds(sPre, cnt, wtmp);
        for (int32_t p = threadIdx.x; p < total; p += BLOCK) {
            const int i = upper_bound_i32(sPre, cnt, p);
            const int32_t o = p - (i ? sPre[i - 1] : 0);
            const int32_t w = col[sSt[i] + o];
            if (w != v && keep_w(w)) fn(i, sA[i], w);
        }
        __syncthreads();
        after_chunk(cnt);
        __syncthreads();
    }
}

// bound on a vertex's 2-hop table: the degrees of its neighbours
__global__ void k_loop_bound(const int64_t *row_ptr, const int32_t *col, int32_t n, unsigned long long *mx) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        u64 sum = 0;
        for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) {
            const int32_t a = col[e];
            sum += (u64)(row_ptr[a + 1] - row_ptr[a]);
        }
        sum = wave_sum(sum);
        if (lane() == 0 && sum) atomicMax(mx, (unsigned long long)sum);
    }
}

// the table of a workgroup for vertex v: the smallest power of two >= 2 *
// (bound), cleared
__device__ __forceinline__ uint32_t loop_table(const int64_t *row_ptr, const int32_t *col, int32_t v,
                                               int32_t *keys, uint32_t *vals, int64_t lsize, u64 *sRed) {
    u64 sum = 0;
    for (int64_t e = row_ptr[v] + threadIdx.x; e < row_ptr[v + 1]; e += BLOCK) {
        const int32_t a = col[e];
        sum += (u64)(row_ptr[a + 1] - row_ptr[a]);
    }
    sum = wave_sum(sum);
    if (lane() == 0) sRed[threadIdx.x / WAVE] = sum;
    __syncthreads();
    u64 tot = 0;
    for (int i = 0; i < WAVES_PER_BLOCK; i++) tot += sRed[i];
    int64_t size = 2;
    while (size < 2 * (int64_t)tot) size <<= 1;
    if (size > lsize) size = lsize;                  // never: lsize covers the graph's largest bound
    for (int64_t i = threadIdx.x; i < size; i += BLOCK) {
        keys[i] = LOOP_EMPTY;
        vals[i] = 0;
    }
    __syncthreads();
    return (uint32_t)(size - 1);
}

// 4-loop pattern-degrees: deg(v) = sum over w of C(2-paths v - . - w, 2);
// one workgroup per vertex, the table in its slice of keys/vals
__global__ __launch_bounds__(BLOCK) void k_loop_degrees(const int64_t *row_ptr, const int32_t *col, int32_t n,
                                                         int32_t *lkey, uint32_t *lval, int64_t lsize, u64 *deg) {
    __shared__ int32_t sA[BLOCK];
    __shared__ int64_t sSt[BLOCK];
    __shared__ int32_t sPre[BLOCK];
    __shared__ int32_t wtmp[WAVES_PER_BLOCK];
    __shared__ u64 sRed[WAVES_PER_BLOCK];
    int32_t *keys = lkey + (size_t)blockIdx.x * lsize;
    uint32_t *vals = lval + (size_t)blockIdx.x * lsize;
    for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
        const uint32_t mask = loop_table(row_ptr, col, (int32_t)v, keys, vals, lsize, sRed);
        loop_two_paths(
            row_ptr, col, (int32_t)v, [](int32_t) { return true; }, [](int32_t) { return true; },
            [&](int, int32_t, int32_t w) { loop_add(keys, vals, mask, w); }, [](int) {}, sA, sSt, sPre, wtmp);
        u64 c = 0;
        for (uint32_t i = threadIdx.x; i <= mask; i += BLOCK) {
            const u64 y = vals[i];
            c += y * (y - (y ? 1 : 0)) / 2;
        }
        c = wave_sum(c);
        __syncthreads();
        if (lane() == 0) sRed[threadIdx.x / WAVE] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 t = 0;
            for (int i = 0; i < WAVES_PER_BLOCK; i++) t += sRed[i];
            deg[v] = t;
        }
        __syncthreads();
    }
}

// One workgroup per frontier vertex v: the loops v - a - w - b whose other
// members may share a clique with v this round (the owner rule) are
// destroyed; w loses C(c, 2) and each middle a loses c - 1 per group of c
// 2-paths to w.
__global__ __launch_bounds__(BLOCK) void k_loop_process(PeelBufs b) {
    __shared__ int32_t sA[BLOCK];
    __shared__ int64_t sSt[BLOCK];
    __shared__ int32_t sPre[BLOCK];
    __shared__ int32_t wtmp[WAVES_PER_BLOCK];
    __shared__ u64 sRed[WAVES_PER_BLOCK];
    __shared__ u64 sLoss[BLOCK];
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    const int32_t *F = b.F + (size_t)cur * b.n;
    int32_t *keys = b.lkey + (size_t)blockIdx.x * b.lsize;
    uint32_t *vals = b.lval + (size_t)blockIdx.x * b.lsize;
    for (int64_t fi = blockIdx.x; fi < nF; fi += gridDim.x) {
        const int32_t v = F[fi];
        const uint32_t mask = loop_table(b.row_ptr, b.col, v, keys, vals, b.lsize, sRed);
        auto ok = [&](int32_t x) { return allowed(b.stamp[x], r, x, v); };
        loop_two_paths(
            b.row_ptr, b.col, v, ok, ok, [&](int, int32_t, int32_t w) { loop_add(keys, vals, mask, w); },
            [](int) {}, sA, sSt, sPre, wtmp);
        // opposite vertices
        u64 destroyed = 0;
        for (uint32_t i = threadIdx.x; i <= mask; i += BLOCK) {
            const int32_t w = keys[i];
            const u64 y = vals[i];
            if (w == LOOP_EMPTY || y < 2) continue;
            const u64 t = y * (y - 1) / 2;
            destroyed += t;
            if (b.stamp[w] > r) dec_deg(b, w, t, r);
        }
        // middle vertices: c - 1 per 2-path, summed per middle over its chunk
        for (int i = threadIdx.x; i < BLOCK; i += BLOCK) sLoss[i] = 0;
        __syncthreads();
        loop_two_paths(
            b.row_ptr, b.col, v, ok, ok,
            [&](int i, int32_t, int32_t w) {
                const u64 y = loop_get(keys, vals, mask, w);
                if (y > 1) atomicAdd(&sLoss[i], y - 1);
            },
            [&](int cnt) {
                for (int i = threadIdx.x; i < cnt; i += BLOCK) {
                    const u64 l = sLoss[i];
                    const int32_t a = sA[i];
                    if (l && b.stamp[a] > r) dec_deg(b, a, l, r);
                    sLoss[i] = 0;
                }
            },
            sA, sSt, sPre, wtmp);
        destroyed = wave_sum(destroyed);
        if (lane() == 0) sRed[threadIdx.x / WAVE] = destroyed;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 t = 0;
            for (int i = 0; i < WAVES_PER_BLOCK; i++) t += sRed[i];
            add_destroyed(b, v, t);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- h >= 4

// Items (v, w): v in the frontier, w an allowed neighbour of v.  The engine
// counts the (h-2)-cliques of the sub-DAG on N+(w) ∩ N(v) ∩ allowed.
struct PeelCtx {
    PeelBufs b;
    int cls;
    __device__ __forceinline__ int32_t root(int64_t it) const { return b.item_w[cls * b.item_cap + it]; }
    __device__ __forceinline__ bool accept(int64_t it, int32_t x) const {
        const int32_t v = b.item_v[cls * b.item_cap + it];
        if (!allowed(b.stamp[x], b.ctl->round, x, v)) return false;
        return eset_has(b.eset, b.eset_bits, v, x);
    }
    __device__ __forceinline__ void add(int32_t x, u64 cnt) const {
        const int32_t r = b.ctl->round;
        if (b.stamp[x] > r) dec_deg(b, x, cnt, r);
    }
    __device__ __forceinline__ void add_prefix(int64_t it, u64 t) const {
        const int32_t r = b.ctl->round;
        const int32_t w = root(it);
        if (b.stamp[w] > r) dec_deg(b, w, t, r);
        add_destroyed(b, b.item_v[cls * b.item_cap + it], t);
    }
};

__device__ __forceinline__ int item_class(int d, int R) {
    if (d < R) return -1;
    if (d <= 64) return 0;
    if (R <= 2) return d <= 2048 ? 1 : 2;
    if (d <= 256) return 1;
    if (d <= 768) return 2;
    if (d <= 1280) return 3;
    return 4;
}

// One wave per chunk item (v, c): the neighbours N(v)[c * CHUNK4, ...) of
// frontier vertex v.  A vertex in no alive clique at the start of the round
// (degree 0) destroys nothing, and a neighbour w of degree 0 shares no clique
// with v: neither makes items.  The degrees do not change during this kernel
// (the engines run after it).
__global__ __launch_bounds__(BLOCK) void k_peel_items(PeelBufs b, int R) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nB = c->nB[cur];
    if (c->nF[cur] == 0 || nB == 0) return;
    const int32_t r = c->round;
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const int wv = threadIdx.x / WAVE;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nB; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int64_t item = Bc[it];
        const int32_t v = (int32_t)(item >> 32), ch = (int32_t)(item & 0xffffffff);
        if (b.deg[v] == 0) continue;                          // wave-uniform
        const int64_t e = b.row_ptr[v] + (int64_t)ch * CHUNK4 + lane();
        int cls = -1;
        int32_t w = -1;
        if (e < b.row_ptr[v + 1]) {
            w = b.col[e];
            if (allowed(b.stamp[w], r, w, v) && b.deg[w] != 0)
                cls = item_class((int)(b.row_ptr[w + 1] - b.dag_off[w]), R);
        }
        for (int q = 0; q < 5; q++) {
            u64 m = __ballot(cls == q);
            if (!m) continue;
            int leader = __builtin_ctzll(m);
            int32_t base = 0;
            if (lane() == leader) base = atomicAdd(&c->nitems[q], __popcll(m));
            base = __shfl(base, leader, WAVE);
            if (cls == q) {
                int64_t pos = (int64_t)q * b.item_cap + base + __popcll(m & lanemask_lt());
                b.item_v[pos] = v;
                b.item_w[pos] = w;
            }
        }
    }
}

// The edge set of the h >= 4 peel: every DAG arc (v, x) with both ends in the
// peel's starting vertex set (one wave per listed vertex, its out-row).
__global__ __launch_bounds__(BLOCK) void k_eset_fill(PeelBufs b, const int32_t *list, const int32_t *count,
                                                     u64 *t) {
    const int32_t cnt = *count;
    const u64 mask = (1ull << b.eset_bits) - 1ull;
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < cnt; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = list[i];
        for (int64_t e = b.dag_off[v] + lane(); e < b.row_ptr[v + 1]; e += WAVE) {
            const int32_t x = b.col[e];
            if (b.stamp[x] != ALIVE) continue;
            const u64 key = eset_key(v, x);
            for (u64 j = eset_slot(key, b.eset_bits);; j = (j + 1) & mask) {
                const u64 prev = atomicCAS((unsigned long long *)&t[j], (unsigned long long)ESET_EMPTY,
                                           (unsigned long long)key);
                if (prev == ESET_EMPTY || prev == key) break;
            }
        }
    }
}


// ---------------------------------------------------------------- h >= 4, root mode
//
// The cliques a frontier vertex v destroys are {v} plus the (h-1)-cliques of
// G[C_v], C_v = the neighbours of v allowed in this round (alive at its
// start and not a frontier vertex of smaller rank: the owner rule).  An item
// is v itself: its row is scanned once into C_v (rank order, so an arc of the
// sub-DAG on C_v goes from a smaller to a larger local index), the arcs are
// found by probing the out-lists of C_v's members against a hash of C_v, and
// the members' (h-1)-clique counts come from the bitmap counting of the
// enumeration engine, with no work per clique.  Every member loses its count
// and v's total is the number of cliques it destroys.  A neighbour of clique-
// degree 0 is in no alive clique and is left out of C_v (a neighbour x that
// shares a clique with v keeps a degree >= 1 until v itself takes that clique
// away, so a 0 read while other items decrement x is still final for v).
// When C_v would exceed ROOT_CAP members, each chunk item of v takes its
// ROOT_CAP neighbours w in turn and counts the (h-2)-cliques of
// N+(w) ∩ C_v, one level shallower: every clique through v is seen once, from
// its member of smallest rank after v.

// the members of C_v (or of N+(w) ∩ C_v) one block keeps
struct RootAccept {
    PeelBufs b;
    int32_t v, r;
    __device__ __forceinline__ bool accept(int64_t, int32_t x) const {
        return allowed(b.stamp[x], r, x, v) && b.deg[x] != 0;
    }
};
struct RootAcceptIn {           // also adjacent to v: a binary search in v's row (sorted by rank)
    PeelBufs b;
    int32_t v, r;
    int64_t s0, s1;
    __device__ __forceinline__ bool accept(int64_t, int32_t x) const {
        return allowed(b.stamp[x], r, x, v) && b.deg[x] != 0 && bsearch_i32(b.col, s0, s1, x) >= 0;
    }
};

// allowed entries of col[s0, s0 + d), counted over the block
template <class Acc>
__device__ int block_count_accepted(const Acc &acc, const int32_t *col, int64_t s0, int64_t d, int32_t *wtmp) {
    int32_t c = 0;
    for (int64_t i = threadIdx.x; i < d; i += BLOCK) c += acc.accept(0, col[s0 + i]) ? 1 : 0;
    c = wave_sum(c);
    if (lane() == 0) wtmp[threadIdx.x / WAVE] = c;
    __syncthreads();
    int32_t t = 0;
    for (int i = 0; i < WAVES_PER_BLOCK; i++) t += wtmp[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void hash_insert16(int32_t *keys, uint16_t *vals, int bits, int32_t x, int v) {
    const uint32_t m = (1u << bits) - 1u;
    uint32_t slot = hash_slot(x, bits);
    while (true) {
        const int32_t prev = atomicCAS(&keys[slot], HASH_EMPTY, x);
        if (prev == HASH_EMPTY || prev == x) {
            vals[slot] = (uint16_t)v;
            return;
        }
        slot = (slot + 1) & m;
    }
}

__device__ __forceinline__ int hash_find16(const int32_t *keys, const uint16_t *vals, int bits, int32_t x) {
    const uint32_t m = (1u << bits) - 1u;
    uint32_t slot = hash_slot(x, bits);
    while (true) {
        const int32_t k = keys[slot];
        if (k == x) return vals[slot];
        if (k == HASH_EMPTY) return -1;
        slot = (slot + 1) & m;
    }
}

struct RootLds {
    int32_t C[ROOT_CAP];
    int32_t key[1 << ROOT_HB];
    uint16_t val[1 << ROOT_HB];
    int32_t pre[ROOT_CAP];
    u64 cnt[ROOT_CAP];
    int32_t wtmp[WAVES_PER_BLOCK];
    u64 tot[WAVES_PER_BLOCK];
};

// One member x of a candidate set, on one wave: the cliques of the set's
// vertex through x, from the bitmap rows (S, W words each, restricted to
// mask).  As first member x passes to every y above it the count of the
// RR-cliques x < y < ... (lanes take the y's, 64 at a time); as last member
// it counts the (RR-1)-cliques below it.  The counts of the y's and of x go
// to cnt (global or LDS); returns the number with x first (every lane).
// sA/sB/q: this wave's LDS (W words, W words, 2 * WAVE ids).
template <int RR, int W>
__device__ u64 root_member_work(int x, const u64 *S, const u64 *mask, u64 *cnt, u64 *sA, u64 *sB, int32_t *q) {
    const int L = lane();
    for (int w = L; w < W; w += WAVE) {
        sA[w] = row_above<W>(S, x, w) & mask[w];
        sB[w] = row_below<W>(S, x, w) & mask[w];
    }
    __builtin_amdgcn_wave_barrier();
    u64 first = 0, last = 0;
    for (int role = 0; role < 2; role++) {
        const u64 *X = role == 0 ? sA : sB;
        // the set bits of X go through a queue of 2 * WAVE ids; whenever it
        // holds a wave's worth (and at the end, whatever is left) each lane
        // takes one y
        auto drain = [&](int take) {
            if (L < take) {
                const int y = q[L];
                if constexpr (RR == 2) {
                    if (role == 0) {
                        atomicAdd(&cnt[y], 1ull);
                        first += 1;
                    } else {
                        last += 1;
                    }
                } else if constexpr (RR == 3) {
                    // popcounts streamed over the words at and above y's
                    u64 cy = 0;
#pragma unroll 4
                    for (int k = y >> 6; k < W; k++) cy += (u64)__popcll(X[k] & row_above<W>(S, y, k));
                    if (role == 0) {
                        if (cy) {
                            atomicAdd(&cnt[y], cy);
                            first += cy;
                        }
                    } else {
                        last += cy;
                    }
                } else {
                    u64 M2[W];
#pragma unroll
                    for (int k = 0; k < W; k++) M2[k] = X[k] & row_above<W>(S, y, k);
                    if (role == 0) {
                        const u64 cy = forward<RR - 3, W>(M2, S, cnt);
                        if (cy) {
                            atomicAdd(&cnt[y], cy);
                            first += cy;
                        }
                    } else {
                        last += count_in<RR - 2, W>(M2, S);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        };
        int qn = 0;
        for (int w = 0; w < W; w++) {
            const u64 m = X[w];
            if (((m >> L) & 1ull) != 0) q[qn + __popcll(m & lanemask_lt())] = w * 64 + L;
            qn += __popcll(m);
            __builtin_amdgcn_wave_barrier();
            if (qn >= WAVE) {
                drain(WAVE);
                // the rest of the queue (fewer than WAVE ids) to its front
                const int rest = qn - WAVE;
                int32_t keep = 0;
                if (L < rest) keep = q[WAVE + L];
                __builtin_amdgcn_wave_barrier();
                if (L < rest) q[L] = keep;
                qn = rest;
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (qn > 0) drain(qn);
    }
    first = wave_sum(first);
    last = wave_sum(last);
    if (L == 0 && first + last) atomicAdd(&cnt[x], first + last);
    __builtin_amdgcn_wave_barrier();
    return first;
}

template <int RR>
__device__ u64 root_member(int x, int W, const u64 *S, const u64 *mask, u64 *cnt, u64 *sA, u64 *sB, int32_t *q) {
    if (W == 4) return root_member_work<RR, 4>(x, S, mask, cnt, sA, sB, q);
    if (W == 12) return root_member_work<RR, 12>(x, S, mask, cnt, sA, sB, q);
    if (W == 20) return root_member_work<RR, 20>(x, S, mask, cnt, sA, sB, q);
    return root_member_work<RR, 32>(x, S, mask, cnt, sA, sB, q);
}

// The RR-cliques of the sub-DAG on L.C[0, dd) (rank order): the members'
// counts in L.cnt, the total returned to every thread.  S: this block's
// bitmap rows in global memory (ROOT_SW words, then W mask words).  pairs:
// out-list entries probed (thread 0).  sA/sB/q: the calling wave's LDS for
// root_member.
template <int RR>
__device__ u64 root_count(const PeelBufs &b, int dd, RootLds &L, u64 *S, u64 *pairs, u64 *sA, u64 *sB, int32_t *q) {
    for (int i = threadIdx.x; i < (1 << ROOT_HB); i += BLOCK) L.key[i] = HASH_EMPTY;
    __syncthreads();
    const int W = dd <= 256 ? 4 : dd <= 768 ? 12 : dd <= 1280 ? 20 : 32;
    for (int i = threadIdx.x; i < dd; i += BLOCK) {
        const int32_t x = L.C[i];
        hash_insert16(L.key, L.val, ROOT_HB, x, i);
        L.cnt[i] = 0;
        L.pre[i] = (int32_t)(b.row_ptr[x + 1] - b.dag_off[x]);
    }
    for (int i = threadIdx.x; i < dd * W; i += BLOCK) S[i] = 0;
    u64 *mask = S + ROOT_SW;                           // every member counts (the accept test applied the owner rule)
    for (int w = threadIdx.x; w < W; w += BLOCK) {
        const int rem = dd - w * 64;
        mask[w] = rem >= 64 ? ~0ull : (rem > 0 ? (1ull << rem) - 1ull : 0ull);
    }
    __syncthreads();
    const int32_t tot_pairs = block_incl_scan_lds(L.pre, dd, L.wtmp);
    if (threadIdx.x == 0) *pairs += (u64)tot_pairs;
    for (int32_t base = 0; base < tot_pairs; base += BLOCK) {
        const int32_t p = base + threadIdx.x;
        if (p >= tot_pairs) continue;
        const int i = upper_bound_i32(L.pre, dd, p);
        const int32_t off = p - (i ? L.pre[i - 1] : 0);
        const int32_t y = b.col[b.dag_off[L.C[i]] + off];
        const int j = hash_find16(L.key, L.val, ROOT_HB, y);
        if (j < 0) continue;
        atomicOr(&S[(size_t)i * W + (j >> 6)], 1ull << (j & 63));
        atomicOr(&S[(size_t)j * W + (i >> 6)], 1ull << (i & 63));
    }
    __threadfence_block();
    __syncthreads();
    u64 hits = 0;
    for (int x = threadIdx.x / WAVE; x < dd; x += WAVES_PER_BLOCK)
        hits += root_member<RR>(x, W, S, mask, L.cnt, sA, sB, q);
    if (lane() == 0) L.tot[threadIdx.x / WAVE] = hits;
    __syncthreads();
    u64 total = 0;
    for (int i = 0; i < WAVES_PER_BLOCK; i++) total += L.tot[i];
    __syncthreads();
    return total;
}

// every member of L.C[0, dd) that survives the round loses its count
__device__ __forceinline__ void root_flush(const PeelBufs &b, int dd, const RootLds &L, int32_t r) {
    for (int i = threadIdx.x; i < dd; i += BLOCK) {
        const u64 c = L.cnt[i];
        const int32_t x = L.C[i];
        if (c && b.stamp[x] > r) dec_deg(b, x, c, r);
    }
    __syncthreads();
}

// the main kernel's counted work (root mode): lane 0 of every wave holds its
// wave's tallies; one atomic each per block
__device__ __forceinline__ void add_work3(const PeelBufs &b, u64 pairs, u64 cands, u64 entries) {
    __shared__ u64 sW[3][WAVES_PER_BLOCK];
    const int wv = threadIdx.x / WAVE;
    if (lane() == 0) {
        sW[0][wv] = pairs;
        sW[1][wv] = cands;
        sW[2][wv] = entries;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        u64 t = 0;
        for (int i = 0; i < WAVES_PER_BLOCK; i++) t += sW[threadIdx.x][i];
        if (t) atomicAdd(&b.ctl->work[threadIdx.x], t);
    }
}

// A single-workgroup item (v, chunk) of Big: v's whole C_v in one workgroup
// (its chunk 0), or, when C_v exceeds ROOT_CAP members, the (h-2)-cliques of
// N+(w) ∩ C_v for every neighbour w of this chunk.
template <int R>
__device__ void root_big_item(const PeelBufs &b, int32_t v, int32_t ch, int32_t r, RootLds &L, u64 *S, u64 &pairs,
                              u64 &cands, u64 &entries, u64 *sA, u64 *sB, int32_t *q) {
    if (b.deg[v] == 0) return;                         // a frontier vertex's degree is fixed in its round
    const int64_t s0 = b.row_ptr[v], d = b.row_ptr[v + 1] - s0;
    const RootAccept acc{b, v, r};
    int dd;
    if (d <= ROOT_CAP) {
        dd = block_load_candidates(acc, 0, b.col, s0, (int)d, L.C, L.wtmp);
        entries += (u64)d;
    } else {
        dd = block_count_accepted(acc, b.col, s0, d, L.wtmp);
        entries += (u64)d;
        if (dd <= ROOT_CAP) {
            if (ch != 0) return;                       // chunk 0 takes the whole vertex
            // the accepted entries in row order, ROOT_CAP at a time (a
            // degree falling to 0 meanwhile only drops an entry: dd stays a bound)
            int got = 0;
            for (int64_t o = 0; o < d; o += ROOT_CAP) {
                const int part = (int)min((int64_t)ROOT_CAP, d - o);
                got += block_load_candidates(acc, 0, b.col, s0 + o, part, L.C + got, L.wtmp);
            }
            dd = got;
        } else {
            // C_v too large for one workgroup: the neighbours w of this chunk in turn
            const int64_t w0 = (int64_t)ch * ROOT_CAP, w1 = min(d, w0 + ROOT_CAP);
            const RootAcceptIn accw{b, v, r, s0, s0 + d};
            u64 destroyed = 0;
            for (int64_t e = s0 + w0; e < s0 + w1; e++) {
                const int32_t w = b.col[e];
                // w's degree may be falling under other items: one thread decides for the block
                if (threadIdx.x == 0) L.wtmp[0] = acc.accept(0, w) ? 1 : 0;
                __syncthreads();
                const bool take = L.wtmp[0] != 0;
                __syncthreads();
                if (!take) continue;
                const int64_t o0 = b.dag_off[w];
                const int dw = (int)(b.row_ptr[w + 1] - o0);   // <= maxdout <= ROOT_CAP in root mode
                if (dw < R - 1) continue;
                const int de = block_load_candidates(accw, 0, b.col, o0, dw, L.C, L.wtmp);
                entries += (u64)dw;
                if (de < R - 1) continue;
                cands += (u64)de;
                const u64 t = root_count<R - 1>(b, de, L, S, &pairs, sA, sB, q);
                root_flush(b, de, L, r);
                if (threadIdx.x == 0 && t) {
                    if (b.stamp[w] > r) dec_deg(b, w, t, r);
                    destroyed += t;
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) add_destroyed(b, v, destroyed);
            return;
        }
    }
    if (dd < R) return;
    cands += (u64)dd;
    const u64 t = root_count<R>(b, dd, L, S, &pairs, sA, sB, q);
    root_flush(b, dd, L, r);
    if (threadIdx.x == 0) add_destroyed(b, v, t);
}

// index of x in the sorted list a[0, n), n <= 4096, or -1: a lower bound
// by halving steps of fixed count, so that independent searches of one lane
// interleave
__device__ __forceinline__ int lds_find_fixed(const int32_t *a, int n, int32_t x) {
    int pos = 0;
#pragma unroll
    for (int step = 2048; step > 0; step >>= 1) {
        const int q = pos + step;
        if (q <= n && a[q - 1] < x) pos = q;
    }
    return pos < n && a[pos] == x ? pos : -1;
}

// first index in the sorted list a[0, n) holding x, or -1
__device__ __forceinline__ int lds_find(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && a[lo] == x ? lo : -1;
}

// one step of a member's out-list walk: EA entries per lane loaded before
// their (fixed-step, interleaved) searches in v's row
template <int EA>
__device__ __forceinline__ void root_walk(const int32_t *col, int64_t e0, int64_t o1, const int32_t *sR, int d, u64 *rw,
                                          int L) {
    int32_t y[EA];
#pragma unroll
    for (int t = 0; t < EA; t++) {
        const int64_t e = e0 + t * WAVE + L;
        y[t] = e < o1 ? col[e] : -1;
    }
#pragma unroll
    for (int t = 0; t < EA; t++) {
        const int j = y[t] >= 0 ? lds_find_fixed(sR, d, y[t]) : -1;
        if (j >= 0) atomicOr((unsigned long long *)&rw[j >> 6], 1ull << (j & 63));
    }
}

// cliques counted per member of a sliced vertex (each clique once for every
// one of its h - 1 members besides v)
__device__ __forceinline__ void add_destroyed_m(const PeelBufs &b, int32_t v, u64 t) {
    if (t) atomicAdd(&b.gs[graph_of(b, v)].destroyed_m, t);
}

// Arc discovery.  A sliced vertex v (a row of ROOT_WAVE_MAX + 1 .. 2048 (4096 at h = 4)
// entries) has a region in this round's half of the arena: one bitmap row
// per entry of v's row, indexed by row position, and the mask of the entries
// that take part in v's cliques (alive, and not a frontier vertex of smaller
// rank: the owner rule).  An item (v, slice) stands for ROOT_SUB
// workgroups; each copies v's row to LDS and gives each of its waves one
// entry x, whose lanes walk N+(x) and find their entries in v's row by
// binary search (both are in rank order), setting the bit of every arc
// (each arc is found once, from its lower end, and set in the lower end's
// row, which the wave builds in LDS and writes out whole: rows hold only the
// bits above their own entry, so no region needs clearing and no arc an
// atomic in global memory).  The first workgroup of v also writes the mask.
// Wave items (rows of at most ROOT_WAVE_MAX entries): one wave does the
// whole count, C_v in one 64-bit word per member.
template <int R>
__global__ __launch_bounds__(BLOCK) void k_root_edges(PeelBufs b) {
    __shared__ int32_t sR[ROOT_SLICED_H4];
    __shared__ int32_t wC[WAVES_PER_BLOCK][64];
    __shared__ int32_t wKey[WAVES_PER_BLOCK][128];
    __shared__ int32_t wVal[WAVES_PER_BLOCK][128];
    __shared__ int32_t wPre[WAVES_PER_BLOCK][64];
    __shared__ int64_t wSt[WAVES_PER_BLOCK][64];
    __shared__ u64 wCnt[WAVES_PER_BLOCK][64];
    __shared__ u64 wS[WAVES_PER_BLOCK][64];
    __shared__ u64 wRow[WAVES_PER_BLOCK][64];
    PeelCtl *c = b.ctl;
    // the round's fields of both halves loaded together, the half in use picked after
    const int32_t cur = c->cur, r = c->round;
    const int64_t nalive = c->n_alive;
    const int2 f2 = *(const int2 *)c->nF, b2 = *(const int2 *)c->nB, t2 = *(const int2 *)c->nT;
    const int32_t nFc = cur ? f2.y : f2.x;
    // a round of the one graph that removes every alive vertex leaves no
    // survivor whose degree could fall: nothing to count (its end sets the
    // graph's clique count to zero)
    if (nFc == 0 || (b.G == 1 && (int64_t)nFc == nalive)) return;
    const int32_t nG = cur ? b2.y : b2.x, nI = cur ? t2.y : t2.x;
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    u64 *bits = b.rbits + (size_t)cur * b.rcap;
    const int wv = threadIdx.x / WAVE, L = lane();
    u64 pairs = 0, cands = 0, entries = 0;
    for (int64_t it = blockIdx.x; it < (int64_t)nG * ROOT_SUB; it += gridDim.x) {
        const int64_t item = Bc[it / ROOT_SUB];
        const int32_t v = (int32_t)(item >> 32), sl = (int32_t)(item & 0xffffffff);
        const int sub = (int)(it % ROOT_SUB);
        const u64 dv = b.deg[v];
        const int64_t s0 = b.row_ptr[v], s1 = b.row_ptr[v + 1], rb = b.rbase[v];
        if (dv == 0) continue;                         // block-uniform: fixed in v's round
        const int d = (int)(s1 - s0);                  // <= root_sliced_max(h) for a sliced vertex
        for (int i = threadIdx.x; i < d; i += BLOCK) sR[i] = b.col[s0 + i];
        __syncthreads();
        const int W = root_words(d);
        u64 *S = bits + rb;
        if (sl == 0 && sub == 0) {
            // the mask: wave wv takes word base / 64 + wv of each pass
            u64 *mask = S + (int64_t)d * W;
            for (int base = 0; base < W * 64; base += BLOCK) {
                const int i = base + threadIdx.x;
                bool ok = false;
                if (i < d) {
                    const int32_t x = sR[i];
                    ok = allowed(b.stamp[x], r, x, v);
                }
                const u64 bm = __ballot(ok);
                if (L == 0 && (i >> 6) < W) mask[i >> 6] = bm;
                if (L == 0) cands += (u64)__popcll(bm);
            }
            if (threadIdx.x == 0) entries += (u64)d;
        }
        const int m = sl * ROOT_SL + sub * WAVES_PER_BLOCK + wv;
        if (m < d) {
            const int32_t x = sR[m];
            const int32_t sx = b.stamp[x];
            const int64_t o0 = b.dag_off[x], o1 = b.row_ptr[x + 1];   // with the stamp
            if (allowed(sx, r, x, v)) {                    // wave-uniform
                // the upper part of row m (bits j > m) in LDS, then written
                // out whole from word m / 64 on
                u64 *rw = wRow[wv];
                for (int w = L; w < W; w += WAVE) rw[w] = 0;
                __builtin_amdgcn_wave_barrier();
                if (L == 0) pairs += (u64)(o1 - o0);
                // a long out-list takes 16 entries per lane a step, a short one 4
                for (int64_t e0 = o0; e0 < o1;) {
                    if (o1 - e0 > 8 * WAVE) {
                        root_walk<16>(b.col, e0, o1, sR, d, rw, L);
                        e0 += 16 * WAVE;
                    } else {
                        root_walk<4>(b.col, e0, o1, sR, d, rw, L);
                        e0 += 4 * WAVE;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                for (int w = (m >> 6) + L; w < W; w += WAVE) S[(size_t)m * W + w] = rw[w];
            }
        }
        __syncthreads();
    }
    // wave items
    for (int i = L; i < 128; i += WAVE) wKey[wv][i] = HASH_EMPTY;
    wCnt[wv][L] = 0;
    wS[wv][L] = 0;
    __builtin_amdgcn_wave_barrier();
    const int64_t *Tc = b.T + (size_t)cur * b.tcap;
    DestroyedTally tally;
    u64 wpairs = 0, wcands = 0, wentries = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nI; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = (int32_t)(Tc[it] >> 32);
        if (b.deg[v] == 0) continue;                   // wave-uniform
        const int64_t s0 = b.row_ptr[v];
        const int d = (int)(b.row_ptr[v + 1] - s0);    // <= ROOT_WAVE_MAX
        int32_t x = -1;
        bool keep = false;
        if (L < d) {
            x = b.col[s0 + L];
            keep = allowed(b.stamp[x], r, x, v) && b.deg[x] != 0;
        }
        const u64 km = __ballot(keep);
        const int dd = __popcll(km);
        wentries += (u64)d;
        if (dd < R) continue;                          // wave-uniform
        wcands += (u64)dd;
        const int li = __popcll(km & lanemask_lt());   // rank order kept
        if (keep) {
            wC[wv][li] = x;
            hash_insert(wKey[wv], wVal[wv], 7, x, li);
        }
        int32_t len = 0;
        int64_t st = 0;
        if (keep) {
            st = b.dag_off[x];
            len = (int32_t)(b.row_ptr[x + 1] - st);
        }
        const int32_t inc = wave_incl_scan(len);
        if (keep) {
            wPre[wv][li] = inc;
            wSt[wv][li] = st;
        }
        const int32_t tot = __shfl(inc, WAVE - 1, WAVE);
        wpairs += (u64)tot;
        __builtin_amdgcn_wave_barrier();
        for (int32_t base = 0; base < tot; base += WAVE) {
            const int32_t p = base + L;
            if (p < tot) {
                const int i = upper_bound_i32(wPre[wv], dd, p);
                const int32_t off = p - (i ? wPre[wv][i - 1] : 0);
                const int32_t y = b.col[wSt[wv][i] + off];
                const int j = hash_find(wKey[wv], wVal[wv], 7, y);
                if (j >= 0) {
                    atomicOr(&wS[wv][i], 1ull << j);
                    atomicOr(&wS[wv][j], 1ull << i);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        u64 t = 0;
        if (L < dd) t = bitmap_node_work<R, 1>(L, &wS[wv][0], &wCnt[wv][0]);
        t = wave_sum(t);
        __builtin_amdgcn_wave_barrier();
        const u64 cL = L < dd ? wCnt[wv][L] : 0;
        const int32_t xL = L < dd ? wC[wv][L] : 0;
        if (cL && b.stamp[xL] > r) dec_deg(b, xL, cL, r);
        if (L == 0) tally.add(b, v, t);
        __builtin_amdgcn_wave_barrier();
        for (int i = L; i < 128; i += WAVE) wKey[wv][i] = HASH_EMPTY;
        wCnt[wv][L] = 0;
        wS[wv][L] = 0;
        __builtin_amdgcn_wave_barrier();
    }
    if (L == 0) tally.flush(b);
    if (b.count_work) {
        // lane 0 of every wave: its wave items, its entries' probes and the
        // masks it wrote; thread 0 also the scanned rows
        add_work3(b, wpairs + (L == 0 ? pairs : 0), wcands + (L == 0 ? cands : 0),
                  wentries + (threadIdx.x == 0 ? entries : 0));
    }
}

// One entry x of a sliced vertex v's row, on one wave: the R-cliques of v's
// candidate graph that hold x, i.e. the (R-1)-cliques among x's neighbours
// there, N (in LDS): the bits above x from row x, those below x from the
// rows of the entries before it (bit x of each), restricted to the mask.  Lanes take the members y of N (through
// a queue of 2 * WAVE ids, 64 at a time) and count the (R-2)-cliques above y
// in N & N(y).  Returns the count to every lane; *words gets the 64-bit
// words this lane ANDed and counted at the first level.
template <int R, int W>
__device__ u64 root_own_work(int x, const u64 *S, const u64 *mask, u64 *sN, int32_t *q, u64 *words) {
    const int L = lane(), xw = x >> 6;
    // x's neighbours: above x from its own row, below x from bit x of the
    // rows before it (one 64-bit ballot per 64 rows)
    for (int w = L; w < W; w += WAVE) sN[w] = w >= xw ? S[(size_t)x * W + w] : 0ull;
    __builtin_amdgcn_wave_barrier();
    // eight loads in flight per lane before their ballots
    constexpr int GB = 8;
    for (int j0 = 0; j0 < x; j0 += GB * WAVE) {
        u64 v[GB];
#pragma unroll
        for (int t = 0; t < GB; t++) {
            const int j = j0 + t * WAVE + L;
            v[t] = j < x ? S[(size_t)j * W + xw] : 0ull;
        }
#pragma unroll
        for (int t = 0; t < GB; t++) {
            const u64 bw = __ballot(((v[t] >> (x & 63)) & 1ull) != 0);
            if (L == 0 && j0 + t * WAVE < x) sN[(j0 >> 6) + t] |= bw;
        }
        __builtin_amdgcn_wave_barrier();
    }
    for (int w = L; w < W; w += WAVE) sN[w] &= mask[w];
    __builtin_amdgcn_wave_barrier();
    u64 c = 0, nw = 0;
    auto drain = [&](int take) {
        if (L < take) {
            const int y = q[L];
            nw += (u64)(W - (y >> 6));
            if constexpr (R == 3) {
                // every word at or above y's, all loads issued before their counts
                const int yw = y >> 6;
#pragma unroll
                for (int k = 0; k < W; k++)
                    if (k >= yw) c += (u64)__popcll(sN[k] & row_above<W>(S, y, k));
            } else {
                u64 M2[W];
#pragma unroll
                for (int k = 0; k < W; k++) M2[k] = sN[k] & row_above<W>(S, y, k);
                c += count_in<R - 2, W>(M2, S);
            }
        }
        __builtin_amdgcn_wave_barrier();
    };
    int qn = 0;
    for (int w = 0; w < W; w++) {
        const u64 m = sN[w];
        if (((m >> L) & 1ull) != 0) q[qn + __popcll(m & lanemask_lt())] = w * 64 + L;
        qn += __popcll(m);
        __builtin_amdgcn_wave_barrier();
        if (qn >= WAVE) {
            drain(WAVE);
            // the rest of the queue (fewer than WAVE ids) to its front
            const int rest = qn - WAVE;
            int32_t keep = 0;
            if (L < rest) keep = q[WAVE + L];
            __builtin_amdgcn_wave_barrier();
            if (L < rest) q[L] = keep;
            qn = rest;
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (qn > 0) drain(qn);
    *words += nw;
    return wave_sum(c);
}

template <int R>
__device__ u64 root_own(int x, int W, const u64 *S, const u64 *mask, u64 *sN, int32_t *q, u64 *words) {
    if (W == 4) return root_own_work<R, 4>(x, S, mask, sN, q, words);
    if (W == 12) return root_own_work<R, 12>(x, S, mask, sN, q, words);
    if (W == 20) return root_own_work<R, 20>(x, S, mask, sN, q, words);
    if constexpr (R == 3) {
        if (W == 64) return root_own_work<R, 64>(x, S, mask, sN, q, words);
    }
    return root_own_work<R, 32>(x, S, mask, sN, q, words);
}

// Counting.  SLICED: one wave per entry of a sliced vertex v's row that the
// mask lets take part; the wave counts the cliques of v that hold its entry
// x and takes them off x's degree at once (x a survivor).  No entry waits
// for another: each clique is counted once by every one of its members.
// BIG: the single-workgroup items, whose 56 KB of LDS would hold the sliced
// counting to two workgroups per CU; they run as a launch of their own.
// (The round ends in its own kernel too: ending it in the last workgroup to
// finish would cost every workgroup a device-scope fence, which writes back
// its L2, every round.)
template <int R, bool SLICED, bool BIG>
__global__ __launch_bounds__(BLOCK) void k_root_count(PeelBufs b, u64 *gS) {
    __shared__ int32_t sQ[WAVES_PER_BLOCK][2 * WAVE];
    __shared__ u64 sN64[WAVES_PER_BLOCK][64];
    __shared__ u64 sAB[WAVES_PER_BLOCK][2][32];
    PeelCtl *c = b.ctl;
    // the round's fields of both halves loaded together, the half in use picked after
    const int32_t cur = c->cur, r = c->round;
    const int64_t nalive = c->n_alive;
    const int2 f2 = *(const int2 *)c->nF, b2 = *(const int2 *)c->nB, g2 = *(const int2 *)c->nBig;
    const int32_t nFc = cur ? f2.y : f2.x;
    const bool any = nFc != 0 && !(b.G == 1 && (int64_t)nFc == nalive);   // (as in k_root_edges)
    const int32_t nG = any ? (cur ? b2.y : b2.x) : 0, nBig = any ? (cur ? g2.y : g2.x) : 0;
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const u64 *bits = b.rbits + (size_t)cur * b.rcap;
    const int wv = threadIdx.x / WAVE;
    u64 pairs = 0, cands = 0, entries = 0, words = 0;
    // wave tasks: entry (slice item, offset) of a sliced vertex
    const int64_t ntask = SLICED ? (int64_t)nG * ROOT_SL : 0, nwaves = (int64_t)gridDim.x * WAVES_PER_BLOCK;
    for (int64_t t = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; t < ntask; t += nwaves) {
        const int64_t item = Bc[t / ROOT_SL];
        const int32_t v = (int32_t)(item >> 32), sl = (int32_t)(item & 0xffffffff);
        const int m = sl * ROOT_SL + (int)(t % ROOT_SL);
        const u64 dv = b.deg[v];
        const int64_t s0 = b.row_ptr[v], s1 = b.row_ptr[v + 1], rb = b.rbase[v];
        if (dv == 0) continue;                         // its items made no arcs either
        const int d = (int)(s1 - s0);
        if (m >= d) continue;
        const int W = root_words(d);
        const u64 *S = bits + rb;
        const u64 *mask = S + (int64_t)d * W;
        const int32_t x = b.col[s0 + m];              // with the mask word
        if (((mask[m >> 6] >> (m & 63)) & 1ull) == 0) continue;
        const int32_t sx = b.stamp[x];                 // in flight during the count
        const u64 cx = root_own<R>(m, W, S, mask, sN64[wv], sQ[wv], &words);
        if (cx && lane() == 0) {
            if (sx > r) dec_deg(b, x, cx, r);
            add_destroyed_m(b, v, cx);
        }
    }
    if constexpr (BIG) {
        __shared__ RootLds L;
        const int64_t *Gc = b.Big + (size_t)cur * b.bigcap;
        u64 *Sg = gS + (size_t)blockIdx.x * ROOT_SLICE;
        for (int64_t it = blockIdx.x; it < nBig; it += gridDim.x) {
            const int64_t item = Gc[it];
            root_big_item<R>(b, (int32_t)(item >> 32), (int32_t)(item & 0xffffffff), r, L, Sg, pairs, cands,
                             entries, sAB[wv][0], sAB[wv][1], sQ[wv]);
        }
    } else {
        (void)nBig;
        (void)gS;
    }
    if (b.count_work) {
        add_work3(b, threadIdx.x == 0 ? pairs : 0, threadIdx.x == 0 ? cands : 0, threadIdx.x == 0 ? entries : 0);
        const u64 wsum = wave_sum(words);
        if (lane() == 0 && wsum) atomicAdd(&c->work[3], wsum);
    }
}

// ---------------------------------------------------------------- adjacency compaction
//
// Between rounds, rows of removed vertices and entries pointing at them are
// dead weight for every later round.  Compaction rebuilds the CSR over the
// vertices still taking part (stamp >= current round: alive, or in the
// pending frontier), keeping each row sorted by rank so that N+(v) is again
// the tail of row v.  Vertex ids do not change.

// one wave per vertex: kept neighbours, and kept out-neighbours
// The compaction walks the alive list (alive vertices and the pending
// frontier, which were alive when the list was last rebuilt; removed ones are
// skipped): a masked peel of a small vertex set then costs its own rows, not
// a pass over every vertex.  cnt and cnt_out are zero on entry.
__global__ __launch_bounds__(BLOCK) void k_compact_count(PeelBufs b, int64_t *cnt, int32_t *cnt_out) {
    const PeelCtl *pc = b.ctl;
    const int32_t r = pc->round, lc = pc->lcur, nl = pc->nlist[lc];
    const int32_t *lst = b.lists + (size_t)lc * b.n;
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nl; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = lst[i];
        if (b.stamp[v] < r) continue;
        int64_t c = 0;
        int32_t co = 0;
        for (int64_t e = b.row_ptr[v] + lane(); e < b.row_ptr[v + 1]; e += WAVE) {
            int32_t w = b.col[e];
            bool keep = b.stamp[w] >= r;
            c += keep ? 1 : 0;
            co += (keep && w > v) ? 1 : 0;
        }
        c = wave_sum(c);
        co = wave_sum(co);
        if (lane() == 0) {
            cnt[v] = c;
            cnt_out[v] = co;
        }
    }
}

// DAG offsets of the compacted rows (a removed vertex's row is empty)
__global__ void k_compact_dag(const int64_t *nrow, const int32_t *cnt_out, int32_t n, int64_t *ndag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        ndag[v] = nrow[v + 1] - cnt_out[v];
}

__global__ __launch_bounds__(BLOCK) void k_compact_fill(PeelBufs b, const int64_t *nrow, int32_t *ncol) {
    const PeelCtl *pc = b.ctl;
    const int32_t r = pc->round, lc = pc->lcur, nl = pc->nlist[lc];
    const int32_t *lst = b.lists + (size_t)lc * b.n;
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nl; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = lst[i];
        if (b.stamp[v] < r) continue;
        int64_t o = nrow[v];
        const int64_t e1 = b.row_ptr[v + 1];
        for (int64_t e = b.row_ptr[v]; e < e1; e += WAVE) {
            int32_t w = -1;
            bool keep = false;
            if (e + lane() < e1) {
                w = b.col[e + lane()];
                keep = b.stamp[w] >= r;
            }
            u64 m = __ballot(keep);
            if (keep) ncol[o + __popcll(m & lanemask_lt())] = w;
            o += __popcll(m);
        }
    }
}

// the pending frontier's chunk items were cut for the old row lengths: redo them
__global__ void k_reset_chunks(PeelBufs b) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.ctl->nB[b.ctl->cur] = 0;
        b.ctl->htop[b.ctl->cur] = 0;
        if (b.rootmode) {
            b.ctl->nT[b.ctl->cur] = 0;
            b.ctl->nBig[b.ctl->cur] = 0;
        }
    }
}
__global__ void k_rechunk(PeelBufs b) {
    const int32_t cur = b.ctl->cur, nF = b.ctl->nF[cur];
    const int32_t *F = b.F + (size_t)cur * b.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nF; i += (int64_t)gridDim.x * blockDim.x)
        push_chunks(b, F[i], cur);
}

__global__ void k_last_row(int64_t *nrow, const int64_t *cnt, int32_t n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) nrow[n] = nrow[n - 1] + cnt[n - 1];
}

// Rebuild b.row_ptr / b.col / b.dag_off over the vertices still taking part.
static void compact_adjacency(PeelBufs &b, hipStream_t s, Scratch &sc) {
    const int32_t n = b.n;
    int64_t *cnt = sc.get_n<int64_t>(n);
    int32_t *cnt_out = sc.get_n<int32_t>(n);
    int64_t *nrow = sc.get_n<int64_t>((int64_t)n + 1);
    fill_u64((u64 *)cnt, 0, n, s);
    fill_i32(cnt_out, 0, n, s);
    k_compact_count<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, cnt, cnt_out);
    scan_exclusive_i64(cnt, nrow, n, s, sc);
    k_last_row<<<1, 1, 0, s>>>(nrow, cnt, n);
    int64_t total = 0;
    DSD_HIP(hipMemcpyAsync(&total, nrow + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    int32_t *ncol = sc.get_n<int32_t>(total);
    int64_t *ndag = sc.get_n<int64_t>(n);
    k_compact_dag<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(nrow, cnt_out, n, ndag);
    k_compact_fill<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, nrow, ncol);
    b.row_ptr = nrow;
    b.col = ncol;
    b.dag_off = ndag;
    if (b.h >= 3) {
        k_reset_chunks<<<1, 1, 0, s>>>(b);
        k_rechunk<<<256, BLOCK, 0, s>>>(b);
    }
}

// ---------------------------------------------------------------- host driver

// 4-loop tables: slots per workgroup (a power of two, twice the largest
// 2-hop bound of the graph) and the number of workgroups that fit in
// LOOP_TABLE_SLOTS slots in all
constexpr int64_t LOOP_TABLE_SLOTS = (int64_t)1 << 28;   // 2 GiB of keys and counts
constexpr int64_t LOOP_MAX_SLOTS = (int64_t)1 << 26;

static int64_t loop_tables(const DevGraph &g, int *groups, hipStream_t s, Scratch &sc) {
    unsigned long long *mx = sc.get_n<unsigned long long>(1);
    fill_u64((u64 *)mx, 0, 1, s);
    if (g.n > 0) k_loop_bound<<<grid_for(g.n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, g.n, mx);
    unsigned long long bound = 0;
    DSD_HIP(hipMemcpyAsync(&bound, mx, sizeof(bound), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    int64_t size = 2;
    while (size < 2 * (int64_t)bound) size <<= 1;
    if (size > LOOP_MAX_SLOTS)
        throw Error(-5, "a 2-hop neighbourhood is too large for the 4-loop tables");
    *groups = (int)std::min<int64_t>(512, std::max<int64_t>(1, LOOP_TABLE_SLOTS / size));
    return size;
}

void loop4_degrees(const DevGraph &g, u64 *deg, hipStream_t s, Scratch &sc) {
    if (g.n == 0) return;
    int groups = 0;
    const int64_t size = loop_tables(g, &groups, s, sc);
    int32_t *keys = sc.get_n<int32_t>((int64_t)groups * size);
    uint32_t *vals = sc.get_n<uint32_t>((int64_t)groups * size);
    k_loop_degrees<<<groups, BLOCK, 0, s>>>(g.row_ptr, g.col, g.n, keys, vals, size, deg);
}

// x-star pattern: residual degrees start as the degrees
__global__ void k_star_init(PeelBufs b) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < b.n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = (int32_t)(b.row_ptr[v + 1] - b.row_ptr[v]);
        b.ydeg[v] = d;
        b.yold[v] = d;
        b.tround[v] = -1;
    }
}

__global__ void k_init_graphs(PeelBufs b, const u64 *mu, const int64_t *lv_base, u64 k_floor) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b.G) return;
    GraphState s{};
    s.k = k_floor;
    s.kcand = ~0ull;
    s.mu_alive = mu[g];
    s.lv_base = lv_base ? lv_base[g] : 0;
    b.gs[g] = s;
}

__global__ void k_peel_init(PeelBufs b, const uint8_t *alive0, int32_t *list0, int32_t *count) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t lim = ((int64_t)b.n + WAVE - 1) / WAVE * WAVE;
    constexpr size_t GS_STRIDE = sizeof(GraphState) / sizeof(int64_t);
    for (int64_t v = blockIdx.x * (int64_t)BLOCK + threadIdx.x; v - lane() < lim; v += stride) {
        bool in = v < b.n && (alive0 == nullptr || alive0[v] != 0);
        if (v < b.n) {
            b.stamp[v] = in ? ALIVE : -1;
            b.core[v] = 0;
        }
        wave_push(in, (int32_t)v, list0, count);
        wave_add_by_graph<unsigned long long>(in ? graph_of(b, (int32_t)v) : -1,
                                              (unsigned long long *)&b.gs[0].n_alive, GS_STRIDE);
    }
}

// every graph with alive vertices opens its first level
__global__ void k_start_graphs(PeelBufs b) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < b.G && b.gs[g].n_alive > 0) {
        b.gs[g].sel = 1;
        atomicAdd(&b.ctl->nsel[0], 1);
    }
    if (g == 0) b.ctl->n_alive = b.ctl->nlist[0];
}

// ---------------------------------------------------------------- tail engine (h = 3 with triangle lists, h = 2)
//
// Once at most TE_MAX vertices are alive, the rest of a single graph's peel
// runs in one launch of one workgroup.  First every CU helps to rewrite the
// tail vertices' rows (h = 3: triangle rows; h = 2: adjacency rows): only
// pairs whose two vertices are still in the tail stay, renumbered to local
// ids that follow the rank order (so the owner rule compares local ids),
// packed two to a 32-bit word, each row padded to a multiple of four words.  The workgroup then keeps the degrees
// and the states of the tail vertices in LDS and takes round after round,
// with only workgroup barriers between them: the level (the rule of the
// round-synchronous peel: the alive vertices of degree <= k, else a new
// level at the smallest alive degree), the frontier, and the frontier's rows
// streamed from HBM.  Each lane takes TE_PL consecutive pairs of a row with
// vector loads, looks up all of their states before it waits, and applies
// each run of one first vertex with a single LDS atomic.

constexpr int TE_MAX = (int)TAIL_ENGINE_VERTICES;   // tail vertices: local ids fit 16 bits
constexpr int TE_BLOCK = 1024;
constexpr int TE_WAVES = TE_BLOCK / WAVE;
constexpr int TE_PER = TE_MAX / TE_BLOCK;     // local ids per thread in the frontier scans
constexpr int TE_PL = 8;                      // consecutive pairs per lane
constexpr int TE_ITEM = WAVE * TE_PL;         // pairs per work item of a round
constexpr int TE_FB = 2048;                   // frontier vertices per batch of items
constexpr int TE_CH = 4096;                   // pairs per item of the row rewrite
constexpr uint32_t TE_NONE = 0xffffffffu;     // padding (local ids are below 2^14)
constexpr uint8_t TE_DEAD = 0, TE_CUR = 1, TE_ALIVE = 2;
constexpr uint32_t TE_HEAVY = 1u << 18;       // a round whose frontier rows hold more pairs goes to the grid
                                              // (DSD_TE_GRID_PAIRS overrides it)
constexpr int TE_HBLOCK = 1024;               // threads per workgroup of the grid round

// The engine's state across a round handed to the grid: the engine stops
// with its frontier marked (TE_CUR) and its rows' items listed, k_te_heavy
// processes those items on every CU, and the engine starts again where the
// round ends.  On a single CU a round of the dense innermost levels (hundreds
// of vertices whose rows hold tens of millions of pairs) takes milliseconds;
// the grid takes tens of microseconds.
struct TeState {
    uint32_t *deg;        // [A] degrees (a removed vertex's slot: its core number)
    uint8_t *st;          // [A] TE_DEAD / TE_CUR / TE_ALIVE
    uint32_t *F;          // [nF] the round's frontier (local ids)
    uint32_t *ipre;       // [nF + 1] each frontier vertex's first item; ipre[nF] = items
    uint32_t *imap;       // [items] item -> frontier position
    int32_t heavy;        // set when the engine stopped for a grid round
    int32_t r, nlevels, open;
    uint32_t nF, items;
    u64 k, mu_alive;
    int64_t n_alive;
    u64 destroyed;        // cliques the grid round destroyed
    u64 pairs;            // pairs of all grid rounds
    u64 rounds;           // grid rounds
};

// tail membership: alive, or in the pending frontier of the next round
__global__ void k_te_flags(const int32_t *stamp, int32_t n, const PeelCtl *c, uint32_t *flag) {
    const int32_t r = c->round;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = stamp[v] >= r ? 1u : 0u;
}

// local id -> vertex, and each tail vertex's rewrite items (roff: the
// triangle rows' offsets for h = 3, the adjacency's for h = 2)
__global__ void k_te_glob(const uint32_t *flag, const uint32_t *loc, int32_t n, const int64_t *roff, int32_t *glob,
                          int64_t *ib, int32_t *count) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[v]) continue;
        const uint32_t l = loc[v];
        glob[l] = (int32_t)v;
        ib[l] = (roff[v + 1] - roff[v] + TE_CH - 1) / TE_CH;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = (int32_t)(loc[n - 1] + flag[n - 1]);
}

// The pairs of one rewrite item that stay inside the tail (a row holds every
// triangle once, as (a, x) with a ranked below x): counted (FILL false, into
// kc[it]) or written from kc[it] on (FILL true), in row order, so every row
// stays grouped by its first vertex.
// H = 2: the rows are adjacency rows (tpairs: the column array), and each
// neighbour x in the tail becomes the word (x, x).
template <bool FILL, int H>
__global__ __launch_bounds__(BLOCK) void k_te_pairs(const int64_t *tvoff, const int32_t *tpairs, const uint32_t *flag,
                                                     const uint32_t *loc, const int32_t *glob, const int64_t *ib,
                                                     int32_t A, int64_t NI, int64_t *kc, uint32_t *lp) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < NI; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        int32_t lo = 0, hi = A - 1;   // the item's vertex: the largest l with ib[l] <= it
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (ib[mid] <= it) lo = mid;
            else hi = mid - 1;
        }
        const int32_t v = glob[lo];
        const int64_t e0 = tvoff[v] + (it - ib[lo]) * TE_CH, e1 = min(tvoff[v + 1], e0 + TE_CH);
        int64_t pos = FILL ? kc[it] : 0;
        for (int64_t base = e0; base < e1; base += WAVE) {
            const int64_t e = base + lane();
            bool keep = false;
            uint32_t val = 0;
            if (e < e1) {
                if (H == 3) {
                    const int32_t a = tpairs[2 * e], x = tpairs[2 * e + 1];
                    keep = flag[a] && flag[x];
                    if (FILL && keep) val = (loc[a] << 16) | loc[x];
                } else {
                    const int32_t x = tpairs[e];
                    keep = flag[x] != 0;
                    if (FILL && keep) val = (loc[x] << 16) | loc[x];
                }
            }
            const u64 m = __ballot(keep);
            if (FILL && keep) lp[pos + __popcll(m & lanemask_lt())] = val;
            pos += __popcll(m);
        }
        if (!FILL && lane() == 0) kc[it] = pos;
    }
}

// kept pairs of every tail vertex (vcnt) and its row length padded to four (rl)
__global__ void k_te_vsum(const int64_t *ib, const int64_t *kc, int32_t A, int64_t *vcnt, int64_t *rl) {
    for (int32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < A; l += gridDim.x * blockDim.x) {
        int64_t s = 0;
        for (int64_t it = ib[l]; it < ib[l + 1]; it++) s += kc[it];
        vcnt[l] = s;
        rl[l] = (s + 3) & ~(int64_t)3;
    }
}

// where every rewrite item starts writing: its row's start plus the kept
// pairs of the row's earlier items (kc: counts in, starts out)
__global__ void k_te_ioff(const int64_t *ib, const int64_t *lrow, int32_t A, int64_t *kc) {
    for (int32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < A; l += gridDim.x * blockDim.x) {
        int64_t run = lrow[l];
        for (int64_t it = ib[l]; it < ib[l + 1]; it++) {
            const int64_t c = kc[it];
            kc[it] = run;
            run += c;
        }
    }
}

__global__ void k_te_pad(const int64_t *lrow, const int64_t *vcnt, int32_t A, uint32_t *lp) {
    for (int32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < A; l += gridDim.x * blockDim.x)
        for (int64_t e = lrow[l] + vcnt[l]; e < lrow[l + 1]; e++) lp[e] = TE_NONE;
}

// workgroup barrier that orders LDS only: a wave's global stores stay in
// flight across it (nothing in the engine reads them back)
__device__ __forceinline__ void te_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ bool te_allowed(uint32_t st, uint32_t x, uint32_t v) {
    return st == TE_ALIVE || (st == TE_CUR && x > v);
}

// Wave reductions in VALU cross-lane operations (DPP: quad permutations and
// row mirrors reduce every 16-lane row, row broadcasts join the rows; lane
// 63 ends with the total, which readlane hands to every lane).  id: the
// operation's identity, taken by lanes a row mask leaves out.
template <bool MIN>
__device__ __forceinline__ uint32_t te_dpp_op(uint32_t a, uint32_t b) {
    return MIN ? (a < b ? a : b) : a + b;
}
template <bool MIN>
__device__ __forceinline__ uint32_t te_wave_reduce(uint32_t v) {
    const int id = MIN ? -1 : 0;
    v = te_dpp_op<MIN>(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0xb1, 0xf, 0xf, false));   // quad [1,0,3,2]
    v = te_dpp_op<MIN>(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x4e, 0xf, 0xf, false));   // quad [2,3,0,1]
    v = te_dpp_op<MIN>(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x141, 0xf, 0xf, false));  // half-row mirror
    v = te_dpp_op<MIN>(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x140, 0xf, 0xf, false));  // row mirror
    v = te_dpp_op<MIN>(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xa, 0xf, false));  // row 15 -> rows 1, 3
    v = te_dpp_op<MIN>(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xc, 0xf, false));  // lane 31 -> rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// exclusive prefix of v over the wave's lanes, from one ballot per bit in use
__device__ __forceinline__ uint32_t te_wave_prefix(uint32_t v, uint32_t *total) {
    uint32_t pre = 0, tot = 0;
    const u64 lt = lanemask_lt();
    for (int bit = 0; bit < 32; bit++) {
        if (__ballot((v >> bit) != 0) == 0) break;
        const u64 m = __ballot((v >> bit) & 1u);
        pre += (uint32_t)__popcll(m & lt) << bit;
        tot += (uint32_t)__popcll(m) << bit;
    }
    *total = tot;
    return pre;
}

// Workgroup reductions, double-buffered so that one barrier suffices: a
// call writes one half and reads it after the barrier; the next call uses
// the other half, and the call after that is behind the next call's barrier.
struct TeRed {
    uint32_t cnt[2][TE_WAVES];
    uint32_t mn[2][TE_WAVES];
    uint32_t sum[2][TE_WAVES];
};

// exclusive prefix (return) and total (*ctot) of c, minimum of m (*mall) and
// sum of s (*sall) over the workgroup; every thread calls it with the same par
__device__ __forceinline__ uint32_t te_reduce(TeRed &R, int &par, uint32_t c, uint32_t m, uint32_t s, uint32_t *ctot,
                                              uint32_t *mall, uint32_t *sall) {
    const int wv = threadIdx.x / WAVE, L = lane();
    uint32_t wtot = 0;
    const uint32_t pre = te_wave_prefix(c, &wtot);
    const uint32_t wmin = te_wave_reduce<true>(m), wsum = te_wave_reduce<false>(s);
    if (L == 0) {
        R.cnt[par][wv] = wtot;
        R.mn[par][wv] = wmin;
        R.sum[par][wv] = wsum;
    }
    te_sync();
    const uint32_t ci = L < TE_WAVES ? R.cnt[par][L] : 0u;
    const uint32_t mi = L < TE_WAVES ? R.mn[par][L] : 0xffffffffu;
    const uint32_t si = L < TE_WAVES ? R.sum[par][L] : 0u;
    const uint32_t before = te_wave_reduce<false>(L < wv ? ci : 0u);
    *ctot = te_wave_reduce<false>(ci);
    *mall = te_wave_reduce<true>(mi);
    *sall = te_wave_reduce<false>(si);
    par ^= 1;
    return before + pre;
}

// this thread's TE_PER local ids: their degrees and states
__device__ __forceinline__ void te_load(const uint32_t *sDeg, const uint8_t *sSt, int l0, uint32_t *d,
                                        uint32_t *st) {
    const uint4 s4 = *(const uint4 *)(sSt + l0);
    const uint32_t sw[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint4 d4 = *(const uint4 *)(sDeg + l0 + 4 * q);
        d[4 * q] = d4.x;
        d[4 * q + 1] = d4.y;
        d[4 * q + 2] = d4.z;
        d[4 * q + 3] = d4.w;
#pragma unroll
        for (int j = 0; j < 4; j++) st[4 * q + j] = (sw[q] >> (8 * j)) & 0xffu;
    }
}

// the frontier flags of this thread's ids at level k
__device__ __forceinline__ uint32_t te_mask(const uint32_t *d, const uint32_t *st, u64 k) {
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < TE_PER; j++) mask |= (st[j] == TE_ALIVE && d[j] <= k) ? 1u << j : 0u;
    return mask;
}

// pairs and items (TE_ITEM pairs each) in the rows of this thread's ids in mask
__device__ __forceinline__ void te_front_work(uint32_t mask, int l0, const uint32_t *sRs, uint32_t *pairs,
                                              uint32_t *items) {
    uint32_t p = 0, it = 0;
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
        const int l = l0 + __builtin_ctz(mm);
        const uint32_t len = sRs[l + 1] - sRs[l];
        p += len;
        it += (len + TE_ITEM - 1) / TE_ITEM;
    }
    *pairs = p;
    *items = it;
}

// A round's frontier from one exchange between the waves.  Each wave offers
// two candidates: its alive ids of degree <= k, and its alive ids at the
// wave's smallest degree; with their counts, item counts and pairs, and the
// previous round's destroyed cliques.  Once the exchange is read, either some
// ids are at degree <= k (the level goes on with them) or none is, and the
// new level opens at the smallest alive degree with the ids of the waves
// whose own minimum it is.  The frontier position (at) and first item (iat)
// of this thread's ids are exclusive prefixes in id order.
struct TeSel {
    uint32_t v[2][8][TE_WAVES];   // [parity][field][wave]
};
constexpr int TS_CK = 0, TS_CM = 1, TS_MIN = 2, TS_DEST = 3, TS_PK = 4, TS_PM = 5, TS_IK = 6, TS_IM = 7;
struct TeRound {
    uint32_t mask, nF, at, iat, items, fpairs, gone, gmin;
    bool fresh;   // a new level at gmin
};
__device__ __forceinline__ TeRound te_select(TeSel &S, int &par, const uint32_t *d, const uint32_t *st, u64 k, int l0,
                                             const uint32_t *sRs, uint32_t destroyed) {
    const int wv = threadIdx.x / WAVE, L = lane();
    const uint32_t mk = te_mask(d, st, k);
    uint32_t mn = 0xffffffffu;
#pragma unroll
    for (int j = 0; j < TE_PER; j++)
        if (st[j] == TE_ALIVE && d[j] < mn) mn = d[j];
    const uint32_t wmin = te_wave_reduce<true>(mn);
    uint32_t mm = 0;
#pragma unroll
    for (int j = 0; j < TE_PER; j++) mm |= (st[j] == TE_ALIVE && d[j] == wmin) ? 1u << j : 0u;
    uint32_t pk, ik, pm, im;
    te_front_work(mk, l0, sRs, &pk, &ik);
    te_front_work(mm, l0, sRs, &pm, &im);
    uint32_t ckw, cmw, ikw, imw;
    const uint32_t prek = te_wave_prefix(__popc(mk), &ckw), prem = te_wave_prefix(__popc(mm), &cmw);
    const uint32_t preik = te_wave_prefix(ik, &ikw), preim = te_wave_prefix(im, &imw);
    const uint32_t dw = te_wave_reduce<false>(destroyed), pkw = te_wave_reduce<false>(pk),
                   pmw = te_wave_reduce<false>(pm);
    if (L == 0) {
        S.v[par][TS_CK][wv] = ckw;
        S.v[par][TS_CM][wv] = cmw;
        S.v[par][TS_MIN][wv] = wmin;
        S.v[par][TS_DEST][wv] = dw;
        S.v[par][TS_PK][wv] = pkw;
        S.v[par][TS_PM][wv] = pmw;
        S.v[par][TS_IK][wv] = ikw;
        S.v[par][TS_IM][wv] = imw;
    }
    te_sync();
    const bool in = L < TE_WAVES;
    const uint32_t ck = in ? S.v[par][TS_CK][L] : 0u, wm = in ? S.v[par][TS_MIN][L] : 0xffffffffu;
    TeRound o;
    o.gone = te_wave_reduce<false>(in ? S.v[par][TS_DEST][L] : 0u);
    o.gmin = te_wave_reduce<true>(wm);
    const uint32_t nfk = te_wave_reduce<false>(ck);
    if (nfk > 0) {
        const uint32_t ic = in ? S.v[par][TS_IK][L] : 0u;
        o.fresh = false;
        o.mask = mk;
        o.nF = nfk;
        o.at = prek + te_wave_reduce<false>(L < wv ? ck : 0u);
        o.iat = preik + te_wave_reduce<false>(L < wv ? ic : 0u);
        o.items = te_wave_reduce<false>(ic);
        o.fpairs = te_wave_reduce<false>(in ? S.v[par][TS_PK][L] : 0u);
    } else {
        const bool eq = in && wm == o.gmin;
        const uint32_t cm = eq ? S.v[par][TS_CM][L] : 0u, ic = eq ? S.v[par][TS_IM][L] : 0u;
        o.fresh = true;
        o.mask = wmin == o.gmin ? mm : 0u;
        o.nF = te_wave_reduce<false>(cm);
        o.at = prem + te_wave_reduce<false>(L < wv ? cm : 0u);
        o.iat = preim + te_wave_reduce<false>(L < wv ? ic : 0u);
        o.items = te_wave_reduce<false>(ic);
        o.fpairs = te_wave_reduce<false>(eq ? S.v[par][TS_PM][L] : 0u);
    }
    par ^= 1;
    return o;
}

// lrow (A + 1 entries) below 2^32: the row starts live in LDS.  H = 2: a
// removed vertex costs each alive neighbour x (the word (x, x)) one edge.
// resume: the state comes from ts, where the engine left it for a grid
// round, and that round ends first.  A round whose frontier rows hold more
// than heavy pairs is left to the grid.
template <int H>
__global__ __launch_bounds__(TE_BLOCK) void k_tail_engine(PeelBufs b, const int32_t *glob, const int64_t *lrow,
                                                          const uint32_t *lp, int32_t A, int32_t *err, TeState *ts,
                                                          int resume, uint32_t heavy) {
    __shared__ __align__(16) uint32_t sDeg[TE_MAX];
    __shared__ __align__(16) uint8_t sSt[TE_MAX];
    __shared__ uint32_t sRs[TE_MAX + 1];
    __shared__ uint16_t sF[TE_FB];
    __shared__ uint32_t sIpre[TE_FB];
    __shared__ TeRed R;
    __shared__ TeSel S;
    PeelCtl *c = b.ctl;
    GraphState *gs = b.gs;
    const int t = threadIdx.x, wv = t / WAVE, L = lane();
    int32_t r, nlevels;
    u64 k, mu_alive;
    int64_t n_alive;
    bool open;
    uint32_t destroyed = 0;   // this thread's share of the current round (summed at the next round's start;
                              // a round destroys at most mu_alive < 2^32 cliques)
    if (!resume) {
        for (int l = t; l < TE_MAX; l += TE_BLOCK) {
            sDeg[l] = l < A ? (uint32_t)b.deg[glob[l]] : 0u;
            sSt[l] = l < A ? TE_ALIVE : TE_DEAD;
        }
        r = c->round;
        k = gs[0].k;
        mu_alive = gs[0].mu_alive;
        n_alive = gs[0].n_alive;
        nlevels = gs[0].nlevels;
        open = gs[0].sel != 0;
    } else {
        for (int l = t; l < TE_MAX; l += TE_BLOCK) {
            sDeg[l] = l < A ? ts->deg[l] : 0u;
            sSt[l] = l < A ? ts->st[l] : TE_DEAD;
        }
        r = ts->r;
        k = ts->k;
        mu_alive = ts->mu_alive;
        n_alive = ts->n_alive;
        nlevels = ts->nlevels;
        open = ts->open != 0;
        if (t == 0) destroyed = (uint32_t)ts->destroyed;
    }
    for (int l = t; l <= A; l += TE_BLOCK) sRs[l] = (uint32_t)lrow[l];
    const int64_t lv_base = gs[0].lv_base;
    int par = 0, spar = 0;
    __syncthreads();
    if (t == 0) ts->heavy = 0;
    const int l0 = t * TE_PER;
    if (resume) {
        // the end of the round the grid processed
        if (open) nlevels += 1;
        n_alive -= ts->nF;
        r += 1;
        open = false;
#pragma unroll
        for (int j = 0; j < TE_PER; j++)
            if (sSt[l0 + j] == TE_CUR) sSt[l0 + j] = TE_DEAD;
    }
    int64_t guard = 0;
    while (n_alive > 0) {
        if (++guard > (int64_t)A + 1) {   // every round removes at least one vertex
            if (t == 0) *err = 1;
            break;
        }
        // the frontier: alive vertices of degree <= k; none left means a new
        // level at the smallest alive degree.  The same reduction ends the
        // previous round (its destroyed cliques).
        TeRound rd;
        {
            uint32_t d[TE_PER], st[TE_PER];
            te_load(sDeg, sSt, l0, d, st);
            rd = te_select(S, spar, d, st, k, l0, sRs, destroyed);
        }
        destroyed = 0;
        mu_alive -= rd.gone;
        if (rd.fresh) {
            open = true;
            k = k > (u64)rd.gmin ? k : (u64)rd.gmin;
        }
        const uint32_t mask = rd.mask, nF = rd.nF, at = rd.at, fpairs = rd.fpairs;
        if (nF == 0) {   // cannot happen while vertices are alive
            if (t == 0) *err = 2;
            break;
        }
        // the level table entry of a new level: the level, |R_k| and mu(R_k)
        // as its first round begins
        if (open && t == 0) {
            const int64_t at_l = lv_base + nlevels;
            b.lv_k[at_l] = k;
            b.lv_size[at_l] = (u64)n_alive;
            b.lv_mu[at_l] = mu_alive;
        }
        // frontier vertices leave: a removed vertex's degree slot keeps its
        // core number (written out at the end)
        for (uint32_t mm = mask; mm; mm &= mm - 1) {
            const int l = l0 + __builtin_ctz(mm);
            sSt[l] = TE_CUR;
            sDeg[l] = (uint32_t)k;
        }
        if (fpairs > heavy) {
            // a heavy round goes to the grid: the frontier with its items'
            // starts, and the whole state, to ts; then the engine stops
            const uint32_t items = rd.items;
            uint32_t run = rd.iat;
            te_sync();   // orders the frontier marks before the state is copied
            uint32_t q = at;
            for (uint32_t mm = mask; mm; mm &= mm - 1, q++) {
                const int l = l0 + __builtin_ctz(mm);
                ts->F[q] = (uint32_t)l;
                ts->ipre[q] = run;
                run += (sRs[l + 1] - sRs[l] + TE_ITEM - 1) / TE_ITEM;
            }
            for (int l = t; l < A; l += TE_BLOCK) {
                ts->deg[l] = sDeg[l];
                ts->st[l] = sSt[l];
            }
            if (t == 0) {
                ts->ipre[nF] = items;
                ts->nF = nF;
                ts->items = items;
                ts->r = r;
                ts->k = k;
                ts->mu_alive = mu_alive;
                ts->n_alive = n_alive;
                ts->nlevels = nlevels;
                ts->open = open ? 1 : 0;
                ts->destroyed = 0;
                ts->pairs += fpairs;
                ts->rounds += 1;
                ts->heavy = 1;
            }
            return;
        }
        // the frontier's rows: the nb vertices listed in sF, their items'
        // starts in sIpre
        auto run_items = [&](int nb, uint32_t items) {
            // each wave takes items wv, wv + TE_WAVES, ...; the next one's
            // pairs are loaded while the current one is processed
            auto locate = [&](uint32_t it, uint32_t *v, uint32_t *p0, uint32_t *p1) {
                int lo = 0, hi = nb - 1;   // the item's frontier vertex: the largest q with sIpre[q] <= it
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sIpre[mid] <= it) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t l = sF[lo], ofs = (it - sIpre[lo]) * TE_ITEM;
                *v = l;
                *p0 = sRs[l] + ofs;
                *p1 = min(sRs[l + 1], *p0 + TE_ITEM);
            };
            auto fetch = [&](uint32_t p0, uint32_t p1, uint32_t *pv) {
                const uint32_t q0 = p0 + (uint32_t)L * TE_PL;
#pragma unroll
                for (int cq = 0; cq < TE_PL / 4; cq++) {
                    uint4 w = make_uint4(TE_NONE, TE_NONE, TE_NONE, TE_NONE);
                    if (q0 + 4 * cq < p1) w = *(const uint4 *)(lp + q0 + 4 * cq);
                    pv[4 * cq] = w.x;
                    pv[4 * cq + 1] = w.y;
                    pv[4 * cq + 2] = w.z;
                    pv[4 * cq + 3] = w.w;
                }
            };
            uint32_t v = 0, pv[TE_PL], p0 = 0, p1 = 0;
            if ((uint32_t)wv < items) {
                locate(wv, &v, &p0, &p1);
                fetch(p0, p1, pv);
            }
            for (uint32_t it = wv; it < items; it += TE_WAVES) {
                uint32_t vn = 0, pn[TE_PL];
#pragma unroll
                for (int j = 0; j < TE_PL; j++) pn[j] = TE_NONE;
                if (it + TE_WAVES < items) {
                    locate(it + TE_WAVES, &vn, &p0, &p1);
                    fetch(p0, p1, pn);
                }
                uint32_t s2[TE_PL];   // states of a (low byte) and x (next byte)
#pragma unroll
                for (int j = 0; j < TE_PL; j++) {
                    const uint32_t qv = pv[j] == TE_NONE ? 0u : pv[j];
                    s2[j] = (uint32_t)sSt[qv >> 16] | ((uint32_t)sSt[qv & 0xffffu] << 8);
                }
                // triangle {v, a, x} costs a and x a clique each: x's loss goes
                // at once (0 for a removed vertex; a padding word touches slot
                // 0 with 0), a's are summed over the lane's run of equal a
                uint32_t acc = 0;
#pragma unroll
                for (int j = 0; j < TE_PL; j++) {
                    const uint32_t qv = pv[j] == TE_NONE ? 0u : pv[j];
                    const uint32_t a = qv >> 16, x = qv & 0xffffu;
                    const uint32_t sa = s2[j] & 0xffu, sx = s2[j] >> 8;
                    const bool ok = pv[j] != TE_NONE && te_allowed(sa, a, v) && te_allowed(sx, x, v);
                    destroyed += ok ? 1u : 0u;
                    if (H == 3) atomicSub(&sDeg[x], (ok && sx == TE_ALIVE) ? 1u : 0u);
                    acc += (ok && sa == TE_ALIVE) ? 1u : 0u;
                    const bool last = j == TE_PL - 1 || (pv[j + (j < TE_PL - 1)] >> 16) != a;
                    if (last && acc) {
                        atomicSub(&sDeg[a], acc);
                        acc = 0;
                    }
                }
                v = vn;
#pragma unroll
                for (int j = 0; j < TE_PL; j++) pv[j] = pn[j];
            }
            te_sync();   // the next batch rewrites sF and sIpre; the next round reads the degrees
        };
        if (nF <= TE_FB) {
            // one batch: the list and the item starts come from the selection
            uint32_t q = at, ip = rd.iat;
            for (uint32_t mm = mask; mm; mm &= mm - 1, q++) {
                const int l = l0 + __builtin_ctz(mm);
                sF[q] = (uint16_t)l;
                sIpre[q] = ip;
                ip += (sRs[l + 1] - sRs[l] + TE_ITEM - 1) / TE_ITEM;
            }
            te_sync();
            run_items((int)nF, rd.items);
        } else {
            // TE_FB vertices at a time
            for (uint32_t f0 = 0; f0 < nF; f0 += TE_FB) {
                const int nb = (int)min((uint32_t)TE_FB, nF - f0);
                uint32_t q = at;
                for (uint32_t mm = mask; mm; mm &= mm - 1, q++)
                    if (q >= f0 && q < f0 + TE_FB) sF[q - f0] = (uint16_t)(l0 + __builtin_ctz(mm));
                te_sync();
                constexpr int PT = TE_FB / TE_BLOCK;
                uint32_t cnt[PT], own = 0;
#pragma unroll
                for (int j = 0; j < PT; j++) {
                    const int qq = t * PT + j;
                    cnt[j] = 0;
                    if (qq < nb) {
                        const uint32_t l = sF[qq];
                        cnt[j] = (sRs[l + 1] - sRs[l] + TE_ITEM - 1) / TE_ITEM;
                    }
                    own += cnt[j];
                }
                uint32_t items = 0, u1, u2;
                uint32_t run = te_reduce(R, par, own, 0xffffffffu, 0u, &items, &u1, &u2);
#pragma unroll
                for (int j = 0; j < PT; j++) {
                    const int qq = t * PT + j;
                    if (qq < nb) sIpre[qq] = run;
                    run += cnt[j];
                }
                te_sync();
                run_items(nb, items);
            }
        }
        // end of the round; each thread retires its own frontier entries (the
        // next round's reduction orders this before any other thread's reads)
        if (open) nlevels += 1;
        n_alive -= nF;
        r += 1;
        open = false;
        for (uint32_t mm = mask; mm; mm &= mm - 1) sSt[l0 + __builtin_ctz(mm)] = TE_DEAD;
    }
    {
        uint32_t u0, u1, gone = 0;
        (void)te_reduce(R, par, 0u, 0xffffffffu, destroyed, &u0, &u1, &gone);
        mu_alive -= gone;
    }
    for (int l = t; l < A; l += TE_BLOCK) b.core[glob[l]] = sDeg[l];
    if (t == 0) {
        GraphState &g0 = gs[0];
        g0.k = k;
        g0.kcand = ~0ull;
        g0.mu_alive = mu_alive;
        g0.destroyed = 0;
        g0.n_alive = n_alive;
        g0.nF[0] = g0.nF[1] = 0;
        g0.nlevels = nlevels;
        g0.sel = 0;
        c->n_alive = n_alive;
        c->round = r;
        c->nF[0] = c->nF[1] = 0;
        c->nsel[0] = c->nsel[1] = 0;
        c->pending = 0;
    }
}

// item -> frontier position for a grid round (one wave per frontier vertex)
__global__ void k_te_expand(const TeState *ts) {
    const uint32_t nF = ts->nF;
    const int wv = threadIdx.x / WAVE;
    for (uint32_t q = blockIdx.x * WAVES_PER_BLOCK + wv; q < nF; q += gridDim.x * WAVES_PER_BLOCK)
        for (uint32_t i = ts->ipre[q] + lane(); i < ts->ipre[q + 1]; i += WAVE) ts->imap[i] = q;
}

// One round of the engine on every CU: a wave per item (TE_ITEM pairs of a
// frontier vertex's row, TE_PL consecutive pairs per lane), the same owner
// rule and losses as the engine.  Each workgroup holds the states and its own
// loss counters in LDS and adds the counters to the degrees at its end, so
// the degrees of the few survivors of a dense level see one atomic per
// workgroup instead of one per pair.
template <int H>
__global__ __launch_bounds__(TE_HBLOCK) void k_te_heavy(TeState *ts, const int64_t *lrow, const uint32_t *lp,
                                                         int32_t A) {
    __shared__ uint8_t sSt[TE_MAX];          // 80 KB in all: two workgroups per CU
    __shared__ uint32_t sLoss[TE_MAX];
    for (int l = threadIdx.x; l < A; l += TE_HBLOCK) {
        sSt[l] = ts->st[l];
        sLoss[l] = 0;
    }
    __syncthreads();
    const uint32_t items = ts->items;
    const int wv = threadIdx.x / WAVE, L = lane();
    uint32_t destroyed = 0;
    for (uint32_t it = blockIdx.x * (TE_HBLOCK / WAVE) + wv; it < items; it += gridDim.x * (TE_HBLOCK / WAVE)) {
        const uint32_t q = ts->imap[it];
        const uint32_t v = ts->F[q];
        const int64_t p0 = lrow[v] + (int64_t)(it - ts->ipre[q]) * TE_ITEM;
        const int64_t p1 = min(lrow[v + 1], p0 + TE_ITEM);
        const int64_t q0 = p0 + (int64_t)L * TE_PL;
        uint32_t pv[TE_PL];
#pragma unroll
        for (int cq = 0; cq < TE_PL / 4; cq++) {
            uint4 w = make_uint4(TE_NONE, TE_NONE, TE_NONE, TE_NONE);
            if (q0 + 4 * cq < p1) w = *(const uint4 *)(lp + q0 + 4 * cq);
            pv[4 * cq] = w.x;
            pv[4 * cq + 1] = w.y;
            pv[4 * cq + 2] = w.z;
            pv[4 * cq + 3] = w.w;
        }
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < TE_PL; j++) {
            const bool real = pv[j] != TE_NONE;
            const uint32_t qv = real ? pv[j] : 0u;
            const uint32_t a = qv >> 16, x = qv & 0xffffu;
            const uint32_t sa = sSt[a], sx = sSt[x];
            const bool ok = real && te_allowed(sa, a, v) && te_allowed(sx, x, v);
            destroyed += ok ? 1u : 0u;
            if (H == 3 && ok && sx == TE_ALIVE) atomicAdd(&sLoss[x], 1u);
            acc += (ok && sa == TE_ALIVE) ? 1u : 0u;
            const bool last = j == TE_PL - 1 || (pv[j + (j < TE_PL - 1)] >> 16) != a;
            if (last && acc) {
                atomicAdd(&sLoss[a], acc);
                acc = 0;
            }
        }
    }
    const uint32_t wd = te_wave_reduce<false>(destroyed);
    if (L == 0 && wd) atomicAdd((unsigned long long *)&ts->destroyed, (unsigned long long)wd);
    __syncthreads();
    for (int l = threadIdx.x; l < A; l += TE_HBLOCK)
        if (sLoss[l]) atomicSub(&ts->deg[l], sLoss[l]);
}

// Times every launch of one kernel: the launch carries a start and a stop
// HIP event recorded by the dispatch itself (hipExtLaunchKernelGGL), so the
// pair spans the kernel and nothing else on the stream.  The events come
// from a process-wide pool that only grows, so a call pays for event
// creation only the first time it needs that many; a second peel running at
// the same time (another thread) goes untimed.
template <int SLOT>
class LaunchTimer {
public:
    explicit LaunchTimer(bool want) : lk_(pool_mu(), std::try_to_lock) { on_ = want && lk_.owns_lock(); }
    bool on() const { return on_; }
    // launch kernel k on s, timed when the timer is on
    template <typename... Args>
    void launch(void (*k)(Args...), dim3 grid, dim3 block, hipStream_t s, Args... args) {
        if (!on_) {
            hipLaunchKernelGGL(k, grid, block, 0, s, args...);
            return;
        }
        std::vector<hipEvent_t> &ev = pool();
        while (ev.size() < used_ + 2) {
            hipEvent_t e;
            DSD_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        hipExtLaunchKernelGGL(k, grid, block, 0, s, ev[used_], ev[used_ + 1], 0, args...);
        used_ += 2;
    }
    // total milliseconds and launches (after the stream has drained)
    double total_ms(u64 *launches) {
        double t = 0;
        std::vector<hipEvent_t> &ev = pool();
        for (size_t i = 0; on_ && i < used_; i += 2) {
            float ms = 0;
            DSD_HIP(hipEventSynchronize(ev[i + 1]));
            DSD_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            t += ms;
        }
        *launches = used_ / 2;
        return t;
    }

private:
    static std::mutex &pool_mu() {
        static std::mutex m;
        return m;
    }
    static std::vector<hipEvent_t> &pool() {
        static std::vector<hipEvent_t> v;
        return v;
    }
    std::unique_lock<std::mutex> lk_;
    bool on_ = false;
    size_t used_ = 0;
};

// The captured round graphs of one peel (plain and tail mode) and the
// stream they are captured on; destroyed with the peel, or when the
// adjacency they name is compacted.
struct RoundGraphs {
    hipStream_t cs = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    void reset() {
        for (auto &e : exec) {
            if (e) (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    }
    ~RoundGraphs() {
        reset();
        if (cs) (void)hipStreamDestroy(cs);
    }
};

template <int R>
// the engines read the peel's current (possibly compacted) adjacency; a
// class whose out-degree range lies above the graph's largest out-degree
// (maxdout) never has items and is not launched
static void launch_peel_items(const PeelBufs &b, hipStream_t s, u64 *gS, int32_t maxdout) {
    PeelCtx ctx{b, 0};
    const int32_t *ni = &b.ctl->nitems[0];
    k_engine_wave<R, PeelCtx><<<1024, BLOCK, 0, s>>>(ctx, b.row_ptr, b.col, b.dag_off, 0, ni + 0);
    if constexpr (R <= 2) {
        ctx.cls = 1;
        if (maxdout > 64)
            k_engine_block<R, 2048, 12, 1, false, PeelCtx><<<512, BLOCK, 0, s>>>(ctx, b.row_ptr, b.col, b.dag_off,
                                                                                    0, ni + 1, nullptr);
        ctx.cls = 2;
        if (maxdout > 2048)
            k_engine_huge_r2<PeelCtx><<<256, BLOCK, 0, s>>>(ctx, b.row_ptr, b.col, b.dag_off, 0, ni + 2);
    } else {
        ctx.cls = 1;
        if (maxdout > 64)
            k_engine_block<R, 256, 9, 4, false, PeelCtx><<<1024, BLOCK, 0, s>>>(ctx, b.row_ptr, b.col, b.dag_off,
                                                                                   0, ni + 1, nullptr);
        ctx.cls = 2;
        if (maxdout > 256)
            k_engine_block<R, 768, 11, 12, false, PeelCtx><<<512, BLOCK, 0, s>>>(ctx, b.row_ptr, b.col, b.dag_off,
                                                                                    0, ni + 2, nullptr);
        ctx.cls = 3;
        if (maxdout > 768)
            k_engine_block<R, 1280, 12, 20, true, PeelCtx><<<256, BLOCK, 0, s>>>(ctx, b.row_ptr, b.col, b.dag_off,
                                                                                    0, ni + 3, gS);
    }
}

// The rest of a single graph's h = 3 peel by the tail engine, once at most
// TE_MAX vertices are alive (the state is between two rounds).  Returns
// false, having changed nothing, when the degrees could exceed 32 bits or
// the rewritten rows would not fit; the environment variable
// DSD_TAIL_ENGINE=0 turns it off.
static bool tail_engine(const PeelBufs &b, int h, int32_t n, int64_t n_alive, hipStream_t s, Scratch &sc,
                        KernelTimes *kt) {
    const char *env = std::getenv("DSD_TAIL_ENGINE");
    if (env && std::strcmp(env, "0") == 0) return false;
    if (n_alive < 1 || n_alive > TE_MAX) return false;
    GraphState g0;
    DSD_HIP(hipMemcpyAsync(&g0, b.gs, sizeof(GraphState), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (g0.mu_alive >= ((u64)1 << 32) || g0.n_alive != n_alive) return false;   // degrees <= mu_alive
    // every clique of the tail sits in ppc words of the rows (a triangle in
    // its three members' rows, an edge in its two ends'), 4 bytes each
    const int64_t ppc = h == 3 ? 3 : 2;
    const int64_t bytes = 4 * ppc * (int64_t)g0.mu_alive + 8 * (int64_t)n + 64 * n_alive;
    const int64_t *roff = h == 3 ? b.tvoff : b.row_ptr;
    const int32_t *rdat = h == 3 ? b.tpairs : b.col;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || bytes > (int64_t)(free_b / 4)) return false;
    const int32_t A = (int32_t)n_alive;
    uint32_t *flag = sc.get_n<uint32_t>(n), *loc = sc.get_n<uint32_t>(n);
    int32_t *glob = sc.get_n<int32_t>(A), *cnt = sc.get_n<int32_t>(2);
    int64_t *ib = sc.get_n<int64_t>(A + 1);
    k_te_flags<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(b.stamp, n, b.ctl, flag);
    scan_exclusive_u32(flag, loc, n, s, sc);
    fill_i32((int32_t *)(ib + A), 0, 2, s);
    k_te_glob<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(flag, loc, n, roff, glob, ib, cnt);
    scan_exclusive_i64(ib, ib, A + 1, s, sc);
    int64_t hv[2] = {0, 0};
    DSD_HIP(hipMemcpyAsync(&hv[0], ib + A, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&hv[1], cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    const int64_t NI = hv[0];
    if ((int32_t)hv[1] != A) throw Error(-3, "tail engine: the tail's vertex count disagrees with the alive count");
    int64_t *kc = sc.get_n<int64_t>(NI + 1);
    const int gp = grid_for(NI, WAVES_PER_BLOCK, 8192), gA = grid_for(A, BLOCK, 64);
    if (NI > 0) {
        if (h == 3) k_te_pairs<false, 3><<<gp, BLOCK, 0, s>>>(roff, rdat, flag, loc, glob, ib, A, NI, kc, nullptr);
        else k_te_pairs<false, 2><<<gp, BLOCK, 0, s>>>(roff, rdat, flag, loc, glob, ib, A, NI, kc, nullptr);
    }
    // rows padded to four pairs, so that lanes load them four at a time
    int64_t *vcnt = sc.get_n<int64_t>(A), *lrow = sc.get_n<int64_t>(A + 1);
    fill_i32((int32_t *)(lrow + A), 0, 2, s);
    k_te_vsum<<<gA, BLOCK, 0, s>>>(ib, kc, A, vcnt, lrow);
    scan_exclusive_i64(lrow, lrow, A + 1, s, sc);
    int64_t total = 0;
    DSD_HIP(hipMemcpyAsync(&total, lrow + A, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (total > ppc * (int64_t)g0.mu_alive + 3 * (int64_t)A)
        throw Error(-3, "tail engine: more pairs than the tail's cliques allow");
    if (total >= ((int64_t)1 << 32)) return false;   // row starts are kept in 32 bits
    u64 walked = 0;   // pairs the engine walks: every kept pair once
    if (kt) {
        u64 *s2 = sc.get_n<u64>(2);
        sum_u64_128((const u64 *)kc, NI, s2, s, sc);
        DSD_HIP(hipMemcpyAsync(&walked, s2, sizeof(u64), hipMemcpyDeviceToHost, s));
    }
    k_te_ioff<<<gA, BLOCK, 0, s>>>(ib, lrow, A, kc);
    uint32_t *lp = sc.get_n<uint32_t>(total);
    if (NI > 0) {
        if (h == 3) k_te_pairs<true, 3><<<gp, BLOCK, 0, s>>>(roff, rdat, flag, loc, glob, ib, A, NI, kc, lp);
        else k_te_pairs<true, 2><<<gp, BLOCK, 0, s>>>(roff, rdat, flag, loc, glob, ib, A, NI, kc, lp);
    }
    k_te_pad<<<gA, BLOCK, 0, s>>>(lrow, vcnt, A, lp);
    fill_i32(cnt, 0, 1, s);
    // the state for grid rounds
    TeState *ts = sc.get_n<TeState>(1);
    TeState hts{};
    hts.deg = sc.get_n<uint32_t>(A);
    hts.st = sc.get_n<uint8_t>(A);
    hts.F = sc.get_n<uint32_t>(A);
    hts.ipre = sc.get_n<uint32_t>(A + 1);
    hts.imap = sc.get_n<uint32_t>(total / TE_ITEM + A + 1);   // items of one round: sum of ceil(row / TE_ITEM)
    DSD_HIP(hipMemcpyAsync(ts, &hts, sizeof(TeState), hipMemcpyHostToDevice, s));
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (kt && kt->time_main)
        for (auto &e : ev) DSD_HIP(hipEventCreate(&e));
    double engine_ms = 0, grid_ms = 0;
    u64 launches = 0;
    int resume = 0;
    uint32_t heavy = TE_HEAVY;
    if (const char *hp = std::getenv("DSD_TE_GRID_PAIRS")) heavy = (uint32_t)std::strtoul(hp, nullptr, 10);
    while (true) {
        if (ev[0]) DSD_HIP(hipEventRecord(ev[0], s));
        if (h == 3) k_tail_engine<3><<<1, TE_BLOCK, 0, s>>>(b, glob, lrow, lp, A, cnt, ts, resume, heavy);
        else k_tail_engine<2><<<1, TE_BLOCK, 0, s>>>(b, glob, lrow, lp, A, cnt, ts, resume, heavy);
        DSD_HIP(hipGetLastError());
        if (ev[1]) DSD_HIP(hipEventRecord(ev[1], s));
        launches += 1;
        int32_t err = 0;
        DSD_HIP(hipMemcpyAsync(&hts, ts, sizeof(TeState), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(&err, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        if (ev[0]) {
            float ms = 0;
            DSD_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            engine_ms += ms;
        }
        if (err) {
            for (auto &e : ev)
                if (e) (void)hipEventDestroy(e);
            throw Error(-3, "tail engine: a round removed no vertex");
        }
        if (!hts.heavy) break;
        // the round the engine stopped at, on every CU; then the engine resumes
        if (ev[2]) DSD_HIP(hipEventRecord(ev[2], s));
        k_te_expand<<<grid_for(hts.nF, WAVES_PER_BLOCK, 1024), BLOCK, 0, s>>>(ts);
        const int gh = (int)std::min<u64>(512, ((u64)hts.items + TE_HBLOCK / WAVE - 1) / (TE_HBLOCK / WAVE));
        if (h == 3) k_te_heavy<3><<<gh, TE_HBLOCK, 0, s>>>(ts, lrow, lp, A);
        else k_te_heavy<2><<<gh, TE_HBLOCK, 0, s>>>(ts, lrow, lp, A);
        DSD_HIP(hipGetLastError());
        if (ev[3]) {
            DSD_HIP(hipEventRecord(ev[3], s));
            DSD_HIP(hipEventSynchronize(ev[3]));
            float ms = 0;
            DSD_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
            grid_ms += ms;
        }
        resume = 1;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (kt) {
        kt->tail_ms += engine_ms;
        kt->tail_launches += launches;
        kt->tail_pairs += walked - hts.pairs;
        kt->tail_vertices += (u64)A;
        kt->tail_grid_ms += grid_ms;
        kt->tail_grid_rounds += hts.rounds;
        kt->tail_grid_pairs += hts.pairs;
    }
    return true;
}

PeelResult peel(const DevGraph &g, int h, const uint8_t *alive0, u64 *deg, u64 mu, u64 k_floor, u64 *core,
                hipStream_t s, Scratch &sc, KernelTimes *kt, const PeelGroups *grp, bool min_degree,
                const TriList *tl, int pattern, int px) {
    PeelResult res;
    const int32_t n = g.n;
    if (n == 0) return res;
    const int32_t G = grp ? grp->G : 1;
    PeelBufs b{};
    b.n = n;
    b.h = h;
    b.G = G;
    b.gid = grp ? grp->gid : nullptr;
    b.row_ptr = g.row_ptr;
    b.col = g.col;
    b.dag_off = g.dag_off;
    b.minpeel = min_degree ? 1 : 0;
    int gloop = 0;
    if (pattern != 0) {
        // special patterns: no clique machinery (h is only the pattern's size)
        b.pattern = pattern;
        b.px = px;
        b.h = 0;
        h = 2;
        tl = nullptr;
        if (pattern == 1) {
            b.ydeg = sc.get_n<int32_t>(n);
            b.yold = sc.get_n<int32_t>(n);
            b.tround = sc.get_n<int32_t>(n);
            b.touch = sc.get_n<int32_t>(n);
            k_star_init<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(b);
        } else {
            b.lsize = loop_tables(g, &gloop, s, sc);
            b.lkey = sc.get_n<int32_t>((int64_t)gloop * b.lsize);
            b.lval = sc.get_n<uint32_t>((int64_t)gloop * b.lsize);
        }
    }
    // h >= 4: one item per frontier vertex (root mode) unless an out-list is
    // longer than a block holds (then the (v, w) items below);
    // DSD_PEEL_ROOT=0 turns root mode off
    const char *rm_env = std::getenv("DSD_PEEL_ROOT");
    const bool rootmode = h >= 4 && pattern == 0 && g.maxdout <= ROOT_CAP && !(rm_env && rm_env[0] == '0');
    b.rootmode = rootmode ? 1 : 0;
    b.count_work = kt != nullptr && (h <= 3 || rootmode);
    b.ctl = sc.get_n<PeelCtl>(1);
    b.gs = sc.get_n<GraphState>(G);
    b.stamp = sc.get_n<int32_t>(n);
    b.deg = deg;
    b.core = core;
    b.F = sc.get_n<int32_t>(2 * (int64_t)n);
    b.lists = sc.get_n<int32_t>(2 * (int64_t)n);
    const int64_t lv_total = grp ? grp->lv_total : (int64_t)n + 1;
    b.lv_k = sc.get_n<u64>(lv_total);
    b.lv_size = sc.get_n<u64>(lv_total);
    b.lv_mu = sc.get_n<u64>(lv_total);
    const bool listed = h == 3 && tl != nullptr && tl->pairs != nullptr;
    if (listed) {
        b.tvoff = tl->voff;
        b.tpairs = tl->pairs;
        // a vertex joins at most one frontier; its items number <= 1 + pairs / TL_CHUNK
        b.tcap = (int64_t)n + tl->entries / TL_CHUNK + 1;
        b.T = sc.get_n<int64_t>(2 * b.tcap);
    } else if (h == 3) {
        // a vertex joins at most one frontier; its chunks number <= 1 + deg / CHUNK
        b.bcap = (int64_t)n + 2 * g.m / CHUNK + 1;
        b.B = sc.get_n<int64_t>(2 * b.bcap);
        // a vertex of degree d > SMALL_DEG takes SLOTS_PER_CHUNK * ceil(d / CHUNK) < 4d
        // slots, and no vertex is in two frontiers: 8m slots per half suffice
        b.hcap = 8 * g.m + SLOTS_PER_CHUNK;
        b.hkey = sc.get_n<int32_t>(2 * b.hcap);
        b.hval = sc.get_n<uint32_t>(2 * b.hcap);
        b.hbase = sc.get_n<int64_t>(n);
        fill_i32(b.hkey, HASH_EMPTY, 2 * b.hcap, s);
        fill_i32((int32_t *)b.hval, 0, 2 * b.hcap, s);
        // one wide item per (frontier vertex, neighbour): at most 2m per round
        b.wcap = 2 * g.m + 1;
        b.W = sc.get_n<int64_t>(b.wcap);
    }
    const int R = h - 2;
    u64 *gS = nullptr, *gSr = nullptr;
    constexpr int ROOT_GRID = 512, ROOT_EDGE_GRID = 1024;
    if (rootmode) {
        // a vertex joins at most one frontier: one wave item, at most
        // 1 + deg / ROOT_SL slice items, or at most 1 + deg / ROOT_CAP
        // single-workgroup items
        b.bcap = (int64_t)n + 2 * g.m / ROOT_SL + 1;
        b.B = sc.get_n<int64_t>(2 * b.bcap);
        b.tcap = (int64_t)n + 1;
        b.T = sc.get_n<int64_t>(2 * b.tcap);
        b.bigcap = (int64_t)n + 2 * g.m / ROOT_CAP + 1;
        b.Big = sc.get_n<int64_t>(2 * b.bigcap);
        // bitmap rows of one round's sliced vertices (a vertex that finds no
        // room becomes a single-workgroup item); every word read is written
        // in the same round (or masked out), so nothing is cleared.  At h = 4
        // a half holds 2^21 words (16 MiB, half the chip's L2): in a round
        // with many long rows the regions beyond that thrash L2 and do better
        // as single-workgroup items, whose bitmaps stay in one workgroup's
        // slice (R-MAT scale 22: CoreApp's peel 0.96 s at 2^26 words, 0.54 s
        // at 2^21; the full peel 4.46 -> 4.24 s); at h >= 5 (rows of at most
        // 2,048 entries) 2^26 measures slightly better.
        const int64_t rmax = h == 4 ? (int64_t)1 << 21 : (int64_t)1 << 26;
        b.rcap = std::min<int64_t>(rmax, std::max<int64_t>((int64_t)1 << 16, 16 * g.m));
        // DSD_ROOT_ARENA_WORDS overrides the arena size (0: every vertex a single-workgroup item)
        if (const char *ra = std::getenv("DSD_ROOT_ARENA_WORDS")) b.rcap = std::max<int64_t>(1, std::atoll(ra));
        b.rbits = sc.get_n<u64>(2 * b.rcap);
        b.rbase = sc.get_n<int64_t>(n);
        gSr = sc.get_n<u64>((int64_t)ROOT_GRID * ROOT_SLICE);
    } else if (h >= 4) {
        // a vertex joins at most one frontier; its chunks number <= 1 + deg / CHUNK4
        b.bcap = (int64_t)n + 2 * g.m / CHUNK4 + 1;
        b.B = sc.get_n<int64_t>(2 * b.bcap);
        // every (v, w) item is an arc of the frontier's adjacency; a round holds at most 2m of them
        b.item_cap = 2 * g.m + 1;
        b.item_v = sc.get_n<int32_t>(5 * b.item_cap);
        b.item_w = sc.get_n<int32_t>(5 * b.item_cap);
        if (R >= 3) gS = sc.get_n<u64>((int64_t)256 * 1280 * 20);
        if (g.maxdout > 1280 && R >= 3)
            throw Error(-5, "an out-neighbourhood exceeds 1280 vertices (limit of the (v, w) item kernels, h >= 5, "
                            "with the per-vertex counting turned off)");
    }
    const u64 *mu_dev = grp ? grp->mu : nullptr;
    if (!mu_dev) {
        u64 *m1 = sc.get_n<u64>(1);
        fill_u64(m1, mu, 1, s);
        mu_dev = m1;
    }
    fill_i32((int32_t *)b.ctl, 0, (int64_t)(sizeof(PeelCtl) / sizeof(int32_t)), s);
    k_init_graphs<<<grid_for(G, 256), 256, 0, s>>>(b, mu_dev, grp ? grp->lv_base : nullptr, k_floor);
    k_peel_init<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(b, alive0, b.lists, &b.ctl->nlist[0]);
    k_start_graphs<<<grid_for(G, 256), 256, 0, s>>>(b);
    int64_t *pinned = (int64_t *)thread_pinned();
    DSD_HIP(hipMemcpyAsync(pinned, &b.ctl->n_alive, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    int64_t n_alive = pinned[0];
    if (h >= 4 && !rootmode && n_alive > 0) {
        // the edges among the starting vertices, at most half the slots filled
        const int64_t pairs = n_alive * (n_alive - 1) / 2;
        const int64_t edges = std::max<int64_t>(1, std::min<int64_t>(g.m, pairs));
        int bits = 10;
        while (((int64_t)1 << bits) < 2 * edges) bits++;
        u64 *t = sc.get_n<u64>((int64_t)1 << bits);
        fill_u64(t, ESET_EMPTY, (int64_t)1 << bits, s);
        b.eset = t;
        b.eset_bits = bits;
        k_eset_fill<<<grid_for(n_alive, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, b.lists, &b.ctl->nlist[0], t);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt) {
        DSD_HIP(hipEventCreate(&e0));
        DSD_HIP(hipEventCreate(&e1));
        DSD_HIP(hipEventRecord(e0, s));
    }
    const int gmin = 256, gbuild = 1024, gproc = 2048, gprobe = 1024, gtail = 256;
    // tail mode from this many alive vertices on (the count only falls)
    constexpr int64_t TAIL_ALIVE = 16384;
    bool tail = false;
    LaunchTimer<0> main_timer(kt != nullptr && kt->time_main && (h <= 3 || rootmode));
    LaunchTimer<1> main2_timer(kt != nullptr && kt->time_main && rootmode);
    // the lists need no adjacency: dead entries are skipped by their bit
    int64_t steps = 0, chunk = 4;
    const int64_t max_steps = 4 * (int64_t)n + 64;
    const bool compacting = !listed;
    int64_t compacted_at = n;
    if (compacting && n_alive > 0 && n_alive < n / 2) {
        compact_adjacency(b, s, sc);
        compacted_at = n_alive;
    }
    const bool engine = (listed || h == 2) && G == 1 && !min_degree && pattern == 0;
    // DSD_PEEL_GRAPH=1: every round's kernels replayed from a captured HIP
    // graph instead of launched one by one (not with per-launch timing)
    const char *pg = std::getenv("DSD_PEEL_GRAPH");
    const bool use_graph = pg && pg[0] == '1' && !main_timer.on() && !main2_timer.on();
    RoundGraphs graphs;
    if (use_graph) DSD_HIP(hipStreamCreateWithFlags(&graphs.cs, hipStreamNonBlocking));
    while (n_alive > 0) {
        if (engine && n_alive <= TE_MAX && tail_engine(b, h, n, n_alive, s, sc, kt)) break;
        if (compacting && n_alive < compacted_at / 2) {
            compact_adjacency(b, s, sc);
            compacted_at = n_alive;
            graphs.reset();
        }
        if (n_alive <= TAIL_ALIVE) tail = true;
        const int gp = tail ? gtail : gprobe, gq = tail ? gtail : gproc, gf = tail ? gtail : gbuild;
        // one round's kernels; they read the round's state from the device,
        // so the same sequence serves every round until the adjacency
        // (a kernel argument) is compacted
        auto one_round = [&](hipStream_t st) {
            if (tail) {
                k_tail_level<<<1, TAIL_BLOCK, 0, st>>>(b);
            } else {
                k_level_min<<<gmin, BLOCK, 0, st>>>(b);
                k_level_build<<<gbuild, BLOCK, 0, st>>>(b);
            }
            if (b.pattern == 1) {
                main_timer.launch(k_star_front, dim3(gq), dim3(BLOCK), st, b);
                k_star_touch<<<gq, BLOCK, 0, st>>>(b);
            } else if (b.pattern == 2) {
                main_timer.launch(k_loop_process, dim3(gloop), dim3(BLOCK), st, b);
            } else if (h == 2) {
                main_timer.launch(k_process_h2, dim3(gq), dim3(BLOCK), st, b);
            } else if (listed) {
                main_timer.launch(k_tl_process, dim3(gp), dim3(BLOCK), st, b);
            } else if (h == 3) {
                k_h3_fill<<<gf, BLOCK, 0, st>>>(b);
                main_timer.launch(k_h3_probe, dim3(gp), dim3(BLOCK), st, b);
                k_h3_flush<<<gf, BLOCK, 0, st>>>(b);
            } else if (rootmode) {
                switch (h) {
                    case 4:
                        main_timer.launch(k_root_edges<3>, dim3(ROOT_EDGE_GRID), dim3(BLOCK), st, b);
                        main2_timer.launch(k_root_count<3, true, false>, dim3(ROOT_GRID), dim3(BLOCK), st, b, gSr);
                        k_root_count<3, false, true><<<ROOT_GRID, BLOCK, 0, st>>>(b, gSr);
                        break;
                    case 5:
                        main_timer.launch(k_root_edges<4>, dim3(ROOT_EDGE_GRID), dim3(BLOCK), st, b);
                        main2_timer.launch(k_root_count<4, true, false>, dim3(ROOT_GRID), dim3(BLOCK), st, b, gSr);
                        k_root_count<4, false, true><<<ROOT_GRID, BLOCK, 0, st>>>(b, gSr);
                        break;
                    case 6:
                        main_timer.launch(k_root_edges<5>, dim3(ROOT_EDGE_GRID), dim3(BLOCK), st, b);
                        main2_timer.launch(k_root_count<5, true, false>, dim3(ROOT_GRID), dim3(BLOCK), st, b, gSr);
                        k_root_count<5, false, true><<<ROOT_GRID, BLOCK, 0, st>>>(b, gSr);
                        break;
                    default: throw Error(-1, "h outside [2, 6]");
                }
            } else {
                k_peel_items<<<gproc, BLOCK, 0, st>>>(b, R);
                switch (R) {
                    case 2: launch_peel_items<2>(b, st, gS, g.maxdout); break;
                    case 3: launch_peel_items<3>(b, st, gS, g.maxdout); break;
                    case 4: launch_peel_items<4>(b, st, gS, g.maxdout); break;
                    default: throw Error(-1, "h outside [2, 6]");
                }
            }
            if (tail) {
                // the next k_tail_level ends this round
            } else if (G == 1) {
                k_finish_one<<<1, 1, 0, st>>>(b);
            } else {
                k_finish_graphs<<<grid_for(G, 256), 256, 0, st>>>(b);
                k_finish_global<<<1, 1, 0, st>>>(b);
            }
        };
        if (use_graph) {
            hipGraphExec_t &ge = graphs.exec[tail ? 1 : 0];
            if (!ge) {
                // captured on a stream of its own (the graph's stream may be
                // the null stream, which cannot be captured), replayed on s
                DSD_HIP(hipStreamBeginCapture(graphs.cs, hipStreamCaptureModeThreadLocal));
                one_round(graphs.cs);
                hipGraph_t gr = nullptr;
                DSD_HIP(hipStreamEndCapture(graphs.cs, &gr));
                const hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (ie != hipSuccess) throw Error(-3, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
            }
            for (int64_t i = 0; i < chunk; i++) DSD_HIP(hipGraphLaunch(ge, s));
        } else {
            for (int64_t i = 0; i < chunk; i++) one_round(s);
        }
        if (tail) k_tail_finish<<<1, TAIL_BLOCK, 0, s>>>(b);
        steps += chunk;
        DSD_HIP(hipMemcpyAsync(pinned, &b.ctl->n_alive, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        n_alive = pinned[0];
        if (steps > max_steps) throw Error(-3, "peel did not converge");
        if (chunk < 32) chunk *= 2;
    }
    if (kt) {
        DSD_HIP(hipEventRecord(e1, s));
        DSD_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DSD_HIP(hipEventElapsedTime(&ms, e0, e1));
        kt->k4_ms += ms;
        kt->k4_launches += 1;
        u64 launches = 0;
        kt->main_ms += main_timer.total_ms(&launches);
        kt->main_launches += launches;
        kt->main2_ms += main2_timer.total_ms(&launches);
        kt->main2_launches += launches;
        if (b.pattern == 1) kt->main_kind = 4;
        else if (b.pattern == 2) kt->main_kind = 5;
        else if (h == 2) kt->main_kind = 1;
        else if (h == 3) kt->main_kind = listed ? 3 : 2;
        else if (rootmode) kt->main_kind = 6;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    PeelCtl fin;
    std::vector<GraphState> gst(G);
    DSD_HIP(hipMemcpyAsync(&fin, b.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(gst.data(), b.gs, G * sizeof(GraphState), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (fin.n_alive != 0) throw Error(-3, "peel ended with alive vertices");
    if (kt && b.count_work) {
        kt->main_pairs += fin.work[0];
        kt->main_nbrs += fin.work[1];
        kt->main_entries += fin.work[2];
        kt->main2_words += fin.work[3];
    }
    res.rounds = fin.round;
    res.graph_levels.resize(G);
    for (int32_t i = 0; i < G; i++) {
        if (gst[i].n_alive != 0) throw Error(-3, "peel ended with alive vertices in a graph");
        res.graph_levels[i] = gst[i].nlevels;
        res.levels += gst[i].nlevels;
    }
    const int64_t ncopy = G == 1 ? (int64_t)gst[0].nlevels : lv_total;
    res.level_k.resize(ncopy);
    res.level_size.resize(ncopy);
    res.level_mu.resize(ncopy);
    if (ncopy > 0) {
        DSD_HIP(hipMemcpyAsync(res.level_k.data(), b.lv_k, ncopy * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(res.level_size.data(), b.lv_size, ncopy * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(res.level_mu.data(), b.lv_mu, ncopy * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
    }
    if (G == 1 && gst[0].nlevels > 0) res.kmax = res.level_k.back();
    return res;
}

}  // namespace dsd
