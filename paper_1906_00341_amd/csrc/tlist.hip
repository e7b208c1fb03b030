// Triangle lists (h = 3): row v holds a pair (a, b) for every triangle
// {v, a, b}, twice (as (a, b) and as (b, a)), grouped by a in the order of
// v's CSR row; the rows hold 6 mu pairs in all.
//
// The peel destroys the triangles of a removed vertex by walking its row in
// fixed-size runs of pairs, so that even a hub's row spreads over thousands
// of waves; each neighbour's losses are summed over its run of pairs before
// they reach its degree.
//
// Listing: every triangle {u, w, x} with rank u < w < x is found once from
// its root u, as w in N+(u) and x in N+(w) ∩ N+(u); N+(u) is hashed in LDS
// with each member's position in row u (one wave per root of out-degree <=
// 64, one workgroup per larger root).  A first pass counts the triangles on
// every edge (its support, for both arcs), a second writes the six pairs
// through per-arc cursors into the segment of each arc.
#include <cstdlib>
#include <cstring>

#include "graph.hpp"
#include "primitives.hpp"

namespace dsd {

namespace {

constexpr int TL_SMALL = 64;          // roots with |N+| <= this take one wave
constexpr int TL_SMALL_BITS = 7;      // their hash: 128 slots
constexpr int TL_MAX_OUT = 2048;      // larger roots take a workgroup, hash of <= 4096 slots
constexpr int TL_BIG_BITS = 12;
constexpr int TL_EMPTY = -1;
constexpr int64_t TL_MAX_BYTES = (int64_t)24 << 30;

struct TlBuild {
    const int64_t *row_ptr;
    const int32_t *col;
    const int64_t *dag_off;
    const int64_t *rev;   // [2m] reverse arc: rev[e] for e = (v, a) is the position of v in row a
    u64 *cnt;             // [2m] pass 0: supports of forward arcs; pass 1: write cursors
    const int64_t *woff;  // [2m + 1] arc segment starts (pass 1)
    int32_t *pairs;       // [2 * 6 mu] (a, b) (pass 1)
    int32_t *big;         // roots with more than TL_SMALL out-neighbours
    int32_t *nbig;
    int32_t *err;         // set if a list would overflow (never, when the supports are right)
    int32_t n;
    int32_t pass;         // 0: count, 1: fill
};

__device__ __forceinline__ void tl_insert(int32_t *keys, int32_t *pos, int bits, int32_t x, int32_t p) {
    const uint32_t mask = (1u << bits) - 1;
    uint32_t slot = hash_slot(x, bits);
    while (true) {
        const int32_t prev = atomicCAS(&keys[slot], TL_EMPTY, x);
        if (prev == TL_EMPTY) {
            pos[slot] = p;
            return;
        }
        if (prev == x) return;
        slot = (slot + 1) & mask;
    }
}

// position (offset in N+(u)) of x, or -1
__device__ __forceinline__ int32_t tl_find(const int32_t *keys, const int32_t *pos, int bits, int32_t x) {
    const uint32_t mask = (1u << bits) - 1;
    uint32_t slot = hash_slot(x, bits);
    while (true) {
        const int32_t k = keys[slot];
        if (k == x) return pos[slot];
        if (k == TL_EMPTY) return -1;
        slot = (slot + 1) & mask;
    }
}

// pair (a, y) into the segment of arc e = (v, a) through its cursor
__device__ __forceinline__ void tl_put(const TlBuild &b, int64_t e, int32_t a, int32_t y) {
    const int64_t p = (int64_t)atomicAdd(&b.cnt[e], (u64)1);
    if (p >= b.woff[e + 1]) {
        atomicOr(b.err, 1);
        return;
    }
    b.pairs[2 * p] = a;
    b.pairs[2 * p + 1] = y;
}

// One wave: the triangles {u, w, x} for the out-neighbours w of u at row
// positions [lo, hi) (hi - lo <= 64; u's out-list starts at ulo), x in N+(w)
// found in the hash of N+(u).  The (w, x) pairs are flattened over the
// lanes.  sPre/sSt/sW: this wave's 64-entry LDS scratch.
__device__ __forceinline__ void tl_range(const TlBuild &b, int32_t u, int64_t ulo, const int32_t *keys,
                                         const int32_t *pos, int bits, int64_t lo, int64_t hi, int32_t *sPre,
                                         int64_t *sSt, int32_t *sW) {
    const int L = lane();
    int32_t w = -1, len = 0;
    int64_t st0 = 0;
    if (lo + L < hi) {
        w = b.col[lo + L];
        st0 = b.dag_off[w];
        len = (int32_t)(b.row_ptr[w + 1] - st0);
    }
    const int32_t inc = wave_incl_scan(len);
    sPre[L] = inc;
    sSt[L] = st0;
    sW[L] = w;
    const int32_t total = __shfl(inc, WAVE - 1, WAVE);
    __builtin_amdgcn_wave_barrier();
    for (int32_t pb = 0; pb < total; pb += WAVE) {
        const int32_t p = pb + L;
        int i = 0;
        int32_t x = -1, px = -1;
        int64_t e_wx = 0;
        if (p < total) {
            i = upper_bound_i32(sPre, WAVE, p);
            const int32_t o = p - (i ? sPre[i - 1] : 0);
            e_wx = sSt[i] + o;
            x = b.col[e_wx];
            px = tl_find(keys, pos, bits, x);
        }
        const bool found = px >= 0;
        const u64 fm = __ballot(found);
        if (!fm) continue;
        // lanes with the same w form a run (i is non-decreasing over the lanes)
        const int prev_i = __shfl_up(i, 1, WAVE);
        const bool head = p < total && (L == 0 || prev_i != i);
        const u64 hm = __ballot(head);
        const u64 le = lanemask_lt() | (1ull << L);
        const int start = 63 - __builtin_clzll(hm & le);             // first lane of this lane's run
        const u64 nxt = hm & ~le;
        const int end = nxt ? __builtin_ctzll(nxt) : WAVE;            // one past the run
        const u64 run = (end == WAVE ? ~0ull : ((1ull << end) - 1)) & ~((1ull << start) - 1);
        const int32_t c = __popcll(fm & run);
        const int64_t e_uw = lo + i, e_ux = ulo + px;
        if (b.pass == 0) {
            if (L == start && c > 0) atomicAdd(&b.cnt[e_uw], (u64)c);
            if (found) {
                atomicAdd(&b.cnt[e_ux], (u64)1);
                atomicAdd(&b.cnt[e_wx], (u64)1);
            }
        } else {
            // the two lists of edge (u, w) take one cursor step per run
            u64 b1 = 0, b2 = 0;
            if (L == start && c > 0) {
                b1 = atomicAdd(&b.cnt[e_uw], (u64)c);
                b2 = atomicAdd(&b.cnt[b.rev[e_uw]], (u64)c);
            }
            b1 = __shfl(b1, start, WAVE);
            b2 = __shfl(b2, start, WAVE);
            if (found) {
                const int32_t k = __popcll(fm & run & lanemask_lt());
                const int32_t wv = sW[i];
                const int64_t q1 = (int64_t)b1 + k, q2 = (int64_t)b2 + k;
                if (q1 < b.woff[e_uw + 1]) {
                    b.pairs[2 * q1] = wv;
                    b.pairs[2 * q1 + 1] = x;
                } else {
                    atomicOr(b.err, 1);
                }
                if (q2 < b.woff[b.rev[e_uw] + 1]) {
                    b.pairs[2 * q2] = u;
                    b.pairs[2 * q2 + 1] = x;
                } else {
                    atomicOr(b.err, 1);
                }
                tl_put(b, e_ux, x, wv);
                tl_put(b, b.rev[e_ux], u, wv);
                tl_put(b, e_wx, x, u);
                tl_put(b, b.rev[e_wx], wv, u);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// roots of out-degree 2 .. TL_SMALL, one wave each; larger roots are queued (pass 0)
__global__ __launch_bounds__(BLOCK) void k_tl_small(TlBuild b) {
    __shared__ int32_t sKey[WAVES_PER_BLOCK][1 << TL_SMALL_BITS];
    __shared__ int32_t sPos[WAVES_PER_BLOCK][1 << TL_SMALL_BITS];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    const int wv = threadIdx.x / WAVE, L = lane();
    for (int64_t u = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; u < b.n; u += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int64_t lo = b.dag_off[u], hi = b.row_ptr[u + 1];
        const int64_t d = hi - lo;
        if (d < 2) continue;
        if (d > TL_SMALL) {
            if (b.pass == 0 && L == 0) b.big[atomicAdd(b.nbig, 1)] = (int32_t)u;
            continue;
        }
        for (int i = L; i < (1 << TL_SMALL_BITS); i += WAVE) sKey[wv][i] = TL_EMPTY;
        __builtin_amdgcn_wave_barrier();
        if (L < d) tl_insert(sKey[wv], sPos[wv], TL_SMALL_BITS, b.col[lo + L], L);
        __builtin_amdgcn_wave_barrier();
        tl_range(b, (int32_t)u, lo, sKey[wv], sPos[wv], TL_SMALL_BITS, lo, hi, sPre[wv], sSt[wv], sW[wv]);
    }
}

// queued roots (out-degree TL_SMALL+1 .. TL_MAX_OUT), one workgroup each
__global__ __launch_bounds__(BLOCK) void k_tl_big(TlBuild b) {
    __shared__ int32_t sKey[1 << TL_BIG_BITS];
    __shared__ int32_t sPos[1 << TL_BIG_BITS];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    const int wv = threadIdx.x / WAVE;
    const int32_t nb = *b.nbig;
    for (int32_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int32_t u = b.big[i];
        const int64_t lo = b.dag_off[u], hi = b.row_ptr[u + 1];
        const int64_t d = hi - lo;
        int bits = 1;
        while ((int64_t)1 << bits < 2 * d) bits++;      // load <= 1/2; d <= TL_MAX_OUT keeps bits <= 12
        for (int j = threadIdx.x; j < (1 << bits); j += BLOCK) sKey[j] = TL_EMPTY;
        __syncthreads();
        for (int64_t j = threadIdx.x; j < d; j += BLOCK) tl_insert(sKey, sPos, bits, b.col[lo + j], (int32_t)j);
        __syncthreads();
        for (int64_t c = lo + (int64_t)wv * WAVE; c < hi; c += (int64_t)WAVES_PER_BLOCK * WAVE)
            tl_range(b, u, lo, sKey, sPos, bits, c, c + WAVE < hi ? c + WAVE : hi, sPre[wv], sSt[wv], sW[wv]);
        __syncthreads();
    }
}

// reverse arcs: for a forward arc e = (v, a) (a in N+(v)), v sits in the
// in-part of row a, which is sorted by rank
__global__ void k_tl_rev(const int64_t *row_ptr, const int32_t *col, const int64_t *dag_off, int32_t n,
                         int64_t *rev) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        for (int64_t e = dag_off[v] + lane(); e < row_ptr[v + 1]; e += WAVE) {
            const int32_t a = col[e];
            const int64_t f = bsearch_i32(col, row_ptr[a], dag_off[a], (int32_t)v);
            rev[e] = f;
            if (f >= 0) rev[f] = e;
        }
    }
}

// supports of reverse arcs from their forward arcs; -1 in rev means a
// broken CSR (never)
__global__ void k_tl_mirror(const int64_t *row_ptr, const int64_t *dag_off, const int64_t *rev, int32_t n, u64 *cnt,
                            int32_t *err) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        for (int64_t e = dag_off[v] + lane(); e < row_ptr[v + 1]; e += WAVE) {
            const int64_t f = rev[e];
            if (f < 0) atomicOr(err, 4);
            else cnt[f] = cnt[e];
        }
    }
}

// every list must be exactly full
__global__ void k_tl_check(const u64 *cur, const int64_t *woff, int64_t arcs, int32_t *err) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < arcs; e += (int64_t)gridDim.x * blockDim.x)
        if ((int64_t)cur[e] != woff[e + 1]) atomicOr(err, 2);
}

__global__ void k_tl_offsets_tail(int64_t *woff, const u64 *cnt, int64_t arcs) {
    if (blockIdx.x == 0 && threadIdx.x == 0) woff[arcs] = woff[arcs - 1] + (int64_t)cnt[arcs - 1];
}

// clique-degrees from the supports: every triangle at v is counted on two of
// v's arcs (one wave per vertex)
__global__ void k_tl_degrees(const int64_t *row_ptr, const u64 *cnt, int32_t n, u64 *deg) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        u64 sum = 0;
        for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) sum += cnt[e];
        sum = wave_sum(sum);
        if (lane() == 0) deg[v] = sum / 2;
    }
}

// clique-degrees from finished lists: row v holds two pairs per triangle at v
__global__ void k_tl_row_degrees(const int64_t *voff, int32_t n, u64 *deg) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = (u64)(voff[v + 1] - voff[v]) / 2;
}

// row starts: voff[v] = start of v's first arc segment
__global__ void k_tl_rows(const int64_t *row_ptr, const int64_t *woff, int32_t n, int64_t *voff) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x)
        voff[v] = woff[row_ptr[v]];
}

}  // namespace

bool tri_list_wanted(const DevGraph &g, u64 mu) {
    const char *e = std::getenv("DSD_TRI_LIST");
    if (e && std::strcmp(e, "0") == 0) return false;
    if (g.n == 0 || mu == 0 || g.maxdout > TL_MAX_OUT) return false;
    if (mu > (u64)0x7fffffff / 6) return false;             // entries are counted in int32 positions
    const int64_t entries = 6 * (int64_t)mu, arcs = 2 * g.m;
    // pairs and row starts, and the build's segment starts, cursors and reverse arcs
    const int64_t bytes = 8 * entries + 8 * ((int64_t)g.n + 1) + 24 * arcs + 8;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    return bytes <= TL_MAX_BYTES && bytes <= (int64_t)(free_b / 4);
}

bool tri_supports_possible(const DevGraph &g) {
    const char *e = std::getenv("DSD_TRI_LIST");
    if (e && std::strcmp(e, "0") == 0) return false;
    if (g.n == 0 || g.m == 0 || g.maxdout > TL_MAX_OUT) return false;
    // reverse arcs, supports and segment starts: 24 B per arc
    const int64_t bytes = 24 * 2 * g.m + 8 * ((int64_t)g.n + 1);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    return bytes <= (int64_t)(free_b / 4);
}

u64 tri_supports(const DevGraph &g, u64 *deg, TlCounts &w, hipStream_t s, Scratch &sc) {
    const int32_t n = g.n;
    const int64_t arcs = 2 * g.m;
    w.rev = sc.get_n<int64_t>(arcs);
    w.cnt = sc.get_n<u64>(arcs);
    w.big = sc.get_n<int32_t>(n);
    w.nbig = sc.get_n<int32_t>(2);
    fill_i32(w.nbig, 0, 2, s);
    fill_u64(w.cnt, 0, arcs, s);
    TlBuild b{};
    b.row_ptr = g.row_ptr;
    b.col = g.col;
    b.dag_off = g.dag_off;
    b.rev = w.rev;
    b.cnt = w.cnt;
    b.big = w.big;
    b.nbig = w.nbig;
    b.err = w.nbig + 1;
    b.n = n;
    k_tl_rev<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, g.dag_off, n, w.rev);
    b.pass = 0;
    k_tl_small<<<grid_for(n, WAVES_PER_BLOCK, 4096), BLOCK, 0, s>>>(b);
    k_tl_big<<<1024, BLOCK, 0, s>>>(b);
    k_tl_mirror<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.dag_off, w.rev, n, w.cnt, b.err);
    k_tl_degrees<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, w.cnt, n, deg);
    u64 *sum = sc.get_n<u64>(2);
    sum_u64_128(deg, n, sum, s, sc);
    u64 hs[2];
    int32_t err = 0;
    DSD_HIP(hipMemcpyAsync(hs, sum, sizeof(hs), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&err, b.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (err) throw Error(-3, "triangle supports: a reverse arc is missing");
    if (hs[1] != 0 || hs[0] % 3 != 0) throw Error(-3, "triangle supports: clique-degree sum not a multiple of 3");
    w.mu = hs[0] / 3;
    return w.mu;
}

void build_tri_list(const DevGraph &g, TlCounts &w, TriList &tl, hipStream_t s, Scratch &sc) {
    free_tri_list(tl);
    const int32_t n = g.n;
    const int64_t arcs = 2 * g.m;
    tl.mu = w.mu;
    tl.entries = 6 * (int64_t)w.mu;
    if (hipMalloc(&tl.voff, (size_t)(n + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&tl.pairs, (size_t)(tl.entries > 0 ? tl.entries : 1) * 2 * sizeof(int32_t)) != hipSuccess) {
        free_tri_list(tl);
        throw Error(-2, "device allocation of the triangle lists failed");
    }
    TlBuild b{};
    b.row_ptr = g.row_ptr;
    b.col = g.col;
    b.dag_off = g.dag_off;
    b.rev = w.rev;
    b.cnt = w.cnt;
    int64_t *woff = sc.get_n<int64_t>(arcs + 1);
    b.woff = woff;
    b.pairs = tl.pairs;
    b.big = w.big;
    b.nbig = w.nbig;
    b.err = w.nbig + 1;
    b.n = n;
    scan_exclusive_i64((const int64_t *)w.cnt, woff, arcs, s, sc);
    k_tl_offsets_tail<<<1, 1, 0, s>>>(woff, w.cnt, arcs);
    int32_t err = 0;
    int64_t total = 0;
    DSD_HIP(hipMemcpyAsync(&err, b.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&total, woff + arcs, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (err || total != tl.entries) {      // every reverse arc found, supports summing to 6 mu
        free_tri_list(tl);
        throw Error(-3, "triangle lists do not match the supports");
    }
    DSD_HIP(hipMemcpyAsync(b.cnt, woff, (size_t)arcs * sizeof(u64), hipMemcpyDeviceToDevice, s));
    k_tl_rows<<<grid_for((int64_t)n + 1, BLOCK, 4096), BLOCK, 0, s>>>(g.row_ptr, woff, n, tl.voff);
    b.pass = 1;
    k_tl_small<<<grid_for(n, WAVES_PER_BLOCK, 4096), BLOCK, 0, s>>>(b);
    k_tl_big<<<1024, BLOCK, 0, s>>>(b);
    k_tl_check<<<grid_for(arcs, BLOCK, 4096), BLOCK, 0, s>>>(b.cnt, woff, arcs, b.err);
    DSD_HIP(hipMemcpyAsync(&err, b.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (err) {
        free_tri_list(tl);
        throw Error(-3, "triangle lists do not match the supports");
    }
}

void build_tri_list(const DevGraph &g, const u64 *deg, u64 mu, TriList &tl, hipStream_t s, Scratch &sc) {
    (void)deg;
    TlCounts w;
    u64 *d = sc.get_n<u64>(g.n);
    if (tri_supports(g, d, w, s, sc) != mu) throw Error(-3, "triangle lists do not match the clique-degrees");
    build_tri_list(g, w, tl, s, sc);
}

void tri_list_degrees(const TriList &tl, int32_t n, u64 *deg, hipStream_t s) {
    k_tl_row_degrees<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(tl.voff, n, deg);
}

void free_tri_list(TriList &tl) {
    (void)hipFree(tl.voff);
    (void)hipFree(tl.pairs);
    tl = TriList();
}

}  // namespace dsd
