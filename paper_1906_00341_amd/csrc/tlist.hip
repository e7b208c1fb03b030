// Triangle lists (h = 3): row v holds a pair (a, b) for every triangle
// {v, a, b}, once, with a ranked below b, in the segment of arc (v, a); the
// segments follow v's CSR row, so a row is grouped by a, and the rows hold
// 3 mu pairs in all.
//
// The peel destroys the triangles of a removed vertex by walking its row in
// fixed-size runs of pairs, so that even a hub's row spreads over thousands
// of waves; the losses of a are summed over its run of pairs before they
// reach its degree, b loses its triangle on its own.
//
// Listing: every triangle {u, w, x} with rank u < w < x is found once from
// its root u, as w in N+(u) and x in N+(w) ∩ N+(u); N+(u) is hashed in LDS
// with each member's position in row u.  A root of out-degree <= 64 takes
// one wave; one of out-degree <= 256 is cut into chunks of 64 out-neighbours
// w, each chunk an item for one wave that hashes N+(u) itself (the hashing
// costs d+(u)/64 steps against the chunk's sum of d+(w) probes, and every
// wave of the chip stays busy); larger roots take a workgroup.  The triangle
// goes to the segments of (u, w) as (w, x), of (w, u) as (u, x) and of
// (x, u) as (u, w), so every segment is written only by the root of its
// triangles, the lower end of its arc.  A first pass counts, on u's own
// forward arcs (u, a), the triangles with a in the middle (r1, summed over a
// run of lanes) and with a on top (r2); segment (u, a) then holds r1 pairs
// and segment (a, u) r1 + r2.  A second pass writes the three pairs through
// per-arc cursors.  Counts and cursors are 32-bit (a count is below n, a
// position below 3 mu < 2^31); a write is bounded by the size of the lists,
// and a final check that every cursor stopped exactly at its segment's end
// catches any miscount.
#include <cstdlib>
#include <cstring>

#include "graph.hpp"
#include "primitives.hpp"

namespace dsd {

namespace {

constexpr int TL_SMALL = 64;          // roots with |N+| <= this take one wave
constexpr int TL_SMALL_BITS = 7;      // their hash: 128 slots
constexpr int TL_MID = 256;           // roots with |N+| <= this are cut into per-wave chunks of 64
constexpr int TL_MID_BITS = 9;        // their hash: <= 512 slots
constexpr int TL_MAX_OUT = 2048;      // larger roots take a workgroup, hash of <= 4096 slots
constexpr int TL_BIG_BITS = 12;
constexpr int TL_EMPTY = -1;
constexpr int64_t TL_MAX_BYTES = (int64_t)24 << 30;

struct TlBuild {
    const int64_t *row_ptr;
    const int32_t *col;
    const int64_t *dag_off;
    const int64_t *rev;   // [2m] reverse arc: rev[e] for e = (v, a) is the position of v in row a
    uint32_t *cnt;        // [2m] pass 0: r1 of forward arcs; pass 1: write cursors
    uint32_t *top;        // [2m] pass 0: r2 of forward arcs
    int64_t entries;      // 3 mu: the pairs' capacity (pass 1)
    int32_t *pairs;       // [2 * 3 mu] (a, b) (pass 1)
    int32_t *big;         // roots with more than TL_MID out-neighbours
    int32_t *nbig;        // [0] their count, [1] the error flags, [2] the count of mid items
    int64_t *mid;         // items (root, chunk): root | chunk << 32 for roots of TL_SMALL+1 .. TL_MID
    int32_t *err;         // set if a list would overflow (never, when the counts are right)
    int32_t n;
    int32_t pass;         // 0: count, 1: fill
};

template <class P>
__device__ __forceinline__ void tl_insert(int32_t *keys, P *pos, int bits, int32_t x, int32_t p) {
    const uint32_t mask = (1u << bits) - 1;
    uint32_t slot = hash_slot(x, bits);
    while (true) {
        const int32_t prev = atomicCAS(&keys[slot], TL_EMPTY, x);
        if (prev == TL_EMPTY) {
            pos[slot] = (P)p;
            return;
        }
        if (prev == x) return;
        slot = (slot + 1) & mask;
    }
}

// position (offset in N+(u)) of x, or -1
template <class P>
__device__ __forceinline__ int32_t tl_find(const int32_t *keys, const P *pos, int bits, int32_t x) {
    const uint32_t mask = (1u << bits) - 1;
    uint32_t slot = hash_slot(x, bits);
    while (true) {
        const int32_t k = keys[slot];
        if (k == x) return (int32_t)pos[slot];
        if (k == TL_EMPTY) return -1;
        slot = (slot + 1) & mask;
    }
}

// pair (a, y) at position p of the lists (p from an arc's cursor)
__device__ __forceinline__ void tl_store(const TlBuild &b, int64_t p, int32_t a, int32_t y) {
    if (p >= b.entries) {
        atomicOr(b.err, 1);
        return;
    }
    *(int2 *)&b.pairs[2 * p] = make_int2(a, y);
}

// pair (a, y) into the segment of arc e = (v, a) through its cursor
__device__ __forceinline__ void tl_put(const TlBuild &b, int64_t e, int32_t a, int32_t y) {
    tl_store(b, (int64_t)atomicAdd(&b.cnt[e], 1u), a, y);
}

// One wave: the triangles {u, w, x} for the out-neighbours w of u at row
// positions [lo, hi) (hi - lo <= 64; u's out-list starts at ulo), x in N+(w)
// found in the hash of N+(u).  The (w, x) pairs are flattened over the
// lanes.  sPre/sSt/sW: this wave's 64-entry LDS scratch.
template <class P>
__device__ __forceinline__ void tl_range(const TlBuild &b, int32_t u, int64_t ulo, const int32_t *keys,
                                         const P *pos, int bits, int64_t lo, int64_t hi, int32_t *sPre,
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
    // a lane's step p lies in the row of w number i = the first with
    // sPre[i] > p; the next step's i (a search from the current one, which
    // mostly ends at its first test) and neighbour are fetched while this
    // step's are probed
    int i_n = 0;
    int64_t e_n = 0;
    int32_t x_n = -1;
    if (L < total) {
        i_n = upper_bound_i32(sPre, WAVE, L);
        e_n = sSt[i_n] + (L - (i_n ? sPre[i_n - 1] : 0));
        x_n = b.col[e_n];
    }
    for (int32_t pb = 0; pb < total; pb += WAVE) {
        const int32_t p = pb + L;
        const int i = i_n;
        const int64_t e_wx = e_n;
        const int32_t x = x_n;
        if (p + WAVE < total) {
            const int32_t q = p + WAVE;     // sPre[WAVE - 1] = total > q bounds both searches
            if (sPre[i_n] <= q) i_n += 1 + upper_bound_i32(sPre + i_n + 1, WAVE - 1 - i_n, q);
            e_n = sSt[i_n] + (q - (i_n ? sPre[i_n - 1] : 0));
            x_n = b.col[e_n];
        }
        int32_t px = -1;
        if (p < total) px = tl_find(keys, pos, bits, x);
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
            if (L == start && c > 0) atomicAdd(&b.cnt[e_uw], (uint32_t)c);
            if (found) atomicAdd(&b.top[e_ux], 1u);
        } else {
            // segments (u, w) and (w, u) take one cursor step per run
            uint32_t b1 = 0, b2 = 0;
            if (L == start && c > 0) {
                b1 = atomicAdd(&b.cnt[e_uw], (uint32_t)c);
                b2 = atomicAdd(&b.cnt[b.rev[e_uw]], (uint32_t)c);
            }
            b1 = __shfl(b1, start, WAVE);
            b2 = __shfl(b2, start, WAVE);
            if (found) {
                const int32_t k = __popcll(fm & run & lanemask_lt());
                const int32_t wv = sW[i];
                tl_store(b, (int64_t)b1 + k, wv, x);
                tl_store(b, (int64_t)b2 + k, u, x);
                tl_put(b, b.rev[e_ux], u, wv);
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
            if (b.pass == 0 && L == 0) {
                if (d > TL_MID) {
                    b.big[atomicAdd(b.nbig, 1)] = (int32_t)u;
                } else {
                    const int32_t k = (int32_t)((d + WAVE - 1) / WAVE);
                    const int32_t q = atomicAdd(b.nbig + 2, k);
                    for (int32_t c = 0; c < k; c++) b.mid[q + c] = u | ((int64_t)c << 32);
                }
            }
            continue;
        }
        for (int i = L; i < (1 << TL_SMALL_BITS); i += WAVE) sKey[wv][i] = TL_EMPTY;
        __builtin_amdgcn_wave_barrier();
        if (L < d) tl_insert(sKey[wv], sPos[wv], TL_SMALL_BITS, b.col[lo + L], L);
        __builtin_amdgcn_wave_barrier();
        tl_range(b, (int32_t)u, lo, sKey[wv], sPos[wv], TL_SMALL_BITS, lo, hi, sPre[wv], sSt[wv], sW[wv]);
    }
}

// chunks of 64 out-neighbours of the queued roots of out-degree
// TL_SMALL+1 .. TL_MID, one wave each; the wave hashes N+(u) first
__global__ __launch_bounds__(BLOCK) void k_tl_mid(TlBuild b) {
    __shared__ int32_t sKey[WAVES_PER_BLOCK][1 << TL_MID_BITS];
    __shared__ int16_t sPos[WAVES_PER_BLOCK][1 << TL_MID_BITS];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    const int wv = threadIdx.x / WAVE, L = lane();
    const int32_t ni = b.nbig[2];
    for (int32_t it = blockIdx.x * WAVES_PER_BLOCK + wv; it < ni; it += gridDim.x * WAVES_PER_BLOCK) {
        const int64_t item = b.mid[it];
        const int32_t u = (int32_t)(item & 0xffffffff);
        const int64_t c = item >> 32;
        const int64_t lo = b.dag_off[u], hi = b.row_ptr[u + 1];
        const int32_t d = (int32_t)(hi - lo);
        int bits = TL_SMALL_BITS;
        while ((1 << bits) < 2 * d) bits++;             // load <= 1/2; d <= TL_MID keeps bits <= TL_MID_BITS
        for (int i = L; i < (1 << bits); i += WAVE) sKey[wv][i] = TL_EMPTY;
        __builtin_amdgcn_wave_barrier();
        for (int32_t j = L; j < d; j += WAVE) tl_insert(sKey[wv], sPos[wv], bits, b.col[lo + j], j);
        __builtin_amdgcn_wave_barrier();
        const int64_t a = lo + c * WAVE;
        tl_range(b, u, lo, sKey[wv], sPos[wv], bits, a, a + WAVE < hi ? a + WAVE : hi, sPre[wv], sSt[wv], sW[wv]);
    }
}

// queued roots (out-degree TL_MID+1 .. TL_MAX_OUT), one workgroup each
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

// segment sizes of reverse arcs: (a, v) for the forward arc (v, a) holds
// r1 + r2 of (v, a); -1 in rev means a broken CSR (never)
__global__ void k_tl_mirror(const int64_t *row_ptr, const int64_t *dag_off, const int64_t *rev, int32_t n, uint32_t *cnt,
                            const uint32_t *top, int32_t *err) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        for (int64_t e = dag_off[v] + lane(); e < row_ptr[v + 1]; e += WAVE) {
            const int64_t f = rev[e];
            if (f < 0) atomicOr(err, 4);
            else cnt[f] = cnt[e] + top[e];
        }
    }
}

// every list must be exactly full
__global__ void k_tl_check(const uint32_t *cur, const uint32_t *woff, int64_t arcs, int32_t *err) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < arcs; e += (int64_t)gridDim.x * blockDim.x)
        if (cur[e] != woff[e + 1]) atomicOr(err, 2);
}

__global__ void k_tl_offsets_tail(uint32_t *woff, const uint32_t *cnt, int64_t arcs) {
    if (blockIdx.x == 0 && threadIdx.x == 0) woff[arcs] = woff[arcs - 1] + cnt[arcs - 1];
}

// clique-degrees from the segment sizes: every triangle at v lies in one of
// v's segments (one wave per vertex)
__global__ void k_tl_degrees(const int64_t *row_ptr, const uint32_t *cnt, int32_t n, u64 *deg) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        u64 sum = 0;
        for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) sum += cnt[e];
        sum = wave_sum(sum);
        if (lane() == 0) deg[v] = sum;
    }
}

// clique-degrees from finished lists: row v holds one pair per triangle at v
__global__ void k_tl_row_degrees(const int64_t *voff, int32_t n, u64 *deg) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = (u64)(voff[v + 1] - voff[v]);
}

// row starts: voff[v] = start of v's first arc segment
__global__ void k_tl_rows(const int64_t *row_ptr, const uint32_t *woff, int32_t n, int64_t *voff) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x)
        voff[v] = (int64_t)woff[row_ptr[v]];
}

}  // namespace

bool tri_list_wanted(const DevGraph &g, u64 mu) {
    const char *e = std::getenv("DSD_TRI_LIST");
    if (e && std::strcmp(e, "0") == 0) return false;
    if (g.n == 0 || mu == 0 || g.maxdout > TL_MAX_OUT) return false;
    if (mu > (u64)0x7fffffff / 3) return false;             // entries are counted in int32 positions
    const int64_t entries = 3 * (int64_t)mu, arcs = 2 * g.m;
    // pairs and row starts, and the listing's segment starts, cursors and reverse arcs
    const int64_t bytes = 8 * entries + 8 * ((int64_t)g.n + 1) + 24 * arcs + 8;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    return bytes <= TL_MAX_BYTES && bytes <= (int64_t)(free_b / 4);
}

bool tri_counts_possible(const DevGraph &g) {
    const char *e = std::getenv("DSD_TRI_LIST");
    if (e && std::strcmp(e, "0") == 0) return false;
    if (g.n == 0 || g.m == 0 || g.maxdout > TL_MAX_OUT) return false;
    // reverse arcs, counts and segment starts: at most 24 B per arc
    const int64_t bytes = 24 * 2 * g.m + 8 * ((int64_t)g.n + 1);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    return bytes <= (int64_t)(free_b / 4);
}

u64 tri_counts(const DevGraph &g, u64 *deg, TlCounts &w, hipStream_t s, Scratch &sc) {
    const int32_t n = g.n;
    const int64_t arcs = 2 * g.m;
    w.rev = sc.get_n<int64_t>(arcs);
    w.cnt = sc.get_n<uint32_t>(arcs);
    w.top = sc.get_n<uint32_t>(arcs);
    w.big = sc.get_n<int32_t>(n);
    w.nbig = sc.get_n<int32_t>(3);
    w.mid = sc.get_n<int64_t>(g.m / 32 + 2);     // sum of ceil(d/64) over roots with d > 64 is below m/32 + 1
    fill_i32(w.nbig, 0, 3, s);
    fill_i32((int32_t *)w.cnt, 0, arcs, s);
    fill_i32((int32_t *)w.top, 0, arcs, s);
    TlBuild b{};
    b.row_ptr = g.row_ptr;
    b.col = g.col;
    b.dag_off = g.dag_off;
    b.rev = w.rev;
    b.cnt = w.cnt;
    b.top = w.top;
    b.big = w.big;
    b.nbig = w.nbig;
    b.mid = w.mid;
    b.err = w.nbig + 1;
    b.n = n;
    k_tl_rev<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, g.dag_off, n, w.rev);
    b.pass = 0;
    k_tl_small<<<grid_for(n, WAVES_PER_BLOCK, 4096), BLOCK, 0, s>>>(b);
    k_tl_mid<<<4096, BLOCK, 0, s>>>(b);
    k_tl_big<<<1024, BLOCK, 0, s>>>(b);
    k_tl_mirror<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.dag_off, w.rev, n, w.cnt, w.top, b.err);
    k_tl_degrees<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, w.cnt, n, deg);
    u64 *sum = sc.get_n<u64>(2);
    sum_u64_128(deg, n, sum, s, sc);
    u64 hs[2];
    int32_t err = 0;
    DSD_HIP(hipMemcpyAsync(hs, sum, sizeof(hs), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&err, b.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (err) throw Error(-3, "triangle lists: a reverse arc is missing");
    if (hs[1] != 0 || hs[0] % 3 != 0) throw Error(-3, "triangle lists: clique-degree sum not a multiple of 3");
    w.mu = hs[0] / 3;
    return w.mu;
}

void build_tri_list(const DevGraph &g, TlCounts &w, TriList &tl, hipStream_t s, Scratch &sc, Scratch *keep) {
    free_tri_list(tl);
    const int32_t n = g.n;
    const int64_t arcs = 2 * g.m;
    tl.mu = w.mu;
    tl.entries = 3 * (int64_t)w.mu;
    if (tl.entries > 0x7fffffff) throw Error(-3, "triangle lists: positions exceed 31 bits");
    if (keep) {
        tl.owned = false;
        tl.voff = keep->get_n<int64_t>((int64_t)n + 1);
        tl.pairs = keep->get_n<int32_t>(2 * tl.entries);
    } else if (hipMalloc(&tl.voff, (size_t)(n + 1) * sizeof(int64_t)) != hipSuccess ||
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
    uint32_t *woff = sc.get_n<uint32_t>(arcs + 1);
    b.entries = tl.entries;
    b.pairs = tl.pairs;
    b.big = w.big;
    b.nbig = w.nbig;
    b.mid = w.mid;
    b.err = w.nbig + 1;
    b.n = n;
    scan_exclusive_u32(w.cnt, woff, arcs, s, sc);
    k_tl_offsets_tail<<<1, 1, 0, s>>>(woff, w.cnt, arcs);
    int32_t err = 0;
    uint32_t total = 0;
    DSD_HIP(hipMemcpyAsync(&err, b.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&total, woff + arcs, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (err || (int64_t)total != tl.entries) {      // every reverse arc found, segments summing to 3 mu
        free_tri_list(tl);
        throw Error(-3, "triangle lists do not match their counts");
    }
    DSD_HIP(hipMemcpyAsync(b.cnt, woff, (size_t)arcs * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    k_tl_rows<<<grid_for((int64_t)n + 1, BLOCK, 4096), BLOCK, 0, s>>>(g.row_ptr, woff, n, tl.voff);
    b.pass = 1;
    k_tl_small<<<grid_for(n, WAVES_PER_BLOCK, 4096), BLOCK, 0, s>>>(b);
    k_tl_mid<<<4096, BLOCK, 0, s>>>(b);
    k_tl_big<<<1024, BLOCK, 0, s>>>(b);
    k_tl_check<<<grid_for(arcs, BLOCK, 4096), BLOCK, 0, s>>>(b.cnt, woff, arcs, b.err);
    DSD_HIP(hipMemcpyAsync(&err, b.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (err) {
        free_tri_list(tl);
        throw Error(-3, "triangle lists do not match their counts");
    }
}

void build_tri_list(const DevGraph &g, const u64 *deg, u64 mu, TriList &tl, hipStream_t s, Scratch &sc,
                    Scratch *keep) {
    (void)deg;
    TlCounts w;
    u64 *d = sc.get_n<u64>(g.n);
    if (tri_counts(g, d, w, s, sc) != mu) throw Error(-3, "triangle lists do not match the clique-degrees");
    build_tri_list(g, w, tl, s, sc, keep);
}

void tri_list_degrees(const TriList &tl, int32_t n, u64 *deg, hipStream_t s) {
    k_tl_row_degrees<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(tl.voff, n, deg);
}

void free_tri_list(TriList &tl) {
    if (tl.owned) {
        (void)hipFree(tl.voff);
        (void)hipFree(tl.pairs);
    }
    tl = TriList();
}

}  // namespace dsd
