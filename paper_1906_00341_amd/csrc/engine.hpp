// Clique-counting engine over candidate sets (device templates).
//
// A work item names a root vertex w of the degree-ordered DAG.  Its
// candidate set C is N+(w) filtered by the item's context (a vertex mask for
// clique-degrees; "inside N(v) and still alive" for the peel).  The engine
// counts the R-cliques of the sub-DAG induced on C and attributes to every
// member x of C the number of those cliques that contain x; the item's
// prefix (w, and v for the peel) receives the total.  With R = h - 1 this is
// the clique-degree of Definition 3 restricted to cliques whose lowest-rank
// member is w; with R = h - 2 and prefix {v, w} it is the set of cliques
// through a removed vertex v that Algorithm 3 must take away.
//
// R = 1: every member of C completes one clique.
// R = 2: edges inside C, found by probing each x's out-list against an LDS
//        hash of C (no bitmap).
// R >= 3: the sub-DAG is stored as a symmetric bitmap S over C (local index
//        = rank order, so "out" = higher index).  Members in prefix positions
//        get their counts from popcounts of intersected rows; the last member
//        y of a clique gets, in one pass, the number of (R-1)-cliques inside
//        its in-neighbourhood Col(y).  No work is done per clique.
//
// Context interface (Ctx):
//   int32_t root(int64_t item)                 -- w
//   bool accept(int64_t item, int32_t x)        -- x in N+(w) kept in C?
//   void add(int32_t x, u64 c)                  -- member x of c cliques
//   void add_prefix(int64_t item, u64 total)    -- the item's prefix, total cliques
#pragma once

#include "common.hpp"

namespace dsd {

constexpr int HASH_EMPTY = -1;

// ---------------------------------------------------------------- bit helpers

template <int W>
__device__ __forceinline__ u64 row_above(const u64 *S, int x, int w) {
    // bits of row x strictly above x (out-neighbours in the sub-DAG)
    u64 v = S[(size_t)x * W + w];
    int xw = x >> 6;
    if (w < xw) return 0;
    if (w == xw) return (x & 63) == 63 ? 0ull : (v & (~0ull << ((x & 63) + 1)));
    return v;
}

template <int W>
__device__ __forceinline__ u64 row_below(const u64 *S, int x, int w) {
    // bits of row x strictly below x (in-neighbours in the sub-DAG)
    u64 v = S[(size_t)x * W + w];
    int xw = x >> 6;
    if (w > xw) return 0;
    if (w == xw) return v & ((1ull << (x & 63)) - 1ull);
    return v;
}

template <int W>
__device__ __forceinline__ u64 popc_w(const u64 (&M)[W]) {
    u64 c = 0;
#pragma unroll
    for (int w = 0; w < W; w++) c += (u64)__popcll(M[w]);
    return c;
}

// number of D-cliques inside the candidate mask M (rank order, each once)
template <int D, int W>
__device__ u64 count_in(const u64 (&M)[W], const u64 *S) {
    if constexpr (D == 1) {
        return popc_w<W>(M);
    } else {
        u64 tot = 0;
#pragma unroll 1
        for (int w = 0; w < W; w++) {
            u64 word = M[w];
            while (word) {
                int x = w * 64 + __builtin_ctzll(word);
                word &= word - 1;
                u64 M2[W];
                bool any = false;
#pragma unroll
                for (int q = 0; q < W; q++) {
                    M2[q] = M[q] & row_above<W>(S, x, q);
                    any |= M2[q] != 0;
                }
                if (any) tot += count_in<D - 1, W>(M2, S);
            }
        }
        return tot;
    }
}

// Prefix enumeration: choose D more members from M; at D == 0 the number of
// completions is popc(M).  Every chosen member gets the completions through
// it (cnt is an LDS array of u64 counters).  Returns the total.
template <int D, int W>
__device__ u64 forward(const u64 (&M)[W], const u64 *S, u64 *cnt) {
    if constexpr (D == 0) {
        return popc_w<W>(M);
    } else {
        u64 tot = 0;
#pragma unroll 1
        for (int w = 0; w < W; w++) {
            u64 word = M[w];
            while (word) {
                int x = w * 64 + __builtin_ctzll(word);
                word &= word - 1;
                u64 M2[W];
                bool any = false;
#pragma unroll
                for (int q = 0; q < W; q++) {
                    M2[q] = M[q] & row_above<W>(S, x, q);
                    any |= M2[q] != 0;
                }
                if (!any) continue;
                u64 c = forward<D - 1, W>(M2, S, cnt);
                if (c) {
                    atomicAdd(&cnt[x], c);
                    tot += c;
                }
            }
        }
        return tot;
    }
}

// Per-member R-clique counts for the sub-DAG over d nodes stored in S
// (symmetric rows of W words).  Work item for one thread: node x.  Adds to
// cnt[] (LDS), returns the number of cliques whose first member is x.
template <int R, int W>
__device__ u64 bitmap_node_work(int x, const u64 *S, u64 *cnt) {
    u64 M[W];
    // x as first member
#pragma unroll
    for (int q = 0; q < W; q++) M[q] = row_above<W>(S, x, q);
    u64 c = forward<R - 2, W>(M, S, cnt);
    u64 tot = c;
    // x as last member: (R-1)-cliques inside its in-neighbourhood
#pragma unroll
    for (int q = 0; q < W; q++) M[q] = row_below<W>(S, x, q);
    c += count_in<R - 1, W>(M, S);
    if (c) atomicAdd(&cnt[x], c);
    return tot;
}

// ---------------------------------------------------------------- LDS hash

__device__ __forceinline__ void hash_insert(int32_t *keys, int32_t *vals, int bits, int32_t x, int32_t v) {
    uint32_t m = (1u << bits) - 1u, slot = hash_slot(x, bits);
    while (true) {
        int32_t prev = atomicCAS(&keys[slot], HASH_EMPTY, x);
        if (prev == HASH_EMPTY || prev == x) {
            vals[slot] = v;
            return;
        }
        slot = (slot + 1) & m;
    }
}

__device__ __forceinline__ int32_t hash_find(const int32_t *keys, const int32_t *vals, int bits, int32_t x) {
    uint32_t m = (1u << bits) - 1u, slot = hash_slot(x, bits);
    while (true) {
        int32_t k = keys[slot];
        if (k == x) return vals[slot];
        if (k == HASH_EMPTY) return -1;
        slot = (slot + 1) & m;
    }
}

// ---------------------------------------------------------------- block helpers

// In-place inclusive scan of a[0, n) (n <= BLOCK * per) in LDS; returns total.
__device__ __forceinline__ int32_t block_incl_scan_lds(int32_t *a, int n, int32_t *wtmp) {
    int per = (n + BLOCK - 1) / BLOCK;
    int lo = threadIdx.x * per, hi = min(n, lo + per);
    int32_t s = 0;
    for (int i = lo; i < hi; i++) s += a[i];
    int32_t inc = wave_incl_scan(s);
    int w = threadIdx.x / WAVE;
    if (lane() == WAVE - 1) wtmp[w] = inc;
    __syncthreads();
    int32_t off = inc - s;
    for (int i = 0; i < w; i++) off += wtmp[i];
    int32_t total = 0;
    for (int i = 0; i < WAVES_PER_BLOCK; i++) total += wtmp[i];
    for (int i = lo; i < hi; i++) {
        off += a[i];
        a[i] = off;
    }
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------- item kernels

// Load the candidate set of an item into out[] in rank order (order-preserving
// block compaction).  Returns |C|.  d <= cap.
template <class Ctx>
__device__ int block_load_candidates(const Ctx &ctx, int64_t item, const int32_t *col, int64_t s0, int d,
                                     int32_t *out, int32_t *wtmp) {
    int per = (d + BLOCK - 1) / BLOCK;
    int lo = threadIdx.x * per, hi = min(d, lo + per);
    int32_t keep = 0;
    for (int i = lo; i < hi; i++) keep += ctx.accept(item, col[s0 + i]) ? 1 : 0;
    int32_t inc = wave_incl_scan(keep);
    int w = threadIdx.x / WAVE;
    if (lane() == WAVE - 1) wtmp[w] = inc;
    __syncthreads();
    int32_t off = inc - keep;
    for (int i = 0; i < w; i++) off += wtmp[i];
    int32_t total = 0;
    for (int i = 0; i < WAVES_PER_BLOCK; i++) total += wtmp[i];
    for (int i = lo; i < hi; i++) {
        int32_t x = col[s0 + i];
        if (ctx.accept(item, x)) out[off++] = x;
    }
    __syncthreads();
    return total;
}

// ---- wave engine: one wave per item, d <= 64 ---------------------------------
// R = 2 uses the hash; R >= 3 the one-word bitmap.
template <int R, class Ctx>
__global__ __launch_bounds__(BLOCK) void k_engine_wave(Ctx ctx, const int64_t *row_ptr, const int32_t *col,
                                                       const int64_t *dag_off, int64_t nitems,
                                                       const int32_t *nitems_dev) {
    if (nitems_dev) nitems = *nitems_dev;
    __shared__ int32_t sC[WAVES_PER_BLOCK][64];
    __shared__ int32_t sKey[WAVES_PER_BLOCK][128];
    __shared__ int32_t sVal[WAVES_PER_BLOCK][128];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][64];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][64];
    __shared__ u64 sCnt[WAVES_PER_BLOCK][64];
    __shared__ u64 sS[WAVES_PER_BLOCK][64];
    const int wv = threadIdx.x / WAVE, L = lane();
    for (int i = L; i < 128; i += WAVE) sKey[wv][i] = HASH_EMPTY;
    sCnt[wv][L] = 0;
    sS[wv][L] = 0;
    __builtin_amdgcn_wave_barrier();
    const int64_t stride = (int64_t)gridDim.x * WAVES_PER_BLOCK;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nitems; it += stride) {
        const int32_t w = ctx.root(it);
        const int64_t s0 = dag_off[w];
        const int d = (int)(row_ptr[w + 1] - s0);
        int32_t x = -1;
        bool keep = false;
        if (L < d) {
            x = col[s0 + L];
            keep = ctx.accept(it, x);
        }
        const u64 km = __ballot(keep);
        const int dd = __popcll(km);
        if (dd < R) continue;                                   // wave-uniform
        const int li = __popcll(km & lanemask_lt());            // rank order kept
        if (keep) {
            sC[wv][li] = x;
            hash_insert(sKey[wv], sVal[wv], 7, x, li);
        }
        __builtin_amdgcn_wave_barrier();
        u64 total = 0;
        if constexpr (R == 1) {
            if (keep) ctx.add(x, 1);
            total = (u64)dd;
        } else {
            // flattened (i, offset) pairs over the out-lists of C
            int32_t len = 0;
            int64_t st = 0;
            if (keep) {
                st = dag_off[x];
                len = (int32_t)(row_ptr[x + 1] - st);
            }
            int32_t inc = wave_incl_scan(keep ? len : 0);
            if (keep) {
                sPre[wv][li] = inc;
                sSt[wv][li] = st;
            }
            const int32_t tot_pairs = __shfl(inc, WAVE - 1, WAVE);
            __builtin_amdgcn_wave_barrier();
            u64 hits = 0;
            for (int32_t base = 0; base < tot_pairs; base += WAVE) {
                int32_t p = base + L;
                bool hit = false;
                int i = 0, j = -1;
                if (p < tot_pairs) {
                    i = upper_bound_i32(sPre[wv], dd, p);
                    int32_t off = p - (i ? sPre[wv][i - 1] : 0);
                    int32_t y = col[sSt[wv][i] + off];
                    j = hash_find(sKey[wv], sVal[wv], 7, y);
                    hit = j >= 0;
                }
                if constexpr (R == 2) {
                    if (hit) {
                        atomicAdd(&sCnt[wv][i], 1ull);
                        atomicAdd(&sCnt[wv][j], 1ull);
                    }
                    hits += (u64)__popcll(__ballot(hit));
                } else {
                    if (hit) {
                        atomicOr(&sS[wv][i], 1ull << j);
                        atomicOr(&sS[wv][j], 1ull << i);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            if constexpr (R == 2) {
                total = hits;
            } else {
                u64 t = 0;
                if (L < dd) t = bitmap_node_work<R, 1>(L, &sS[wv][0], &sCnt[wv][0]);
                total = wave_sum(t);
            }
            __builtin_amdgcn_wave_barrier();
            if (L < dd) {
                u64 c = sCnt[wv][L];
                if (c) ctx.add(sC[wv][L], c);
            }
        }
        if (L == 0 && total) ctx.add_prefix(it, total);
        __builtin_amdgcn_wave_barrier();
        // reset the wave's LDS for the next item
        for (int i = L; i < 128; i += WAVE) sKey[wv][i] = HASH_EMPTY;
        sCnt[wv][L] = 0;
        sS[wv][L] = 0;
        __builtin_amdgcn_wave_barrier();
    }
}

// ---- block engine: one block per item -------------------------------------
// CAP: max |N+(w)|; HB: hash bits (2^HB >= 2*CAP); W: bitmap words (R >= 3);
// GLOBAL_S: the bitmap lives in a per-block slice of global scratch.
template <int R, int CAP, int HB, int W, bool GLOBAL_S, class Ctx>
__global__ __launch_bounds__(BLOCK) void k_engine_block(Ctx ctx, const int64_t *row_ptr, const int32_t *col,
                                                        const int64_t *dag_off, int64_t nitems,
                                                        const int32_t *nitems_dev, u64 *gS) {
    if (nitems_dev) nitems = *nitems_dev;
    __shared__ int32_t sC[CAP];
    __shared__ int32_t sKey[1 << HB];
    __shared__ int32_t sVal[1 << HB];
    __shared__ int32_t sPre[CAP];
    __shared__ u64 sCnt[CAP];
    __shared__ int32_t wtmp[WAVES_PER_BLOCK];
    __shared__ u64 sTot[WAVES_PER_BLOCK];
    constexpr int SW = (R >= 3 && !GLOBAL_S) ? CAP * W : 1;
    __shared__ u64 sSl[SW];
    u64 *S = GLOBAL_S ? gS + (size_t)blockIdx.x * CAP * W : sSl;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int32_t w = ctx.root(it);
        const int64_t s0 = dag_off[w];
        const int d = (int)(row_ptr[w + 1] - s0);
        for (int i = threadIdx.x; i < (1 << HB); i += BLOCK) sKey[i] = HASH_EMPTY;
        const int dd = block_load_candidates(ctx, it, col, s0, d, sC, wtmp);
        if (dd < R) continue;                                  // block-uniform
        for (int i = threadIdx.x; i < dd; i += BLOCK) {
            hash_insert(sKey, sVal, HB, sC[i], i);
            sCnt[i] = 0;
            int32_t x = sC[i];
            sPre[i] = (int32_t)(row_ptr[x + 1] - dag_off[x]);
        }
        if constexpr (R >= 3) {
            for (int i = threadIdx.x; i < dd * W; i += BLOCK) S[i] = 0;
        }
        __syncthreads();
        u64 total = 0;
        if constexpr (R == 1) {
            for (int i = threadIdx.x; i < dd; i += BLOCK) ctx.add(sC[i], 1);
            total = (u64)dd;
        } else {
            const int32_t tot_pairs = block_incl_scan_lds(sPre, dd, wtmp);
            u64 hits = 0;
            for (int32_t base = 0; base < tot_pairs; base += BLOCK) {
                int32_t p = base + threadIdx.x;
                if (p < tot_pairs) {
                    int i = upper_bound_i32(sPre, dd, p);
                    int32_t off = p - (i ? sPre[i - 1] : 0);
                    int32_t x = sC[i];
                    int32_t y = col[dag_off[x] + off];
                    int j = hash_find(sKey, sVal, HB, y);
                    if (j >= 0) {
                        if constexpr (R == 2) {
                            atomicAdd(&sCnt[i], 1ull);
                            atomicAdd(&sCnt[j], 1ull);
                            hits++;
                        } else {
                            atomicOr(&S[(size_t)i * W + (j >> 6)], 1ull << (j & 63));
                            atomicOr(&S[(size_t)j * W + (i >> 6)], 1ull << (i & 63));
                        }
                    }
                }
            }
            if constexpr (R >= 3) {
                if (GLOBAL_S) __threadfence_block();
                __syncthreads();
                for (int x = threadIdx.x; x < dd; x += BLOCK) hits += bitmap_node_work<R, W>(x, S, sCnt);
            }
            hits = wave_sum(hits);
            if (lane() == 0) sTot[threadIdx.x / WAVE] = hits;
            __syncthreads();
            for (int i = 0; i < WAVES_PER_BLOCK; i++) total += sTot[i];
            for (int i = threadIdx.x; i < dd; i += BLOCK) {
                u64 c = sCnt[i];
                if (c) ctx.add(sC[i], c);
            }
        }
        if (threadIdx.x == 0 && total) ctx.add_prefix(it, total);
        __syncthreads();
    }
}

// ---- huge engine for R == 2 (any |N+(w)|): global binary searches ----------
template <class Ctx>
__global__ __launch_bounds__(BLOCK) void k_engine_huge_r2(Ctx ctx, const int64_t *row_ptr, const int32_t *col,
                                                          const int64_t *dag_off, int64_t nitems,
                                                          const int32_t *nitems_dev) {
    if (nitems_dev) nitems = *nitems_dev;
    __shared__ u64 sTot[WAVES_PER_BLOCK];
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int32_t w = ctx.root(it);
        const int64_t s0 = dag_off[w], e0 = row_ptr[w + 1];
        const int64_t d = e0 - s0;
        u64 tot = 0;
        for (int64_t i = threadIdx.x; i < d; i += BLOCK) {
            int32_t x = col[s0 + i];
            if (!ctx.accept(it, x)) continue;
            u64 cx = 0;
            for (int64_t e = dag_off[x]; e < row_ptr[x + 1]; e++) {
                int32_t y = col[e];
                if (!ctx.accept(it, y)) continue;
                if (bsearch_i32(col, s0, e0, y) >= 0) {
                    ctx.add(y, 1);
                    cx++;
                }
            }
            if (cx) ctx.add(x, cx);
            tot += cx;
        }
        tot = wave_sum(tot);
        if (lane() == 0) sTot[threadIdx.x / WAVE] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 t = 0;
            for (int i = 0; i < WAVES_PER_BLOCK; i++) t += sTot[i];
            if (t) ctx.add_prefix(it, t);
        }
        __syncthreads();
    }
}

}  // namespace dsd
