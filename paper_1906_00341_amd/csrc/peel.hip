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
// State lives on the device (PeelCtl).  One round is a fixed sequence of
// grid-wide kernels (level-min, level-build, process, finish) that read the
// state themselves, so the host enqueues many rounds without waiting.  For
// h = 3 a large frontier vertex is split into items of CHUNK neighbours plus
// one item per neighbour with a long out-list, so that even a round that
// removes a single hub keeps thousands of waves busy; its neighbourhood hash
// sits in global memory, shared by those items.  An optional single-workgroup
// tail (DSD_TAIL_T) runs the last rounds in one launch instead.
#include "engine.hpp"
#include "graph.hpp"

namespace dsd {

struct PeelCtl {
    u64 k;          // current level
    u64 kcand;      // smallest alive degree (next level)
    u64 mu_alive;   // cliques among alive vertices
    u64 destroyed;  // cliques destroyed in this round
    int64_t n_alive;
    int64_t tail_T;    // the single-workgroup tail takes over at or below this many alive vertices
    int32_t round;
    int32_t cur;       // frontier buffer in use
    int32_t nF[2];     // frontier sizes
    int32_t nB[2];     // chunk items of large frontier vertices (h = 3)
    int32_t nlist[2];  // alive-list sizes
    int32_t lcur;      // alive list in use
    int32_t nlevels;
    uint32_t done;     // finished blocks (last-block finalisation)
    int32_t selecting; // set by level-min: this round starts a new level
    int32_t nitems[8]; // (v, w) work items per class (h >= 4)
    int64_t htop[2];   // slots handed out in the global neighbourhood hashes (h = 3)
    int64_t nW;        // wide (v, w) items of this round (h = 3)
};

struct PeelBufs {
    PeelCtl *ctl;
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
    u64 *lv_k, *lv_size, *lv_mu;  // level table [n + 1]
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
};

constexpr int SMALL_DEG = 64;           // h = 3: larger frontier vertices are split into chunks
constexpr int CHUNK = 32;               // neighbours per chunk item (one wave)
constexpr int SLOTS_PER_CHUNK = 64;     // global hash slots per chunk (load factor <= 1/2)
constexpr int WIDE_OUT = 32;            // neighbours w with |N+(w)| >= this get a wave of their own
constexpr int BIG_HASH_BITS = 14;       // single-workgroup tail: 16384 slots = 64 KB of LDS
constexpr int BIG_HASH_CAP = 8192;      // larger neighbourhoods use binary search
constexpr int SMALL_HASH_BITS = 7;      // per-wave hash for degree <= SMALL_DEG

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

// the last block to arrive returns true (block-uniform)
__device__ __forceinline__ bool last_block(uint32_t *done) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = atomicAdd(done, 1u) == gridDim.x - 1;
    __syncthreads();
    return is_last;
}

// chunk items of a large frontier vertex, and the slots of its neighbourhood
// hash (h = 3)
__device__ __forceinline__ void push_chunks(const PeelBufs &b, int32_t x, int which) {
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

__device__ __forceinline__ void dec_deg(const PeelBufs &b, int32_t x, u64 c, u64 k, int32_t r) {
    u64 old = atomic_sub_u64(&b.deg[x], c);
    if (old > k && old - c <= k) {
        const int nx = b.ctl->cur ^ 1;
        int32_t *Fn = b.F + (size_t)nx * b.n;
        int32_t pos = atomicAdd(&b.ctl->nF[nx], 1);
        Fn[pos] = x;
        b.stamp[x] = r + 1;
        b.core[x] = k;
        push_chunks(b, x, nx);
    }
}

// a clique through frontier vertex v may use x iff x was alive at the start
// of the round and is not a frontier vertex of smaller rank (owner rule)
__device__ __forceinline__ bool allowed(int32_t st, int32_t r, int32_t x, int32_t v) {
    return st > r || (st == r && x > v);
}

// ---------------------------------------------------------------- level selection

__device__ __forceinline__ bool grid_rounds_on(const PeelCtl *c) { return c->n_alive > c->tail_T; }

// the level of the current round: a round that opens a level records it only
// when it finishes, so until then the level is max(k, smallest alive degree)
__device__ __forceinline__ u64 round_level(const PeelCtl *c) {
    return c->selecting ? (c->k > c->kcand ? c->k : c->kcand) : c->k;
}

// the alive list is copied (compacted) by level-build once more than an
// eighth of it are removed vertices; n_alive and the list length do not
// change between level-build and the end of the round, so every reader of
// this test agrees
__device__ __forceinline__ bool list_compacts(const PeelCtl *c) {
    const int32_t cnt = c->nlist[c->lcur];
    return (int64_t)(cnt - c->n_alive) * 8 > (int64_t)cnt;
}

__global__ __launch_bounds__(BLOCK) void k_level_min(PeelBufs b) {
    PeelCtl *c = b.ctl;
    // nF and n_alive do not change during this kernel, so every block takes
    // the same decision; level-build reads the flag because it grows nF itself
    const bool sel = c->nF[c->cur] == 0 && c->n_alive > 0 && grid_rounds_on(c);
    if (blockIdx.x == 0 && threadIdx.x == 0) c->selecting = sel ? 1 : 0;
    if (!sel) return;
    const int32_t *list = b.lists + (size_t)c->lcur * b.n;
    const int32_t cnt = c->nlist[c->lcur];
    u64 m = ~0ull;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * BLOCK) {
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
        if (m != ~0ull) atomicMin(&c->kcand, m);
    }
}

// compacted: the survivors were copied to the other alive list
__device__ __forceinline__ void record_level(const PeelBufs &b, PeelCtl *c, u64 k, bool compacted) {
    int32_t L = c->nlevels;
    b.lv_k[L] = k;
    b.lv_size[L] = (u64)c->n_alive;
    b.lv_mu[L] = c->mu_alive;
    c->nlevels = L + 1;
    c->k = k;
    c->kcand = ~0ull;
    if (compacted) {
        c->nlist[c->lcur] = 0;
        c->lcur ^= 1;
    }
}

__global__ __launch_bounds__(BLOCK) void k_level_build(PeelBufs b) {
    PeelCtl *c = b.ctl;
    if (!c->selecting) return;
    const u64 k = round_level(c);
    const int32_t r = c->round, lc = c->lcur, cur = c->cur;
    const int32_t *in = b.lists + (size_t)lc * b.n;
    int32_t *out = b.lists + (size_t)(lc ^ 1) * b.n;
    int32_t *F = b.F + (size_t)cur * b.n;
    const int32_t cnt = c->nlist[lc];
    const bool compact = list_compacts(c);
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = blockIdx.x * (int64_t)BLOCK; base < cnt; base += stride) {
        const int64_t i = base + threadIdx.x;
        int32_t v = -1;
        bool alive = false, take = false;
        if (i < cnt) {
            v = in[i];
            alive = b.stamp[v] == ALIVE;
            take = alive && b.deg[v] <= k;
        }
        if (take) {
            b.stamp[v] = r;
            b.core[v] = k;
            push_chunks(b, v, cur);
        }
        wave_push(take, v, F, &c->nF[cur]);
        if (compact) block_push(alive && !take, v, out, &c->nlist[lc ^ 1]);
    }
}

// end of a round: the frontier is gone
__device__ __forceinline__ void finish_round(PeelCtl *c) {
    int32_t cur = c->cur;
    c->n_alive -= c->nF[cur];
    c->mu_alive -= c->destroyed;
    c->destroyed = 0;
    c->nF[cur] = 0;
    c->nB[cur] = 0;
    c->htop[cur] = 0;
    c->nW = 0;
    c->cur = cur ^ 1;
    c->round += 1;
    c->done = 0;
    for (int i = 0; i < 8; i++) c->nitems[i] = 0;
}

// ---------------------------------------------------------------- h = 2

__global__ __launch_bounds__(BLOCK) void k_process_h2(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0 || !grid_rounds_on(c)) return;
    const int32_t r = c->round;
    const u64 k = round_level(c);
    const int32_t *F = b.F + (size_t)cur * b.n;
    u64 destroyed = 0;
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nF; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[i];
        for (int64_t e = b.row_ptr[v] + lane(); e < b.row_ptr[v + 1]; e += WAVE) {
            int32_t w = b.col[e];
            int32_t st = b.stamp[w];
            if (st == r) {
                destroyed += (v < w) ? 1 : 0;       // both ends leave: count the edge once
            } else if (st > r) {
                destroyed += 1;
                dec_deg(b, w, 1, k, r);
            }
        }
    }
    destroyed = wave_sum(destroyed);
    if (lane() == 0 && destroyed) atomicAdd(&c->destroyed, destroyed);
}

// ---------------------------------------------------------------- h = 3

// LDS hash over the allowed neighbourhood of frontier vertex v.  The value of
// a slot counts the cliques through v found so far that contain that
// neighbour; the counts go to global memory once per neighbour (flush), so
// the pair loop itself never waits on a global atomic.
// size: any number of slots >= 2 (a power of two in LDS; chunk-sized in
// global memory); at most half of them are ever filled
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

__device__ __forceinline__ int hash_bits_for(int64_t d) {
    int bits = 7;
    while (bits < BIG_HASH_BITS && ((int64_t)1 << bits) < 2 * d) bits++;
    return bits;
}

// insert the allowed neighbours N(v)[rv0, rv1) (threads t, t + step, ...)
__device__ __forceinline__ void hash_fill(const PeelBufs &b, const NbHash &hs, int32_t v, int64_t rv0, int64_t rv1,
                                          int32_t r, int t, int step) {
    for (int64_t e = rv0 + t; e < rv1; e += step) {
        int32_t x = b.col[e];
        if (allowed(b.stamp[x], r, x, v)) hs.put(x);
    }
}

// apply the pending counts of slots t, t + step, ... and empty them
__device__ __forceinline__ void hash_flush(const PeelBufs &b, const NbHash &hs, int32_t r, u64 k, int t, int step) {
    for (uint32_t i = t; i < hs.size; i += step) {
        int32_t key = hs.keys[i];
        if (key == HASH_EMPTY) continue;
        uint32_t c = hs.vals[i];
        if (c && b.stamp[key] > r) dec_deg(b, key, c, k, r);
        hs.keys[i] = HASH_EMPTY;
        hs.vals[i] = 0;
    }
}

// One wave handles the neighbours N(v)[lo, hi) of frontier vertex v: for each
// allowed neighbour w it probes N+(w) against the allowed neighbourhood of v,
// so every triangle {v, w, x} with w before x is seen once.  HASHED: counts
// go to the hash values; otherwise membership is a binary search in the
// sorted row N(v)[rv0, rv1) and survivors are decremented at once.
// sPre/sSt/sW/sCnt: this wave's 64-entry LDS scratch.
// Neighbours w whose out-list holds wide_out or more entries are skipped (a
// wide item of their own covers them).
template <bool HASHED>
__device__ __forceinline__ u64 h3_wave_range(const PeelBufs &b, int32_t v, int64_t lo, int64_t hi, int64_t rv0,
                                            int64_t rv1, int32_t r, u64 k, const NbHash &hs, int32_t *sPre,
                                            int64_t *sSt, int32_t *sW, uint32_t *sCnt,
                                            int32_t wide_out = 0x7fffffff) {
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
                if (HASHED) wslot = hs.find(w);
            }
        }
        int32_t inc = wave_incl_scan(len);
        sPre[L] = inc;
        sSt[L] = st0;
        sW[L] = HASHED ? wslot : w;
        sCnt[L] = 0;
        const int32_t total = __shfl(inc, WAVE - 1, WAVE);
        __builtin_amdgcn_wave_barrier();
        for (int32_t pb = 0; pb < total; pb += WAVE) {
            int32_t p = pb + L;
            if (p < total) {
                int i = upper_bound_i32(sPre, WAVE, p);
                int32_t off = p - (i ? sPre[i - 1] : 0);
                int32_t x = b.col[sSt[i] + off];
                if (HASHED) {
                    int slot = hs.find(x);
                    if (slot >= 0) {                      // triangle {v, w, x}, owned by v
                        destroyed++;
                        atomicAdd(&sCnt[i], 1u);
                        atomicAdd(&hs.vals[slot], 1u);
                    }
                } else if (allowed(b.stamp[x], r, x, v) && bsearch_i32(b.col, rv0, rv1, x) >= 0) {
                    destroyed++;
                    atomicAdd(&sCnt[i], 1u);
                    if (b.stamp[x] > r) dec_deg(b, x, 1, k, r);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t cw = sCnt[L];
        if (cw) {
            if (HASHED) atomicAdd(&hs.vals[sW[L]], cw);
            else if (b.stamp[sW[L]] > r) dec_deg(b, sW[L], cw, k, r);
        }
        __builtin_amdgcn_wave_barrier();
    }
    return destroyed;
}

// small frontier vertices (degree <= SMALL_DEG): one wave each, per-wave hash
__global__ __launch_bounds__(BLOCK) void k_process_h3_small(PeelBufs b) {
    __shared__ int32_t sKey[WAVES_PER_BLOCK][1 << SMALL_HASH_BITS];
    __shared__ uint32_t sVal[WAVES_PER_BLOCK][1 << SMALL_HASH_BITS];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    __shared__ uint32_t sCnt[WAVES_PER_BLOCK][WAVE];
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0 || !grid_rounds_on(c)) return;
    const int32_t r = c->round;
    const u64 k = round_level(c);
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE, L = lane();
    const NbHash hs{sKey[wv], sVal[wv], 1u << SMALL_HASH_BITS};
    u64 destroyed = 0;
    for (int i = L; i < (1 << SMALL_HASH_BITS); i += WAVE) {
        hs.keys[i] = HASH_EMPTY;
        hs.vals[i] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    for (int64_t fi = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; fi < nF; fi += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[fi];
        const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
        if (rv1 - rv0 > SMALL_DEG) continue;                     // chunk items cover it
        hash_fill(b, hs, v, rv0, rv1, r, L, WAVE);
        __builtin_amdgcn_wave_barrier();
        destroyed += h3_wave_range<true>(b, v, rv0, rv1, rv0, rv1, r, k, hs, sPre[wv], sSt[wv], sW[wv], sCnt[wv]);
        __builtin_amdgcn_wave_barrier();
        hash_flush(b, hs, r, k, L, WAVE);
        __builtin_amdgcn_wave_barrier();
    }
    destroyed = wave_sum(destroyed);
    if (L == 0 && destroyed) atomicAdd(&c->destroyed, destroyed);
}

// All waves of a workgroup handle the neighbours N(v)[lo, hi) of v (64 at a
// time, round-robin); the hash covers all of N(v).  Used by the grid kernel
// for chunk items and by the tail for whole frontier vertices.
template <int NW>
__device__ __forceinline__ u64 h3_block_range(const PeelBufs &b, int32_t v, int64_t lo, int64_t hi, int32_t r, u64 k,
                                             int32_t *keys, uint32_t *vals, int32_t (*sPre)[WAVE],
                                             int64_t (*sSt)[WAVE], int32_t (*sW)[WAVE], uint32_t (*sCnt)[WAVE]) {
    const int wv = threadIdx.x / WAVE;
    const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
    const bool hashed = rv1 - rv0 <= BIG_HASH_CAP;
    const NbHash hs{keys, vals, 1u << hash_bits_for(rv1 - rv0)};
    u64 destroyed = 0;
    if (hashed) hash_fill(b, hs, v, rv0, rv1, r, threadIdx.x, NW * WAVE);
    __syncthreads();
    for (int64_t plo = lo + (int64_t)wv * WAVE; plo < hi; plo += (int64_t)NW * WAVE) {
        const int64_t phi = min(hi, plo + WAVE);
        if (hashed)
            destroyed += h3_wave_range<true>(b, v, plo, phi, rv0, rv1, r, k, hs, sPre[wv], sSt[wv], sW[wv], sCnt[wv]);
        else
            destroyed += h3_wave_range<false>(b, v, plo, phi, rv0, rv1, r, k, hs, sPre[wv], sSt[wv], sW[wv], sCnt[wv]);
    }
    __syncthreads();
    if (hashed) hash_flush(b, hs, r, k, threadIdx.x, NW * WAVE);
    __syncthreads();
    return destroyed;
}

// Larger frontier vertices (degree > SMALL_DEG) are cut into chunks of CHUNK
// neighbours, one wave each, so that the pairs of a hub spread over the whole
// chip.  Their neighbourhood hashes live in global memory (SLOTS_PER_CHUNK
// slots per chunk): fill inserts the allowed neighbours, probe counts the
// triangles, flush hands each neighbour's count to dec_deg once and empties
// the slots for later rounds.

__device__ __forceinline__ NbHash big_hash(const PeelBufs &b, int32_t cur, int32_t v, int64_t d) {
    const int64_t nc = (d + CHUNK - 1) / CHUNK;
    const size_t off = (size_t)cur * b.hcap + b.hbase[v];
    return NbHash{b.hkey + off, b.hval + off, (uint32_t)(nc * SLOTS_PER_CHUNK)};
}

__global__ __launch_bounds__(BLOCK) void k_h3_fill(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0 || !grid_rounds_on(c)) return;
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

__global__ __launch_bounds__(BLOCK) void k_h3_probe(PeelBufs b) {
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    __shared__ uint32_t sCnt[WAVES_PER_BLOCK][WAVE];
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0 || !grid_rounds_on(c)) return;
    const int32_t r = c->round, nB = c->nB[cur];
    const int64_t nW = c->nW;
    const u64 k = round_level(c);
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const int wv = threadIdx.x / WAVE;
    u64 destroyed = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nB + nW; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        if (it < nB) {
            // chunk item: the neighbours with short out-lists, their pairs flattened over the wave
            const int64_t item = Bc[it];
            const int32_t v = (int32_t)(item >> 32), ch = (int32_t)(item & 0xffffffff);
            const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
            const int64_t lo = rv0 + (int64_t)ch * CHUNK, hi = min(rv1, lo + CHUNK);
            const NbHash hs = big_hash(b, cur, v, rv1 - rv0);
            destroyed += h3_wave_range<true>(b, v, lo, hi, rv0, rv1, r, k, hs, sPre[wv], sSt[wv], sW[wv], sCnt[wv],
                                             WIDE_OUT);
        } else {
            // wide item (v, w): the lanes walk N+(w)
            const int64_t item = b.W[it - nB];
            const int32_t v = (int32_t)(item >> 32), w = (int32_t)(item & 0xffffffff);
            const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
            const NbHash hs = big_hash(b, cur, v, rv1 - rv0);
            uint32_t cw = 0;
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
            destroyed += lane() == 0 ? cw : 0;
        }
    }
    destroyed = wave_sum(destroyed);
    if (lane() == 0 && destroyed) atomicAdd(&c->destroyed, destroyed);
}

__global__ __launch_bounds__(BLOCK) void k_h3_flush(PeelBufs b) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur;
    if (c->nF[cur] == 0 || !grid_rounds_on(c)) return;
    const int32_t r = c->round, nB = c->nB[cur];
    const u64 k = round_level(c);
    const int64_t *Bc = b.B + (size_t)cur * b.bcap;
    const int wv = threadIdx.x / WAVE;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; it < nB; it += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int64_t item = Bc[it];
        const int32_t v = (int32_t)(item >> 32), ch = (int32_t)(item & 0xffffffff);
        const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
        const NbHash hs = big_hash(b, cur, v, rv1 - rv0);
        const uint32_t s0 = (uint32_t)ch * SLOTS_PER_CHUNK;
        for (uint32_t i = s0 + lane(); i < s0 + SLOTS_PER_CHUNK && i < hs.size; i += WAVE) {
            const int32_t key = hs.keys[i];
            if (key == HASH_EMPTY) continue;
            const uint32_t cnt = hs.vals[i];
            if (cnt && b.stamp[key] > r) dec_deg(b, key, cnt, k, r);
            hs.keys[i] = HASH_EMPTY;
            hs.vals[i] = 0;
        }
    }
}

// ---------------------------------------------------------------- tail: one workgroup

constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_WAVES = TAIL_THREADS / WAVE;

// Runs every remaining round inside one workgroup: level selection, frontier
// build and clique destruction are separated by workgroup barriers.  Each
// frontier vertex is handled by the whole workgroup in turn.
template <int H>
__global__ __launch_bounds__(TAIL_THREADS) void k_peel_tail(PeelBufs b) {
    __shared__ int32_t sKey[1 << BIG_HASH_BITS];
    __shared__ uint32_t sVal[1 << BIG_HASH_BITS];
    __shared__ int32_t sPre[TAIL_WAVES][WAVE];
    __shared__ int64_t sSt[TAIL_WAVES][WAVE];
    __shared__ int32_t sW[TAIL_WAVES][WAVE];
    __shared__ uint32_t sCnt[TAIL_WAVES][WAVE];
    __shared__ u64 sRed[TAIL_WAVES];
    __shared__ u64 sK;
    __shared__ int64_t sAlive;
    __shared__ int32_t sCur, sNF;
    PeelCtl *c = b.ctl;
    const int wv = threadIdx.x / WAVE, L = lane();
    for (int i = threadIdx.x; i < (1 << BIG_HASH_BITS); i += TAIL_THREADS) {
        sKey[i] = HASH_EMPTY;
        sVal[i] = 0;
    }
    while (true) {
        // one thread reads the control state, so every wave takes the same path
        // (other waves' pushes would otherwise be visible to some reads only)
        __syncthreads();
        if (threadIdx.x == 0) {
            sAlive = c->n_alive;
            sCur = c->cur;
            sNF = c->nF[c->cur];
        }
        __syncthreads();
        if (sAlive == 0) break;
        const int32_t cur = sCur;
        if (sNF == 0) {
            // new level: k = max(k, smallest alive degree)
            const int32_t lc = c->lcur, cnt = c->nlist[lc];
            const int32_t *in = b.lists + (size_t)lc * b.n;
            u64 m = ~0ull;
            for (int32_t i = threadIdx.x; i < cnt; i += TAIL_THREADS) {
                int32_t v = in[i];
                if (b.stamp[v] == ALIVE) m = b.deg[v] < m ? b.deg[v] : m;
            }
            m = wave_min(m);
            if (L == 0) sRed[wv] = m;
            __syncthreads();
            if (threadIdx.x == 0) {
                u64 mm = ~0ull;
                for (int i = 0; i < TAIL_WAVES; i++) mm = sRed[i] < mm ? sRed[i] : mm;
                sK = c->k > mm ? c->k : mm;
            }
            __syncthreads();
            const u64 k = sK;
            const int32_t r = c->round;
            int32_t *out = b.lists + (size_t)(lc ^ 1) * b.n;
            int32_t *F = b.F + (size_t)cur * b.n;
            const int32_t lim = (cnt + WAVE - 1) / WAVE * WAVE;
            for (int32_t i = threadIdx.x; i - L < lim; i += TAIL_THREADS) {
                int32_t v = -1;
                bool alive = false, take = false;
                if (i < cnt) {
                    v = in[i];
                    alive = b.stamp[v] == ALIVE;
                    take = alive && b.deg[v] <= k;
                }
                if (take) {
                    b.stamp[v] = r;
                    b.core[v] = k;
                }
                wave_push(take, v, F, &c->nF[cur]);
                wave_push(alive && !take, v, out, &c->nlist[lc ^ 1]);
            }
            __syncthreads();
            if (threadIdx.x == 0) record_level(b, c, k, true);
            __syncthreads();
        }
        // destroy the cliques through the frontier, one frontier vertex at a time
        const int32_t nF = c->nF[cur], r = c->round;
        const u64 k = c->k;
        const int32_t *F = b.F + (size_t)cur * b.n;
        u64 destroyed = 0;
        for (int32_t fi = 0; fi < nF; fi++) {
            const int32_t v = F[fi];
            const int64_t rv0 = b.row_ptr[v], rv1 = b.row_ptr[v + 1];
            if constexpr (H == 2) {
                for (int64_t e = rv0 + threadIdx.x; e < rv1; e += TAIL_THREADS) {
                    int32_t w = b.col[e];
                    int32_t st = b.stamp[w];
                    if (st == r) {
                        destroyed += (v < w) ? 1 : 0;
                    } else if (st > r) {
                        destroyed += 1;
                        dec_deg(b, w, 1, k, r);
                    }
                }
            } else {
                destroyed += h3_block_range<TAIL_WAVES>(b, v, rv0, rv1, r, k, sKey, sVal, sPre, sSt, sW, sCnt);
            }
        }
        destroyed = wave_sum(destroyed);
        if (L == 0) sRed[wv] = destroyed;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 t = 0;
            for (int i = 0; i < TAIL_WAVES; i++) t += sRed[i];
            c->destroyed += t;
            finish_round(c);
        }
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
        return bsearch_i32(b.col, b.row_ptr[v], b.row_ptr[v + 1], x) >= 0;
    }
    __device__ __forceinline__ void add(int32_t x, u64 cnt) const {
        const int32_t r = b.ctl->round;
        if (b.stamp[x] > r) dec_deg(b, x, cnt, round_level(b.ctl), r);
    }
    __device__ __forceinline__ void add_prefix(int64_t it, u64 t) const {
        const int32_t r = b.ctl->round;
        const int32_t w = root(it);
        if (b.stamp[w] > r) dec_deg(b, w, t, round_level(b.ctl), r);
        atomicAdd(&b.ctl->destroyed, t);
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

__global__ __launch_bounds__(BLOCK) void k_peel_items(PeelBufs b, int R) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE;
    for (int64_t fi = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; fi < nF; fi += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[fi];
        const int64_t e1 = b.row_ptr[v + 1];
        for (int64_t e = b.row_ptr[v]; e < e1; e += WAVE) {
            int cls = -1;
            int32_t w = -1;
            if (e + lane() < e1) {
                w = b.col[e + lane()];
                if (allowed(b.stamp[w], r, w, v)) cls = item_class((int)(b.row_ptr[w + 1] - b.dag_off[w]), R);
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
}

// end of every grid round: a round that opened a level records it, then the
// frontier is retired
__global__ void k_finish_round(PeelBufs b) {
    PeelCtl *c = b.ctl;
    if (c->selecting) {
        record_level(b, c, round_level(c), list_compacts(c));
        c->selecting = 0;
    }
    if (c->nF[c->cur] == 0) return;
    finish_round(c);
}

// ---------------------------------------------------------------- adjacency compaction
//
// Between rounds, rows of removed vertices and entries pointing at them are
// dead weight for every later round.  Compaction rebuilds the CSR over the
// vertices still taking part (stamp >= current round: alive, or in the
// pending frontier), keeping each row sorted by rank so that N+(v) is again
// the tail of row v.  Vertex ids do not change.

// one wave per vertex: kept neighbours, and kept out-neighbours
__global__ __launch_bounds__(BLOCK) void k_compact_count(PeelBufs b, int64_t *cnt, int32_t *cnt_out) {
    const int32_t r = b.ctl->round;
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < b.n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        int64_t c = 0;
        int32_t co = 0;
        if (b.stamp[v] >= r) {
            for (int64_t e = b.row_ptr[v] + lane(); e < b.row_ptr[v + 1]; e += WAVE) {
                int32_t w = b.col[e];
                bool keep = b.stamp[w] >= r;
                c += keep ? 1 : 0;
                co += (keep && w > (int32_t)v) ? 1 : 0;
            }
        }
        c = wave_sum(c);
        co = wave_sum(co);
        if (lane() == 0) {
            cnt[v] = c;
            cnt_out[v] = co;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_compact_fill(PeelBufs b, const int64_t *nrow, const int32_t *cnt_out,
                                                         int32_t *ncol, int64_t *ndag) {
    const int32_t r = b.ctl->round;
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < b.n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        int64_t o = nrow[v];
        if (lane() == 0) ndag[v] = nrow[v + 1] - cnt_out[v];
        if (b.stamp[v] < r) continue;
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
    k_compact_count<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, cnt, cnt_out);
    scan_exclusive_i64(cnt, nrow, n, s, sc);
    k_last_row<<<1, 1, 0, s>>>(nrow, cnt, n);
    int64_t total = 0;
    DSD_HIP(hipMemcpyAsync(&total, nrow + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    int32_t *ncol = sc.get_n<int32_t>(total);
    int64_t *ndag = sc.get_n<int64_t>(n);
    k_compact_fill<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, nrow, cnt_out, ncol, ndag);
    b.row_ptr = nrow;
    b.col = ncol;
    b.dag_off = ndag;
    if (b.h == 3) {
        k_reset_chunks<<<1, 1, 0, s>>>(b);
        k_rechunk<<<256, BLOCK, 0, s>>>(b);
    }
}

// ---------------------------------------------------------------- host driver

__global__ void k_peel_init(PeelBufs b, const uint8_t *alive0, int32_t *list0, int32_t *count) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t lim = ((int64_t)b.n + WAVE - 1) / WAVE * WAVE;
    for (int64_t v = blockIdx.x * (int64_t)BLOCK + threadIdx.x; v - lane() < lim; v += stride) {
        bool in = v < b.n && (alive0 == nullptr || alive0[v] != 0);
        if (v < b.n) {
            b.stamp[v] = in ? ALIVE : -1;
            b.core[v] = 0;
        }
        wave_push(in, (int32_t)v, list0, count);
    }
}

__global__ void k_set_alive(PeelBufs b) {
    if (blockIdx.x == 0 && threadIdx.x == 0) b.ctl->n_alive = b.ctl->nlist[0];
}

template <int R>
static void launch_peel_items(const DevGraph &g, const PeelBufs &b, hipStream_t s, u64 *gS) {
    PeelCtx ctx{b, 0};
    const int32_t *ni = &b.ctl->nitems[0];
    k_engine_wave<R, PeelCtx><<<1024, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off, 0, ni + 0);
    if constexpr (R <= 2) {
        ctx.cls = 1;
        k_engine_block<R, 2048, 12, 1, false, PeelCtx><<<512, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                0, ni + 1, nullptr);
        ctx.cls = 2;
        k_engine_huge_r2<PeelCtx><<<256, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off, 0, ni + 2);
    } else {
        ctx.cls = 1;
        k_engine_block<R, 256, 9, 4, false, PeelCtx><<<1024, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                               0, ni + 1, nullptr);
        ctx.cls = 2;
        k_engine_block<R, 768, 11, 12, false, PeelCtx><<<512, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                0, ni + 2, nullptr);
        ctx.cls = 3;
        k_engine_block<R, 1280, 12, 20, true, PeelCtx><<<256, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                0, ni + 3, gS);
    }
}

// Alive-vertex count at or below which the single-workgroup tail finishes the
// peel (h <= 3).  Grid rounds spread a hub's pairs over the whole chip and
// beat the tail on power-law graphs, so by default the tail is off;
// DSD_TAIL_T sets it for experiments.
static int64_t tail_threshold(int h) {
    if (h > 3) return 0;
    const char *e = getenv("DSD_TAIL_T");
    return e ? atoll(e) : 0;
}

PeelResult peel(const DevGraph &g, int h, const uint8_t *alive0, u64 *deg, u64 mu, u64 k_floor, u64 *core,
                hipStream_t s, Scratch &sc, KernelTimes *kt) {
    PeelResult res;
    const int32_t n = g.n;
    if (n == 0) return res;
    PeelBufs b{};
    b.n = n;
    b.h = h;
    b.row_ptr = g.row_ptr;
    b.col = g.col;
    b.dag_off = g.dag_off;
    b.ctl = sc.get_n<PeelCtl>(1);
    b.stamp = sc.get_n<int32_t>(n);
    b.deg = deg;
    b.core = core;
    b.F = sc.get_n<int32_t>(2 * (int64_t)n);
    b.lists = sc.get_n<int32_t>(2 * (int64_t)n);
    b.lv_k = sc.get_n<u64>(n + 1);
    b.lv_size = sc.get_n<u64>(n + 1);
    b.lv_mu = sc.get_n<u64>(n + 1);
    if (h == 3) {
        // a vertex joins at most one frontier; its chunks number <= 1 + deg / CHUNK
        b.bcap = (int64_t)n + 2 * g.m / CHUNK + 1;
        b.B = sc.get_n<int64_t>(2 * b.bcap);
        // a vertex of degree d > CHUNK takes SLOTS_PER_CHUNK * ceil(d / CHUNK) <= 4d
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
    u64 *gS = nullptr;
    if (h >= 4) {
        // every (v, w) item is an arc of the frontier's adjacency; a round holds at most 2m of them
        b.item_cap = 2 * g.m + 1;
        b.item_v = sc.get_n<int32_t>(5 * b.item_cap);
        b.item_w = sc.get_n<int32_t>(5 * b.item_cap);
        if (R >= 3) gS = sc.get_n<u64>((int64_t)256 * 1280 * 20);
        if (g.maxdout > 1280 && R >= 3)
            throw Error(-5, "an out-neighbourhood exceeds 1280 vertices (limit of the bitmap kernels, h >= 5)");
    }
    PeelCtl init{};
    init.k = k_floor;
    init.kcand = ~0ull;
    init.mu_alive = mu;
    init.tail_T = tail_threshold(h);
    DSD_HIP(hipMemcpyAsync(b.ctl, &init, sizeof(PeelCtl), hipMemcpyHostToDevice, s));
    k_peel_init<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(b, alive0, b.lists, &b.ctl->nlist[0]);
    k_set_alive<<<1, 1, 0, s>>>(b);
    int64_t *pinned = nullptr;
    DSD_HIP(hipHostMalloc((void **)&pinned, 2 * sizeof(int64_t), hipHostMallocDefault));
    DSD_HIP(hipMemcpyAsync(pinned, &b.ctl->n_alive, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    int64_t n_alive = pinned[0];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt) {
        DSD_HIP(hipEventCreate(&e0));
        DSD_HIP(hipEventCreate(&e1));
        DSD_HIP(hipEventRecord(e0, s));
    }
    const int gmin = 256, gbuild = 1024, gproc = 2048;
    int64_t steps = 0, chunk = 4;
    const int64_t max_steps = 4 * (int64_t)n + 64;
    const bool compacting = h <= 3;
    int64_t compacted_at = n;
    if (compacting && n_alive > 0 && n_alive < n / 2) {
        compact_adjacency(b, s, sc);
        compacted_at = n_alive;
    }
    while (n_alive > init.tail_T) {
        if (compacting && n_alive < compacted_at / 2) {
            compact_adjacency(b, s, sc);
            compacted_at = n_alive;
        }
        for (int64_t i = 0; i < chunk; i++) {
            k_level_min<<<gmin, BLOCK, 0, s>>>(b);
            k_level_build<<<gbuild, BLOCK, 0, s>>>(b);
            if (h == 2) {
                k_process_h2<<<gproc, BLOCK, 0, s>>>(b);
                k_finish_round<<<1, 1, 0, s>>>(b);
            } else if (h == 3) {
                k_process_h3_small<<<gproc, BLOCK, 0, s>>>(b);
                k_h3_fill<<<gbuild, BLOCK, 0, s>>>(b);
                k_h3_probe<<<gproc, BLOCK, 0, s>>>(b);
                k_h3_flush<<<gbuild, BLOCK, 0, s>>>(b);
                k_finish_round<<<1, 1, 0, s>>>(b);
            } else {
                k_peel_items<<<gproc, BLOCK, 0, s>>>(b, R);
                switch (R) {
                    case 2: launch_peel_items<2>(g, b, s, gS); break;
                    case 3: launch_peel_items<3>(g, b, s, gS); break;
                    case 4: launch_peel_items<4>(g, b, s, gS); break;
                    default: throw Error(-1, "h outside [2, 6]");
                }
                k_finish_round<<<1, 1, 0, s>>>(b);
            }
        }
        steps += chunk;
        DSD_HIP(hipMemcpyAsync(pinned, &b.ctl->n_alive, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        n_alive = pinned[0];
        if (steps > max_steps) {
            (void)hipHostFree(pinned);
            throw Error(-3, "peel did not converge");
        }
        if (chunk < 32) chunk *= 2;
    }
    if (n_alive > 0) {
        if (compacting && n_alive < compacted_at) compact_adjacency(b, s, sc);
        if (h == 2) k_peel_tail<2><<<1, TAIL_THREADS, 0, s>>>(b);
        else k_peel_tail<3><<<1, TAIL_THREADS, 0, s>>>(b);
    }
    (void)hipHostFree(pinned);
    if (kt) {
        DSD_HIP(hipEventRecord(e1, s));
        DSD_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DSD_HIP(hipEventElapsedTime(&ms, e0, e1));
        kt->k4_ms += ms;
        kt->k4_launches += 1;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    PeelCtl fin;
    DSD_HIP(hipMemcpyAsync(&fin, b.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (fin.n_alive != 0) throw Error(-3, "peel ended with alive vertices");
    res.rounds = fin.round;
    res.levels = fin.nlevels;
    res.level_k.resize(fin.nlevels);
    res.level_size.resize(fin.nlevels);
    res.level_mu.resize(fin.nlevels);
    if (fin.nlevels > 0) {
        DSD_HIP(hipMemcpyAsync(res.level_k.data(), b.lv_k, fin.nlevels * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(res.level_size.data(), b.lv_size, fin.nlevels * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(res.level_mu.data(), b.lv_mu, fin.nlevels * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        res.kmax = res.level_k.back();
    }
    return res;
}

}  // namespace dsd
