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
// State lives on the device (PeelCtl).  One step is a fixed sequence of
// kernels (level-min, level-build, process, [finalize]) that read the state
// themselves, so the host enqueues many steps without waiting and only polls
// the number of alive vertices now and then.
#include "engine.hpp"
#include "graph.hpp"

namespace dsd {

struct PeelCtl {
    u64 k;          // current level
    u64 kcand;      // smallest alive degree (next level)
    u64 mu_alive;   // cliques among alive vertices
    u64 destroyed;  // cliques destroyed in this round
    int64_t n_alive;
    int32_t round;
    int32_t cur;       // frontier buffer in use
    int32_t nF[2];     // frontier sizes
    int32_t nlist[2];  // alive-list sizes
    int32_t lcur;      // alive list in use
    int32_t nlevels;
    uint32_t done;     // finished blocks (last-block finalisation)
    int32_t selecting; // set by level-min: this step starts a new level
    int32_t nitems[8]; // (v, w) work items per class (h >= 4)
};

struct PeelBufs {
    PeelCtl *ctl;
    int32_t *stamp;    // ALIVE, removal round, or -1 (not taking part)
    u64 *deg;          // current clique-degree
    u64 *core;
    int32_t *F;        // [2][n] frontiers
    int32_t *lists;    // [2][n] alive lists
    u64 *lv_k, *lv_size, *lv_mu;  // level table [n + 1]
    int32_t *item_v, *item_w;     // [8][cap] work items (h >= 4)
    int64_t item_cap;
    int32_t n;
};

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

// the last block to arrive returns true (block-uniform)
__device__ __forceinline__ bool last_block(uint32_t *done) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = atomicAdd(done, 1u) == gridDim.x - 1;
    __syncthreads();
    return is_last;
}

__device__ __forceinline__ void dec_deg(const PeelBufs &b, int32_t x, u64 c, u64 k, int32_t r) {
    u64 old = atomic_sub_u64(&b.deg[x], c);
    if (old > k && old - c <= k) {
        int32_t *Fn = b.F + (size_t)(b.ctl->cur ^ 1) * b.n;
        int32_t pos = atomicAdd(&b.ctl->nF[b.ctl->cur ^ 1], 1);
        Fn[pos] = x;
        b.stamp[x] = r + 1;
        b.core[x] = k;
    }
}

// ---------------------------------------------------------------- level selection

__global__ __launch_bounds__(BLOCK) void k_level_min(PeelBufs b) {
    PeelCtl *c = b.ctl;
    // nF and n_alive do not change during this kernel, so every block takes
    // the same decision; level-build reads the flag because it grows nF itself
    const bool sel = c->nF[c->cur] == 0 && c->n_alive > 0;
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
    m = wave_min(m);
    if (lane() == 0 && m != ~0ull) atomicMin(&c->kcand, m);
}

__global__ __launch_bounds__(BLOCK) void k_level_build(PeelBufs b) {
    PeelCtl *c = b.ctl;
    if (!c->selecting) return;
    const u64 k = c->k > c->kcand ? c->k : c->kcand;
    const int32_t r = c->round, lc = c->lcur, cur = c->cur;
    const int32_t *in = b.lists + (size_t)lc * b.n;
    int32_t *out = b.lists + (size_t)(lc ^ 1) * b.n;
    int32_t *F = b.F + (size_t)cur * b.n;
    const int32_t cnt = c->nlist[lc];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t lim = ((int64_t)cnt + WAVE - 1) / WAVE * WAVE;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i - lane() < lim; i += stride) {
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
    if (last_block(&c->done) && threadIdx.x == 0) {
        int32_t L = c->nlevels;
        b.lv_k[L] = k;
        b.lv_size[L] = (u64)c->n_alive;
        b.lv_mu[L] = c->mu_alive;
        c->nlevels = L + 1;
        c->k = k;
        c->kcand = ~0ull;
        c->nlist[lc] = 0;
        c->lcur = lc ^ 1;
        c->done = 0;
    }
}

// end of a round: the frontier is gone
__device__ __forceinline__ void finish_round(PeelCtl *c) {
    int32_t cur = c->cur;
    c->n_alive -= c->nF[cur];
    c->mu_alive -= c->destroyed;
    c->destroyed = 0;
    c->nF[cur] = 0;
    c->cur = cur ^ 1;
    c->round += 1;
    c->done = 0;
    for (int i = 0; i < 8; i++) c->nitems[i] = 0;
}

// ---------------------------------------------------------------- h = 2

__global__ __launch_bounds__(BLOCK) void k_process_h2(PeelBufs b, const int64_t *row_ptr, const int32_t *col) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    const u64 k = c->k;
    const int32_t *F = b.F + (size_t)cur * b.n;
    u64 destroyed = 0;
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < nF; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[i];
        for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) {
            int32_t w = col[e];
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
    if (last_block(&c->done) && threadIdx.x == 0) finish_round(c);
}

// ---------------------------------------------------------------- h = 3

constexpr int H3_HASH_BITS = 10;              // 1024 slots per wave
constexpr int H3_HASH_CAP = 512;              // neighbourhoods up to this size use the hash

__global__ __launch_bounds__(BLOCK) void k_process_h3(PeelBufs b, const int64_t *row_ptr, const int32_t *col,
                                                      const int64_t *dag_off) {
    __shared__ int32_t sKey[WAVES_PER_BLOCK][1 << H3_HASH_BITS];
    __shared__ int32_t sVal[WAVES_PER_BLOCK][1 << H3_HASH_BITS];
    __shared__ int32_t sPre[WAVES_PER_BLOCK][WAVE];
    __shared__ int64_t sSt[WAVES_PER_BLOCK][WAVE];
    __shared__ int32_t sW[WAVES_PER_BLOCK][WAVE];
    __shared__ uint32_t sCnt[WAVES_PER_BLOCK][WAVE];
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    const u64 k = c->k;
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE, L = lane();
    u64 destroyed = 0;
    for (int i = L; i < (1 << H3_HASH_BITS); i += WAVE) sKey[wv][i] = HASH_EMPTY;
    __builtin_amdgcn_wave_barrier();
    for (int64_t fi = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; fi < nF; fi += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[fi];
        const int64_t rv0 = row_ptr[v], rv1 = row_ptr[v + 1];
        const int64_t dv = rv1 - rv0;
        const bool use_hash = dv <= H3_HASH_CAP;
        if (use_hash) {
            for (int64_t e = rv0 + L; e < rv1; e += WAVE) {
                int32_t x = col[e];
                int32_t st = b.stamp[x];
                if (st > r || (st == r && x > v)) hash_insert(sKey[wv], sVal[wv], H3_HASH_BITS, x, 0);
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int64_t base = 0; base < dv; base += WAVE) {
            int32_t w = -1, len = 0;
            int64_t st0 = 0;
            if (base + L < dv) {
                w = col[rv0 + base + L];
                int32_t st = b.stamp[w];
                if (st > r || (st == r && w > v)) {
                    st0 = dag_off[w];
                    len = (int32_t)(row_ptr[w + 1] - st0);
                }
            }
            int32_t inc = wave_incl_scan(len);
            sPre[wv][L] = inc;
            sSt[wv][L] = st0;
            sW[wv][L] = w;
            sCnt[wv][L] = 0;
            const int32_t total = __shfl(inc, WAVE - 1, WAVE);
            __builtin_amdgcn_wave_barrier();
            for (int32_t pb = 0; pb < total; pb += WAVE) {
                int32_t p = pb + L;
                if (p < total) {
                    int i = upper_bound_i32(sPre[wv], WAVE, p);
                    int32_t off = p - (i ? sPre[wv][i - 1] : 0);
                    int32_t x = col[sSt[wv][i] + off];
                    bool found;
                    if (use_hash) {
                        found = hash_find(sKey[wv], sVal[wv], H3_HASH_BITS, x) >= 0;
                    } else {
                        int32_t st = b.stamp[x];
                        found = (st > r || (st == r && x > v)) && bsearch_i32(col, rv0, rv1, x) >= 0;
                    }
                    if (found) {                       // triangle {v, w, x}, owned by v
                        destroyed++;
                        atomicAdd(&sCnt[wv][i], 1u);
                        if (b.stamp[x] > r) dec_deg(b, x, 1, k, r);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            uint32_t cw = sCnt[wv][L];
            if (cw && b.stamp[sW[wv][L]] > r) dec_deg(b, sW[wv][L], cw, k, r);
            __builtin_amdgcn_wave_barrier();
        }
        if (use_hash) {
            for (int i = L; i < (1 << H3_HASH_BITS); i += WAVE) sKey[wv][i] = HASH_EMPTY;
            __builtin_amdgcn_wave_barrier();
        }
    }
    destroyed = wave_sum(destroyed);
    if (L == 0 && destroyed) atomicAdd(&c->destroyed, destroyed);
    if (last_block(&c->done) && threadIdx.x == 0) finish_round(c);
}

// ---------------------------------------------------------------- h >= 4

// Items (v, w): v in the frontier, w an allowed neighbour of v.  The engine
// counts the (h-2)-cliques of the sub-DAG on N+(w) ∩ N(v) ∩ allowed.
struct PeelCtx {
    PeelBufs b;
    const int64_t *row_ptr;
    const int32_t *col;
    int cls;
    __device__ __forceinline__ int32_t root(int64_t it) const { return b.item_w[cls * b.item_cap + it]; }
    __device__ __forceinline__ bool accept(int64_t it, int32_t x) const {
        const int32_t v = b.item_v[cls * b.item_cap + it];
        const int32_t r = b.ctl->round;
        const int32_t st = b.stamp[x];
        if (!(st > r || (st == r && x > v))) return false;
        return bsearch_i32(col, row_ptr[v], row_ptr[v + 1], x) >= 0;
    }
    __device__ __forceinline__ void add(int32_t x, u64 cnt) const {
        const int32_t r = b.ctl->round;
        if (b.stamp[x] > r) dec_deg(b, x, cnt, b.ctl->k, r);
    }
    __device__ __forceinline__ void add_prefix(int64_t it, u64 t) const {
        const int32_t r = b.ctl->round;
        const int32_t w = root(it);
        if (b.stamp[w] > r) dec_deg(b, w, t, b.ctl->k, r);
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

__global__ __launch_bounds__(BLOCK) void k_peel_items(PeelBufs b, const int64_t *row_ptr, const int32_t *col,
                                                      const int64_t *dag_off, int R) {
    PeelCtl *c = b.ctl;
    const int32_t cur = c->cur, nF = c->nF[cur];
    if (nF == 0) return;
    const int32_t r = c->round;
    const int32_t *F = b.F + (size_t)cur * b.n;
    const int wv = threadIdx.x / WAVE;
    for (int64_t fi = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; fi < nF; fi += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = F[fi];
        const int64_t e1 = row_ptr[v + 1];
        for (int64_t e = row_ptr[v]; e < e1; e += WAVE) {
            int cls = -1;
            int32_t w = -1;
            if (e + lane() < e1) {
                w = col[e + lane()];
                int32_t st = b.stamp[w];
                if (st > r || (st == r && w > v)) cls = item_class((int)(row_ptr[w + 1] - dag_off[w]), R);
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

__global__ void k_finish_round(PeelBufs b) {
    PeelCtl *c = b.ctl;
    if (c->nF[c->cur] == 0) return;
    finish_round(c);
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
    PeelCtx ctx{b, g.row_ptr, g.col, 0};
    const int32_t *ni = &b.ctl->nitems[0];
    ctx.cls = 0;
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

PeelResult peel(const DevGraph &g, int h, const uint8_t *alive0, u64 *deg, u64 mu, u64 k_floor, u64 *core,
                hipStream_t s, Scratch &sc) {
    PeelResult res;
    const int32_t n = g.n;
    if (n == 0) return res;
    PeelBufs b{};
    b.n = n;
    b.ctl = sc.get_n<PeelCtl>(1);
    b.stamp = sc.get_n<int32_t>(n);
    b.deg = deg;
    b.core = core;
    b.F = sc.get_n<int32_t>(2 * (int64_t)n);
    b.lists = sc.get_n<int32_t>(2 * (int64_t)n);
    b.lv_k = sc.get_n<u64>(n + 1);
    b.lv_size = sc.get_n<u64>(n + 1);
    b.lv_mu = sc.get_n<u64>(n + 1);
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
    DSD_HIP(hipMemcpyAsync(b.ctl, &init, sizeof(PeelCtl), hipMemcpyHostToDevice, s));
    k_peel_init<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(b, alive0, b.lists, &b.ctl->nlist[0]);
    k_set_alive<<<1, 1, 0, s>>>(b);
    int64_t *pinned = nullptr;
    DSD_HIP(hipHostMalloc((void **)&pinned, 2 * sizeof(int64_t), hipHostMallocDefault));
    DSD_HIP(hipMemcpyAsync(pinned, &b.ctl->n_alive, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    int64_t n_alive = pinned[0];
    const int gmin = 1024, gbuild = 1024, gproc = 2048;
    int64_t steps = 0, chunk = 4;
    const int64_t max_steps = 4 * (int64_t)n + 64;
    while (n_alive > 0) {
        for (int64_t i = 0; i < chunk; i++) {
            k_level_min<<<gmin, BLOCK, 0, s>>>(b);
            k_level_build<<<gbuild, BLOCK, 0, s>>>(b);
            if (h == 2) {
                k_process_h2<<<gproc, BLOCK, 0, s>>>(b, g.row_ptr, g.col);
            } else if (h == 3) {
                k_process_h3<<<gproc, BLOCK, 0, s>>>(b, g.row_ptr, g.col, g.dag_off);
            } else {
                k_peel_items<<<gproc, BLOCK, 0, s>>>(b, g.row_ptr, g.col, g.dag_off, R);
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
        if (chunk < 64) chunk *= 2;
    }
    (void)hipHostFree(pinned);
    PeelCtl fin;
    DSD_HIP(hipMemcpyAsync(&fin, b.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
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
