// K3: clique-degrees (Definition 3) on the degree-ordered DAG.
//
// Every h-clique is listed once, from its lowest-rank member r: the other
// h-1 members form an (h-1)-clique of the sub-DAG induced on N+(r).  Roots
// are binned by out-degree into a wave class (one wave per root, |N+| <= 64)
// and block classes (one workgroup per root, candidate set, hash and bitmap
// staged in LDS); each root flushes at most |N+(r)| + 1 global 64-bit atomics.
#include "engine.hpp"
#include "graph.hpp"

namespace dsd {

struct EnumCtx {
    const int32_t *roots;
    const uint8_t *mask;
    u64 *deg;
    __device__ __forceinline__ int32_t root(int64_t it) const { return roots[it]; }
    __device__ __forceinline__ bool accept(int64_t, int32_t x) const { return mask == nullptr || mask[x] != 0; }
    __device__ __forceinline__ void add(int32_t x, u64 c) const { atomic_add_u64(&deg[x], c); }
    __device__ __forceinline__ void add_prefix(int64_t it, u64 t) const { atomic_add_u64(&deg[roots[it]], t); }
};

// h = 2: the clique-degree is the degree (inside the mask: one wave per
// vertex, since a hub's row is long)
__global__ void k_deg_h2(const int64_t *row_ptr, int32_t n, u64 *deg) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = (u64)(row_ptr[v + 1] - row_ptr[v]);
}

__global__ __launch_bounds__(BLOCK) void k_deg_h2_masked(const int64_t *row_ptr, const int32_t *col,
                                                          const uint8_t *mask, int32_t n, u64 *deg) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        u64 c = 0;
        if (mask[v])
            for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) c += mask[col[e]] ? 1 : 0;
        c = wave_sum(c);
        if (lane() == 0) deg[v] = c;
    }
}

__device__ __forceinline__ u64 binom_sat_dev(u64 x, int r) {
    if ((u64)r > x) return 0;
    unsigned __int128 acc = 1;
    for (int i = 1; i <= r; i++) {
        acc = acc * (unsigned __int128)(x - (u64)r + (u64)i) / (unsigned __int128)i;
        if (acc > (unsigned __int128)~0ull) return ~0ull;
    }
    return (u64)acc;
}

constexpr int NCLASS = 6;

// class of a root by its out-degree; -1 = no clique can be rooted here
__device__ __forceinline__ int root_class(int d, int R) {
    if (d < R) return -1;
    if (d <= 64) return 0;
    if (R <= 2) return d <= 2048 ? 1 : 2;
    if (d <= 256) return 1;
    if (d <= 768) return 2;
    if (d <= 1280) return 3;
    if (d <= 2048) return 4;
    return 5;   // beyond the bitmap kernels
}

__device__ __forceinline__ u64 sat_add(u64 a, u64 b) { return (a + b < a) ? ~0ull : a + b; }

// pass 0: per-class counts and a saturating bound sum_r C(d+(r), R) on the
// number of cliques; pass 1: fill the class lists.  Wave-aggregated atomics.
__global__ void k_classify(const int64_t *row_ptr, const int64_t *dag_off, const uint8_t *mask, int32_t n, int R,
                           int pass, int32_t *cursor, int32_t *lists, const int32_t *class_off, u64 *bound) {
    u64 b = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t lim = ((int64_t)n + WAVE - 1) / WAVE * WAVE;   // whole waves stay in the loop
    for (int64_t r = start; r < lim + stride; r += stride) {
        if (r - threadIdx.x % WAVE >= lim) break;                    // wave-uniform exit
        int c = -1, d = 0;
        if (r < n && (!mask || mask[r])) {
            d = (int)(row_ptr[r + 1] - dag_off[r]);
            c = root_class(d, R);
        }
        if (pass == 0 && c >= 0) b = sat_add(b, binom_sat_dev((u64)d, R));
        for (int k = 0; k < NCLASS; k++) {
            u64 m = __ballot(c == k);
            if (!m) continue;
            int leader = __builtin_ctzll(m);
            int32_t basepos = 0;
            if (lane() == leader) basepos = atomicAdd(&cursor[k], __popcll(m));
            basepos = __shfl(basepos, leader, WAVE);
            if (pass == 1 && c == k) lists[class_off[k] + basepos + __popcll(m & lanemask_lt())] = (int32_t)r;
        }
    }
    if (pass == 0) {
        for (int d = WAVE / 2; d > 0; d >>= 1) b = sat_add(b, __shfl_xor(b, d, WAVE));
        if (lane() == 0 && b) {
            u64 old = atomicAdd(bound, b);
            if (old + b < old) atomicExch(bound, ~0ull);
        }
    }
}

template <int R>
static void launch_engine(const DevGraph &g, const EnumCtx &base, const int32_t *lists, const int32_t *off,
                          const int32_t *cnt, hipStream_t s, Scratch &sc, int gs_blocks) {
    EnumCtx c = base;
    if (cnt[0]) {
        c.roots = lists + off[0];
        int blocks = grid_for(cnt[0], WAVES_PER_BLOCK, 8192);
        k_engine_wave<R, EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col, g.dag_off, cnt[0], nullptr);
    }
    if constexpr (R <= 2) {
        if (cnt[1]) {
            c.roots = lists + off[1];
            int blocks = grid_for(cnt[1], 1, 4096);
            k_engine_block<R, 2048, 12, 1, false, EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col, g.dag_off,
                                                                                   cnt[1], nullptr, nullptr);
        }
        if (cnt[2]) {
            c.roots = lists + off[2];
            int blocks = grid_for(cnt[2], 1, 1024);
            k_engine_huge_r2<EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col, g.dag_off, cnt[2], nullptr);
        }
    } else {
        if (cnt[1]) {
            c.roots = lists + off[1];
            int blocks = grid_for(cnt[1], 1, 4096);
            k_engine_block<R, 256, 9, 4, false, EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col, g.dag_off,
                                                                                 cnt[1], nullptr, nullptr);
        }
        if (cnt[2]) {
            c.roots = lists + off[2];
            int blocks = grid_for(cnt[2], 1, 2048);
            k_engine_block<R, 768, 11, 12, false, EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col,
                                                                                   g.dag_off, cnt[2], nullptr, nullptr);
        }
        if (cnt[3]) {
            c.roots = lists + off[3];
            int blocks = grid_for(cnt[3], 1, gs_blocks);
            u64 *gS = sc.get_n<u64>((int64_t)blocks * 1280 * 20);
            k_engine_block<R, 1280, 12, 20, true, EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col, g.dag_off,
                                                                                  cnt[3], nullptr, gS);
        }
        if (cnt[4]) {
            // hubs of out-degree 1281..2048: 32-word bitmap rows in global memory
            c.roots = lists + off[4];
            int blocks = grid_for(cnt[4], 1, gs_blocks);
            u64 *gS = sc.get_n<u64>((int64_t)blocks * 2048 * 32);
            k_engine_block<R, 2048, 12, 32, true, EnumCtx><<<blocks, BLOCK, 0, s>>>(c, g.row_ptr, g.col, g.dag_off,
                                                                                  cnt[4], nullptr, gS);
        }
    }
}

bool clique_degrees(const DevGraph &g, int h, const uint8_t *mask, u64 *deg, hipStream_t s, Scratch &sc,
                    KernelTimes *kt, int gs_blocks) {
    const int32_t n = g.n;
    if (n == 0) return true;
    if (h == 2) {
        if (mask) k_deg_h2_masked<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, mask, n, deg);
        else k_deg_h2<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, n, deg);
        return true;
    }
    const int R = h - 1;
    fill_u64(deg, 0, n, s);
    int32_t *cursor = sc.get_n<int32_t>(NCLASS);
    u64 *bound = sc.get_n<u64>(1);
    fill_i32(cursor, 0, NCLASS, s);
    fill_u64(bound, 0, 1, s);
    int blocks = grid_for(n, BLOCK, 4096);
    k_classify<<<blocks, BLOCK, 0, s>>>(g.row_ptr, g.dag_off, mask, n, R, 0, cursor, nullptr, nullptr, bound);
    int32_t hc[NCLASS];
    u64 hb = 0;
    DSD_HIP(hipMemcpyAsync(hc, cursor, sizeof(hc), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&hb, bound, sizeof(u64), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (hb == ~0ull || hb > ~0ull / (u64)h) return false;          // counts could overflow 64 bits
    if (hc[5]) throw Error(-5, "an out-neighbourhood exceeds 2048 vertices (limit of the bitmap kernels, h >= 4)");
    int32_t off[NCLASS + 1];
    off[0] = 0;
    for (int c = 0; c < NCLASS; c++) off[c + 1] = off[c] + hc[c];
    int32_t *lists = sc.get_n<int32_t>(off[NCLASS]);
    int32_t *d_off = sc.get_n<int32_t>(NCLASS + 1);
    DSD_HIP(hipMemcpyAsync(d_off, off, sizeof(off), hipMemcpyHostToDevice, s));
    fill_i32(cursor, 0, NCLASS, s);
    k_classify<<<blocks, BLOCK, 0, s>>>(g.row_ptr, g.dag_off, mask, n, R, 1, cursor, lists, d_off, bound);
    EnumCtx ctx{nullptr, mask, deg};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt) {
        DSD_HIP(hipEventCreate(&e0));
        DSD_HIP(hipEventCreate(&e1));
        DSD_HIP(hipEventRecord(e0, s));
    }
    switch (R) {
        case 2: launch_engine<2>(g, ctx, lists, off, hc, s, sc, gs_blocks); break;
        case 3: launch_engine<3>(g, ctx, lists, off, hc, s, sc, gs_blocks); break;
        case 4: launch_engine<4>(g, ctx, lists, off, hc, s, sc, gs_blocks); break;
        case 5: launch_engine<5>(g, ctx, lists, off, hc, s, sc, gs_blocks); break;
        default: throw Error(-1, "h outside [2, 6]");
    }
    if (kt) {
        DSD_HIP(hipEventRecord(e1, s));
        DSD_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DSD_HIP(hipEventElapsedTime(&ms, e0, e1));
        kt->k3_ms += ms;
        for (int c = 0; c < NCLASS; c++) kt->k3_launches += hc[c] ? 1 : 0;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    // the host copy of `off` must outlive the async H2D copy above
    DSD_HIP(hipStreamSynchronize(s));
    return true;
}

}  // namespace dsd
