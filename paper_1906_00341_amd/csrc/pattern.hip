// Special patterns (the appendix on core decomposition for special
// patterns): pattern-degrees and (k, Psi)-cores for x-stars and 4-loops.
//
// An x-star is a centre joined to x tails (x >= 2).  A vertex v with y
// neighbours is the centre of C(y, x) of them and a tail of C(z_u - 1, x - 1)
// stars centred at each neighbour u of degree z_u, so its pattern-degree is a
// pass over its row: no instance is ever listed.  The peel removes the
// frontier and updates the same closed form (peel.hip).
//
// A 4-loop (the appendix's diamond) through v consists of two 2-paths from v
// to one vertex w: v lies in C(c, 2) loops opposite w when c of its
// neighbours are also w's.  Its pattern-degree and its peel group the 2-paths
// of a vertex by their end w in a table of the vertex's workgroup
// (peel.hip).
#include "handle.hpp"

namespace dsd {
namespace {

// C(n, k), k <= 8; sets *ovf and saturates when the value passes 2^64 - 1
__device__ __forceinline__ u64 binom_sat_flag(int64_t n, int k, int *ovf) {
    if (n < k || n < 0) return 0;
    unsigned __int128 acc = 1;
    for (int i = 1; i <= k; i++) {
        acc = acc * (unsigned __int128)(n - k + i) / (unsigned __int128)i;
        if (acc > (unsigned __int128)~0ull) {
            *ovf = 1;
            return ~0ull;
        }
    }
    return (u64)acc;
}

// one wave per vertex: C(y, x) plus the tail terms of its neighbours
__global__ __launch_bounds__(BLOCK) void k_star_degrees(const int64_t *row_ptr, const int32_t *col, int32_t n, int x,
                                                         u64 *deg, int32_t *err) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t v = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; v < n; v += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        int ovf = 0;
        u64 acc = 0;
        for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) {
            const int32_t u = col[e];
            const u64 t = binom_sat_flag(row_ptr[u + 1] - row_ptr[u] - 1, x - 1, &ovf);
            if (acc + t < acc) ovf = 1;
            acc += t;
        }
        // wave sum with overflow detection
        for (int d = WAVE / 2; d > 0; d >>= 1) {
            const u64 o = __shfl_xor(acc, d, WAVE);
            if (acc + o < acc) ovf = 1;
            acc += o;
        }
        if (lane() == 0) {
            const u64 own = binom_sat_flag(row_ptr[v + 1] - row_ptr[v], x, &ovf);
            if (acc + own < acc) ovf = 1;
            deg[v] = acc + own;
        }
        if (__ballot(ovf) && lane() == 0) atomicOr(err, 1);
    }
}

}  // namespace

bool star_degrees(const DevGraph &g, int x, u64 *deg, hipStream_t s, Scratch &sc) {
    int32_t *err = sc.get_n<int32_t>(1);
    fill_i32(err, 0, 1, s);
    if (g.n > 0) k_star_degrees<<<grid_for(g.n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, g.n, x, deg, err);
    int32_t e = 0;
    DSD_HIP(hipMemcpyAsync(&e, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    return e == 0;
}

// pattern-degrees of the whole graph and their instance count
static u64 pattern_degrees_run(dsd_graph_s *G, int pattern, int x, u64 *d) {
    hipStream_t s = G->stream;
    if (pattern == DSD_PATTERN_STAR) {
        if (!star_degrees(G->g, x, d, s, G->sc)) throw Error(DSD_EOVERFLOW, "pattern-degrees could exceed 64 bits");
    } else {
        loop4_degrees(G->g, d, s, G->sc);
        x = 3;                           // four vertices per instance
    }
    u64 *sum = G->sc.get_n<u64>(2);
    sum_u64_128(d, G->g.n, sum, s, G->sc);
    u64 hs[2];
    DSD_HIP(hipMemcpyAsync(hs, sum, sizeof(hs), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (hs[1] != 0) throw Error(DSD_EOVERFLOW, "sum of pattern-degrees exceeds 64 bits");
    if (hs[0] % (u64)(x + 1) != 0) throw Error(DSD_EDEVICE, "pattern-degree sum not divisible by the pattern size");
    return hs[0] / (u64)(x + 1);
}

static void check_pattern(int pattern, int x) {
    if (pattern == DSD_PATTERN_STAR) {
        if (x < 2 || x > 8) throw Error(DSD_EINVAL, "an x-star needs 2 <= x <= 8 tails");
        return;
    }
    if (pattern == DSD_PATTERN_LOOP4) return;
    throw Error(DSD_EINVAL, "unknown pattern");
}

}  // namespace dsd

using namespace dsd;

extern "C" {

dsd_status dsd_pattern_degrees(dsd_graph G, int pattern, int x, int out_mem, uint64_t *deg, uint64_t *count) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_pattern(pattern, x);
        const int32_t n = G->g.n;
        if (n > 0) check_out(deg, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        u64 *d = G->sc.get_n<u64>(n);
        const u64 mu = n > 0 ? pattern_degrees_run(G, pattern, x, d) : 0;
        G->stats.t_enum_ms = tm.stop();
        G->stats.num_cliques = mu;
        write_u64(G, d, deg, out_mem);
        if (count) *count = mu;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

dsd_status dsd_pattern_core(dsd_graph G, int pattern, int x, int out_mem, uint64_t *core, uint64_t *kmax) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_pattern(pattern, x);
        const int32_t n = G->g.n;
        if (n > 0) check_out(core, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        hipStream_t s = G->stream;
        Timer tm(s);
        u64 *d = G->sc.get_n<u64>(n), *c = G->sc.get_n<u64>(n);
        u64 km = 0;
        if (n > 0) {
            KernelTimes kt;
            kt.time_main = G->time_main;
            Timer te(s);
            const u64 mu = pattern_degrees_run(G, pattern, x, d);
            G->stats.t_enum_ms = te.stop();
            G->stats.num_cliques = mu;
            Timer tp(s);
            if (mu > 0) {
                const int size = pattern == DSD_PATTERN_STAR ? x + 1 : 4;
                PeelResult pr = peel(G->g, size, nullptr, d, mu, 0, c, s, G->sc, &kt, nullptr, false, nullptr,
                                     pattern, x);
                G->stats.peel_rounds = pr.rounds;
                G->stats.peel_levels = pr.levels;
                km = pr.kmax;
            } else {
                fill_u64(c, 0, n, s);
            }
            G->stats.t_peel_ms = tp.stop();
            end_stats(G, kt);
        }
        write_u64(G, c, core, out_mem);
        if (kmax) *kmax = km;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

}  // extern "C"
