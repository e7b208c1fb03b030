// Maximum preflow and minimum cut on the GPU for the exact step's networks
// (Algorithm 1's network, Goldberg's network for h = 2).
//
// Synchronous push-relabel.  A pass is two kernels: every active node (excess
// > 0, height < n) pushes along all of its admissible arcs (residual > 0,
// one level lower) with heights fixed for the whole kernel, then every node
// still active with no admissible arc left is relabelled to one above its
// lowest residual neighbour.  With heights fixed, an arc and its reverse are
// never both admissible, so a push writes its arc pair without races; only
// the receivers' excess needs atomics.  Relabels only raise heights, so a
// neighbour relabelled concurrently leaves the new label valid.  Global
// relabelling (breadth-first search from t over residual arcs, level by
// level) sets exact distances, and marks the nodes that cannot reach t: they
// hold the source side of the maximal minimum cut.  Only the maximum preflow
// is computed: its value is the maximum flow value.
//
// One wave per node (its lanes scan the arcs 64 at a time), except nodes with
// more than BIG_ARCS residual arcs, which take a 1024-thread block each; a
// node's excess is spread over its admissible arcs by a prefix sum.
#include <vector>

#include "common.hpp"
#include "flow.hpp"
#include "primitives.hpp"

namespace dsd {

namespace {

// inclusive prefix sum of non-negative values, saturating at SAT (saturating
// addition of non-negative numbers is associative, so the scan is exact
// below SAT)
constexpr int64_t SAT = (int64_t)1 << 62;
__device__ __forceinline__ int64_t wave_incl_scan_sat(int64_t v) {
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t t = __shfl_up(v, o, WAVE);
        if (lane() >= o) v = (v > SAT - t) ? SAT : v + t;
    }
    return v;
}

__device__ __forceinline__ int wave_min_i32(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        int t = __shfl_xor(v, o, WAVE);
        v = t < v ? t : v;
    }
    return v;
}

constexpr int BIG_ARCS = 4096;
constexpr int BIG_BLOCK = 1024;
constexpr int BIG_WAVES = BIG_BLOCK / WAVE;

struct FlowBufs {
    int n, s, t;
    const int *big;   // nodes with more than BIG_ARCS arcs
    int nbig;
    const int *first, *to, *rev;
    int64_t *cf, *ex;
    int *ht;
    int *front[2];
    int *nfront;   // [2] frontier sizes
    int *active;   // active node count
};

// residual CSR from the arc list: degrees, then every arc and its reverse
__global__ void k_csr_count(const int *eu, const int *ev, int64_t E, uint32_t *cnt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
        atomicAdd(&cnt[eu[i]], 1u);
        atomicAdd(&cnt[ev[i]], 1u);
    }
}

// The same two passes with the arcs of the hot nodes (s, t and the vertex
// nodes, ids < hot: they hold almost every arc) counted in LDS per
// workgroup, so that a global atomic is paid once per hot node per
// workgroup; every workgroup walks one contiguous range of arcs.
constexpr int CSR_HOT = 8192;

__device__ __forceinline__ void csr_range(int64_t E, int64_t *lo, int64_t *hi) {
    const int64_t per = (E + gridDim.x - 1) / gridDim.x;
    *lo = min(E, (int64_t)blockIdx.x * per);
    *hi = min(E, *lo + per);
}

__global__ __launch_bounds__(BLOCK) void k_csr_count_hot(const int *eu, const int *ev, int64_t E, int hot,
                                                          uint32_t *cnt) {
    __shared__ uint32_t sc[CSR_HOT];
    for (int i = threadIdx.x; i < hot; i += BLOCK) sc[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    csr_range(E, &lo, &hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += BLOCK) {
        const int u = eu[i], v = ev[i];
        if (u < hot) atomicAdd(&sc[u], 1u);
        else atomicAdd(&cnt[u], 1u);
        if (v < hot) atomicAdd(&sc[v], 1u);
        else atomicAdd(&cnt[v], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < hot; i += BLOCK)
        if (sc[i]) atomicAdd(&cnt[i], sc[i]);
}

__global__ __launch_bounds__(BLOCK) void k_csr_fill_hot(const int *eu, const int *ev, int64_t E, int hot,
                                                         uint32_t *fill, int *to, int *rev, int *fwd) {
    __shared__ uint32_t sc[CSR_HOT];
    for (int i = threadIdx.x; i < hot; i += BLOCK) sc[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    csr_range(E, &lo, &hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += BLOCK) {
        const int u = eu[i], v = ev[i];
        if (u < hot) atomicAdd(&sc[u], 1u);
        if (v < hot) atomicAdd(&sc[v], 1u);
    }
    __syncthreads();
    // this workgroup's range of each hot node's row
    for (int i = threadIdx.x; i < hot; i += BLOCK)
        if (sc[i]) sc[i] = atomicAdd(&fill[i], sc[i]);
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += BLOCK) {
        const int u = eu[i], v = ev[i];
        const int pu = (int)(u < hot ? atomicAdd(&sc[u], 1u) : atomicAdd(&fill[u], 1u));
        const int pv = (int)(v < hot ? atomicAdd(&sc[v], 1u) : atomicAdd(&fill[v], 1u));
        to[pu] = v;
        to[pv] = u;
        rev[pu] = pv;
        rev[pv] = pu;
        fwd[i] = pu;
    }
}

__global__ void k_csr_last(const uint32_t *cnt, int n, int *first) {
    if (blockIdx.x == 0 && threadIdx.x == 0) first[n] = first[n - 1] + (int)cnt[n - 1];
}

__global__ void k_csr_fill(const int *eu, const int *ev, int64_t E, uint32_t *fill, int *to, int *rev, int *fwd) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
        const int u = eu[i], v = ev[i];
        const int pu = (int)atomicAdd(&fill[u], 1u), pv = (int)atomicAdd(&fill[v], 1u);
        to[pu] = v;
        to[pv] = u;
        rev[pu] = pv;
        rev[pv] = pu;
        fwd[i] = pu;
    }
}

// capacities of one test (see FlowTest), and zero excess
__global__ void k_flow_caps(FlowBufs b, const int *eu, const int *ev, const uint8_t *cls, const int *fwd,
                            const int64_t *deg, int64_t E, FlowTest t) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0, rc = 0;
        switch (cls[i]) {
            case ARC_SRC: c = t.h == 2 ? t.b * t.m : t.b * deg[ev[i] - 2]; break;
            case ARC_SNK: c = t.h == 2 ? t.b * t.m + 2 * t.a - t.b * deg[eu[i] - 2] : (int64_t)t.h * t.a; break;
            case ARC_INF: c = t.inf; break;
            default:
                c = t.b;
                rc = t.h == 2 ? t.b : 0;
        }
        const int p = fwd[i];
        b.cf[p] = c;
        b.cf[b.rev[p]] = rc;
    }
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < b.n; v += (int64_t)gridDim.x * blockDim.x)
        b.ex[v] = 0;
}

// saturate every arc out of s (one wave)
__global__ void k_flow_saturate(FlowBufs b) {
    int64_t sent = 0;
    for (int a = b.first[b.s] + lane(); a < b.first[b.s + 1]; a += WAVE) {
        const int64_t c = b.cf[a];
        if (c <= 0) continue;
        b.cf[a] = 0;
        b.cf[b.rev[a]] += c;
        atomicAdd((unsigned long long *)&b.ex[b.to[a]], (unsigned long long)c);
        sent += c;
    }
    sent = wave_sum(sent);
    if (lane() == 0) atomicAdd((unsigned long long *)&b.ex[b.s], (unsigned long long)(-sent));
}

// breadth-first search from t over residual arcs (u -> v with residual > 0
// means u reaches v): start
__global__ void k_bfs_start(FlowBufs b) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < b.n; v += gridDim.x * blockDim.x)
        b.ht[v] = v == b.t ? 0 : b.n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.front[0][0] = b.t;
        b.nfront[0] = 1;
        b.nfront[1] = 0;
    }
}

// one level: every node of front[cur] (height `level`) labels its unlabelled
// in-neighbours (u with a residual arc u -> v) level + 1
__global__ __launch_bounds__(BLOCK) void k_bfs_level(FlowBufs b, int cur, int level) {
    const int nf = b.nfront[cur];
    const int *F = b.front[cur];
    int *N = b.front[cur ^ 1];
    const int wv = threadIdx.x / WAVE;
    for (int i = blockIdx.x * WAVES_PER_BLOCK + wv; i < nf; i += gridDim.x * WAVES_PER_BLOCK) {
        const int v = F[i];
        if (b.first[v + 1] - b.first[v] > BIG_ARCS) continue;     // k_bfs_level_big
        for (int a0 = b.first[v]; a0 < b.first[v + 1]; a0 += WAVE) {
            const int a = a0 + lane();
            bool take = false;
            int u = -1;
            if (a < b.first[v + 1]) {
                u = b.to[a];
                // the arc u -> v is rev[a]
                if (u != b.s && b.cf[b.rev[a]] > 0 && b.ht[u] == b.n)
                    take = atomicCAS(&b.ht[u], b.n, level + 1) == b.n;
            }
            const u64 m = __ballot(take);
            if (m) {
                const int leader = __builtin_ctzll(m);
                int base = 0;
                if (lane() == leader) base = atomicAdd(&b.nfront[cur ^ 1], __popcll(m));
                base = __shfl(base, leader, WAVE);
                if (take) N[base + __popcll(m & lanemask_lt())] = u;
            }
        }
    }
}

// the same for frontier nodes with more than BIG_ARCS arcs: one block each
__global__ __launch_bounds__(BIG_BLOCK) void k_bfs_level_big(FlowBufs b, int cur, int level) {
    __shared__ int sBase[BIG_WAVES];
    const int nf = b.nfront[cur];
    const int *F = b.front[cur];
    int *N = b.front[cur ^ 1];
    const int wv = threadIdx.x / WAVE;
    for (int i = blockIdx.x; i < nf; i += gridDim.x) {
        const int v = F[i];
        if (b.first[v + 1] - b.first[v] <= BIG_ARCS) continue;    // block-uniform
        for (int a0 = b.first[v]; a0 < b.first[v + 1]; a0 += BIG_BLOCK) {
            const int a = a0 + threadIdx.x;
            bool take = false;
            int u = -1;
            if (a < b.first[v + 1]) {
                u = b.to[a];
                if (u != b.s && b.cf[b.rev[a]] > 0 && b.ht[u] == b.n)
                    take = atomicCAS(&b.ht[u], b.n, level + 1) == b.n;
            }
            const u64 m = __ballot(take);
            if (lane() == 0) sBase[wv] = m ? atomicAdd(&b.nfront[cur ^ 1], __popcll(m)) : 0;
            __builtin_amdgcn_wave_barrier();
            if (take) N[sBase[wv] + __popcll(m & lanemask_lt())] = u;
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ void k_bfs_reset(FlowBufs b, int cur) {
    if (blockIdx.x == 0 && threadIdx.x == 0) b.nfront[cur] = 0;
}

// push phase: heights are read-only here (nodes up to BIG_ARCS arcs)
__global__ __launch_bounds__(BLOCK) void k_flow_push(FlowBufs b) {
    const int wv = threadIdx.x / WAVE;
    for (int u = blockIdx.x * WAVES_PER_BLOCK + wv; u < b.n; u += gridDim.x * WAVES_PER_BLOCK) {
        if (u == b.s || u == b.t || b.first[u + 1] - b.first[u] > BIG_ARCS) continue;
        const int hu = __shfl(b.ht[u], 0, WAVE);
        int64_t rem = __shfl(b.ex[u], 0, WAVE);   // one snapshot for the whole wave
        if (rem <= 0 || hu >= b.n) continue;
        const int64_t start = rem;
        for (int a0 = b.first[u]; a0 < b.first[u + 1] && rem > 0; a0 += WAVE) {
            const int a = a0 + lane();
            int64_t c = 0;
            int v = -1;
            if (a < b.first[u + 1]) {
                v = b.to[a];
                const int64_t r = b.cf[a];
                if (r > 0 && b.ht[v] == hu - 1) c = r < rem ? r : rem;
            }
            const int64_t inc = wave_incl_scan_sat(c);
            const int64_t before = inc - c;
            int64_t d = rem - before;
            d = d < 0 ? 0 : (d > c ? c : d);
            if (d > 0) {
                b.cf[a] -= d;
                b.cf[b.rev[a]] += d;
                atomicAdd((unsigned long long *)&b.ex[v], (unsigned long long)d);
            }
            const int64_t total = __shfl(inc, WAVE - 1, WAVE);
            rem -= total < rem ? total : rem;
        }
        if (lane() == 0 && rem != start)
            atomicAdd((unsigned long long *)&b.ex[u], (unsigned long long)(rem - start));
    }
}

// relabel phase: an active node without admissible arcs rises to one above
// its lowest residual neighbour (n when it has none: it cannot reach t)
__global__ __launch_bounds__(BLOCK) void k_flow_relabel(FlowBufs b) {
    const int wv = threadIdx.x / WAVE;
    int act = 0;
    for (int u = blockIdx.x * WAVES_PER_BLOCK + wv; u < b.n; u += gridDim.x * WAVES_PER_BLOCK) {
        if (u == b.s || u == b.t || b.first[u + 1] - b.first[u] > BIG_ARCS) continue;
        const int hu = __shfl(b.ht[u], 0, WAVE);
        const int64_t eu = __shfl(b.ex[u], 0, WAVE);
        if (eu <= 0 || hu >= b.n) continue;
        int hmin = 0x7fffffff;
        for (int a0 = b.first[u]; a0 < b.first[u + 1]; a0 += WAVE) {
            const int a = a0 + lane();
            if (a < b.first[u + 1] && b.cf[a] > 0) {
                const int hv = b.ht[b.to[a]];
                hmin = hv < hmin ? hv : hmin;
            }
        }
        hmin = wave_min_i32(hmin);
        if (hmin >= hu) {
            const int nh = hmin >= b.n - 1 ? b.n : hmin + 1;
            if (lane() == 0) b.ht[u] = nh;
            if (nh < b.n) act++;
        } else {
            act++;
        }
    }
    if (lane() == 0 && act) atomicAdd(b.active, act);
}

// block-wide inclusive saturating scan of one value per thread; sW: BIG_WAVES entries
__device__ __forceinline__ int64_t block_scan_sat(int64_t c, int64_t *sW, int64_t *total) {
    const int wv = threadIdx.x / WAVE;
    int64_t inc = wave_incl_scan_sat(c);
    if (lane() == WAVE - 1) sW[wv] = inc;
    __syncthreads();
    int64_t before = 0;
    for (int w = 0; w < wv; w++) before = (before > SAT - sW[w]) ? SAT : before + sW[w];
    int64_t all = 0;
    for (int w = 0; w < BIG_WAVES; w++) all = (all > SAT - sW[w]) ? SAT : all + sW[w];
    __syncthreads();
    *total = all;
    return (inc > SAT - before) ? SAT : inc + before;
}

// push phase for the nodes with more than BIG_ARCS arcs: one block each
__global__ __launch_bounds__(BIG_BLOCK) void k_flow_push_big(FlowBufs b) {
    __shared__ int64_t sW[BIG_WAVES];
    __shared__ int64_t sEx;
    __shared__ int sHt;
    for (int i = blockIdx.x; i < b.nbig; i += gridDim.x) {
        const int u = b.big[i];
        if (u == b.s || u == b.t) continue;
        // one snapshot of the node for the whole block (others add to its
        // excess concurrently), so every thread takes the same path
        if (threadIdx.x == 0) {
            sHt = b.ht[u];
            sEx = b.ex[u];
        }
        __syncthreads();
        const int hu = sHt;
        int64_t rem = sEx;
        __syncthreads();
        if (rem <= 0 || hu >= b.n) continue;
        const int64_t start = rem;
        for (int a0 = b.first[u]; a0 < b.first[u + 1] && rem > 0; a0 += BIG_BLOCK) {
            const int a = a0 + threadIdx.x;
            int64_t c = 0;
            int v = -1;
            if (a < b.first[u + 1]) {
                v = b.to[a];
                const int64_t r = b.cf[a];
                if (r > 0 && b.ht[v] == hu - 1) c = r < rem ? r : rem;
            }
            int64_t total;
            const int64_t inc = block_scan_sat(c, sW, &total);
            const int64_t before = inc - c;
            int64_t d = rem - before;
            d = d < 0 ? 0 : (d > c ? c : d);
            if (d > 0) {
                b.cf[a] -= d;
                b.cf[b.rev[a]] += d;
                atomicAdd((unsigned long long *)&b.ex[v], (unsigned long long)d);
            }
            rem -= total < rem ? total : rem;
        }
        if (threadIdx.x == 0 && rem != start)
            atomicAdd((unsigned long long *)&b.ex[u], (unsigned long long)(rem - start));
    }
}

// relabel phase for the nodes with more than BIG_ARCS arcs: one block each;
// the scan stops once an admissible arc shows there is nothing to relabel
__global__ __launch_bounds__(BIG_BLOCK) void k_flow_relabel_big(FlowBufs b) {
    __shared__ int sMin[BIG_WAVES];
    __shared__ int sAdm;
    int act = 0;
    __shared__ int64_t sEx;
    __shared__ int sHt;
    for (int i = blockIdx.x; i < b.nbig; i += gridDim.x) {
        const int u = b.big[i];
        if (u == b.s || u == b.t) continue;
        if (threadIdx.x == 0) {
            sHt = b.ht[u];
            sEx = b.ex[u];
            sAdm = 0;
        }
        __syncthreads();
        const int hu = sHt;
        const int64_t eu = sEx;
        __syncthreads();
        if (eu <= 0 || hu >= b.n) continue;
        int hmin = 0x7fffffff;
        for (int a0 = b.first[u]; a0 < b.first[u + 1]; a0 += BIG_BLOCK) {
            const int a = a0 + threadIdx.x;
            if (a < b.first[u + 1] && b.cf[a] > 0) {
                const int hv = b.ht[b.to[a]];
                hmin = hv < hmin ? hv : hmin;
                if (hv < hu) sAdm = 1;
            }
            __syncthreads();
            const bool stop = sAdm != 0;        // the same value for every thread
            __syncthreads();                    // no thread writes sAdm before all have read it
            if (stop) break;
        }
        hmin = wave_min_i32(hmin);
        if (lane() == 0) sMin[threadIdx.x / WAVE] = hmin;
        __syncthreads();
        if (threadIdx.x == 0) {
            int m = 0x7fffffff;
            for (int w = 0; w < BIG_WAVES; w++) m = sMin[w] < m ? sMin[w] : m;
            if (!sAdm && m >= hu) {
                const int nh = m >= b.n - 1 ? b.n : m + 1;
                b.ht[u] = nh;
                if (nh < b.n) act++;
            } else {
                act++;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && act) atomicAdd(b.active, act);
}

__global__ void k_zero_i32(int *p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0;
}

__global__ void k_reach(FlowBufs b, uint8_t *out) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < b.n; v += gridDim.x * blockDim.x)
        out[v] = b.ht[v] < b.n ? 1 : 0;
}

}  // namespace

struct GpuFlow::Impl {
    hipStream_t s = nullptr;
    Scratch sc;
    FlowBufs b{};
    int64_t E = 0;
    int *eu = nullptr, *ev = nullptr, *fwd = nullptr;
    uint8_t *cls = nullptr;
    int64_t *deg = nullptr;
    int *pinned = nullptr;
    ~Impl() {
        if (s) (void)hipStreamSynchronize(s);
        if (pinned) (void)hipHostFree(pinned);
        if (s) (void)hipStreamDestroy(s);
    }
    int global_relabel();
};

GpuFlow::GpuFlow(int n, int64_t E, const int *eu, const int *ev, const uint8_t *cls, int nv,
                 const uint64_t *deg)
    : p_(new Impl) {
    Impl &I = *p_;
    DSD_HIP(hipStreamCreateWithFlags(&I.s, hipStreamNonBlocking));
    I.E = E;
    const int64_t A = 2 * E;
    FlowBufs &b = I.b;
    b.n = n;
    I.eu = I.sc.get_n<int>(E);
    I.ev = I.sc.get_n<int>(E);
    I.cls = I.sc.get_n<uint8_t>(E);
    I.deg = I.sc.get_n<int64_t>(nv);
    DSD_HIP(hipMemcpyAsync(I.eu, eu, (size_t)E * sizeof(int), hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(I.ev, ev, (size_t)E * sizeof(int), hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(I.cls, cls, (size_t)E, hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(I.deg, deg, (size_t)nv * sizeof(int64_t), hipMemcpyHostToDevice, I.s));
    // residual CSR: count, scan, fill
    uint32_t *cnt = I.sc.get_n<uint32_t>(n), *fill = I.sc.get_n<uint32_t>(n);
    int *first = I.sc.get_n<int>(n + 1);
    int *to = I.sc.get_n<int>(A), *rev = I.sc.get_n<int>(A);
    I.fwd = I.sc.get_n<int>(E);
    fill_i32((int32_t *)cnt, 0, n, I.s);
    // s, t and the vertex nodes take LDS counters when they fit
    const int hot = 2 + nv <= CSR_HOT ? 2 + nv : 0;
    const int gcsr = (int)std::min<int64_t>(1024, std::max<int64_t>(1, E / 4096));
    if (hot) k_csr_count_hot<<<gcsr, BLOCK, 0, I.s>>>(I.eu, I.ev, E, hot, cnt);
    else k_csr_count<<<grid_for(E, BLOCK, 16384), BLOCK, 0, I.s>>>(I.eu, I.ev, E, cnt);
    scan_exclusive_u32(cnt, (uint32_t *)first, n, I.s, I.sc);
    k_csr_last<<<1, 1, 0, I.s>>>(cnt, n, first);
    DSD_HIP(hipMemcpyAsync(fill, first, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, I.s));
    if (hot) k_csr_fill_hot<<<gcsr, BLOCK, 0, I.s>>>(I.eu, I.ev, E, hot, fill, to, rev, I.fwd);
    else k_csr_fill<<<grid_for(E, BLOCK, 16384), BLOCK, 0, I.s>>>(I.eu, I.ev, E, fill, to, rev, I.fwd);
    b.first = first;
    b.to = to;
    b.rev = rev;
    b.cf = I.sc.get_n<int64_t>(A);
    b.ex = I.sc.get_n<int64_t>(n);
    b.ht = I.sc.get_n<int>(n);
    b.front[0] = I.sc.get_n<int>(n);
    b.front[1] = I.sc.get_n<int>(n);
    b.nfront = I.sc.get_n<int>(2);
    b.active = I.sc.get_n<int>(1);
    // nodes with more than BIG_ARCS residual arcs
    std::vector<int> hfirst(n + 1);
    DSD_HIP(hipMemcpyAsync(hfirst.data(), first, (size_t)(n + 1) * sizeof(int), hipMemcpyDeviceToHost, I.s));
    DSD_HIP(hipStreamSynchronize(I.s));
    std::vector<int> big;
    for (int v = 0; v < n; v++)
        if (hfirst[v + 1] - hfirst[v] > BIG_ARCS) big.push_back(v);
    b.nbig = (int)big.size();
    int *d_big = I.sc.get_n<int>(b.nbig > 0 ? b.nbig : 1);
    if (b.nbig > 0)
        DSD_HIP(hipMemcpyAsync(d_big, big.data(), big.size() * sizeof(int), hipMemcpyHostToDevice, I.s));
    b.big = d_big;
    DSD_HIP(hipHostMalloc((void **)&I.pinned, 4 * sizeof(int), hipHostMallocDefault));
    DSD_HIP(hipStreamSynchronize(I.s));
}

GpuFlow::~GpuFlow() = default;

// global relabel (the scratch stays allocated until the Impl goes); returns
// the number of levels
int GpuFlow::Impl::global_relabel() {
    k_bfs_start<<<grid_for(b.n, BLOCK, 4096), BLOCK, 0, s>>>(b);
    int cur = 0, level = 0;
    while (true) {
        k_bfs_level<<<grid_for(b.n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, cur, level);
        if (b.nbig > 0) k_bfs_level_big<<<1024, BIG_BLOCK, 0, s>>>(b, cur, level);
        k_bfs_reset<<<1, 1, 0, s>>>(b, cur);
        DSD_HIP(hipMemcpyAsync(pinned, b.nfront + (cur ^ 1), sizeof(int), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        cur ^= 1;
        level++;
        if (pinned[0] == 0 || level > b.n) break;
    }
    return level;
}

int64_t GpuFlow::maxflow(const FlowTest &test, std::vector<char> &reach_t, int64_t max_passes, bool *converged) {
    Impl &I = *p_;
    FlowBufs &b = I.b;
    const int t = 1;
    b.s = 0;
    b.t = t;
    k_flow_caps<<<grid_for(I.E, BLOCK, 16384), BLOCK, 0, I.s>>>(b, I.eu, I.ev, I.cls, I.fwd, I.deg, I.E, test);
    k_flow_saturate<<<1, WAVE, 0, I.s>>>(b);
    I.global_relabel();
    const int gpass = grid_for(b.n, WAVES_PER_BLOCK, 16384);
    int64_t passes = 0;
    *converged = false;
    int since_relabel = 0;
    while (passes < max_passes) {
        for (int i = 0; i < 8; i++) {
            k_zero_i32<<<1, 1, 0, I.s>>>(b.active);
            k_flow_push<<<gpass, BLOCK, 0, I.s>>>(b);
            if (b.nbig > 0) k_flow_push_big<<<b.nbig < 4096 ? b.nbig : 4096, BIG_BLOCK, 0, I.s>>>(b);
            k_flow_relabel<<<gpass, BLOCK, 0, I.s>>>(b);
            if (b.nbig > 0) k_flow_relabel_big<<<b.nbig < 4096 ? b.nbig : 4096, BIG_BLOCK, 0, I.s>>>(b);
        }
        passes += 8;
        since_relabel += 8;
        DSD_HIP(hipMemcpyAsync(I.pinned, b.active, sizeof(int), hipMemcpyDeviceToHost, I.s));
        DSD_HIP(hipStreamSynchronize(I.s));
        if (I.pinned[0] == 0) {
            *converged = true;
            break;
        }
        if (since_relabel >= 32) {
            I.global_relabel();
            since_relabel = 0;
        }
    }
    int64_t flow = 0;
    DSD_HIP(hipMemcpyAsync(&flow, b.ex + t, sizeof(int64_t), hipMemcpyDeviceToHost, I.s));
    // the final search marks the nodes that still reach t
    I.global_relabel();
    uint8_t *r = I.sc.get_n<uint8_t>(b.n);
    k_reach<<<grid_for(b.n, BLOCK, 4096), BLOCK, 0, I.s>>>(b, r);
    std::vector<uint8_t> hr(b.n);
    DSD_HIP(hipMemcpyAsync(hr.data(), r, b.n, hipMemcpyDeviceToHost, I.s));
    DSD_HIP(hipStreamSynchronize(I.s));
    reach_t.assign(hr.begin(), hr.end());
    return flow;
}

}  // namespace dsd
