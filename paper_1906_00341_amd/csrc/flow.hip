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
    int *bfront[2];   // the frontier's nodes with more than BIG_ARCS arcs
    int *nbfront;     // [2] their numbers
    int *active;   // active node count
    int *act_s, *act_b;   // this pass's active nodes (up to / more than BIG_ARCS arcs)
    int *nact;            // [2] their numbers
    // A big node whose push scan saw every arc with excess left over (so it
    // saturated every admissible arc) records the lowest height behind the
    // arcs still residual after its pushes (rlm, with the pass in rlp); the
    // only residual arcs it did not see are those that nodes pushing into it
    // opened, whose heights are its own plus one (pin: the last pass that
    // pushed into the node).  Its relabel then needs no second scan.
    int *rlp, *rlm, *pin;
    int pass;
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

// ---- Algorithm 1's network for h = 3, built on the device ----
// Nodes: s = 0, t = 1, vertex i -> 2 + i, edge e -> 2 + nv + e.  Edges are
// numbered row by row: the edges (i, j), j > i, of row i (its forward part,
// from fwd[i] on) take ebase[i] .. ebase[i+1].  Arcs:
//   [0, nv)             s -> i
//   [nv, 2 nv)          i -> t
//   [2 nv, 2 nv + 2 np) edge (i, j) -> i and edge (i, j) -> j (infinite)
//   then for every edge (i, j) in edge order and every triangle {i, j, k},
//   k > j, in ascending k: i -> (j, k), j -> (i, k), k -> (i, j).

// the source, sink and infinite arcs (one wave per vertex)
__global__ __launch_bounds__(BLOCK) void k_tn_fixed(const int64_t *so, const int32_t *sa, const int64_t *fwd,
                                                     const int64_t *ebase, int nv, int *eu, int *ev, uint8_t *cls) {
    const int nw = gridDim.x * WAVES_PER_BLOCK;
    for (int i = blockIdx.x * WAVES_PER_BLOCK + threadIdx.x / WAVE; i < nv; i += nw) {
        if (lane() == 0) {
            eu[i] = 0;
            ev[i] = 2 + i;
            cls[i] = ARC_SRC;
            eu[nv + i] = 2 + i;
            ev[nv + i] = 1;
            cls[nv + i] = ARC_SNK;
        }
        const int64_t f0 = fwd[i], f1 = so[i + 1];
        for (int64_t a = f0 + lane(); a < f1; a += WAVE) {
            const int64_t e = ebase[i] + (a - f0);
            const int node = 2 + nv + (int)e;
            const int64_t at = 2 * (int64_t)nv + 2 * e;
            eu[at] = node;
            ev[at] = 2 + i;
            cls[at] = ARC_INF;
            eu[at + 1] = node;
            ev[at + 1] = 2 + sa[a];
            cls[at + 1] = ARC_INF;
        }
    }
}

// Triangles by their lowest vertex i: one workgroup per i keeps a bitmap of
// i's forward part in LDS (W words, and with EMIT the number of its bits
// before every word, so that the rank of k in the forward part is one
// lookup); each wave takes an edge (i, j) of the forward part and tests j's
// forward part against the bitmap 64 entries at a time.  Count pass: the
// triangles of every edge into tcnt.  Emit pass: with toff the exclusive
// scan of those counts, the three arcs of every triangle from arc m0 on.
template <bool EMIT>
__global__ __launch_bounds__(BLOCK) void k_tn_tri(const int64_t *so, const int32_t *sa, const int64_t *fwd,
                                                   const int64_t *ebase, int nv, int W, int64_t *tcnt,
                                                   const int64_t *toff, int64_t m0, int *eu, int *ev,
                                                   uint8_t *cls) {
    extern __shared__ uint32_t tn_lds[];
    __shared__ uint32_t wsum[WAVES_PER_BLOCK];
    uint32_t *bm = tn_lds, *pre = tn_lds + W;
    const int wid = threadIdx.x / WAVE;
    for (int i = blockIdx.x; i < nv; i += gridDim.x) {
        const int64_t f0 = fwd[i], f1 = so[i + 1];
        if (f1 - f0 < 2) {   // no triangle has i as its lowest vertex
            if (!EMIT)
                for (int64_t a = f0 + threadIdx.x; a < f1; a += BLOCK) tcnt[ebase[i] + (a - f0)] = 0;
            continue;
        }
        for (int w = threadIdx.x; w < W; w += BLOCK) bm[w] = 0;
        __syncthreads();
        for (int64_t a = f0 + threadIdx.x; a < f1; a += BLOCK) {
            const int k = sa[a];
            atomicOr(&bm[k >> 5], 1u << (k & 31));
        }
        __syncthreads();
        if (EMIT) {
            // pre[w] = bits set in words before w: each thread sums a run of
            // words, then a block scan of the run totals
            const int per = (W + BLOCK - 1) / BLOCK;
            const int w0 = min(W, (int)threadIdx.x * per), w1 = min(W, w0 + per);
            uint32_t own = 0;
            for (int w = w0; w < w1; w++) own += __popc(bm[w]);
            const uint32_t inc = wave_incl_scan(own);
            if (lane() == WAVE - 1) wsum[wid] = inc;
            __syncthreads();
            uint32_t run = inc - own;
            for (int x = 0; x < wid; x++) run += wsum[x];
            for (int w = w0; w < w1; w++) {
                pre[w] = run;
                run += __popc(bm[w]);
            }
            __syncthreads();
        }
        for (int64_t a = f0 + wid; a < f1; a += WAVES_PER_BLOCK) {
            const int j = sa[a];
            const int64_t e = ebase[i] + (a - f0);
            const int64_t g0 = fwd[j], g1 = so[j + 1];
            int64_t pos = EMIT ? toff[e] : 0;
            for (int64_t q0 = g0; q0 < g1; q0 += WAVE) {
                const int64_t q = q0 + lane();
                int k = 0;
                bool hit = false;
                if (q < g1) {
                    k = sa[q];
                    hit = (bm[k >> 5] >> (k & 31)) & 1u;
                }
                const u64 m = __ballot(hit);
                if (EMIT && hit) {
                    const int64_t at = m0 + 3 * (pos + __popcll(m & lanemask_lt()));
                    const uint32_t below = bm[k >> 5] & ((1u << (k & 31)) - 1u);
                    const int64_t p = (int64_t)pre[k >> 5] + __popc(below);   // rank of k in i's forward part
                    eu[at] = 2 + i;
                    ev[at] = 2 + nv + (int)(ebase[j] + (q - g0));
                    eu[at + 1] = 2 + j;
                    ev[at + 1] = 2 + nv + (int)(ebase[i] + p);
                    eu[at + 2] = 2 + k;
                    ev[at + 2] = 2 + nv + (int)e;
                    cls[at] = ARC_MID;
                    cls[at + 1] = ARC_MID;
                    cls[at + 2] = ARC_MID;
                }
                pos += __popcll(m);
            }
            if (!EMIT && lane() == 0) tcnt[e] = pos;
        }
        __syncthreads();   // the next vertex rewrites the bitmap
    }
}

// triangles through vertex i: its residual row holds the reverse of s -> i,
// i -> t, one infinite arc per edge at i and one arc per triangle at i
__global__ void k_tn_deg(const int *first, const int64_t *so, int nv, int64_t *deg) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x)
        deg[i] = (int64_t)(first[3 + i] - first[2 + i]) - 2 - (so[i + 1] - so[i]);
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
        const bool big = b.first[b.t + 1] - b.first[b.t] > BIG_ARCS;
        (big ? b.bfront : b.front)[0][0] = b.t;
        b.nfront[0] = big ? 0 : 1;
        b.nbfront[0] = big ? 1 : 0;
        b.nfront[1] = 0;
        b.nbfront[1] = 0;
    }
}

// a newly labelled node u joins the next frontier of its kind (all lanes
// of the wave call this together)
__device__ __forceinline__ void bfs_push(const FlowBufs &b, bool take, int u, int nx) {
    const bool big = take && b.first[u + 1] - b.first[u] > BIG_ARCS;
    const u64 ms = __ballot(take && !big), mb = __ballot(big);
    const int leader_s = ms ? __builtin_ctzll(ms) : 0, leader_b = mb ? __builtin_ctzll(mb) : 0;
    int base_s = 0, base_b = 0;
    if (ms && lane() == leader_s) base_s = atomicAdd(&b.nfront[nx], __popcll(ms));
    if (mb && lane() == leader_b) base_b = atomicAdd(&b.nbfront[nx], __popcll(mb));
    base_s = __shfl(base_s, leader_s, WAVE);
    base_b = __shfl(base_b, leader_b, WAVE);
    if (take && !big) b.front[nx][base_s + __popcll(ms & lanemask_lt())] = u;
    if (big) b.bfront[nx][base_b + __popcll(mb & lanemask_lt())] = u;
}

// one level: every node of front[cur] (height `level`; the frontier nodes
// with at most BIG_ARCS arcs) labels its unlabelled
// in-neighbours (u with a residual arc u -> v) level + 1
__global__ __launch_bounds__(BLOCK) void k_bfs_level(FlowBufs b, int cur, int level) {
    const int nf = b.nfront[cur];
    const int *F = b.front[cur];
    const int wv = threadIdx.x / WAVE;
    for (int i = blockIdx.x * WAVES_PER_BLOCK + wv; i < nf; i += gridDim.x * WAVES_PER_BLOCK) {
        const int v = F[i];
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
            if (__ballot(take)) bfs_push(b, take, u, cur ^ 1);
        }
    }
}

// the same for frontier nodes with more than BIG_ARCS arcs: one block each
__global__ __launch_bounds__(BIG_BLOCK) void k_bfs_level_big(FlowBufs b, int cur, int level) {
    const int nf = b.nbfront[cur];
    const int *F = b.bfront[cur];
    constexpr int K = 4;   // arcs per thread per step: their loads go out together
    for (int i = blockIdx.x; i < nf; i += gridDim.x) {
        const int v = F[i];
        const int end = b.first[v + 1];
        for (int a0 = b.first[v]; a0 < end; a0 += BIG_BLOCK * K) {
            int u[K];
            bool cand[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int a = a0 + k * BIG_BLOCK + threadIdx.x;
                u[k] = -1;
                cand[k] = false;
                if (a < end) {
                    u[k] = b.to[a];
                    cand[k] = u[k] != b.s && b.cf[b.rev[a]] > 0 && b.ht[u[k]] == b.n;
                }
            }
#pragma unroll
            for (int k = 0; k < K; k++) {
                const bool take = cand[k] && atomicCAS(&b.ht[u[k]], b.n, level + 1) == b.n;
                if (__ballot(take)) bfs_push(b, take, u[k], cur ^ 1);
            }
        }
    }
}

__global__ void k_bfs_reset(FlowBufs b, int cur) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.nfront[cur] = 0;
        b.nbfront[cur] = 0;
    }
}

// The active nodes of a pass (excess > 0, height < n, not s or t), listed
// once so that the pass's kernels walk the list rather than every node: a
// few hundred nodes stay active for most of the passes.  nact (two
// counters) must be zero on entry.
__device__ __forceinline__ void flow_list_push(bool pred, int u, int *list, int *count) {
    const u64 m = __ballot(pred);
    if (!m) return;
    const int leader = __builtin_ctzll(m);
    int base = 0;
    if (lane() == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader, WAVE);
    if (pred) list[base + __popcll(m & lanemask_lt())] = u;
}

__global__ __launch_bounds__(BLOCK) void k_flow_active(FlowBufs b) {
    const int stride = gridDim.x * BLOCK;
    const int lim = (b.n + WAVE - 1) / WAVE * WAVE;   // whole waves take part in the ballots
    for (int u = blockIdx.x * BLOCK + threadIdx.x; u - lane() < lim; u += stride) {
        bool act = false, big = false;
        if (u < b.n && u != b.s && u != b.t) {
            act = b.ex[u] > 0 && b.ht[u] < b.n;
            big = b.first[u + 1] - b.first[u] > BIG_ARCS;
        }
        flow_list_push(act && !big, u, b.act_s, &b.nact[0]);
        flow_list_push(act && big, u, b.act_b, &b.nact[1]);
    }
}

__global__ void k_zero_act(FlowBufs b) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.nact[0] = 0;
        b.nact[1] = 0;
    }
}

// push phase: heights are read-only here (nodes up to BIG_ARCS arcs, from
// the pass's active list)
__global__ __launch_bounds__(BLOCK) void k_flow_push(FlowBufs b) {
    const int wv = threadIdx.x / WAVE;
    const int na = b.nact[0];
    for (int i = blockIdx.x * WAVES_PER_BLOCK + wv; i < na; i += gridDim.x * WAVES_PER_BLOCK) {
        const int u = b.act_s[i];
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
                b.pin[v] = b.pass;
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
    const int na = b.nact[0];
    for (int i = blockIdx.x * WAVES_PER_BLOCK + wv; i < na; i += gridDim.x * WAVES_PER_BLOCK) {
        const int u = b.act_s[i];
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
    constexpr int K = 4;   // arcs per thread per step: their loads go out together
    __shared__ int64_t sW[BIG_WAVES];
    __shared__ int sMn[BIG_WAVES];
    __shared__ int64_t sEx;
    __shared__ int sHt;
    const int na = b.nact[1];
    for (int i = blockIdx.x; i < na; i += gridDim.x) {
        const int u = b.act_b[i];
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
        const int end = b.first[u + 1];
        int hmin = 0x7fffffff;   // heights behind this thread's arcs still residual after the pushes
        for (int a0 = b.first[u]; a0 < end && rem > 0; a0 += BIG_BLOCK * K) {
            int64_t c[K], r[K];
            int v[K], hv[K];
            int64_t own = 0;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int a = a0 + k * BIG_BLOCK + threadIdx.x;
                c[k] = 0;
                r[k] = 0;
                v[k] = -1;
                hv[k] = 0x7fffffff;
                if (a < end) {
                    v[k] = b.to[a];
                    r[k] = b.cf[a];
                    if (r[k] > 0) {
                        hv[k] = b.ht[v[k]];
                        if (hv[k] == hu - 1) c[k] = r[k] < rem ? r[k] : rem;
                    }
                }
                own = (own > SAT - c[k]) ? SAT : own + c[k];
            }
            if (!__syncthreads_or(own > 0)) {   // no admissible arc in this step
#pragma unroll
                for (int k = 0; k < K; k++)
                    if (r[k] > 0 && hv[k] < hmin) hmin = hv[k];
                continue;
            }
            int64_t total;
            const int64_t inc = block_scan_sat(own, sW, &total);
            int64_t before = inc - own;
#pragma unroll
            for (int k = 0; k < K; k++) {
                int64_t d = rem - before;
                d = d < 0 ? 0 : (d > c[k] ? c[k] : d);
                if (d > 0) {
                    const int a = a0 + k * BIG_BLOCK + threadIdx.x;
                    b.cf[a] -= d;
                    b.cf[b.rev[a]] += d;
                    atomicAdd((unsigned long long *)&b.ex[v[k]], (unsigned long long)d);
                    b.pin[v[k]] = b.pass;
                }
                if (r[k] - d > 0 && hv[k] < hmin) hmin = hv[k];
                before = (before > SAT - c[k]) ? SAT : before + c[k];
            }
            rem -= total < rem ? total : rem;
        }
        if (threadIdx.x == 0 && rem != start)
            atomicAdd((unsigned long long *)&b.ex[u], (unsigned long long)(rem - start));
        if (rem > 0) {   // (the same for every thread) every arc seen, every admissible one saturated
            hmin = wave_min_i32(hmin);
            if (lane() == 0) sMn[threadIdx.x / WAVE] = hmin;
            __syncthreads();
            if (threadIdx.x == 0) {
                int m = 0x7fffffff;
                for (int w = 0; w < BIG_WAVES; w++) m = sMn[w] < m ? sMn[w] : m;
                b.rlm[u] = m;
                b.rlp[u] = b.pass;
            }
        }
    }
}

// relabel phase for the nodes with more than BIG_ARCS arcs: one block each;
// the scan stops once an admissible arc shows there is nothing to relabel
__global__ __launch_bounds__(BIG_BLOCK) void k_flow_relabel_big(FlowBufs b) {
    __shared__ int sMin[BIG_WAVES];
    __shared__ int sAdm;
    int act = 0;
    __shared__ int64_t sEx;
    __shared__ int sHt, sFast, sPin;
    const int na = b.nact[1];
    for (int i = blockIdx.x; i < na; i += gridDim.x) {
        const int u = b.act_b[i];
        if (u == b.s || u == b.t) continue;
        if (threadIdx.x == 0) {
            sHt = b.ht[u];
            sEx = b.ex[u];
            sAdm = 0;
            sFast = b.rlp[u] == b.pass ? 1 : 0;
            sPin = b.pin[u] == b.pass ? 1 : 0;
        }
        __syncthreads();
        const int hu = sHt;
        const int64_t eu = sEx;
        const bool fast = sFast != 0, pin = sPin != 0;
        __syncthreads();
        if (eu <= 0 || hu >= b.n) continue;
        if (fast) {
            // the push scan saw every arc: the lowest residual neighbour is
            // the one it recorded, or one that pushed into the node
            if (threadIdx.x == 0) {
                int m = b.rlm[u];
                if (pin && hu + 1 < m) m = hu + 1;
                if (m >= hu) {
                    const int nh = m >= b.n - 1 ? b.n : m + 1;
                    b.ht[u] = nh;
                    if (nh < b.n) act++;
                } else {
                    act++;
                }
            }
            continue;
        }
        int hmin = 0x7fffffff;
        constexpr int K = 4;   // arcs per thread per step: their loads go out together
        const int end = b.first[u + 1];
        for (int a0 = b.first[u]; a0 < end; a0 += BIG_BLOCK * K) {
            bool adm = false;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int a = a0 + k * BIG_BLOCK + threadIdx.x;
                if (a < end && b.cf[a] > 0) {
                    const int hv = b.ht[b.to[a]];
                    hmin = hv < hmin ? hv : hmin;
                    adm = adm || hv < hu;
                }
            }
            if (__syncthreads_or(adm)) {   // the same value for every thread
                if (threadIdx.x == 0) sAdm = 1;
                break;
            }
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
    int *pinned = nullptr;   // the thread's pinned buffer
    int nv = 0;
    ~Impl() {
        if (s) (void)hipStreamSynchronize(s);
        sc.recycle();
        if (s) (void)hipStreamDestroy(s);
    }
    int global_relabel();
    void residual(int n);
};

GpuFlow::GpuFlow() : p_(new Impl) { DSD_HIP(hipStreamCreateWithFlags(&p_->s, hipStreamNonBlocking)); }

GpuFlow::GpuFlow(int n, int64_t E, const int *eu, const int *ev, const uint8_t *cls, int nv,
                 const uint64_t *deg)
    : GpuFlow() {
    Impl &I = *p_;
    I.E = E;
    I.nv = nv;
    I.eu = I.sc.get_n<int>(E);
    I.ev = I.sc.get_n<int>(E);
    I.cls = I.sc.get_n<uint8_t>(E);
    I.deg = I.sc.get_n<int64_t>(nv);
    DSD_HIP(hipMemcpyAsync(I.eu, eu, (size_t)E * sizeof(int), hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(I.ev, ev, (size_t)E * sizeof(int), hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(I.cls, cls, (size_t)E, hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(I.deg, deg, (size_t)nv * sizeof(int64_t), hipMemcpyHostToDevice, I.s));
    I.residual(n);
}

std::unique_ptr<GpuFlow> GpuFlow::triangles(int nv, const int64_t *so, const int32_t *sa, const int64_t *fwd,
                                            std::vector<uint64_t> &deg, uint64_t *tri) {
    if (nv < 1 || nv > TRI_NET_MAX_NV) throw Error(-5, "triangle network: vertex count out of range");
    std::unique_ptr<GpuFlow> g(new GpuFlow());
    Impl &I = *g->p_;
    I.nv = nv;
    const int64_t ns = so[nv];
    std::vector<int64_t> ebase(nv + 1, 0);
    for (int i = 0; i < nv; i++) ebase[i + 1] = ebase[i] + (so[i + 1] - fwd[i]);
    const int64_t np = ebase[nv];
    if (2 + (int64_t)nv + np > 0x7fffffff) throw Error(-5, "flow network too large");
    int64_t *d_so = I.sc.get_n<int64_t>(nv + 1), *d_fwd = I.sc.get_n<int64_t>(nv);
    int64_t *d_eb = I.sc.get_n<int64_t>(nv + 1), *tcnt = I.sc.get_n<int64_t>(np + 1);
    int32_t *d_sa = I.sc.get_n<int32_t>(ns);
    DSD_HIP(hipMemcpyAsync(d_so, so, (size_t)(nv + 1) * sizeof(int64_t), hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(d_fwd, fwd, (size_t)nv * sizeof(int64_t), hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipMemcpyAsync(d_eb, ebase.data(), (size_t)(nv + 1) * sizeof(int64_t), hipMemcpyHostToDevice, I.s));
    if (ns > 0) DSD_HIP(hipMemcpyAsync(d_sa, sa, (size_t)ns * sizeof(int32_t), hipMemcpyHostToDevice, I.s));
    const int W = (nv + 31) / 32;
    const size_t lds = (size_t)2 * W * sizeof(uint32_t);
    // triangles per edge, then their offsets (tcnt[np] = total)
    k_tn_tri<false><<<nv, BLOCK, lds, I.s>>>(d_so, d_sa, d_fwd, d_eb, nv, W, tcnt, nullptr, 0, nullptr, nullptr,
                                             nullptr);
    fill_i32((int32_t *)(tcnt + np), 0, 2, I.s);
    scan_exclusive_i64(tcnt, tcnt, np + 1, I.s, I.sc);
    int64_t total = 0;
    DSD_HIP(hipMemcpyAsync(&total, tcnt + np, sizeof(int64_t), hipMemcpyDeviceToHost, I.s));
    DSD_HIP(hipStreamSynchronize(I.s));
    const int64_t m0 = 2 * (int64_t)nv + 2 * np;
    if (m0 > 0x7fffffff / 2 || total > (0x7fffffff / 2 - m0) / 3) throw Error(-5, "flow network too large");
    const int64_t E = m0 + 3 * total;
    I.E = E;
    I.eu = I.sc.get_n<int>(E);
    I.ev = I.sc.get_n<int>(E);
    I.cls = I.sc.get_n<uint8_t>(E);
    I.deg = I.sc.get_n<int64_t>(nv);
    k_tn_fixed<<<grid_for(nv, WAVES_PER_BLOCK, 16384), BLOCK, 0, I.s>>>(d_so, d_sa, d_fwd, d_eb, nv, I.eu, I.ev,
                                                                        I.cls);
    if (total > 0)
        k_tn_tri<true><<<nv, BLOCK, lds, I.s>>>(d_so, d_sa, d_fwd, d_eb, nv, W, nullptr, tcnt, m0, I.eu, I.ev,
                                                I.cls);
    I.residual((int)(2 + nv + np));
    k_tn_deg<<<grid_for(nv, BLOCK, 4096), BLOCK, 0, I.s>>>(I.b.first, d_so, nv, I.deg);
    deg.resize(nv);
    DSD_HIP(hipMemcpyAsync(deg.data(), I.deg, (size_t)nv * sizeof(int64_t), hipMemcpyDeviceToHost, I.s));
    DSD_HIP(hipStreamSynchronize(I.s));
    *tri = (uint64_t)total;
    return g;
}

uint64_t count_triangles_device(int nv, const int64_t *so, const int32_t *sa, const int64_t *fwd) {
    if (nv < 1 || nv > TRI_NET_MAX_NV) throw Error(-5, "triangle count: vertex count out of range");
    std::vector<int64_t> ebase(nv + 1, 0);
    for (int i = 0; i < nv; i++) ebase[i + 1] = ebase[i] + (so[i + 1] - fwd[i]);
    const int64_t np = ebase[nv], ns = so[nv];
    if (np == 0) return 0;
    hipStream_t s = nullptr;
    DSD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    uint64_t total[2] = {0, 0};
    try {
        Scratch sc;
        int64_t *d_so = sc.get_n<int64_t>(nv + 1), *d_fwd = sc.get_n<int64_t>(nv);
        int64_t *d_eb = sc.get_n<int64_t>(nv + 1), *tcnt = sc.get_n<int64_t>(np);
        int32_t *d_sa = sc.get_n<int32_t>(ns);
        u64 *d_tot = sc.get_n<u64>(2);
        DSD_HIP(hipMemcpyAsync(d_so, so, (size_t)(nv + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        DSD_HIP(hipMemcpyAsync(d_fwd, fwd, (size_t)nv * sizeof(int64_t), hipMemcpyHostToDevice, s));
        DSD_HIP(hipMemcpyAsync(d_eb, ebase.data(), (size_t)(nv + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        DSD_HIP(hipMemcpyAsync(d_sa, sa, (size_t)ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
        const int W = (nv + 31) / 32;
        k_tn_tri<false><<<nv, BLOCK, (size_t)2 * W * sizeof(uint32_t), s>>>(d_so, d_sa, d_fwd, d_eb, nv, W, tcnt,
                                                                            nullptr, 0, nullptr, nullptr, nullptr);
        sum_u64_128((const u64 *)tcnt, np, d_tot, s, sc);
        DSD_HIP(hipMemcpyAsync(total, d_tot, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamDestroy(s);
        throw;
    }
    DSD_HIP(hipStreamDestroy(s));
    return total[0];
}

int GpuFlow::nodes() const { return p_->b.n; }
int64_t GpuFlow::arcs() const { return p_->E; }

void GpuFlow::download_arcs(int *eu, int *ev) const {
    Impl &I = *p_;
    DSD_HIP(hipMemcpyAsync(eu, I.eu, (size_t)I.E * sizeof(int), hipMemcpyDeviceToHost, I.s));
    DSD_HIP(hipMemcpyAsync(ev, I.ev, (size_t)I.E * sizeof(int), hipMemcpyDeviceToHost, I.s));
    DSD_HIP(hipStreamSynchronize(I.s));
}

void GpuFlow::force_sources(const std::vector<char> &forced) {
    Impl &I = *p_;
    if ((int)forced.size() != I.nv) throw Error(-5, "force_sources: one flag per vertex expected");
    std::vector<uint8_t> c(I.nv);
    for (int i = 0; i < I.nv; i++) c[i] = forced[i] ? ARC_INF : ARC_SRC;
    DSD_HIP(hipMemcpyAsync(I.cls, c.data(), (size_t)I.nv, hipMemcpyHostToDevice, I.s));
    DSD_HIP(hipStreamSynchronize(I.s));
}

// residual CSR of the E arcs in eu/ev: count, scan, fill
void GpuFlow::Impl::residual(int n) {
    Impl &I = *this;
    const int64_t A = 2 * E;
    b.n = n;
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
    b.bfront[0] = I.sc.get_n<int>(n);
    b.bfront[1] = I.sc.get_n<int>(n);
    b.nbfront = I.sc.get_n<int>(2);
    b.active = I.sc.get_n<int>(1);
    b.act_s = I.sc.get_n<int>(n);
    b.act_b = I.sc.get_n<int>(n);
    b.nact = I.sc.get_n<int>(2);
    b.rlp = I.sc.get_n<int>(n);
    b.rlm = I.sc.get_n<int>(n);
    b.pin = I.sc.get_n<int>(n);
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
    I.pinned = (int *)thread_pinned();
    DSD_HIP(hipStreamSynchronize(I.s));
}

GpuFlow::~GpuFlow() = default;

// global relabel (the scratch stays allocated until the Impl goes); returns
// the number of levels launched (a multiple of eight)
int GpuFlow::Impl::global_relabel() {
    k_bfs_start<<<grid_for(b.n, BLOCK, 4096), BLOCK, 0, s>>>(b);
    // levels go out eight at a time (a level whose frontier is empty does
    // nothing), and the host looks at the frontier after each batch
    int cur = 0, level = 0;
    while (true) {
        for (int j = 0; j < 8; j++) {
            k_bfs_level<<<grid_for(b.n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(b, cur, level);
            if (b.nbig > 0) k_bfs_level_big<<<b.nbig < 1024 ? b.nbig : 1024, BIG_BLOCK, 0, s>>>(b, cur, level);
            k_bfs_reset<<<1, 1, 0, s>>>(b, cur);
            cur ^= 1;
            level++;
        }
        DSD_HIP(hipMemcpyAsync(pinned, b.nfront + cur, sizeof(int), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(pinned + 1, b.nbfront + cur, sizeof(int), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        if ((pinned[0] == 0 && pinned[1] == 0) || level > b.n) break;
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
    fill_i32(b.rlp, -1, b.n, I.s);
    fill_i32(b.pin, -1, b.n, I.s);
    I.global_relabel();
    // a pass: list the active nodes, push, relabel; the passes' kernels
    // walk the lists with grids sized for the busy first passes
    const int gpass = grid_for(b.n, WAVES_PER_BLOCK, 2048), gact = grid_for(b.n, BLOCK, 1024);
    const int gbig = b.nbig < 4096 ? b.nbig : 4096;
    int64_t passes = 0;
    *converged = false;
    int since_relabel = 0;
    // The list made after a pass's pushes serves its relabels and the next
    // pass's pushes (relabelling adds no excess; a node raised to n is
    // skipped by the push).
    auto list_active = [&]() {
        k_zero_act<<<1, 1, 0, I.s>>>(b);
        k_flow_active<<<gact, BLOCK, 0, I.s>>>(b);
    };
    list_active();
    while (passes < max_passes) {
        for (int i = 0; i < 8; i++) {
            b.pass = (int)(passes + i);
            k_flow_push<<<gpass, BLOCK, 0, I.s>>>(b);
            if (b.nbig > 0) k_flow_push_big<<<gbig, BIG_BLOCK, 0, I.s>>>(b);
            list_active();
            k_flow_relabel<<<gpass, BLOCK, 0, I.s>>>(b);
            if (b.nbig > 0) k_flow_relabel_big<<<gbig, BIG_BLOCK, 0, I.s>>>(b);
        }
        passes += 8;
        since_relabel += 8;
        // converged when no node was active after the last pass's pushes
        DSD_HIP(hipMemcpyAsync(I.pinned, b.nact, 2 * sizeof(int), hipMemcpyDeviceToHost, I.s));
        DSD_HIP(hipStreamSynchronize(I.s));
        if (I.pinned[0] + I.pinned[1] == 0) {
            *converged = true;
            break;
        }
        if (since_relabel >= 32) {
            I.global_relabel();
            since_relabel = 0;
            list_active();   // heights changed: nodes that cannot reach t leave the list
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
