// K1 (CSR build) and K2 (degree-ordered DAG orientation).
//
// The paper's data model is a simple undirected graph (Section 3).  Raw pairs
// are canonicalised to (min, max) keys, radix-sorted and de-duplicated; the
// degree order (deg, id) ascending gives every vertex a rank; the edges are
// re-keyed in rank space in both directions and sorted again, which yields a
// CSR whose rows are sorted by rank.  The out-neighbours of r in the DAG
// u -> v iff (deg u, u) < (deg v, v) are then the tail of row r.  Listing
// each clique from its lowest-rank member is the ordered enumeration the
// paper borrows for Algorithm 3 (Section 5.3); the degree order keeps the
// out-degrees small.
#include "graph.hpp"

namespace dsd {

static int bits_for(int64_t n) {
    int b = 1;
    while (((int64_t)1 << b) - 1 < n) b++;
    return b;   // n <= 2^b - 1, so every id < 2^b - 1
}

__global__ void k_pair_keys(const int32_t *src, const int32_t *dst, int64_t P, int32_t n, int bits, u64 *keys,
                            int32_t *bad) {
    const u64 invalid = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1ull);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            *bad = 1;
            keys[i] = invalid;
            continue;
        }
        if (u == v) { keys[i] = invalid; continue; }
        u64 a = (u64)(u < v ? u : v), b = (u64)(u < v ? v : u);
        keys[i] = (a << bits) | b;
    }
}

// flags[i] = 1 if keys[i] is a valid key that differs from its predecessor
__global__ void k_unique_flags(const u64 *keys, int64_t P, u64 invalid, int64_t *flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        u64 k = keys[i];
        flags[i] = (k != invalid && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
    }
}

__global__ void k_unique_compact(const u64 *keys, int64_t P, u64 invalid, const int64_t *pos, u64 *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        u64 k = keys[i];
        if (k != invalid && (i == 0 || keys[i - 1] != k)) out[pos[i]] = k;
    }
}

__global__ void k_edge_degrees(const u64 *edges, int64_t m, int bits, int32_t *deg) {
    const u64 mask = (1ull << bits) - 1ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        u64 k = edges[i];
        atomicAdd(&deg[(int32_t)(k >> bits)], 1);
        atomicAdd(&deg[(int32_t)(k & mask)], 1);
    }
}

__global__ void k_rank_keys(const int32_t *deg, int32_t n, int bits, u64 *keys) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        keys[v] = ((u64)deg[v] << bits) | (u64)v;
}

__global__ void k_rank_perm(const u64 *keys, int32_t n, int bits, int32_t *orig_of, int32_t *rank_of) {
    const u64 mask = (1ull << bits) - 1ull;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = (int32_t)(keys[r] & mask);
        orig_of[r] = v;
        rank_of[v] = (int32_t)r;
    }
}

// K2: re-key every edge in rank space, both directions
__global__ void k_orient_keys(const u64 *edges, int64_t m, int bits, const int32_t *rank_of, u64 *keys) {
    const u64 mask = (1ull << bits) - 1ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        u64 k = edges[i];
        u64 ru = (u64)rank_of[(int32_t)(k >> bits)];
        u64 rv = (u64)rank_of[(int32_t)(k & mask)];
        keys[2 * i] = (ru << bits) | rv;
        keys[2 * i + 1] = (rv << bits) | ru;
    }
}

// col from the sorted keys; row_ptr by row boundaries (empty rows included)
__global__ void k_csr_from_keys(const u64 *keys, int64_t E, int32_t n, int bits, int32_t *col, int64_t *row_ptr) {
    const u64 mask = (1ull << bits) - 1ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= E; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t cur = (i == E) ? (int64_t)n : (int64_t)(keys[i] >> bits);
        int64_t prev = (i == 0) ? -1 : (int64_t)(keys[i - 1] >> bits);
        if (i < E) col[i] = (int32_t)(keys[i] & mask);
        for (int64_t q = prev + 1; q <= cur; q++) row_ptr[q] = i;
    }
}

// dag_off[r] = first position of row r holding a rank > r; also max degrees
__global__ void k_dag_off(const int64_t *row_ptr, const int32_t *col, int32_t n, int64_t *dag_off, int32_t *maxes) {
    int32_t md = 0, mo = 0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = row_ptr[r], hi = row_ptr[r + 1], e = hi;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (col[mid] > (int32_t)r) hi = mid; else lo = mid + 1;
        }
        dag_off[r] = lo;
        int32_t d = (int32_t)(e - row_ptr[r]), o = (int32_t)(e - lo);
        md = d > md ? d : md;
        mo = o > mo ? o : mo;
    }
    md = wave_max(md);
    mo = wave_max(mo);
    if (lane() == 0) {
        atomicMax(&maxes[0], md);
        atomicMax(&maxes[1], mo);
    }
}

__global__ void k_wedges(const int64_t *row_ptr, const int64_t *dag_off, int32_t n, u64 *out) {
    u64 w2 = 0, s2 = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        u64 din = (u64)(dag_off[v] - row_ptr[v]), dout = (u64)(row_ptr[v + 1] - dag_off[v]);
        w2 += din * dout;
        s2 += (din + dout) * dout;
    }
    w2 = wave_sum(w2);
    s2 = wave_sum(s2);
    if (lane() == 0) {
        atomicAdd(&out[0], w2);
        atomicAdd(&out[1], s2);
    }
}

void build_graph(int32_t n, int64_t P, const int32_t *src, const int32_t *dst, DevGraph &g, hipStream_t s,
                 Scratch &sc, float *t_orient_ms, Scratch *keep) {
    g.n = n;
    g.bits = bits_for(n > 0 ? n : 1);
    const int bits = g.bits;
    const u64 invalid = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1ull);
    int64_t m = 0;
    int32_t *d_bad = sc.get_n<int32_t>(4);
    fill_i32(d_bad, 0, 4, s);
    u64 *edges = nullptr;
    if (P > 0) {
        u64 *keys = sc.get_n<u64>(P), *tmp = sc.get_n<u64>(P);
        k_pair_keys<<<grid_for(P, BLOCK, 8192), BLOCK, 0, s>>>(src, dst, P, n, bits, keys, d_bad);
        radix_sort_u64(keys, tmp, P, 2 * bits, s, sc);
        int64_t *pos = sc.get_n<int64_t>(P);
        k_unique_flags<<<grid_for(P, BLOCK, 8192), BLOCK, 0, s>>>(keys, P, invalid, pos);
        scan_exclusive_i64(pos, pos, P, s, sc);
        int64_t last_pos = 0;
        u64 last_key = 0, prev_key = 0;
        DSD_HIP(hipMemcpyAsync(&last_pos, pos + P - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(&last_key, keys + P - 1, sizeof(u64), hipMemcpyDeviceToHost, s));
        if (P > 1) DSD_HIP(hipMemcpyAsync(&prev_key, keys + P - 2, sizeof(u64), hipMemcpyDeviceToHost, s));
        int32_t bad = 0;
        DSD_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        if (bad) throw Error(-1, "vertex id outside [0, n)");
        m = last_pos + ((last_key != invalid && (P == 1 || prev_key != last_key)) ? 1 : 0);
        edges = tmp;   // reuse: unique keys
        if (m > 0) k_unique_compact<<<grid_for(P, BLOCK, 8192), BLOCK, 0, s>>>(keys, P, invalid, pos, edges);
    }
    g.m = m;
    const int64_t E = 2 * m;
    if (E > (int64_t)0x7fffffff) throw Error(-5, "more than 2^31-1 adjacency entries");
    hipEvent_t e0, e1;
    DSD_HIP(hipEventCreate(&e0));
    DSD_HIP(hipEventCreate(&e1));
    DSD_HIP(hipEventRecord(e0, s));
    // degrees in caller ids -> rank order
    int32_t *deg = sc.get_n<int32_t>(n);
    if (keep) {
        g.owned = false;
        g.row_ptr = keep->get_n<int64_t>((int64_t)n + 1);
        g.col = keep->get_n<int32_t>(E);
        g.dag_off = keep->get_n<int64_t>(n);
        g.orig_of = keep->get_n<int32_t>(n);
        g.rank_of = keep->get_n<int32_t>(n);
    } else {
        g.owned = true;
        DSD_HIP(hipMalloc(&g.row_ptr, ((size_t)n + 1) * sizeof(int64_t)));
        DSD_HIP(hipMalloc(&g.col, (size_t)(E > 0 ? E : 1) * sizeof(int32_t)));
        DSD_HIP(hipMalloc(&g.dag_off, (size_t)(n > 0 ? n : 1) * sizeof(int64_t)));
        DSD_HIP(hipMalloc(&g.orig_of, (size_t)(n > 0 ? n : 1) * sizeof(int32_t)));
        DSD_HIP(hipMalloc(&g.rank_of, (size_t)(n > 0 ? n : 1) * sizeof(int32_t)));
    }
    int32_t *maxes = d_bad + 2;
    if (n > 0) {
        fill_i32(deg, 0, n, s);
        if (m > 0) k_edge_degrees<<<grid_for(m, BLOCK, 8192), BLOCK, 0, s>>>(edges, m, bits, deg);
        u64 *rk = sc.get_n<u64>(n), *rtmp = sc.get_n<u64>(n);
        k_rank_keys<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(deg, n, bits, rk);
        radix_sort_u64(rk, rtmp, n, 2 * bits, s, sc);
        k_rank_perm<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(rk, n, bits, g.orig_of, g.rank_of);
    }
    u64 *k3 = nullptr;
    if (E > 0) {
        k3 = sc.get_n<u64>(E);
        u64 *t3 = sc.get_n<u64>(E);
        k_orient_keys<<<grid_for(m, BLOCK, 8192), BLOCK, 0, s>>>(edges, m, bits, g.rank_of, k3);
        radix_sort_u64(k3, t3, E, 2 * bits, s, sc);
    }
    k_csr_from_keys<<<grid_for(E + 1, BLOCK, 8192), BLOCK, 0, s>>>(k3, E, n, bits, g.col, g.row_ptr);
    if (n > 0) k_dag_off<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, n, g.dag_off, maxes);
    DSD_HIP(hipEventRecord(e1, s));
    u64 *wed = sc.get_n<u64>(2);
    fill_u64(wed, 0, 2, s);
    if (n > 0) k_wedges<<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(g.row_ptr, g.dag_off, n, wed);
    int32_t hm[2] = {0, 0};
    u64 hw[2] = {0, 0};
    DSD_HIP(hipMemcpyAsync(hm, maxes, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(hw, wed, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    g.w2 = hw[0];
    g.s2 = hw[1];
    g.maxdeg = hm[0];
    g.maxdout = hm[1];
    if (t_orient_ms) DSD_HIP(hipEventElapsedTime(t_orient_ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void free_graph(DevGraph &g) {
    if (g.owned) {
        (void)hipFree(g.row_ptr);
        (void)hipFree(g.col);
        (void)hipFree(g.dag_off);
        (void)hipFree(g.orig_of);
        (void)hipFree(g.rank_of);
    }
    g = DevGraph();
}

}  // namespace dsd
