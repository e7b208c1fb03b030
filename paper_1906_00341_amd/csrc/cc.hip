// K5: connected components of a core (Pruning2, Section 6.1) and the small
// mask / gather / reduction kernels used by the drivers.
//
// Components: union-find over the edges inside the mask.  Every root points
// to the smallest rank of its tree; an edge (u, v) links the larger of the
// two roots under the smaller one with a compare-and-swap and retries when
// it loses a race; finds halve paths.  A final pass points every vertex at
// its root, so label[r] = smallest rank in r's component.
#include "graph.hpp"

namespace dsd {

__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x) {
    int32_t p = parent[x];
    while (p != x) {
        int32_t gp = parent[p];
        if (gp != p) parent[x] = gp;   // path halving; parents only move toward the root
        x = p;
        p = gp;
    }
    return x;
}

__global__ void k_cc_init(const uint8_t *mask, int32_t n, int32_t *parent) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        parent[v] = (mask == nullptr || mask[v]) ? (int32_t)v : -1;
}

// one wave per vertex u; lanes over N(u) ∩ (u, n)
__global__ __launch_bounds__(BLOCK) void k_cc_hook(const int64_t *row_ptr, const int32_t *col, const int64_t *dag_off,
                                                   const uint8_t *mask, int32_t n, int32_t *parent) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t u = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; u < n; u += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        if (mask && !mask[u]) continue;
        for (int64_t e = dag_off[u] + lane(); e < row_ptr[u + 1]; e += WAVE) {
            int32_t v = col[e];
            if (mask && !mask[v]) continue;
            int32_t a = (int32_t)u, b = v;
            while (true) {
                a = uf_find(parent, a);
                b = uf_find(parent, b);
                if (a == b) break;
                int32_t hi = a > b ? a : b, lo = a > b ? b : a;
                if (atomicCAS(&parent[hi], hi, lo) == hi) break;
                a = hi;
                b = lo;
            }
        }
    }
}

__global__ void k_cc_flatten(int32_t n, int32_t *parent) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (parent[v] < 0) continue;
        int32_t x = (int32_t)v;
        while (parent[x] != x) x = parent[x];
        parent[v] = x;
    }
}

void components(const DevGraph &g, const uint8_t *mask, int32_t *label, hipStream_t s, Scratch &) {
    const int32_t n = g.n;
    if (n == 0) return;
    k_cc_init<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(mask, n, label);
    k_cc_hook<<<grid_for(n, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(g.row_ptr, g.col, g.dag_off, mask, n, label);
    k_cc_flatten<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(n, label);
}

// ---------------------------------------------------------------- small kernels

__global__ void k_mask_core_ge(const u64 *core, int32_t n, u64 k, uint8_t *mask) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        mask[v] = core[v] >= k ? 1 : 0;
}
void mask_core_at_least(const u64 *core, int32_t n, u64 k, uint8_t *mask, hipStream_t s) {
    if (n > 0) k_mask_core_ge<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(core, n, k, mask);
}

__global__ void k_mask_core_eq(const u64 *core, int32_t n, u64 k, uint8_t *mask) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        mask[v] = core[v] == k ? 1 : 0;
}
void mask_core_equal(const u64 *core, int32_t n, u64 k, uint8_t *mask, hipStream_t s) {
    if (n > 0) k_mask_core_eq<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(core, n, k, mask);
}

// order[i] holds (key << bits | vertex); the first w entries form the mask
__global__ void k_mask_prefix(const u64 *order, int32_t n, int64_t w, int bits, uint8_t *mask) {
    const u64 m = (1ull << bits) - 1ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mask[(int32_t)(order[i] & m)] = i < w ? 1 : 0;
}
void mask_from_order_prefix(const u64 *order, int32_t n, int64_t w, int bits, uint8_t *mask, hipStream_t s) {
    if (n > 0) k_mask_prefix<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(order, n, w, bits, mask);
}

template <typename T>
__global__ void k_gather_orig(const int32_t *rank_of, int32_t n, const T *in, T *out) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = in[rank_of[v]];
}
void gather_to_orig_u64(const DevGraph &g, const u64 *in, u64 *out, hipStream_t s) {
    if (g.n > 0) k_gather_orig<u64><<<grid_for(g.n, BLOCK, 8192), BLOCK, 0, s>>>(g.rank_of, g.n, in, out);
}
void gather_to_orig_u8(const DevGraph &g, const uint8_t *in, uint8_t *out, hipStream_t s) {
    if (g.n > 0) k_gather_orig<uint8_t><<<grid_for(g.n, BLOCK, 8192), BLOCK, 0, s>>>(g.rank_of, g.n, in, out);
}

__global__ void k_component_sums(const int32_t *label, const u64 *deg, int32_t n, u64 *size, u64 *dsum) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t l = label[v];
        if (l < 0) continue;
        atomicAdd(&size[l], 1ull);
        if (deg[v]) atomicAdd(&dsum[l], deg[v]);
    }
}
void component_sums(const int32_t *label, const u64 *deg, int32_t n, u64 *size, u64 *dsum, hipStream_t s) {
    if (n == 0) return;
    fill_u64(size, 0, n, s);
    fill_u64(dsum, 0, n, s);
    k_component_sums<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(label, deg, n, size, dsum);
}

__global__ void k_masked_ext(const u64 *a, const uint8_t *mask, int32_t n, u64 *out, int want_max) {
    u64 m = want_max ? 0ull : ~0ull;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (mask && !mask[v]) continue;
        u64 x = a[v];
        m = want_max ? (x > m ? x : m) : (x < m ? x : m);
    }
    m = want_max ? wave_max(m) : wave_min(m);
    if (lane() == 0) {
        if (want_max) atomicMax(out, m); else atomicMin(out, m);
    }
}
void masked_max_u64(const u64 *a, const uint8_t *mask, int32_t n, u64 *out, hipStream_t s) {
    fill_u64(out, 0, 1, s);
    if (n > 0) k_masked_ext<<<grid_for(n, BLOCK, 2048), BLOCK, 0, s>>>(a, mask, n, out, 1);
}
void masked_min_u64(const u64 *a, const uint8_t *mask, int32_t n, u64 *out, hipStream_t s) {
    fill_u64(out, ~0ull, 1, s);
    if (n > 0) k_masked_ext<<<grid_for(n, BLOCK, 2048), BLOCK, 0, s>>>(a, mask, n, out, 0);
}

}  // namespace dsd

// ---------------------------------------------------------------- hand-over to the host

namespace dsd {

__global__ void k_flag_mask(const uint8_t *mask, int32_t n, int64_t *flags) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flags[v] = mask[v] ? 1 : 0;
}

__global__ void k_compact_verts(const uint8_t *mask, const int64_t *pos, int32_t n, int32_t *verts) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (mask[v]) verts[pos[v]] = (int32_t)v;
}

// One wave per located vertex (they are the graph's hubs, with the longest
// rows): its neighbours inside the mask, counted, then written in row order.
__global__ __launch_bounds__(BLOCK) void k_local_deg(const int32_t *verts, int64_t cnt, const int64_t *row_ptr,
                                                      const int32_t *col, const uint8_t *mask, int64_t *ldeg) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < cnt; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = verts[i];
        int64_t c = 0;
        for (int64_t e = row_ptr[v] + lane(); e < row_ptr[v + 1]; e += WAVE) c += mask[col[e]] ? 1 : 0;
        c = wave_sum(c);
        if (lane() == 0) ldeg[i] = c;
    }
}

__global__ __launch_bounds__(BLOCK) void k_local_fill(const int32_t *verts, int64_t cnt, const int64_t *row_ptr,
                                                       const int32_t *col, const uint8_t *mask, const int64_t *pos,
                                                       const int64_t *loff, int32_t *ladj) {
    const int wv = threadIdx.x / WAVE;
    for (int64_t i = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; i < cnt; i += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
        const int32_t v = verts[i];
        int64_t o = loff[i];
        const int64_t e1 = row_ptr[v + 1];
        for (int64_t e0 = row_ptr[v]; e0 < e1; e0 += WAVE) {
            const int64_t e = e0 + lane();
            int32_t w = -1;
            bool keep = false;
            if (e < e1) {
                w = col[e];
                keep = mask[w] != 0;
            }
            const u64 m = __ballot(keep);
            if (keep) ladj[o + __popcll(m & lanemask_lt())] = (int32_t)pos[w];
            o += __popcll(m);
        }
    }
}

__global__ void k_gather_located(const int32_t *verts, int64_t cnt, const u64 *core, const int32_t *label,
                                 u64 *ocore, int32_t *olabel) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        ocore[i] = core[verts[i]];
        olabel[i] = label[verts[i]];
    }
}

void extract_induced(const DevGraph &g, const uint8_t *mask, const int32_t *label, const u64 *core,
                     LocatedCore &out, hipStream_t s, Scratch &sc) {
    const int32_t n = g.n;
    out = LocatedCore();
    out.off.assign(1, 0);
    if (n == 0) return;
    int64_t *pos = sc.get_n<int64_t>(n);
    k_flag_mask<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(mask, n, pos);
    scan_exclusive_i64(pos, pos, n, s, sc);
    int64_t last = 0;
    uint8_t lastm = 0;
    DSD_HIP(hipMemcpyAsync(&last, pos + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&lastm, mask + n - 1, 1, hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    const int64_t cnt = last + (lastm ? 1 : 0);
    if (cnt == 0) return;
    int32_t *verts = sc.get_n<int32_t>(cnt);
    int64_t *loff = sc.get_n<int64_t>(cnt);
    k_compact_verts<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(mask, pos, n, verts);
    k_local_deg<<<grid_for(cnt, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(verts, cnt, g.row_ptr, g.col, mask, loff);
    int64_t lastdeg = 0;
    DSD_HIP(hipMemcpyAsync(&lastdeg, loff + cnt - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    scan_exclusive_i64(loff, loff, cnt, s, sc);
    int64_t lastoff = 0;
    DSD_HIP(hipMemcpyAsync(&lastoff, loff + cnt - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    const int64_t tot = lastoff + lastdeg;
    int32_t *ladj = sc.get_n<int32_t>(tot);
    u64 *ocore = sc.get_n<u64>(cnt);
    int32_t *olabel = sc.get_n<int32_t>(cnt);
    k_local_fill<<<grid_for(cnt, WAVES_PER_BLOCK, 8192), BLOCK, 0, s>>>(verts, cnt, g.row_ptr, g.col, mask, pos, loff,
                                                                        ladj);
    k_gather_located<<<grid_for(cnt, BLOCK, 8192), BLOCK, 0, s>>>(verts, cnt, core, label, ocore, olabel);
    out.rank.resize(cnt);
    out.off.resize(cnt + 1);
    out.adj.resize(tot);
    out.core.resize(cnt);
    out.label.resize(cnt);
    DSD_HIP(hipMemcpyAsync(out.rank.data(), verts, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(out.off.data(), loff, cnt * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (tot) DSD_HIP(hipMemcpyAsync(out.adj.data(), ladj, tot * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(out.core.data(), ocore, cnt * sizeof(u64), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(out.label.data(), olabel, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    out.off[cnt] = tot;
}

__global__ void k_collect_roots(const int32_t *label, const u64 *size, const u64 *dsum, int32_t n, int32_t *cnt,
                                int32_t *root, u64 *osize, u64 *odsum) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (label[v] != (int32_t)v) continue;
        int32_t p = atomicAdd(cnt, 1);
        root[p] = (int32_t)v;
        osize[p] = size[v];
        odsum[p] = dsum[v];
    }
}

void collect_components(const int32_t *label, const u64 *size, const u64 *dsum, int32_t n,
                        std::vector<CompInfo> &out, hipStream_t s, Scratch &sc) {
    out.clear();
    if (n == 0) return;
    int32_t *cnt = sc.get_n<int32_t>(1);
    int32_t *root = sc.get_n<int32_t>(n);
    u64 *osize = sc.get_n<u64>(n), *odsum = sc.get_n<u64>(n);
    fill_i32(cnt, 0, 1, s);
    k_collect_roots<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(label, size, dsum, n, cnt, root, osize, odsum);
    int32_t hc = 0;
    DSD_HIP(hipMemcpyAsync(&hc, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> r(hc);
    std::vector<u64> a(hc), b(hc);
    if (hc) {
        DSD_HIP(hipMemcpyAsync(r.data(), root, hc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(a.data(), osize, hc * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipMemcpyAsync(b.data(), odsum, hc * sizeof(u64), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
    }
    out.resize(hc);
    for (int32_t i = 0; i < hc; i++) out[i] = CompInfo{r[i], a[i], b[i]};
}

__global__ void k_mask_label_eq(const int32_t *label, int32_t n, int32_t l, uint8_t *mask) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        mask[v] = label[v] == l ? 1 : 0;
}
void mask_label_equal(const int32_t *label, int32_t n, int32_t l, uint8_t *mask, hipStream_t s) {
    if (n > 0) k_mask_label_eq<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(label, n, l, mask);
}

}  // namespace dsd
