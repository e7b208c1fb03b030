// C ABI of libdsd (declared in include/dsd.h) and the drivers that chain the
// kernels: clique-degrees, (k, Psi)-core decomposition, CoreApp (Algorithm 6)
// and CoreExact (Algorithm 4, exact step on the host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "handle.hpp"

using namespace dsd;

static thread_local std::string g_err;

namespace dsd {

dsd_status fail(int st, const std::string &msg) {
    g_err = msg;
    return (dsd_status)st;
}



void check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) throw Error(DSD_EDEVICE, "no HIP device available");
}

void check_h(int h) {
    if (h < 2 || h > 6) throw Error(DSD_EINVAL, "h must be in [2, 6]");
}

void check_out(const void *p, int mem) {
    if (!p) throw Error(DSD_EINVAL, "NULL output pointer");
    if (mem != DSD_MEM_HOST && mem != DSD_MEM_DEVICE) throw Error(DSD_EINVAL, "bad memory flag");
}

u64 gcd64(u64 a, u64 b) {
    while (b) {
        u64 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

dsd_rational make_rational(u64 num, u64 den) {
    if (num == 0 || den == 0) return {0, 1};
    u64 g = gcd64(num, den);
    return {num / g, den / g};
}

bool rat_gt(u64 a, u64 b, u64 c, u64 d) { return (unsigned __int128)a * d > (unsigned __int128)c * b; }

u64 ceil_div_u(u64 a, u64 b) { return a / b + (a % b != 0); }

void begin_stats(dsd_graph_s *G) {
    G->stats = dsd_stats{};
    G->stats.n = (uint64_t)G->g.n;
    G->stats.m = (uint64_t)G->g.m;
    G->stats.w2 = G->g.w2;
    G->stats.s2 = G->g.s2;
}

void end_stats(dsd_graph_s *G, const KernelTimes &kt) {
    G->stats.k3_ms = kt.k3_ms;
    G->stats.k4_ms = kt.k4_ms;
    G->stats.k3_launches = kt.k3_launches;
    G->stats.k4_main_ms = kt.main_ms;
    G->stats.k4_main_launches = kt.main_launches;
    G->stats.k4_main_pairs = kt.main_pairs;
    G->stats.k4_main_nbrs = kt.main_nbrs;
    G->stats.k4_main_entries = kt.main_entries;
    G->stats.k4_main2_ms = kt.main2_ms;
    G->stats.k4_main2_launches = kt.main2_launches;
    G->stats.k4_main2_words = kt.main2_words;
    G->stats.k4_launches = kt.k4_launches;
    G->stats.k4_main_kind = (uint64_t)kt.main_kind;
    G->stats.k4_tail_ms = kt.tail_ms;
    G->stats.k4_tail_launches = kt.tail_launches;
    G->stats.k4_tail_pairs = kt.tail_pairs;
    G->stats.k4_tail_vertices = kt.tail_vertices;
    G->stats.k4_tail_grid_ms = kt.tail_grid_ms;
    G->stats.k4_tail_grid_rounds = kt.tail_grid_rounds;
    G->stats.k4_tail_grid_pairs = kt.tail_grid_pairs;
}

// clique-degrees (rank space) and mu; throws on overflow
u64 degrees_and_mu(dsd_graph_s *G, int h, const uint8_t *mask, u64 *deg, KernelTimes *kt) {
    hipStream_t s = G->stream;
    if (!clique_degrees(G->g, h, mask, deg, s, G->sc, kt))
        throw Error(DSD_EOVERFLOW, "clique counts could exceed 64 bits");
    u64 *sum = G->sc.get_n<u64>(2);
    sum_u64_128(deg, G->g.n, sum, s, G->sc);
    u64 hs[2];
    DSD_HIP(hipMemcpyAsync(hs, sum, sizeof(hs), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (hs[1] != 0) throw Error(DSD_EOVERFLOW, "sum of clique-degrees exceeds 64 bits");
    if (hs[0] % (u64)h != 0) throw Error(DSD_EDEVICE, "clique-degree sum not divisible by h");
    return hs[0] / (u64)h;
}

const TriList *tri_lists(dsd_graph_s *G, const u64 *deg, u64 mu) {
    if (!G->tl.pairs && !G->tl_tried) {
        G->tl_tried = true;
        if (tri_list_wanted(G->g, mu)) {
            try {
                build_tri_list(G->g, deg, mu, G->tl, G->stream, G->sc, &G->keep);
            } catch (const Error &e) {
                if (e.status != DSD_ENOMEM) throw;     // no room: the peel intersects neighbourhoods instead
            }
        }
    }
    if (!G->tl.pairs || G->tl.mu != mu) return nullptr;
    return &G->tl;
}

// The decomposition for h, computed once per handle (Algorithm 3 via the
// round-synchronous peel).
const Decomp &decompose(dsd_graph_s *G, int h) {
    Decomp &D = G->dec[h];
    if (D.valid) return D;
    hipStream_t s = G->stream;
    const int32_t n = G->g.n;
    if (!D.core) {
        D.core = G->keep.get_n<u64>(n);
    }
    D.kt = KernelTimes();
    D.kt.time_main = G->time_main;
    Timer te(s);
    u64 *d = G->sc.get_n<u64>(n);
    const TriList *tl = nullptr;
    if (h == 3 && n > 0 && G->tl.pairs) {
        // lists from an earlier call: the clique-degrees are their row lengths
        tri_list_degrees(G->tl, n, d, s);
        D.mu = G->tl.mu;
        tl = &G->tl;
    } else if (h == 3 && n > 0 && !G->tl_tried && tri_counts_possible(G->g)) {
        // the lists' first pass gives the clique-degrees; its segment sizes
        // then serve the second pass
        TlCounts w;
        Timer tk(s);
        D.mu = tri_counts(G->g, d, w, s, G->sc);
        D.kt.k3_ms += tk.stop();
        D.kt.k3_launches += 1;
        G->tl_tried = true;
        if (D.mu > 0 && tri_list_wanted(G->g, D.mu)) {
            try {
                build_tri_list(G->g, w, G->tl, s, G->sc, &G->keep);
            } catch (const Error &e) {
                if (e.status != DSD_ENOMEM) throw;     // no room: the peel intersects neighbourhoods instead
            }
        }
        if (G->tl.pairs && G->tl.mu == D.mu) tl = &G->tl;
    } else {
        D.mu = n > 0 ? degrees_and_mu(G, h, nullptr, d, &D.kt) : 0;
        tl = h == 3 && D.mu > 0 ? tri_lists(G, d, D.mu) : nullptr;
    }
    D.t_enum_ms = te.stop();
    Timer tp(s);
    D.levels = PeelResult();
    if (n > 0) {
        if (D.mu > 0) D.levels = peel(G->g, h, nullptr, d, D.mu, 0, D.core, s, G->sc, &D.kt, nullptr, false, tl);
        else fill_u64(D.core, 0, n, s);
    }
    D.t_peel_ms = tp.stop();
    D.valid = true;
    return D;
}

void decomp_stats(dsd_graph_s *G, const Decomp &D) {
    G->stats.t_enum_ms = D.t_enum_ms;
    G->stats.t_peel_ms = D.t_peel_ms;
    G->stats.num_cliques = D.mu;
    G->stats.peel_rounds = D.levels.rounds;
    G->stats.peel_levels = D.levels.levels;
    end_stats(G, D.kt);
}

template <typename T>
void write_out(dsd_graph_s *G, const T *rank_space, T *out, int mem,
               void (*gather)(const DevGraph &, const T *, T *, hipStream_t)) {
    hipStream_t s = G->stream;
    const int32_t n = G->g.n;
    if (n == 0) return;
    if (mem == DSD_MEM_DEVICE) {
        gather(G->g, rank_space, out, s);
        DSD_HIP(hipStreamSynchronize(s));
    } else {
        T *tmp = G->sc.get_n<T>(n);
        gather(G->g, rank_space, tmp, s);
        DSD_HIP(hipMemcpyAsync(out, tmp, (size_t)n * sizeof(T), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
    }
}

void write_u64(dsd_graph_s *G, const u64 *r, uint64_t *out, int mem) {
    write_out<u64>(G, r, (u64 *)out, mem, gather_to_orig_u64);
}
void write_u8(dsd_graph_s *G, const uint8_t *r, uint8_t *out, int mem) {
    write_out<uint8_t>(G, r, out, mem, gather_to_orig_u8);
}


// CoreExact (Algorithm 4) on a handle: Pruning1 and Pruning2 on the GPU from
// the cached decomposition, the exact search over the located components on
// the host.
dsd_rational core_exact_run(dsd_graph_s *G, int h, uint8_t *res) {
    const int32_t n = G->g.n;
    hipStream_t s = G->stream;
    const Decomp &D = decompose(G, h);
    decomp_stats(G, D);
    fill_u8(res, 0, n, s);
    dsd_rational rho{0, 1};
    const u64 mu = D.mu;
    u64 *core = D.core;
    if (mu == 0) return rho;
    const PeelResult &pr = D.levels;
    Timer tl(s);
    // Pruning1: rho' = max over levels of mu(R_k) / |R_k|
    u64 a = 0, b = 1;
    int64_t best_level = -1;
    for (int64_t i = 0; i < (int64_t)pr.level_k.size(); i++)
        if (pr.level_size[i] > 0 && rat_gt(pr.level_mu[i], pr.level_size[i], a, b)) {
            a = pr.level_mu[i];
            b = pr.level_size[i];
            best_level = i;
        }
    const u64 k1 = ceil_div_u(a, b);
    // Pruning2: components of R_{k'} and their densities
    uint8_t *m1 = G->sc.get_n<uint8_t>(n);
    int32_t *lab1 = G->sc.get_n<int32_t>(n);
    u64 *d1 = G->sc.get_n<u64>(n), *sz = G->sc.get_n<u64>(n), *ds = G->sc.get_n<u64>(n);
    mask_core_at_least(core, n, k1, m1, s);
    components(G->g, m1, lab1, s, G->sc);
    degrees_and_mu(G, h, m1, d1);
    component_sums(lab1, d1, n, sz, ds, s);
    std::vector<CompInfo> c1;
    collect_components(lab1, sz, ds, n, c1, s, G->sc);
    u64 rn = 0, rd = 1;
    int32_t best_root = -1;
    for (const CompInfo &c : c1)
        if (c.size > 0 && c.dsum > 0 && (best_root < 0 || rat_gt(c.dsum, c.size * (u64)h, rn, rd))) {
            rn = c.dsum;
            rd = c.size * (u64)h;
            best_root = c.root;
        }
    dsd_rational r2 = make_rational(rn, rd);
    const u64 k2 = std::max(k1, ceil_div_u(r2.num, r2.den));
    {
        const dsd_rational r1 = make_rational(a, b);
        G->stats.locate_rho1_num = r1.num;
        G->stats.locate_rho1_den = r1.den;
        G->stats.locate_k1 = k1;
        G->stats.locate_rho2_num = r2.num;
        G->stats.locate_rho2_den = r2.den;
        G->stats.locate_k2 = k2;
        u64 nc = 0;
        for (const CompInfo &c : c1) nc += c.size > 0 ? 1 : 0;
        G->stats.locate_components = nc;
    }
    // D starts as the better of the level set attaining rho' and the
    // component attaining rho''; both densities are lower bounds on rho_opt
    if (rat_gt(a, b, r2.num, r2.den) && best_level >= 0) {
        mask_core_at_least(core, n, pr.level_k[best_level], res, s);
        rho = make_rational(a, b);
    } else {
        if (best_root >= 0) mask_label_equal(lab1, n, best_root, res, s);
        rho = r2;
    }
    // components of R_{k''} go to the host
    uint8_t *m2 = m1;
    int32_t *lab2 = lab1;
    if (k2 > k1) {
        m2 = G->sc.get_n<uint8_t>(n);
        lab2 = G->sc.get_n<int32_t>(n);
        mask_core_at_least(core, n, k2, m2, s);
        components(G->g, m2, lab2, s, G->sc);
    }
    LocatedCore lc;
    extract_induced(G->g, m2, lab2, core, lc, s, G->sc);
    G->stats.located_vertices = lc.rank.size();
    // h-cliques of every located component, counted here so that the exact
    // search can refuse a component whose network would be too large before
    // it lists anything: one component is R_{k''} itself, whose cliques the
    // level table holds (mu(R_k) of the first level k >= k''); otherwise the
    // components of R_{k'} (k'' = k') or a masked enumeration of R_{k''}
    {
        std::vector<int32_t> labs(lc.label);
        std::sort(labs.begin(), labs.end());
        labs.erase(std::unique(labs.begin(), labs.end()), labs.end());
        if (labs.size() == 1) {
            for (size_t i = 0; i < pr.level_k.size(); i++)
                if (pr.level_k[i] >= k2) {
                    lc.comp_mu.push_back({labs[0], pr.level_mu[i]});
                    break;
                }
        } else if (labs.size() > 1) {
            std::vector<CompInfo> c2;
            if (k2 == k1) {
                c2 = c1;
            } else {
                u64 *d2 = G->sc.get_n<u64>(n), *sz2 = G->sc.get_n<u64>(n), *ds2 = G->sc.get_n<u64>(n);
                degrees_and_mu(G, h, m2, d2);
                component_sums(lab2, d2, n, sz2, ds2, s);
                collect_components(lab2, sz2, ds2, n, c2, s, G->sc);
            }
            for (const CompInfo &c : c2) lc.comp_mu.push_back({c.root, c.dsum / (u64)h});
            std::sort(lc.comp_mu.begin(), lc.comp_mu.end());
        }
    }
    G->stats.t_locate_ms = tl.stop();
    auto t0 = std::chrono::steady_clock::now();
    Rational l{rho.num, rho.den};
    std::vector<int32_t> bestset;
    ExactStats es;
    bool improved = exact_search(lc, h, k2, l, bestset, es);
    G->stats.t_exact_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    G->stats.flow_calls = es.flow_calls;
    G->stats.flow_nodes_max = es.max_nodes;
    G->stats.t_flow_build_ms = es.build_ms;
    G->stats.t_flow_ms = es.flow_ms;
    G->stats.t_flow_setup_ms = es.setup_ms;
    G->stats.flow_gpu_calls = es.gpu_flow_calls;
    G->stats.flow_gpu_networks = es.gpu_networks;
    if (improved) {
        rho = dsd_rational{l.num, l.den};
        std::vector<uint8_t> hm(n, 0);
        for (int32_t v : bestset) hm[lc.rank[v]] = 1;
        DSD_HIP(hipMemcpyAsync(res, hm.data(), n, hipMemcpyHostToDevice, s));
        DSD_HIP(hipStreamSynchronize(s));
    }
    return rho;
}

// rank and clique-core number of every query vertex
__global__ void k_query_core(const int32_t *rank_of, const u64 *core, const int32_t *q, int32_t nq, int32_t *rank,
                             u64 *qcore) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += gridDim.x * blockDim.x) {
        const int32_t r = rank_of[q[i]];
        rank[i] = r;
        qcore[i] = core[r];
    }
}

__global__ void k_mark(uint8_t *mask, const int32_t *ids, int32_t nq) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += gridDim.x * blockDim.x) mask[ids[i]] = 1;
}

// The densest subgraph containing every query vertex (Section 6.3, for
// h-cliques).  With x the least clique-core number over Q, the (x, Psi)-core
// contains Q and has density l >= x/h (Theorem 1); any densest set D
// containing Q has every vertex outside Q at clique-degree >= rho(D) >= l
// inside D, so D together with the (x, Psi)-core has least degree >=
// min(x, ceil(l)): D lies in that core.  The GPU locates it; the host
// searches it with Q forced to the source side of every cut.
dsd_rational core_exact_query_run(dsd_graph_s *G, int h, const std::vector<int32_t> &q, uint8_t *res) {
    const int32_t n = G->g.n, nq = (int32_t)q.size();
    hipStream_t s = G->stream;
    const Decomp &D = decompose(G, h);
    decomp_stats(G, D);
    fill_u8(res, 0, n, s);
    int32_t *dq = G->sc.get_n<int32_t>(nq), *dr = G->sc.get_n<int32_t>(nq);
    u64 *dc = G->sc.get_n<u64>(nq);
    DSD_HIP(hipMemcpyAsync(dq, q.data(), (size_t)nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    k_query_core<<<grid_for(nq, 256, 1024), 256, 0, s>>>(G->g.rank_of, D.core, dq, nq, dr, dc);
    std::vector<int32_t> qr(nq);
    std::vector<u64> qc(nq);
    DSD_HIP(hipMemcpyAsync(qr.data(), dr, (size_t)nq * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(qc.data(), dc, (size_t)nq * sizeof(u64), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (D.mu == 0) {                  // no clique anywhere: Q itself, at density 0
        k_mark<<<grid_for(nq, 256, 1024), 256, 0, s>>>(res, dr, nq);
        DSD_HIP(hipStreamSynchronize(s));
        return dsd_rational{0, 1};
    }
    const u64 x = *std::min_element(qc.begin(), qc.end());
    // the (x, Psi)-core: Q's first candidate, its density from the level table
    const PeelResult &pr = D.levels;
    int64_t li = -1;
    for (int64_t i = 0; i < (int64_t)pr.level_k.size(); i++)
        if (pr.level_k[i] == x) li = i;
    if (li < 0) throw Error(DSD_EDEVICE, "query vertex core number missing from the level table");
    Rational l{pr.level_mu[li], pr.level_size[li]};
    {
        const dsd_rational r = make_rational(l.num, l.den);
        l = Rational{r.num, r.den};
    }
    const u64 kstar = std::min<u64>(x, ceil_div_u(l.num, l.den));
    Timer tl(s);
    uint8_t *m = G->sc.get_n<uint8_t>(n);
    int32_t *lab = G->sc.get_n<int32_t>(n);
    mask_core_at_least(D.core, n, kstar, m, s);
    components(G->g, m, lab, s, G->sc);
    LocatedCore lc;
    extract_induced(G->g, m, lab, D.core, lc, s, G->sc);
    G->stats.located_vertices = lc.rank.size();
    G->stats.t_locate_ms = tl.stop();
    std::vector<int32_t> local(n, -1);
    for (size_t i = 0; i < lc.rank.size(); i++) local[lc.rank[i]] = (int32_t)i;
    std::vector<int32_t> ql;
    for (int32_t r : qr)
        if (local[r] >= 0) ql.push_back(local[r]);
    auto t0 = std::chrono::steady_clock::now();
    std::vector<int32_t> bestset;
    ExactStats es;
    const bool improved = exact_search_query(lc, h, x, ql, l, bestset, es);
    G->stats.t_exact_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    G->stats.flow_calls = es.flow_calls;
    G->stats.flow_nodes_max = es.max_nodes;
    G->stats.t_flow_build_ms = es.build_ms;
    G->stats.t_flow_ms = es.flow_ms;
    G->stats.t_flow_setup_ms = es.setup_ms;
    G->stats.flow_gpu_calls = es.gpu_flow_calls;
    G->stats.flow_gpu_networks = es.gpu_networks;
    if (improved) {
        std::vector<uint8_t> hm(n, 0);
        for (int32_t v : bestset) hm[lc.rank[v]] = 1;
        DSD_HIP(hipMemcpyAsync(res, hm.data(), n, hipMemcpyHostToDevice, s));
        DSD_HIP(hipStreamSynchronize(s));
    } else {
        mask_core_at_least(D.core, n, x, res, s);
    }
    return dsd_rational{l.num, l.den};
}

}  // namespace dsd

extern "C" {

const char *dsd_status_str(dsd_status s) {
    switch (s) {
        case DSD_OK: return "DSD_OK";
        case DSD_EINVAL: return "DSD_EINVAL";
        case DSD_ENOMEM: return "DSD_ENOMEM";
        case DSD_EDEVICE: return "DSD_EDEVICE";
        case DSD_EOVERFLOW: return "DSD_EOVERFLOW";
        case DSD_EUNSUPPORTED: return "DSD_EUNSUPPORTED";
        case DSD_EBUSY: return "DSD_EBUSY";
        case DSD_ETIMEDOUT: return "DSD_ETIMEDOUT";
        case DSD_ECANCELED: return "DSD_ECANCELED";
    }
    return "DSD_UNKNOWN";
}

const char *dsd_last_error(void) { return g_err.c_str(); }

dsd_status dsd_build_csr(int32_t n, int64_t num_pairs, const int32_t *src, const int32_t *dst, int in_mem,
                         void *stream, dsd_graph *out) {
    if (!out) return fail(DSD_EINVAL, "NULL output handle");
    *out = nullptr;
    if (n < 0 || num_pairs < 0) return fail(DSD_EINVAL, "negative n or pair count");
    if (num_pairs > 0 && (!src || !dst)) return fail(DSD_EINVAL, "NULL pair arrays");
    if (in_mem != DSD_MEM_HOST && in_mem != DSD_MEM_DEVICE) return fail(DSD_EINVAL, "bad memory flag");
    std::unique_ptr<dsd_graph_s> holder;
    DSD_TRY({
        check_device();
        holder.reset(new dsd_graph_s());
        dsd_graph_s *G = holder.get();
        G->stream = (hipStream_t)stream;
        hipStream_t s = G->stream;
        const int32_t *ds = src, *dd = dst;
        if (in_mem == DSD_MEM_HOST && num_pairs > 0) {
            int32_t *a = G->sc.get_n<int32_t>(num_pairs), *b = G->sc.get_n<int32_t>(num_pairs);
            DSD_HIP(hipMemcpyAsync(a, src, (size_t)num_pairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DSD_HIP(hipMemcpyAsync(b, dst, (size_t)num_pairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
            ds = a;
            dd = b;
        }
        float t = 0;
        Timer tm(s);
        build_graph(n, num_pairs, ds, dd, G->g, s, G->sc, &t, &G->keep);
        begin_stats(G);
        G->stats.t_total_ms = tm.stop();
        G->stats.t_orient_ms = t;
        G->sc.reset();
        ScratchRelease release_scratch{G};
        *out = holder.release();
        return DSD_OK;
    })
}

dsd_status dsd_graph_info(dsd_graph g, int32_t *n, int64_t *m) {
    if (!g) return fail(DSD_EINVAL, "NULL graph");
    if (n) *n = g->g.n;
    if (m) *m = g->g.m;
    return DSD_OK;
}

dsd_status dsd_graph_free(dsd_graph g) {
    if (!g) return DSD_OK;
    DSD_TRY({
        (void)hipStreamSynchronize(g->stream);
        delete g;
        return DSD_OK;
    })
}

dsd_status dsd_last_stats(dsd_graph g, dsd_stats *out) {
    if (!g || !out) return fail(DSD_EINVAL, "NULL argument");
    *out = g->stats;
    return DSD_OK;
}

dsd_status dsd_release_cache(void) {
    dsd::release_chunk_pool();
    return DSD_OK;
}

dsd_status dsd_autotune(dsd_graph G, int h, const char *path, int32_t cap, dsd_tune_result *out, int32_t *count) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    if (cap < 0 || (cap > 0 && !out)) return fail(DSD_EINVAL, "bad result array");
    if (h < 3 || h > 6) return fail(DSD_EINVAL, "tuning needs h in [3, 6]");
    DSD_TRY({
        check_device();
        G->sc.reset();
        ScratchRelease release_scratch{G};
        const std::vector<TuneResult> res = autotune(G->g, h, G->stream, G->sc);
        if (path) tune_write(path);
        int32_t k = 0;
        for (const TuneResult &r : res) {
            if (k < cap) out[k] = dsd_tune_result{r.cls, r.roots, r.cap_default, r.cap_best, r.ms_default, r.ms_best};
            k++;
        }
        if (count) *count = k;
        return DSD_OK;
    })
}

dsd_status dsd_tune_load(const char *path) {
    DSD_TRY({
        tune_load(path);
        return DSD_OK;
    })
}

dsd_status dsd_set_kernel_timing(dsd_graph g, int on) {
    if (!g) return fail(DSD_EINVAL, "NULL graph");
    g->time_main = on != 0;
    return DSD_OK;
}

dsd_status dsd_clique_degrees(dsd_graph G, int h, int out_mem, uint64_t *deg, uint64_t *num_cliques) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_h(h);
        if (G->g.n > 0) check_out(deg, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        u64 *d = G->sc.get_n<u64>(G->g.n);
        KernelTimes kt;
        u64 mu = degrees_and_mu(G, h, nullptr, d, &kt);
        G->stats.t_enum_ms = tm.stop();
        end_stats(G, kt);
        write_u64(G, d, deg, out_mem);
        if (num_cliques) *num_cliques = mu;
        G->stats.num_cliques = mu;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

dsd_status dsd_clique_core(dsd_graph G, int h, int out_mem, uint64_t *core, uint64_t *kmax) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_h(h);
        if (G->g.n > 0) check_out(core, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        const Decomp &D = decompose(G, h);
        decomp_stats(G, D);
        write_u64(G, D.core, core, out_mem);
        if (kmax) *kmax = D.levels.kmax;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

// C(x, r), saturating at 2^64 - 1
static u64 binom_sat(u64 x, int r) {
    if ((u64)r > x) return 0;
    unsigned __int128 acc = 1;
    for (int i = 1; i <= r; i++) {
        acc = acc * (unsigned __int128)(x - (u64)r + (u64)i) / (unsigned __int128)i;
        if (acc > (unsigned __int128)~0ull) return ~0ull;
    }
    return (u64)acc;
}

__global__ void k_gamma_keys(const u64 *x, int32_t n, int bits, u64 xsat, u64 keymax, int r, u64 *keys) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        u64 xv = x[v];
        u64 g = xv < (u64)r ? 0 : (xv < xsat ? xv : xsat);   // gamma = C(g, r) is increasing in g
        keys[v] = ((keymax - g) << bits) | (u64)v;
    }
}

__global__ void k_count_top(const u64 *keys, int32_t n, int bits, int32_t *cnt) {
    const u64 top = keys[0] >> bits;
    int32_t c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += (keys[i] >> bits) == top ? 1 : 0;
    c = wave_sum(c);
    if (lane() == 0 && c) atomicAdd(cnt, c);
}

}  // extern "C"

namespace dsd {

// CoreApp (Algorithm 6, in the corrected reading) on a handle: best (device,
// rank space, length n) receives the (k_max, Psi)-core; returns k_max and
// its density.
u64 core_app_run(dsd_graph_s *G, int h, uint8_t *best, dsd_rational *density) {
    const int32_t n = G->g.n;
    hipStream_t s = G->stream;
    u64 kmax = 0, best_mu = 0, best_size = 0;
    fill_u8(best, 0, n, s);
    if (n > 0) {
        // gamma(v) = C(x_v, h-1) from the classic core numbers x_v (Section 6.2)
        u64 *d = G->sc.get_n<u64>(n), *x = G->sc.get_n<u64>(n), *core = G->sc.get_n<u64>(n);
        u64 m = degrees_and_mu(G, 2, nullptr, d);
        Timer tp(s);
        PeelResult xr = peel(G->g, 2, nullptr, d, m, 0, x, s, G->sc);
        G->stats.t_peel_ms += tp.stop();
        // the smallest core number whose C(x, h-1) saturates 64 bits (n + 1
        // if none up to n does); C(x, h-1) only grows with x
        u64 xlo = 0, xsat = (u64)n + 1;
        while (xlo < xsat) {
            const u64 mid = xlo + (xsat - xlo) / 2;
            if (binom_sat(mid, h - 1) == ~0ull) xsat = mid;
            else xlo = mid + 1;
        }
        const u64 keymax = std::min<u64>(xsat, (u64)n);
        u64 *keys = G->sc.get_n<u64>(n), *tmp = G->sc.get_n<u64>(n);
        k_gamma_keys<<<grid_for(n, BLOCK, 8192), BLOCK, 0, s>>>(x, n, G->g.bits, keymax, keymax, h - 1, keys);
        int kb = G->g.bits + 1;
        while ((keymax >> (kb - G->g.bits)) != 0) kb++;
        radix_sort_u64(keys, tmp, n, kb, s, G->sc);
        int32_t *cnt = G->sc.get_n<int32_t>(1);
        fill_i32(cnt, 0, 1, s);
        k_count_top<<<grid_for(n, BLOCK, 2048), BLOCK, 0, s>>>(keys, n, G->g.bits, cnt);
        int32_t ntop = 0;
        DSD_HIP(hipMemcpyAsync(&ntop, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DSD_HIP(hipStreamSynchronize(s));
        auto gamma_at = [&](int64_t i) -> u64 {
            u64 k = 0;
            DSD_HIP(hipMemcpyAsync(&k, keys + i, sizeof(u64), hipMemcpyDeviceToHost, s));
            DSD_HIP(hipStreamSynchronize(s));
            return binom_sat(keymax - (k >> G->g.bits), h - 1);
        };
        int64_t w = std::min<int64_t>(n, std::max<int64_t>(64, ntop));
        uint8_t *inW = G->sc.get_n<uint8_t>(n);
        u64 *mn = G->sc.get_n<u64>(1);
        while (true) {
            mask_from_order_prefix(keys, n, w, G->g.bits, inW, s);
            Timer te(s);
            u64 muW = degrees_and_mu(G, h, inW, d);
            G->stats.t_enum_ms += te.stop();
            masked_min_u64(d, inW, n, mn, s);
            u64 kl = 0;
            DSD_HIP(hipMemcpyAsync(&kl, mn, sizeof(u64), hipMemcpyDeviceToHost, s));
            DSD_HIP(hipStreamSynchronize(s));
            const u64 k0 = std::max(kl, kmax);
            // G[W]'s k_max is at least its density mu(W)/|W| (its densest
            // subgraph lies in the ceil(rho)-core, Lemma 7), so the levels
            // below that need not be peeled one by one
            const u64 dens_ceil = (muW + (u64)w - 1) / (u64)w;
            const u64 kf = std::max(k0, dens_ceil);
            const u64 floor_k = kf > 0 ? kf - 1 : 0;
            Timer tq(s);
            // (no triangle lists here: their rows hold every triangle of the whole graph, and a
            // hub's row in G[W] is mostly triangles that leave W; rewriting them for the tail
            // engine at every W costs more than the peel of G[W])
            PeelResult pr = peel(G->g, h, inW, d, muW, floor_k, core, s, G->sc);
            G->stats.t_peel_ms += tq.stop();
            G->stats.peel_rounds += pr.rounds;
            G->stats.peel_levels += pr.levels;
            if (pr.levels > 0 && pr.kmax > 0 && pr.kmax >= k0) {
                kmax = pr.kmax;
                best_mu = pr.level_mu.back();
                best_size = pr.level_size.back();
                mask_core_equal(core, n, kmax, best, s);
            }
            // stop once every vertex outside W has gamma < kmax (its clique-core number is smaller)
            if (w >= n || gamma_at(w) < kmax) break;
            // W doubles (Algorithm 6), or, when more vertices than that have
            // gamma >= the k_max found so far, grows to take all of them at
            // once (up to 8 |W|): the stopping test can pass only once they
            // are all in W, and the core it returns does not depend on the
            // sizes W passes through
            int64_t lo = w, hi = n;                    // first position whose gamma < kmax
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (gamma_at(mid) >= kmax) lo = mid + 1;
                else hi = mid;
            }
            w = std::min<int64_t>(n, std::max<int64_t>(2 * w, std::min<int64_t>(lo, 8 * w)));
        }
    }
    if (density) *density = kmax > 0 ? make_rational(best_mu, best_size) : dsd_rational{0, 1};
    return kmax;
}

// PeelApp (Algorithm 2) on a handle, every minimum-degree vertex per round:
// the peel's min-degree mode records |S| and mu(S) before every round and
// each vertex's removal round; the answer is the first densest of those
// residual graphs, i.e. the vertices removed in its round or later.
dsd_rational peel_app_run(dsd_graph_s *G, int h, uint8_t *best, int64_t *rounds, int64_t *best_round) {
    const int32_t n = G->g.n;
    hipStream_t s = G->stream;
    fill_u8(best, 0, n, s);
    *rounds = 0;
    *best_round = -1;
    if (n == 0) return dsd_rational{0, 1};
    KernelTimes kt;
    kt.time_main = G->time_main;
    Timer te(s);
    u64 *d = G->sc.get_n<u64>(n);
    const u64 mu = degrees_and_mu(G, h, nullptr, d, &kt);
    const TriList *tl = h == 3 && mu > 0 ? tri_lists(G, d, mu) : nullptr;
    G->stats.t_enum_ms = te.stop();
    G->stats.num_cliques = mu;
    if (mu == 0) {                 // every vertex is at the minimum, 0: one round empties S
        end_stats(G, kt);
        *rounds = 1;
        return dsd_rational{0, 1};
    }
    u64 *round = G->sc.get_n<u64>(n);
    Timer tp(s);
    PeelResult pr = peel(G->g, h, nullptr, d, mu, 0, round, s, G->sc, &kt, nullptr, true, tl);
    G->stats.t_peel_ms = tp.stop();
    G->stats.peel_rounds = pr.rounds;
    G->stats.peel_levels = pr.levels;
    end_stats(G, kt);
    u64 a = 0, b = 1;
    for (int64_t j = 0; j < (int64_t)pr.level_size.size(); j++)
        if (pr.level_size[j] > 0 && rat_gt(pr.level_mu[j], pr.level_size[j], a, b)) {
            a = pr.level_mu[j];
            b = pr.level_size[j];
            *best_round = j;
        }
    *rounds = pr.rounds;
    if (*best_round < 0) return dsd_rational{0, 1};
    mask_core_at_least(round, n, (u64)*best_round, best, s);
    return make_rational(a, b);
}

}  // namespace dsd

extern "C" {

dsd_status dsd_core_app(dsd_graph G, int h, int out_mem, uint8_t *member, uint64_t *kmax_out,
                        dsd_rational *density) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_h(h);
        const int32_t n = G->g.n;
        if (n > 0) check_out(member, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        uint8_t *best = G->sc.get_n<uint8_t>(n);
        const u64 kmax = core_app_run(G, h, best, density);
        write_u8(G, best, member, out_mem);
        if (kmax_out) *kmax_out = kmax;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

dsd_status dsd_peel_app(dsd_graph G, int h, int out_mem, uint8_t *member, dsd_rational *density, int64_t *rounds,
                        int64_t *best_round) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_h(h);
        const int32_t n = G->g.n;
        if (n > 0) check_out(member, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        uint8_t *best = G->sc.get_n<uint8_t>(n);
        int64_t r = 0, br = -1;
        const dsd_rational rho = peel_app_run(G, h, best, &r, &br);
        write_u8(G, best, member, out_mem);
        if (density) *density = rho;
        if (rounds) *rounds = r;
        if (best_round) *best_round = br;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

dsd_status dsd_core_exact_query(dsd_graph G, int h, int32_t nq, const int32_t *q, int out_mem, uint8_t *member,
                                dsd_rational *rho) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    if (nq < 1 || !q) return fail(DSD_EINVAL, "the query needs at least one vertex");
    for (int32_t i = 0; i < nq; i++)
        if (q[i] < 0 || q[i] >= G->g.n) return fail(DSD_EINVAL, "query vertex outside [0, n)");
    DSD_TRY({
        check_h(h);
        const int32_t n = G->g.n;
        check_out(member, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        uint8_t *res = G->sc.get_n<uint8_t>(n);
        const dsd_rational r = core_exact_query_run(G, h, std::vector<int32_t>(q, q + nq), res);
        write_u8(G, res, member, out_mem);
        if (rho) *rho = r;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

dsd_status dsd_core_exact(dsd_graph G, int h, int out_mem, uint8_t *member, dsd_rational *rho_opt) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_h(h);
        const int32_t n = G->g.n;
        if (n > 0) check_out(member, out_mem);
        G->sc.reset();
        ScratchRelease release_scratch{G};
        begin_stats(G);
        Timer tm(G->stream);
        uint8_t *res = G->sc.get_n<uint8_t>(n);
        const dsd_rational rho = core_exact_run(G, h, res);
        write_u8(G, res, member, out_mem);
        if (rho_opt) *rho_opt = rho;
        G->stats.t_total_ms = tm.stop();
        return DSD_OK;
    })
}

}  // extern "C"
