// dsd_batch_run: one operation over many graphs, each group of graphs with
// the same h enumerated and peeled as one disjoint union.
//
// The union needs no sort.  Every handle already holds its graph in rank
// space (rows sorted by rank, N+(r) the tail of row r); concatenating those
// CSRs with vertex offsets gives a graph whose rows are still sorted and
// whose out-lists still orient every clique from its lowest-rank member,
// because no edge joins two graphs.  Vertex offsets double as the bases of
// the per-graph level tables.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "handle.hpp"

namespace dsd {
namespace {

// sub-batches stay within these sizes (the h = 3 peel keeps about 100 bytes
// per arc of scratch)
constexpr int64_t BATCH_MAX_ARCS = (int64_t)1 << 27;
constexpr int64_t BATCH_MAX_VERTICES = (int64_t)1 << 28;
constexpr int EXACT_THREADS = 16;
// CoreApp on a graph this large runs its own top-down search (Algorithm 6)
// instead of joining the union's full decomposition, which would also hold
// every small graph of the group for the large graph's many levels
constexpr int64_t APP_ALONE_EDGES = (int64_t)1 << 20;

struct UnionDesc {
    const int64_t *row_ptr;
    const int32_t *col;
    const int64_t *dag_off;
    int64_t voff, eoff;
};

// the last g with off[g] <= x (off ascending, off[0] = 0 <= x)
__device__ __forceinline__ int32_t find_seg(const int64_t *off, int32_t G, int64_t x) {
    int32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_union_rows(const UnionDesc *d, const int64_t *voff, int32_t G, int64_t N, int64_t E,
                             int64_t *row_ptr, int64_t *dag_off, int32_t *gid) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= N; v += (int64_t)gridDim.x * blockDim.x) {
        if (v == N) {
            row_ptr[N] = E;
            continue;
        }
        const int32_t g = find_seg(voff, G, v);
        const int64_t local = v - d[g].voff;
        row_ptr[v] = d[g].eoff + d[g].row_ptr[local];
        dag_off[v] = d[g].eoff + d[g].dag_off[local];
        gid[v] = g;
    }
}

__global__ void k_union_cols(const UnionDesc *d, const int64_t *eoff, int32_t G, int64_t E, int32_t *col) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = find_seg(eoff, G, e);
        col[e] = d[g].col[e - d[g].eoff] + (int32_t)d[g].voff;
    }
}

// sum of clique-degrees per graph (lanes of a wave mostly share a graph)
__global__ void k_graph_sums(const u64 *deg, const int32_t *gid, int64_t N, u64 *sum) {
    const int64_t lim = (N + WAVE - 1) / WAVE * WAVE;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v - lane() < lim;
         v += (int64_t)gridDim.x * blockDim.x) {
        const bool in = v < N;
        const int32_t g = in ? gid[v] : -1;
        const u64 d = in ? deg[v] : 0;
        const u64 act = __ballot(in);
        if (!act) continue;
        const int first = __builtin_ctzll(act);
        const int32_t g0 = __shfl(g, first, WAVE);
        if (__ballot(in && g != g0) == 0) {
            const u64 t = wave_sum(d);
            if (lane() == first && t) atomicAdd(&sum[g0], t);
        } else if (in && d) {
            atomicAdd(&sum[g], d);
        }
    }
}

__global__ void k_divide(u64 *a, int32_t G, u64 h) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G) a[g] /= h;
}

// member flags of the (k_max, Psi)-core of every graph
__global__ void k_member_kmax(const u64 *core, const int32_t *gid, const u64 *kmax, int64_t N, uint8_t *mem) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < N; v += (int64_t)gridDim.x * blockDim.x) {
        const u64 k = kmax[gid[v]];
        mem[v] = (k > 0 && core[v] == k) ? 1 : 0;
    }
}

// member flags of every graph's densest residual graph in PeelApp's order:
// the vertices removed in its best round or later (none when best < 0)
__global__ void k_member_round(const u64 *round, const int32_t *gid, const int64_t *best, int64_t N, uint8_t *mem) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < N; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = best[gid[v]];
        mem[v] = (b >= 0 && round[v] >= (u64)b) ? 1 : 0;
    }
}

int bits_for_n(int64_t n) {
    int b = 1;
    while (((int64_t)1 << b) <= n) b++;
    return b;
}

// One group: graphs idx (all with this h), one union, one enumeration, one peel.
void run_group(const std::vector<int32_t> &idx, int h, int op, const dsd_graph *graphs, int out_mem,
               void *const *outs, dsd_result *results) {
    auto t0 = std::chrono::steady_clock::now();
    const int32_t G = (int32_t)idx.size();
    dsd_graph_s *G0 = graphs[idx[0]];
    hipStream_t s = G0->stream;
    for (int32_t i : idx) DSD_HIP(hipStreamSynchronize(graphs[i]->stream));
    Scratch sc;
    std::vector<UnionDesc> desc(G);
    std::vector<int64_t> voff(G), eoff(G), lvb(G);
    int64_t N = 0, E = 0;
    DevGraph U;
    for (int32_t j = 0; j < G; j++) {
        const DevGraph &g = graphs[idx[j]]->g;
        desc[j] = UnionDesc{g.row_ptr, g.col, g.dag_off, N, E};
        voff[j] = N;
        eoff[j] = E;
        lvb[j] = N + j;
        N += g.n;
        E += 2 * g.m;
        U.maxdeg = std::max(U.maxdeg, g.maxdeg);
        U.maxdout = std::max(U.maxdout, g.maxdout);
        U.w2 += g.w2;
        U.s2 += g.s2;
    }
    if (N >= 0x7fffffff) throw Error(DSD_EINVAL, "batch group holds too many vertices");
    U.n = (int32_t)N;
    U.m = E / 2;
    U.bits = bits_for_n(N);
    UnionDesc *d_desc = sc.get_n<UnionDesc>(G);
    int64_t *d_voff = sc.get_n<int64_t>(G), *d_eoff = sc.get_n<int64_t>(G), *d_lvb = sc.get_n<int64_t>(G);
    DSD_HIP(hipMemcpyAsync(d_desc, desc.data(), G * sizeof(UnionDesc), hipMemcpyHostToDevice, s));
    DSD_HIP(hipMemcpyAsync(d_voff, voff.data(), G * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DSD_HIP(hipMemcpyAsync(d_eoff, eoff.data(), G * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DSD_HIP(hipMemcpyAsync(d_lvb, lvb.data(), G * sizeof(int64_t), hipMemcpyHostToDevice, s));
    U.row_ptr = sc.get_n<int64_t>(N + 1);
    U.dag_off = sc.get_n<int64_t>(N);
    U.col = sc.get_n<int32_t>(E);
    int32_t *gid = sc.get_n<int32_t>(N);
    k_union_rows<<<grid_for(N + 1, BLOCK, 8192), BLOCK, 0, s>>>(d_desc, d_voff, G, N, E, U.row_ptr, U.dag_off, gid);
    if (E > 0) k_union_cols<<<grid_for(E, BLOCK, 16384), BLOCK, 0, s>>>(d_desc, d_eoff, G, E, U.col);

    // clique-degrees of every graph in one pass
    KernelTimes kt;
    u64 *deg = sc.get_n<u64>(N);
    double t_enum = 0, t_peel = 0;
    {
        Timer te(s);
        if (N > 0 && !clique_degrees(U, h, nullptr, deg, s, sc, &kt))
            throw Error(DSD_EOVERFLOW, "clique counts of the batch group could exceed 64 bits");
        t_enum = te.stop();
    }
    u64 *mu = sc.get_n<u64>(G);
    fill_u64(mu, 0, G, s);
    if (N > 0) k_graph_sums<<<grid_for(N, BLOCK, 4096), BLOCK, 0, s>>>(deg, gid, N, mu);
    k_divide<<<grid_for(G, 256), 256, 0, s>>>(mu, G, (u64)h);
    std::vector<u64> hmu(G);
    DSD_HIP(hipMemcpyAsync(hmu.data(), mu, G * sizeof(u64), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    u64 mu_all = 0;
    for (int32_t j = 0; j < G; j++) {
        dsd_result &r = results[idx[j]];
        r.num_cliques = hmu[j];
        mu_all += hmu[j];
    }
    // h = 3: the union's triangle lists for the peel, freed with the group
    struct ListHolder {
        TriList tl;
        ~ListHolder() { free_tri_list(tl); }
    } lists;
    const TriList *tl = nullptr;
    if (h == 3 && op != DSD_OP_DEGREES && N > 0 && tri_list_wanted(U, mu_all)) {
        try {
            Timer tb(s);
            build_tri_list(U, deg, mu_all, lists.tl, s, sc);
            t_enum += tb.stop();
            tl = &lists.tl;
        } catch (const Error &e) {
            if (e.status != DSD_ENOMEM) throw;   // no room: the peel intersects neighbourhoods instead
        }
    }

    // host staging for host outputs: one copy for the whole group
    auto deliver = [&](const void *dev_union, size_t elem,
                       void (*gather)(const DevGraph &, const void *, void *, hipStream_t)) {
        if (!outs) return;
        void *stage = out_mem == DSD_MEM_HOST ? sc.get((size_t)(N > 0 ? N : 1) * elem) : nullptr;
        for (int32_t j = 0; j < G; j++) {
            void *dst = outs[idx[j]];
            const DevGraph &g = graphs[idx[j]]->g;
            if (!dst || g.n == 0) continue;
            const char *src = (const char *)dev_union + (size_t)voff[j] * elem;
            gather(g, src, out_mem == DSD_MEM_HOST ? (char *)stage + (size_t)voff[j] * elem : dst, s);
        }
        if (out_mem == DSD_MEM_HOST && N > 0) {
            std::vector<char> host((size_t)N * elem);
            DSD_HIP(hipMemcpyAsync(host.data(), stage, host.size(), hipMemcpyDeviceToHost, s));
            DSD_HIP(hipStreamSynchronize(s));
            for (int32_t j = 0; j < G; j++) {
                void *dst = outs[idx[j]];
                const int32_t n = graphs[idx[j]]->g.n;
                if (dst && n > 0) std::memcpy(dst, host.data() + (size_t)voff[j] * elem, (size_t)n * elem);
            }
        }
        DSD_HIP(hipStreamSynchronize(s));
    };
    auto gather64 = [](const DevGraph &g, const void *in, void *out, hipStream_t st) {
        gather_to_orig_u64(g, (const u64 *)in, (u64 *)out, st);
    };
    auto gather8 = [](const DevGraph &g, const void *in, void *out, hipStream_t st) {
        gather_to_orig_u8(g, (const uint8_t *)in, (uint8_t *)out, st);
    };

    if (op == DSD_OP_DEGREES) {
        deliver(deg, sizeof(u64), gather64);
    } else if (op == DSD_OP_PEEL) {
        // PeelApp's order: every graph's level table holds |S| and mu(S) before each of its rounds
        u64 *round = sc.get_n<u64>(N);
        PeelGroups grp;
        grp.G = G;
        grp.gid = gid;
        grp.mu = mu;
        grp.lv_base = d_lvb;
        grp.lv_total = N + G;
        PeelResult pr;
        {
            Timer tp(s);
            if (N > 0) pr = peel(U, h, nullptr, deg, 0, 0, round, s, sc, &kt, &grp, true, tl);
            t_peel = tp.stop();
        }
        std::vector<int64_t> best(G, -1);
        for (int32_t j = 0; j < G; j++) {
            const int32_t L = N > 0 ? pr.graph_levels[j] : 0;
            u64 a = 0, b = 1;
            for (int32_t i = 0; i < L; i++) {
                const u64 sz = pr.level_size[lvb[j] + i], m = pr.level_mu[lvb[j] + i];
                if (sz > 0 && rat_gt(m, sz, a, b)) {
                    a = m;
                    b = sz;
                    best[j] = i;
                }
            }
            dsd_result &r = results[idx[j]];
            r.peel_rounds = (uint64_t)L;
            if (best[j] >= 0) {
                r.density = make_rational(a, b);
                r.members = b;
            }
        }
        int64_t *dbest = sc.get_n<int64_t>(G);
        DSD_HIP(hipMemcpyAsync(dbest, best.data(), G * sizeof(int64_t), hipMemcpyHostToDevice, s));
        uint8_t *mem = sc.get_n<uint8_t>(N);
        if (N > 0) k_member_round<<<grid_for(N, BLOCK, 8192), BLOCK, 0, s>>>(round, gid, dbest, N, mem);
        deliver(mem, 1, gather8);
        DSD_HIP(hipStreamSynchronize(s));
    } else {
        // the peel: every graph keeps its own level
        u64 *core = sc.get_n<u64>(N);
        PeelGroups grp;
        grp.G = G;
        grp.gid = gid;
        grp.mu = mu;
        grp.lv_base = d_lvb;
        grp.lv_total = N + G;
        PeelResult pr;
        {
            Timer tp(s);
            if (N > 0) pr = peel(U, h, nullptr, deg, 0, 0, core, s, sc, &kt, &grp, false, tl);
            t_peel = tp.stop();
        }
        // keep every graph's decomposition on its handle
        std::vector<u64> kmax(G, 0);
        for (int32_t j = 0; j < G; j++) {
            dsd_graph_s *Gi = graphs[idx[j]];
            const int32_t n = Gi->g.n;
            Decomp &D = Gi->dec[h];
            if (!D.core) D.core = Gi->keep.get_n<u64>(n);
            if (n > 0)
                DSD_HIP(hipMemcpyAsync(D.core, core + voff[j], (size_t)n * sizeof(u64), hipMemcpyDeviceToDevice, s));
            const int32_t L = N > 0 ? pr.graph_levels[j] : 0;
            PeelResult lv;
            lv.rounds = pr.rounds;
            lv.levels = L;
            lv.level_k.assign(pr.level_k.begin() + lvb[j], pr.level_k.begin() + lvb[j] + L);
            lv.level_size.assign(pr.level_size.begin() + lvb[j], pr.level_size.begin() + lvb[j] + L);
            lv.level_mu.assign(pr.level_mu.begin() + lvb[j], pr.level_mu.begin() + lvb[j] + L);
            lv.kmax = L > 0 ? lv.level_k.back() : 0;
            kmax[j] = lv.kmax;
            D.mu = hmu[j];
            D.levels = std::move(lv);
            D.t_enum_ms = t_enum;
            D.t_peel_ms = t_peel;
            D.kt = kt;
            D.valid = true;
            dsd_result &r = results[idx[j]];
            r.kmax = kmax[j];
            r.peel_rounds = (uint64_t)pr.rounds;
            if (op == DSD_OP_APP && kmax[j] > 0) {
                r.density = make_rational(D.levels.level_mu.back(), D.levels.level_size.back());
                r.members = D.levels.level_size.back();
            }
        }
        if (op == DSD_OP_CORE) {
            deliver(core, sizeof(u64), gather64);
        } else if (op == DSD_OP_APP) {
            u64 *dk = sc.get_n<u64>(G);
            DSD_HIP(hipMemcpyAsync(dk, kmax.data(), G * sizeof(u64), hipMemcpyHostToDevice, s));
            uint8_t *mem = sc.get_n<uint8_t>(N);
            if (N > 0) k_member_kmax<<<grid_for(N, BLOCK, 8192), BLOCK, 0, s>>>(core, gid, dk, N, mem);
            deliver(mem, 1, gather8);
        }
        DSD_HIP(hipStreamSynchronize(s));
    }
    DSD_HIP(hipStreamSynchronize(s));   // the group's scratch is freed on return
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int32_t i : idx) results[i].t_ms = ms;
}

// CoreApp for one large graph of the batch, alone
void run_app_alone(dsd_graph_s *Gi, int h, int out_mem, void *out, dsd_result &r) {
    auto t0 = std::chrono::steady_clock::now();
    const int32_t n = Gi->g.n;
    Gi->sc.reset();
    ScratchRelease release_scratch{Gi};
    begin_stats(Gi);
    uint8_t *best = Gi->sc.get_n<uint8_t>(n);
    dsd_rational dens{0, 1};
    const u64 kmax = core_app_run(Gi, h, best, &dens);
    std::vector<uint8_t> hm(n);
    if (n > 0) {
        DSD_HIP(hipMemcpyAsync(hm.data(), best, n, hipMemcpyDeviceToHost, Gi->stream));
        DSD_HIP(hipStreamSynchronize(Gi->stream));
    }
    if (out) write_u8(Gi, best, (uint8_t *)out, out_mem);
    r.kmax = kmax;
    r.density = dens;
    r.members = (uint64_t)std::count(hm.begin(), hm.end(), (uint8_t)1);
    r.num_cliques = 0;   // CoreApp does not count the whole graph's cliques
    r.peel_rounds = Gi->stats.peel_rounds;
    r.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// CoreExact for one graph of the batch (its decomposition is on its handle)
void run_exact(dsd_graph_s *Gi, int h, int out_mem, void *out, dsd_result &r) {
    auto t0 = std::chrono::steady_clock::now();
    const int32_t n = Gi->g.n;
    Gi->sc.reset();
    ScratchRelease release_scratch{Gi};
    begin_stats(Gi);
    uint8_t *res = Gi->sc.get_n<uint8_t>(n);
    const dsd_rational rho = core_exact_run(Gi, h, res);
    std::vector<uint8_t> hm(n);
    if (n > 0) {
        DSD_HIP(hipMemcpyAsync(hm.data(), res, n, hipMemcpyDeviceToHost, Gi->stream));
        DSD_HIP(hipStreamSynchronize(Gi->stream));
    }
    if (out) write_u8(Gi, res, (uint8_t *)out, out_mem);
    r.density = rho;
    r.members = (uint64_t)std::count(hm.begin(), hm.end(), (uint8_t)1);
    r.kmax = Gi->dec[h].levels.kmax;
    r.num_cliques = Gi->dec[h].mu;
    r.t_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace dsd

using namespace dsd;

extern "C" dsd_status dsd_batch_run(int32_t count, const dsd_graph *graphs, const int *h, int op, int out_mem,
                                    void *const *outs, dsd_result *results) {
    if (count < 0) return fail(DSD_EINVAL, "negative batch size");
    if (count == 0) return DSD_OK;
    if (!graphs || !h || !results) return fail(DSD_EINVAL, "NULL batch array");
    if (op < DSD_OP_DEGREES || op > DSD_OP_PEEL) return fail(DSD_EINVAL, "unknown batch operation");
    if (outs && out_mem != DSD_MEM_HOST && out_mem != DSD_MEM_DEVICE) return fail(DSD_EINVAL, "bad memory flag");
    std::vector<dsd_graph> sorted(graphs, graphs + count);
    for (int32_t i = 0; i < count; i++) {
        if (!graphs[i]) return fail(DSD_EINVAL, "NULL graph in batch");
        if (h[i] < 2 || h[i] > 6) return fail(DSD_EINVAL, "h must be in [2, 6]");
    }
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(DSD_EINVAL, "a graph appears twice in one batch");
    for (int32_t i = 0; i < count; i++) {
        results[i] = dsd_result{};
        results[i].status = DSD_OK;
        results[i].density = dsd_rational{0, 1};
        results[i].h = h[i];
        results[i].op = op;
    }
    std::vector<std::string> errs(count);
    DSD_TRY({
        check_device();
        // groups by h, cut into sub-batches of bounded size
        for (int hh = 2; hh <= 6; hh++) {
            std::vector<int32_t> grp;
            int64_t arcs = 0, verts = 0;
            auto flush = [&]() {
                if (grp.empty()) return;
                try {
                    run_group(grp, hh, op, graphs, out_mem, outs, results);
                } catch (const Error &e) {
                    for (int32_t i : grp) {
                        results[i].status = (dsd_status)e.status;
                        errs[i] = e.what();
                    }
                }
                grp.clear();
                arcs = verts = 0;
            };
            for (int32_t i = 0; i < count; i++) {
                if (h[i] != hh) continue;
                if (op == DSD_OP_APP && graphs[i]->g.m >= APP_ALONE_EDGES) continue;
                const int64_t a = 2 * graphs[i]->g.m, v = graphs[i]->g.n;
                if (!grp.empty() && (arcs + a > BATCH_MAX_ARCS || verts + v > BATCH_MAX_VERTICES)) flush();
                grp.push_back(i);
                arcs += a;
                verts += v;
            }
            flush();
        }
        const bool app_alone = op == DSD_OP_APP;
        if (op == DSD_OP_EXACT || app_alone) {
            std::atomic<int32_t> next{0};
            auto worker = [&]() {
                while (true) {
                    const int32_t i = next.fetch_add(1);
                    if (i >= count) return;
                    if (results[i].status != DSD_OK) continue;
                    if (app_alone && graphs[i]->g.m < APP_ALONE_EDGES) continue;
                    try {
                        if (app_alone) run_app_alone(graphs[i], h[i], out_mem, outs ? outs[i] : nullptr, results[i]);
                        else run_exact(graphs[i], h[i], out_mem, outs ? outs[i] : nullptr, results[i]);
                    } catch (const Error &e) {
                        results[i].status = (dsd_status)e.status;
                        errs[i] = e.what();
                    } catch (const std::exception &e) {
                        results[i].status = DSD_EDEVICE;
                        errs[i] = e.what();
                    }
                }
            };
            const int nt = std::max(1, std::min<int>(EXACT_THREADS, count));
            std::vector<std::thread> pool;
            for (int t = 1; t < nt; t++) pool.emplace_back(worker);
            worker();
            for (std::thread &t : pool) t.join();
        }
        for (int32_t i = 0; i < count; i++)
            if (results[i].status != DSD_OK) return fail(results[i].status, errs[i]);
        return DSD_OK;
    })
}
