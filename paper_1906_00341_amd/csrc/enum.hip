// K3: clique-degrees (Definition 3) on the degree-ordered DAG.
//
// Every h-clique is listed once, from its lowest-rank member r: the other
// h-1 members form an (h-1)-clique of the sub-DAG induced on N+(r).  Roots
// are binned by out-degree into a wave class (one wave per root, |N+| <= 64)
// and block classes (one workgroup per root, candidate set, hash and bitmap
// staged in LDS); each root flushes at most |N+(r)| + 1 global 64-bit atomics.
#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

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

// ---------------------------------------------------------------- launch grids and their tuning
//
// Each out-degree class of roots is one launch whose grid is capped: the
// workgroups loop over the class's roots, so the cap trades occupancy and
// tail balance against per-workgroup start-up (and, for the classes whose
// bitmaps live in global memory, scratch).  The caps below are the
// defaults; dsd_autotune times a set of caps per class on a caller's graph
// and keeps the fastest in a process-wide table keyed by (architecture, h,
// class), which dsd_tune_load (or DSD_TUNE_FILE, read once) fills from a
// JSON file and dsd_autotune can write back.

static int default_cap(int R, int c) {
    if (c == 0) return 8192;
    if (R <= 2) return c == 1 ? 4096 : 1024;
    return c == 1 ? 4096 : c == 2 ? 2048 : 512;
}

struct TuneTable {
    std::mutex mu;
    std::map<std::string, int> cap;
    bool env_read = false;
};
static TuneTable &tune_table() {
    static TuneTable *t = new TuneTable();   // never destroyed: launches may run during static destruction
    return *t;
}

// the current device's architecture, e.g. gfx950 (the name up to its feature suffix)
static std::string arch_name() {
    static std::mutex mu;
    static std::map<int, std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t p;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
        a = p.gcnArchName;
        const size_t colon = a.find(':');
        if (colon != std::string::npos) a = a.substr(0, colon);
    }
    names[dev] = a;
    return a;
}

static std::string tune_key(const std::string &arch, int h, int c) {
    return arch + "/h" + std::to_string(h) + "/c" + std::to_string(c);
}

// the JSON file: one flat object, "gfx950/h4/c2": 1024, ...
static void tune_parse(const std::string &text, std::map<std::string, int> &out) {
    size_t i = 0;
    auto ws = [&] {
        while (i < text.size() && std::isspace((unsigned char)text[i])) i++;
    };
    auto bad = [] { throw Error(-1, "tuning file is not a flat JSON object of \"key\": integer pairs"); };
    ws();
    if (i >= text.size() || text[i] != '{') bad();
    i++;
    ws();
    if (i < text.size() && text[i] == '}') return;
    while (true) {
        ws();
        if (i >= text.size() || text[i] != '"') bad();
        const size_t k0 = ++i;
        while (i < text.size() && text[i] != '"') i++;
        if (i >= text.size()) bad();
        const std::string key = text.substr(k0, i - k0);
        i++;
        ws();
        if (i >= text.size() || text[i] != ':') bad();
        i++;
        ws();
        const size_t v0 = i;
        while (i < text.size() && std::isdigit((unsigned char)text[i])) i++;
        if (i == v0 || i - v0 > 9) bad();
        const int v = std::atoi(text.substr(v0, i - v0).c_str());
        if (v < 1 || v > 65536) bad();
        out[key] = v;
        ws();
        if (i < text.size() && text[i] == ',') {
            i++;
            continue;
        }
        if (i < text.size() && text[i] == '}') break;
        bad();
    }
}

void tune_load(const char *path) {
    std::map<std::string, int> m;
    if (path) {
        FILE *f = std::fopen(path, "rb");
        if (!f) throw Error(-1, std::string("cannot open tuning file ") + path);
        std::string text;
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
        std::fclose(f);
        tune_parse(text, m);
    }
    TuneTable &t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    t.cap = m;
    t.env_read = true;
}

static void tune_save(const char *path) {
    std::map<std::string, int> m;
    if (FILE *f = std::fopen(path, "rb")) {
        std::string text;
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
        std::fclose(f);
        try {
            tune_parse(text, m);
        } catch (const Error &) {
            m.clear();   // an unreadable old file is replaced
        }
    }
    TuneTable &t = tune_table();
    {
        std::lock_guard<std::mutex> lk(t.mu);
        for (auto &kv : t.cap) m[kv.first] = kv.second;
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) throw Error(-1, std::string("cannot write tuning file ") + path);
    std::fprintf(f, "{");
    bool first = true;
    for (auto &kv : m) {
        std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    std::fprintf(f, "\n}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) throw Error(-1, std::string("cannot write tuning file ") + path);
}

// the grid cap of class c for R = h - 1: the tuned one, else the default
static int class_cap(int R, int c) {
    TuneTable &t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.env_read) {
        t.env_read = true;
        if (const char *e = std::getenv("DSD_TUNE_FILE")) {
            std::map<std::string, int> m;
            if (FILE *f = std::fopen(e, "rb")) {
                std::string text;
                char buf[4096];
                size_t got;
                while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
                std::fclose(f);
                try {
                    tune_parse(text, m);
                } catch (const Error &) {
                    m.clear();   // a malformed file leaves the defaults
                }
            }
            t.cap = m;
        }
    }
    if (t.cap.empty()) return default_cap(R, c);
    auto it = t.cap.find(tune_key(arch_name(), R + 1, c));
    return it == t.cap.end() ? default_cap(R, c) : it->second;
}

// one class's launch; cap: its grid cap (gs_blocks bounds the global-bitmap classes)
template <int R>
static void launch_class(int c, int cap, const DevGraph &g, const EnumCtx &base, const int32_t *lists,
                         const int32_t *off, const int32_t *cnt, hipStream_t s, Scratch &sc, int gs_blocks) {
    EnumCtx ctx = base;
    ctx.roots = lists + off[c];
    if (c == 0) {
        const int blocks = grid_for(cnt[0], WAVES_PER_BLOCK, cap);
        k_engine_wave<R, EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off, cnt[0], nullptr);
        return;
    }
    if constexpr (R <= 2) {
        if (c == 1) {
            const int blocks = grid_for(cnt[1], 1, cap);
            k_engine_block<R, 2048, 12, 1, false, EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                     cnt[1], nullptr, nullptr);
        } else if (c == 2) {
            const int blocks = grid_for(cnt[2], 1, cap);
            k_engine_huge_r2<EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off, cnt[2], nullptr);
        }
    } else {
        if (c == 1) {
            const int blocks = grid_for(cnt[1], 1, cap);
            k_engine_block<R, 256, 9, 4, false, EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                   cnt[1], nullptr, nullptr);
        } else if (c == 2) {
            const int blocks = grid_for(cnt[2], 1, cap);
            k_engine_block<R, 768, 11, 12, false, EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col,
                                                                                     g.dag_off, cnt[2], nullptr, nullptr);
        } else if (c == 3) {
            const int blocks = grid_for(cnt[3], 1, std::min(cap, gs_blocks));
            u64 *gS = sc.get_n<u64>((int64_t)blocks * 1280 * 20);
            k_engine_block<R, 1280, 12, 20, true, EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                    cnt[3], nullptr, gS);
        } else if (c == 4) {
            // hubs of out-degree 1281..2048: 32-word bitmap rows in global memory
            const int blocks = grid_for(cnt[4], 1, std::min(cap, gs_blocks));
            u64 *gS = sc.get_n<u64>((int64_t)blocks * 2048 * 32);
            k_engine_block<R, 2048, 12, 32, true, EnumCtx><<<blocks, BLOCK, 0, s>>>(ctx, g.row_ptr, g.col, g.dag_off,
                                                                                    cnt[4], nullptr, gS);
        }
    }
}

static int nclass_of(int R) { return R <= 2 ? 3 : 5; }

template <int R>
static void launch_engine(const DevGraph &g, const EnumCtx &base, const int32_t *lists, const int32_t *off,
                          const int32_t *cnt, hipStream_t s, Scratch &sc, int gs_blocks) {
    for (int c = 0; c < nclass_of(R); c++)
        if (cnt[c]) launch_class<R>(c, class_cap(R, c), g, base, lists, off, cnt, s, sc, gs_blocks);
}

static void launch_one_class(int R, int c, int cap, const DevGraph &g, const EnumCtx &ctx, const int32_t *lists,
                             const int32_t *off, const int32_t *cnt, hipStream_t s, Scratch &sc) {
    switch (R) {
        case 2: launch_class<2>(c, cap, g, ctx, lists, off, cnt, s, sc, 1 << 20); break;
        case 3: launch_class<3>(c, cap, g, ctx, lists, off, cnt, s, sc, 1 << 20); break;
        case 4: launch_class<4>(c, cap, g, ctx, lists, off, cnt, s, sc, 1 << 20); break;
        case 5: launch_class<5>(c, cap, g, ctx, lists, off, cnt, s, sc, 1 << 20); break;
        default: throw Error(-1, "h outside [2, 6]");
    }
}

// roots binned by class (rank order kept within a class); false if the
// counts could overflow 64 bits.  The host copy of off must outlive the
// stream's use of d_off (the callers synchronise before returning).
struct RootClasses {
    int32_t hc[NCLASS];
    int32_t off[NCLASS + 1];
    int32_t *lists = nullptr;
};
static bool classify_roots(const DevGraph &g, int h, const uint8_t *mask, hipStream_t s, Scratch &sc, RootClasses &rc) {
    const int32_t n = g.n;
    const int R = h - 1;
    int32_t *cursor = sc.get_n<int32_t>(NCLASS);
    u64 *bound = sc.get_n<u64>(1);
    fill_i32(cursor, 0, NCLASS, s);
    fill_u64(bound, 0, 1, s);
    int blocks = grid_for(n, BLOCK, 4096);
    k_classify<<<blocks, BLOCK, 0, s>>>(g.row_ptr, g.dag_off, mask, n, R, 0, cursor, nullptr, nullptr, bound);
    u64 hb = 0;
    DSD_HIP(hipMemcpyAsync(rc.hc, cursor, sizeof(rc.hc), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipMemcpyAsync(&hb, bound, sizeof(u64), hipMemcpyDeviceToHost, s));
    DSD_HIP(hipStreamSynchronize(s));
    if (hb == ~0ull || hb > ~0ull / (u64)h) return false;          // counts could overflow 64 bits
    if (rc.hc[5]) throw Error(-5, "an out-neighbourhood exceeds 2048 vertices (limit of the bitmap kernels, h >= 4)");
    rc.off[0] = 0;
    for (int c = 0; c < NCLASS; c++) rc.off[c + 1] = rc.off[c] + rc.hc[c];
    rc.lists = sc.get_n<int32_t>(rc.off[NCLASS]);
    int32_t *d_off = sc.get_n<int32_t>(NCLASS + 1);
    DSD_HIP(hipMemcpyAsync(d_off, rc.off, sizeof(rc.off), hipMemcpyHostToDevice, s));
    fill_i32(cursor, 0, NCLASS, s);
    k_classify<<<blocks, BLOCK, 0, s>>>(g.row_ptr, g.dag_off, mask, n, R, 1, cursor, rc.lists, d_off, bound);
    return true;
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
    RootClasses rc;
    if (!classify_roots(g, h, mask, s, sc, rc)) return false;
    EnumCtx ctx{nullptr, mask, deg};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt) {
        DSD_HIP(hipEventCreate(&e0));
        DSD_HIP(hipEventCreate(&e1));
        DSD_HIP(hipEventRecord(e0, s));
    }
    switch (R) {
        case 2: launch_engine<2>(g, ctx, rc.lists, rc.off, rc.hc, s, sc, gs_blocks); break;
        case 3: launch_engine<3>(g, ctx, rc.lists, rc.off, rc.hc, s, sc, gs_blocks); break;
        case 4: launch_engine<4>(g, ctx, rc.lists, rc.off, rc.hc, s, sc, gs_blocks); break;
        case 5: launch_engine<5>(g, ctx, rc.lists, rc.off, rc.hc, s, sc, gs_blocks); break;
        default: throw Error(-1, "h outside [2, 6]");
    }
    if (kt) {
        DSD_HIP(hipEventRecord(e1, s));
        DSD_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DSD_HIP(hipEventElapsedTime(&ms, e0, e1));
        kt->k3_ms += ms;
        for (int c = 0; c < NCLASS; c++) kt->k3_launches += rc.hc[c] ? 1 : 0;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    // the host copy of `off` must outlive the async H2D copy above
    DSD_HIP(hipStreamSynchronize(s));
    return true;
}

std::vector<TuneResult> autotune(const DevGraph &g, int h, hipStream_t s, Scratch &sc) {
    std::vector<TuneResult> out;
    if (h < 3 || h > 6) throw Error(-1, "tuning needs h in [3, 6]");
    const int32_t n = g.n;
    if (n == 0) return out;
    const int R = h - 1;
    RootClasses rc;
    if (!classify_roots(g, h, nullptr, s, sc, rc)) throw Error(-4, "clique counts could exceed 64 bits");
    u64 *deg = sc.get_n<u64>(n);
    fill_u64(deg, 0, n, s);
    EnumCtx ctx{nullptr, nullptr, deg};
    DSD_HIP(hipStreamSynchronize(s));
    hipEvent_t e0, e1;
    DSD_HIP(hipEventCreate(&e0));
    DSD_HIP(hipEventCreate(&e1));
    const std::string arch = arch_name();
    for (int c = 0; c < nclass_of(R); c++) {
        if (!rc.hc[c]) continue;
        // caps in workgroups; the wave class counts four roots a workgroup
        const int per = c == 0 ? WAVES_PER_BLOCK : 1;
        const int need = (int)std::min<int64_t>(((int64_t)rc.hc[c] + per - 1) / per, 1 << 20);
        const bool global = R >= 3 && c >= 3;
        std::vector<int> cands = global ? std::vector<int>{64, 128, 256, 512, 1024}
                                        : std::vector<int>{256, 512, 1024, 2048, 4096, 8192};
        const int def = default_cap(R, c);
        if (std::find(cands.begin(), cands.end(), def) == cands.end()) cands.push_back(def);
        TuneResult tr{c, rc.hc[c], def, def, 0.0, 0.0};
        std::map<int, double> seen;   // by effective grid
        double best = 1e300;
        for (int cap : cands) {
            const int eff = std::min(cap, need);
            double ms;
            auto it = seen.find(eff);
            if (it != seen.end()) {
                ms = it->second;
            } else {
                ms = 1e300;
                for (int rep = 0; rep < 2; rep++) {   // the faster of two runs
                    DSD_HIP(hipEventRecord(e0, s));
                    launch_one_class(R, c, cap, g, ctx, rc.lists, rc.off, rc.hc, s, sc);
                    DSD_HIP(hipEventRecord(e1, s));
                    DSD_HIP(hipEventSynchronize(e1));
                    float t = 0;
                    DSD_HIP(hipEventElapsedTime(&t, e0, e1));
                    ms = std::min(ms, (double)t);
                }
                seen[eff] = ms;
            }
            if (cap == def) tr.ms_default = ms;
            // a tie keeps the smaller grid (less scratch, fewer idle workgroups)
            if (ms < best * 0.98 || (ms <= best && cap < tr.cap_best)) {
                best = ms;
                tr.cap_best = cap;
            }
        }
        tr.ms_best = best;
        out.push_back(tr);
        TuneTable &t = tune_table();
        std::lock_guard<std::mutex> lk(t.mu);
        t.env_read = true;
        t.cap[tune_key(arch, h, c)] = tr.cap_best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    DSD_HIP(hipStreamSynchronize(s));
    return out;
}

void tune_write(const char *path) { tune_save(path); }

}  // namespace dsd
