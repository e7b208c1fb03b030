// Host exact step of CoreExact (Algorithm 4): minimum cuts over the located
// core, component by component.
//
// Networks (capacities scaled by the denominator b of alpha = a/b so that
// every capacity is an integer):
//   h = 2 (Goldberg's network, Section 4.1): s->v: b*m, v->t: b*m + 2a -
//         b*deg(v), u<->v: b for every edge.
//   h >= 3 (Algorithm 1): s->v: b*deg(v, Psi), v->t: h*a, psi->v: infinite
//         for v in psi, v->psi: b when psi + v is an h-clique; psi ranges over
//         the (h-1)-cliques that extend to an h-clique (the others carry no
//         flow).
// A subgraph denser than alpha exists iff the maximum flow is below the
// total source capacity (Lemma 14); the source side of the maximal minimum
// cut then maximises mu(S) - alpha |S| and so has density > alpha.
//
// Search: each component C (in descending density) is first tested at the
// best density l found so far; if nothing in C beats l it is skipped.
// Otherwise the density l is raised to that of the set just found and the
// test repeated until it fails (a parametric / Dinkelbach iteration on the
// same networks as Algorithm 4's binary search; densities strictly increase,
// so it ends, and the last set found is densest in C).  Before every test C
// is cut down to the ceil(l)-clique-core (Lemma 7), as Algorithm 4 does when
// its lower bound rises.
#include "exact.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <atomic>
#include <cstdlib>
#include <numeric>
#include <thread>

#include "common.hpp"
#include "flow.hpp"

namespace dsd {

typedef __int128 i128;
static const int64_t CAP_LIMIT = (int64_t)1 << 62;
// Every network is bounded before it is built: at most this many h-cliques
// (about h arcs each); the environment variable DSD_EXACT_MAX_CLIQUES lowers
// or raises it (read at every call).
static const uint64_t MAX_HOST_CLIQUES_DEFAULT = 100000000ull;
static uint64_t max_host_cliques() {
    const char *e = getenv("DSD_EXACT_MAX_CLIQUES");
    return e ? (uint64_t)strtoull(e, nullptr, 10) : MAX_HOST_CLIQUES_DEFAULT;
}
static void too_many_cliques() {
    throw Error(-5, "a flow network of the exact step would hold more h-cliques than its limit (1e8 unless "
                    "DSD_EXACT_MAX_CLIQUES says otherwise)");
}
// Networks with at least this many residual arcs get their minimum cut on the
// GPU (DSD_FLOW_GPU_MIN_ARCS overrides; a negative value keeps every cut on
// the host).  A device run that has not converged after GPU_FLOW_MAX_PASSES
// push/relabel passes is redone by the host push-relabel.
static const int64_t GPU_FLOW_MAX_PASSES = 200000;
static int64_t gpu_flow_min_arcs() {
    const char *e = getenv("DSD_FLOW_GPU_MIN_ARCS");
    return e ? (int64_t)atoll(e) : (int64_t)1 << 21;
}
// h = 3 networks of components with at least this many edges (and at most
// TRI_NET_MAX_NV vertices) are built on the device; the environment variable
// DSD_NET_GPU_MIN_EDGES overrides it (negative: always on the host)
static int64_t gpu_net_min_edges() {
    const char *e = getenv("DSD_NET_GPU_MIN_EDGES");
    return e ? (int64_t)atoll(e) : (int64_t)8192;
}

// ---------------------------------------------------------------- host threads

static int host_threads() {
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, hc ? hc : 1u));
}

// f(t, lo, hi) on T contiguous slices of [0, n) (uniform work per index)
template <class F>
static void parallel_slices(int64_t n, int T, F &&f) {
    if (T <= 1 || n < 2 * (int64_t)T) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < T; t++) {
        const int64_t lo = n * t / T, hi = n * (t + 1) / T;
        th.emplace_back([&f, t, lo, hi] { f(t, lo, hi); });
    }
    for (std::thread &x : th) x.join();
}

// f(t, i) for every i in [0, n), handed out `grain` at a time (uneven work per index)
template <class F>
static void parallel_dynamic(int64_t n, int T, int64_t grain, F &&f) {
    if (T <= 1 || n <= grain) {
        for (int64_t i = 0; i < n; i++) f(0, i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < T; t++)
        th.emplace_back([&, t] {
            while (true) {
                const int64_t lo = next.fetch_add(grain);
                if (lo >= n) return;
                const int64_t hi = std::min(n, lo + grain);
                for (int64_t i = lo; i < hi; i++) f(t, i);
            }
        });
    for (std::thread &x : th) x.join();
}

// an array that is never zero-filled: every entry is written before it is read
template <typename T>
struct RawArray {
    std::unique_ptr<T[]> p;
    int64_t n = 0;
    void alloc(int64_t k) {
        p.reset(new T[k > 0 ? k : 1]);
        n = k;
    }
    T &operator[](int64_t i) { return p[i]; }
    const T &operator[](int64_t i) const { return p[i]; }
};

// ---------------------------------------------------------------- push-relabel

class PushRelabel {
public:
    explicit PushRelabel(int n) : n_(n) {}
    void reserve(int64_t arcs) {
        if (arcs <= cap_arcs_) return;
        RawArray<int> nu, nv;
        nu.alloc(arcs);
        nv.alloc(arcs);
        for (int64_t i = 0; i < E_; i++) {
            nu[i] = eu_[i];
            nv[i] = ev_[i];
        }
        eu_ = std::move(nu);
        ev_ = std::move(nv);
        cap_arcs_ = arcs;
    }
    int arc(int u, int v) {   // capacities are set per test
        if (E_ == cap_arcs_) reserve(std::max<int64_t>(1024, 2 * cap_arcs_));
        eu_[E_] = u;
        ev_[E_] = v;
        return (int)E_++;
    }
    // room for `more` arcs written in place by set_arc; returns the first index
    int64_t grow(int64_t more) {
        reserve(E_ + more);
        const int64_t at = E_;
        E_ += more;
        return at;
    }
    void set_arc(int64_t i, int u, int v) {
        eu_[i] = u;
        ev_[i] = v;
    }
    // Residual CSR: every arc and its reverse.  Each thread takes a slice of
    // the arcs; per-thread counts per node give every thread its own range in
    // every node's list.
    void build() {
        const int64_t E = E_;
        if (2 * E > (int64_t)0x7fffffff)
            throw Error(-5, "flow network has more than 2^31 residual arcs (limit of the host solver)");
        const int T = E < (1 << 20) ? 1 : host_threads();
        std::vector<std::vector<int>> cnt(T, std::vector<int>(n_, 0));
        parallel_slices(E, T, [&](int t, int64_t lo, int64_t hi) {
            int *c = cnt[t].data();
            for (int64_t i = lo; i < hi; i++) {
                c[eu_[i]]++;
                c[ev_[i]]++;
            }
        });
        first_.assign(n_ + 1, 0);
        {
            int64_t run = 0;
            for (int v = 0; v < n_; v++) {
                first_[v] = (int)run;
                for (int t = 0; t < T; t++) {
                    const int c = cnt[t][v];
                    cnt[t][v] = (int)run;        // thread t's next slot in v's list
                    run += c;
                }
            }
            first_[n_] = (int)run;
        }
        const int64_t A = 2 * E;
        to_.alloc(A);     // every slot is written once below
        rev_.alloc(A);
        fwd_.alloc(E);
        cap_.alloc(A);    // every arc's capacity is set (set()) before each flow
        parallel_slices(E, T, [&](int t, int64_t lo, int64_t hi) {
            int *fill = cnt[t].data();
            for (int64_t i = lo; i < hi; i++) {
                const int pu = fill[eu_[i]]++, pv = fill[ev_[i]]++;
                to_[pu] = ev_[i];
                to_[pv] = eu_[i];
                rev_[pu] = pv;
                rev_[pv] = pu;
                fwd_[i] = pu;
            }
        });
    }
    // capacity of arc i (forward) and of its reverse
    void set(int i, int64_t c, int64_t rc = 0) {
        cap_[fwd_[i]] = c;
        cap_[rev_[fwd_[i]]] = rc;
    }
    int nodes() const { return n_; }
    int64_t arcs() const { return E_; }
    int64_t residual_arcs() const { return 2 * E_; }
    // all arcs at once: f(eu, ev) fills arrays of `arcs` entries
    template <class F>
    void load(int64_t arcs, F &&f) {
        reserve(arcs);
        E_ = arcs;
        f(eu_.p.get(), ev_.p.get());
    }
    const int *eu_data() const { return eu_.p.get(); }
    const int *ev_data() const { return ev_.p.get(); }
    // the residual CSR is built on first use by the host maximum flow
    void ensure_built() {
        if (!built_) build();
        built_ = true;
    }

    int64_t maxflow(int s, int t) {
        ex_.assign(n_, 0);
        ht_.assign(n_, 0);
        cnt_.assign(2 * n_ + 2, 0);
        cur_.assign(first_.begin(), first_.end() - 1);
        s_ = s;
        t_ = t;
        for (int a = first_[s]; a < first_[s + 1]; a++) {
            int64_t f = cap_[a];
            if (f <= 0) continue;
            cap_[a] = 0;
            cap_[rev_[a]] += f;
            ex_[to_[a]] += f;
            ex_[s] -= f;
        }
        global_relabel();
        int64_t work = 0;
        while (!q_.empty()) {
            int u = q_.front();
            q_.pop_front();
            inq_[u] = 0;
            if (ht_[u] >= n_ || ex_[u] <= 0) continue;
            discharge(u, work);
            if (work > 6 * (int64_t)n_ + to_.n / 2) {
                work = 0;
                global_relabel();
            }
        }
        return ex_[t];
    }

    // nodes that still reach t in the residual network
    void reach_sink(int t, std::vector<char> &seen) const {
        seen.assign(n_, 0);
        std::vector<int> st{t};
        seen[t] = 1;
        while (!st.empty()) {
            int v = st.back();
            st.pop_back();
            for (int a = first_[v]; a < first_[v + 1]; a++) {
                int u = to_[a];
                if (!seen[u] && cap_[rev_[a]] > 0) {
                    seen[u] = 1;
                    st.push_back(u);
                }
            }
        }
    }

private:
    void global_relabel() {
        std::fill(ht_.begin(), ht_.end(), n_);
        std::fill(cnt_.begin(), cnt_.end(), 0);
        std::vector<int> bfs{t_};
        ht_[t_] = 0;
        for (size_t i = 0; i < bfs.size(); i++) {
            int v = bfs[i];
            for (int a = first_[v]; a < first_[v + 1]; a++) {
                int u = to_[a];
                if (ht_[u] == n_ && u != s_ && cap_[rev_[a]] > 0) {
                    ht_[u] = ht_[v] + 1;
                    bfs.push_back(u);
                }
            }
        }
        ht_[s_] = n_;
        q_.clear();
        inq_.assign(n_, 0);
        for (int v = 0; v < n_; v++) {
            if (ht_[v] < n_) cnt_[ht_[v]]++;
            cur_[v] = first_[v];
            if (v != s_ && v != t_ && ex_[v] > 0 && ht_[v] < n_) {
                q_.push_back(v);
                inq_[v] = 1;
            }
        }
    }

    void discharge(int u, int64_t &work) {
        while (ex_[u] > 0) {
            if (cur_[u] == first_[u + 1]) {
                relabel(u);
                work += first_[u + 1] - first_[u] + 12;
                if (ht_[u] >= n_) return;
                cur_[u] = first_[u];
                continue;
            }
            int a = cur_[u], v = to_[a];
            if (cap_[a] > 0 && ht_[u] == ht_[v] + 1) {
                int64_t d = ex_[u] < cap_[a] ? ex_[u] : cap_[a];
                cap_[a] -= d;
                cap_[rev_[a]] += d;
                ex_[u] -= d;
                ex_[v] += d;
                if (v != s_ && v != t_ && !inq_[v]) {
                    q_.push_back(v);
                    inq_[v] = 1;
                }
            } else {
                cur_[u]++;
            }
        }
    }

    void relabel(int u) {
        int old = ht_[u], nh = 2 * n_;
        for (int a = first_[u]; a < first_[u + 1]; a++)
            if (cap_[a] > 0 && ht_[to_[a]] + 1 < nh) nh = ht_[to_[a]] + 1;
        if (old < n_ && --cnt_[old] == 0) {
            // gap: nothing at height `old` any more, so nothing above it reaches t
            for (int w = 0; w < n_; w++)
                if (ht_[w] > old && ht_[w] < n_) {
                    cnt_[ht_[w]]--;
                    ht_[w] = n_;
                }
            ht_[u] = n_;
            return;
        }
        ht_[u] = nh < n_ ? nh : n_;
        if (ht_[u] < n_) cnt_[ht_[u]]++;
    }

    int n_, s_ = 0, t_ = 1;
    bool built_ = false;
    int64_t E_ = 0, cap_arcs_ = 0;
    RawArray<int> eu_, ev_, fwd_, to_, rev_;
    RawArray<int64_t> cap_;
    std::vector<int> first_, ht_, cnt_, cur_;
    std::vector<char> inq_;
    std::vector<int64_t> ex_;
    std::deque<int> q_;
};

// ---------------------------------------------------------------- host clique listing

// Lists the cliques of size `size` inside `in` (membership over local ids)
// whose smallest member is `root`, in increasing id order; calls
// f(const int32_t *members).  One lister per thread.
struct CliqueLister {
    const LocatedCore &lc;
    const std::vector<char> &in;
    int size;
    std::vector<std::vector<int32_t>> cand;
    std::vector<int32_t> mem;
    CliqueLister(const LocatedCore &l, const std::vector<char> &i, int sz)
        : lc(l), in(i), size(sz), cand(sz + 1), mem(sz) {}

    template <class F>
    void go(int depth, F &f) {
        const std::vector<int32_t> &c = cand[depth];
        for (size_t i = 0; i < c.size(); i++) {
            int32_t x = c[i];
            mem[depth] = x;
            if (depth + 1 == size) {
                f(mem.data());
                continue;
            }
            std::vector<int32_t> &nx = cand[depth + 1];
            nx.clear();
            const int32_t *a = lc.adj.data() + lc.off[x], *ae = lc.adj.data() + lc.off[x + 1];
            size_t j = i + 1;
            while (j < c.size() && a < ae) {
                if (c[j] < *a) j++;
                else if (c[j] > *a) a++;
                else { nx.push_back(c[j]); j++; a++; }
            }
            if (!nx.empty()) go(depth + 1, f);
        }
    }

    template <class F>
    void root(int32_t v, F &&f) {
        if (!in[v]) return;
        mem[0] = v;
        if (size == 1) {
            f(mem.data());
            return;
        }
        cand[1].clear();
        for (int64_t e = lc.off[v]; e < lc.off[v + 1]; e++) {
            int32_t w = lc.adj[e];
            if (w > v && in[w]) cand[1].push_back(w);
        }
        if (!cand[1].empty()) go(1, f);
    }
};

template <class F>
static void list_cliques(const LocatedCore &lc, const std::vector<char> &in, int size, F &&f) {
    CliqueLister L(lc, in, size);
    for (int32_t v = 0; v < (int32_t)lc.rank.size(); v++) L.root(v, f);
}

// h-cliques inside verts, counted on all host threads (roots handed out
// dynamically); throws once the count passes MAX_HOST_CLIQUES
uint64_t count_cliques_host(const LocatedCore &lc, int h, const std::vector<int32_t> &verts) {
    std::vector<char> in(lc.rank.size(), 0);
    for (int32_t v : verts) in[v] = 1;
    const int T = host_threads();
    std::vector<uint64_t> cnt(T, 0);
    std::atomic<uint64_t> total{0};
    std::atomic<bool> over{false};
    std::vector<CliqueLister> lister;
    for (int t = 0; t < T; t++) lister.emplace_back(lc, in, h);
    const uint64_t limit = max_host_cliques();
    parallel_dynamic((int64_t)verts.size(), T, 4, [&](int t, int64_t i) {
        if (over.load(std::memory_order_relaxed)) return;
        uint64_t c = 0;
        lister[t].root(verts[i], [&](const int32_t *) { c++; });
        cnt[t] += c;
        if (total.fetch_add(c) + c > limit) over = true;
    });
    if (over) too_many_cliques();
    uint64_t c = 0;
    for (uint64_t x : cnt) c += x;
    return c;
}

// h-cliques inside verts: the triangles of a large set on the device (the
// listing that builds the h = 3 networks), everything else on the host
static uint64_t count_cliques(const LocatedCore &lc, int h, const std::vector<int32_t> &verts) {
    if (h == 3 && gpu_net_min_edges() >= 0 && verts.size() >= 2 && verts.size() <= (size_t)TRI_NET_MAX_NV) {
        std::vector<int32_t> sorted(verts);
        std::sort(sorted.begin(), sorted.end());
        std::vector<int32_t> idx(lc.rank.size(), -1);
        for (size_t i = 0; i < sorted.size(); i++) idx[sorted[i]] = (int32_t)i;
        const int nv = (int)sorted.size();
        std::vector<int64_t> so(nv + 1, 0), fwd(nv);
        std::vector<int32_t> sa;
        for (int i = 0; i < nv; i++) {
            const int32_t v = sorted[i];
            for (int64_t e = lc.off[v]; e < lc.off[v + 1]; e++)
                if (idx[lc.adj[e]] >= 0) sa.push_back(idx[lc.adj[e]]);   // idx is increasing: rows stay sorted
            so[i + 1] = (int64_t)sa.size();
        }
        for (int i = 0; i < nv; i++) {
            int64_t a = so[i];
            while (a < so[i + 1] && sa[a] < i) a++;
            fwd[i] = a;
        }
        if ((int64_t)sa.size() / 2 >= std::max<int64_t>(1, gpu_net_min_edges()))
            return count_triangles_device(nv, so.data(), sa.data(), fwd.data());
    }
    return count_cliques_host(lc, h, verts);
}

// ---------------------------------------------------------------- one component

static uint64_t ceil_div_u(uint64_t a, uint64_t b) { return a / b + (a % b != 0); }
static bool frac_less(const Rational &x, const Rational &y) {   // x < y
    return (unsigned __int128)x.num * y.den < (unsigned __int128)y.num * x.den;
}
static Rational reduced(uint64_t a, uint64_t b) {
    if (a == 0) return {0, 1};
    uint64_t x = a, y = b;
    while (y) { uint64_t t = x % y; x = y; y = t; }
    return {a / x, b / x};
}

// Network over the vertex set `verts` of one component.
class CompNet {
public:
    CompNet(const LocatedCore &lc, int h, const std::vector<int32_t> &verts) : lc_(lc), h_(h), verts_(verts) {
        const int32_t S = (int32_t)lc.rank.size();
        in_.assign(S, 0);
        for (int32_t v : verts) in_[v] = 1;
        idx_.assign(S, -1);
        for (size_t i = 0; i < verts.size(); i++) idx_[verts[i]] = (int32_t)i;
        const int nv = (int)verts.size();
        deg_.assign(nv, 0);
        if (h == 2) {
            net_ = new PushRelabel(2 + nv);
            m_ = 0;
            for (int i = 0; i < nv; i++) {
                src_.push_back(net_->arc(0, 2 + i));
                snk_.push_back(net_->arc(2 + i, 1));
                int32_t v = verts[i];
                for (int64_t e = lc.off[v]; e < lc.off[v + 1]; e++) {
                    int32_t w = lc.adj[e];
                    if (!in_[w]) continue;
                    deg_[i]++;
                    if (w > v) {
                        mid_.push_back(net_->arc(2 + i, 2 + idx_[w]));
                        m_++;
                    }
                }
            }
            mu_ = m_;
        } else if (h == 3) {
            build_triangle_net(verts);
        } else {
            // bounded first: the listing below holds every clique in memory
            (void)count_cliques_host(lc, h, verts);
            // h-cliques, and the (h-1)-cliques they contain, as sorted tuples
            const int r = h - 1;
            std::vector<int32_t> cl;
            list_cliques(lc, in_, h, [&](const int32_t *mem) { cl.insert(cl.end(), mem, mem + h); });
            mu_ = cl.size() / h;
            std::vector<int32_t> tup;
            tup.reserve(mu_ * h * r);
            for (uint64_t c = 0; c < mu_; c++) {
                const int32_t *K = &cl[c * h];
                for (int i = 0; i < h; i++) deg_[idx_[K[i]]]++;
                for (int drop = 0; drop < h; drop++)
                    for (int i = 0; i < h; i++)
                        if (i != drop) tup.push_back(K[i]);
            }
            const uint64_t T = mu_ * h;
            if (T > 0xffffffffull) too_many_cliques();   // tuple ids are 32-bit
            std::vector<uint32_t> ord(T);
            std::iota(ord.begin(), ord.end(), 0u);
            std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
                const int32_t *ta = &tup[(size_t)a * r], *tb = &tup[(size_t)b * r];
                return std::lexicographical_compare(ta, ta + r, tb, tb + r);
            });
            std::vector<int32_t> psi_of(T);
            int64_t npsi = 0;
            for (uint64_t i = 0; i < T; i++) {
                if (i > 0 && std::equal(&tup[(size_t)ord[i] * r], &tup[(size_t)ord[i] * r] + r,
                                        &tup[(size_t)ord[i - 1] * r])) {
                    psi_of[ord[i]] = psi_of[ord[i - 1]];
                } else {
                    psi_of[ord[i]] = (int32_t)npsi;
                    psi_first_.push_back(ord[i]);
                    npsi++;
                }
            }
            const int64_t base = 2 + nv;
            if (base + npsi > 0x7fffffff) throw Error(-5, "flow network too large");
            net_ = new PushRelabel((int)(base + npsi));
            for (int i = 0; i < nv; i++) {
                src_.push_back(net_->arc(0, 2 + i));
                snk_.push_back(net_->arc(2 + i, 1));
            }
            for (int64_t p = 0; p < npsi; p++)
                for (int i = 0; i < r; i++)
                    inf_.push_back(net_->arc((int)(base + p), 2 + idx_[tup[(size_t)psi_first_[p] * r + i]]));
            for (uint64_t c = 0; c < mu_; c++) {
                const int32_t *K = &cl[c * h];
                for (int drop = 0; drop < h; drop++)
                    mid_.push_back(net_->arc(2 + idx_[K[drop]], (int)(base + psi_of[c * h + drop])));
            }
        }
    }
    // h = 3: psi ranges over the edges of the vertex set (an edge is the
    // 2-clique left when one vertex of a triangle is taken away).  Triangles
    // i < j < k come from merging the forward parts of rows i and j; the
    // merge yields the positions, and hence the edge ids, of (i,k) and (j,k).
    void build_triangle_net(const std::vector<int32_t> &verts) {
        const int nv = (int)verts.size();
        std::vector<int64_t> so(nv + 1, 0);
        std::vector<int32_t> sa;
        for (int i = 0; i < nv; i++) {
            int32_t v = verts[i];
            for (int64_t e = lc_.off[v]; e < lc_.off[v + 1]; e++)
                if (in_[lc_.adj[e]]) sa.push_back(idx_[lc_.adj[e]]);   // idx_ is increasing: rows stay sorted
            so[i + 1] = (int64_t)sa.size();
        }
        std::vector<int64_t> fwd(nv);
        for (int i = 0; i < nv; i++) {
            int64_t a = so[i];
            while (a < so[i + 1] && sa[a] < i) a++;
            fwd[i] = a;
        }
        const int64_t edges = (int64_t)sa.size() / 2;
        if (gpu_net_min_edges() >= 0 && edges >= std::max<int64_t>(1, gpu_net_min_edges()) && nv <= TRI_NET_MAX_NV) {
            // the same network, node and arc numbering built on the device
            gpu_ = GpuFlow::triangles(nv, so.data(), sa.data(), fwd.data(), deg_, &mu_);
            dev_ = true;
            np_ = edges;
            return;
        }
        std::vector<int32_t> eid(sa.size(), -1);
        int64_t npsi = 0;
        for (int i = 0; i < nv; i++)
            for (int64_t e = fwd[i]; e < so[i + 1]; e++) eid[e] = (int32_t)npsi++;
        const int64_t base = 2 + nv;
        if (base + npsi > 0x7fffffff) throw Error(-5, "flow network too large");
        // triangles per vertex i (i the lowest of the three), so that every
        // vertex's arcs go to a range of their own
        const int T = host_threads();
        std::vector<uint64_t> tri_of(nv + 1, 0);
        auto merge = [&](int i, int64_t a, auto &&emit) {
            const int j = sa[a];
            int64_t p = a + 1, q = fwd[j];
            while (p < so[i + 1] && q < so[j + 1]) {
                if (sa[p] < sa[q]) p++;
                else if (sa[p] > sa[q]) q++;
                else {
                    emit(j, p, q);
                    p++;
                    q++;
                }
            }
        };
        parallel_dynamic(nv, T, 4, [&](int, int64_t i) {
            uint64_t c = 0;
            for (int64_t a = fwd[i]; a < so[i + 1]; a++) merge((int)i, a, [&](int, int64_t, int64_t) { c++; });
            tri_of[i + 1] = c;
        });
        for (int i = 0; i < nv; i++) tri_of[i + 1] += tri_of[i];
        const uint64_t tri = tri_of[nv];
        if (tri > max_host_cliques()) too_many_cliques();
        mu_ = tri;
        net_ = new PushRelabel((int)(base + npsi));
        net_->reserve(2 * (int64_t)nv + 2 * npsi + 3 * (int64_t)tri);
        for (int i = 0; i < nv; i++) {
            src_.push_back(net_->arc(0, 2 + i));
            snk_.push_back(net_->arc(2 + i, 1));
        }
        inf_.reserve(2 * npsi);
        for (int i = 0; i < nv; i++)
            for (int64_t a = fwd[i]; a < so[i + 1]; a++) {
                inf_.push_back(net_->arc((int)(base + eid[a]), 2 + i));
                inf_.push_back(net_->arc((int)(base + eid[a]), 2 + sa[a]));
            }
        const int64_t m0 = net_->grow(3 * (int64_t)tri);
        mid_.resize(3 * tri);
        std::vector<uint64_t> tdeg((size_t)T * nv, 0);   // per-thread triangle counts per vertex
        parallel_dynamic(nv, T, 4, [&](int t, int64_t i) {
            uint64_t *dg = tdeg.data() + (size_t)t * nv;
            {
                int64_t at = 3 * (int64_t)tri_of[i];
                for (int64_t a = fwd[i]; a < so[i + 1]; a++)
                    merge((int)i, a, [&](int j, int64_t p, int64_t q) {
                        const int k = sa[p];
                        net_->set_arc(m0 + at, 2 + (int)i, (int)(base + eid[q]));   // i with edge (j, k)
                        net_->set_arc(m0 + at + 1, 2 + j, (int)(base + eid[p]));    // j with edge (i, k)
                        net_->set_arc(m0 + at + 2, 2 + k, (int)(base + eid[a]));    // k with edge (i, j)
                        mid_[at] = (int)(m0 + at);
                        mid_[at + 1] = (int)(m0 + at + 1);
                        mid_[at + 2] = (int)(m0 + at + 2);
                        dg[i]++;
                        dg[j]++;
                        dg[k]++;
                        at += 3;
                    });
            }
        });
        for (int t = 0; t < T; t++)
            for (int i = 0; i < nv; i++) deg_[i] += tdeg[(size_t)t * nv + i];
    }

    ~CompNet() { delete net_; }
    CompNet(const CompNet &) = delete;
    CompNet &operator=(const CompNet &) = delete;

    uint64_t mu() const { return mu_; }
    bool built_on_device() const { return dev_; }
    int nodes() const { return net_ ? net_->nodes() : gpu_->nodes(); }
    int64_t gpu_calls() const { return gpu_calls_; }
    double setup_ms() const { return setup_ms_; }

    // Vertices (local ids of the located core, members of this network) that
    // every cut must keep on the source side: their source arcs become
    // infinite.  Call before the first test.
    void force(const std::vector<int32_t> &q) {
        forced_.assign(verts_.size(), 0);
        for (int32_t v : q)
            if (idx_[v] >= 0) forced_[idx_[v]] = 1;
        if (dev_ && gpu_) gpu_->force_sources(forced_);
    }

    // Strict test at alpha = a/b.  Returns true and the found set (local ids)
    // when some subgraph of this vertex set is denser than alpha.
    bool denser_than(uint64_t a, uint64_t b, std::vector<int32_t> &found) {
        const int nv = (int)verts_.size();
        // every capacity must fit in 63 bits, and the infinite arcs above the total
        i128 srcsum = 0;
        for (int i = 0; i < nv; i++) {
            i128 cs, ct;
            if (h_ == 2) {
                cs = (i128)b * (i128)m_;
                ct = cs + 2 * (i128)a - (i128)b * (i128)deg_[i];
            } else {
                cs = (i128)b * (i128)deg_[i];
                ct = (i128)h_ * (i128)a;
            }
            if (cs >= CAP_LIMIT || ct >= CAP_LIMIT || ct < 0) throw Error(-4, "scaled capacity overflow");
            srcsum += cs;
        }
        if (srcsum * 2 >= CAP_LIMIT) throw Error(-4, "scaled capacity overflow");
        // infinity: above every finite cut.  Without forced vertices the cut
        // {s} bounds the minimum by the source total; with them the minimum
        // can exceed it, so infinity must exceed every finite capacity.
        i128 inf = srcsum + 1;
        if (!forced_.empty()) {
            i128 fin = srcsum;
            for (int i = 0; i < nv; i++)
                fin += h_ == 2 ? (i128)b * (i128)m_ + 2 * (i128)a : (i128)h_ * (i128)a;
            fin += (i128)b * (i128)mids();
            if (h_ == 2) fin += (i128)b * (i128)mids();
            inf = fin + 1;
            if (inf >= CAP_LIMIT) throw Error(-4, "scaled capacity overflow");
        }
        const FlowTest test{h_, (int64_t)a, (int64_t)b, (int64_t)m_, (int64_t)inf};
        int64_t f = 0;
        std::vector<char> reach;
        bool done = false;
        const int64_t res_arcs = net_ ? net_->residual_arcs() : 2 * gpu_->arcs();
        const bool use_gpu = gpu_flow_min_arcs() >= 0 && res_arcs >= gpu_flow_min_arcs();
        if (use_gpu) {
            // the arcs go to the device once; the device sets each test's capacities
            if (!gpu_) {
                std::vector<uint8_t> cls(net_->arcs());
                for (int e : src_) cls[e] = ARC_SRC;
                for (size_t i = 0; i < forced_.size(); i++)
                    if (forced_[i]) cls[src_[i]] = ARC_INF;
                for (int e : snk_) cls[e] = ARC_SNK;
                for (int e : inf_) cls[e] = ARC_INF;
                parallel_slices((int64_t)mid_.size(), host_threads(), [&](int, int64_t lo, int64_t hi) {
                    for (int64_t i = lo; i < hi; i++) cls[mid_[i]] = ARC_MID;
                });
                const auto t0 = std::chrono::steady_clock::now();
                gpu_.reset(new GpuFlow(net_->nodes(), net_->arcs(), net_->eu_data(), net_->ev_data(), cls.data(), nv,
                                       deg_.data()));
                setup_ms_ += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            f = gpu_->maxflow(test, reach, GPU_FLOW_MAX_PASSES, &done);
            if (done) gpu_calls_++;
        }
        if (!done) {
            if (!net_) {
                adopt_device_net();
                if (!use_gpu) gpu_.reset();
            }
            net_->ensure_built();
            for (int i = 0; i < nv; i++) {
                const bool fv = !forced_.empty() && forced_[i];
                if (h_ == 2) {
                    const int64_t cs = test.b * test.m;
                    net_->set(src_[i], fv ? test.inf : cs);
                    net_->set(snk_[i], cs + 2 * test.a - test.b * (int64_t)deg_[i]);
                } else {
                    net_->set(src_[i], fv ? test.inf : test.b * (int64_t)deg_[i]);
                    net_->set(snk_[i], (int64_t)h_ * test.a);
                }
            }
            if (h_ == 2) {
                set_all(mid_, test.b, test.b);
            } else {
                set_all(inf_, test.inf, 0);
                set_all(mid_, test.b, 0);
            }
            f = net_->maxflow(0, 1);
            if ((i128)f < srcsum) net_->reach_sink(1, reach);
        }
        if ((i128)f >= srcsum) return false;
        found.clear();
        for (int i = 0; i < nv; i++)
            if (!reach[2 + i]) found.push_back(verts_[i]);
        return !found.empty();
    }

private:
    int64_t mids() const { return dev_ && !net_ ? 3 * (int64_t)mu_ : (int64_t)mid_.size(); }

    // a device-built network copied to the host maximum flow, in the arc
    // order the device built it (source, sink, infinite, then triangle arcs)
    void adopt_device_net() {
        const int nv = (int)verts_.size();
        net_ = new PushRelabel(gpu_->nodes());
        net_->load(gpu_->arcs(), [&](int *eu, int *ev) { gpu_->download_arcs(eu, ev); });
        src_.resize(nv);
        snk_.resize(nv);
        for (int i = 0; i < nv; i++) {
            src_[i] = i;
            snk_[i] = nv + i;
        }
        inf_.resize(2 * np_);
        std::iota(inf_.begin(), inf_.end(), 2 * nv);
        mid_.resize(3 * mu_);
        std::iota(mid_.begin(), mid_.end(), (int)(2 * nv + 2 * np_));
    }

    void set_all(const std::vector<int> &arcs, int64_t c, int64_t rc) {
        parallel_slices((int64_t)arcs.size(), arcs.size() < (1u << 20) ? 1 : host_threads(),
                        [&](int, int64_t lo, int64_t hi) {
                            for (int64_t i = lo; i < hi; i++) net_->set(arcs[i], c, rc);
                        });
    }

    const LocatedCore &lc_;
    int h_;
    std::vector<int32_t> verts_;
    std::vector<char> in_;
    std::vector<int32_t> idx_;
    std::vector<uint64_t> deg_;
    std::vector<int> src_, snk_, mid_, inf_;
    std::vector<char> forced_;
    std::vector<uint32_t> psi_first_;
    uint64_t mu_ = 0, m_ = 0;
    PushRelabel *net_ = nullptr;
    std::unique_ptr<GpuFlow> gpu_;
    bool dev_ = false;   // built on the device (h = 3): gpu_ holds the network until the host needs it
    int64_t np_ = 0;     // edge nodes of a device-built network
    int64_t gpu_calls_ = 0;
    double setup_ms_ = 0;
};

bool exact_search(const LocatedCore &lc, int h, uint64_t kpp, Rational &l, std::vector<int32_t> &best,
                  ExactStats &st) {
    const int32_t S = (int32_t)lc.rank.size();
    // group vertices by component
    std::vector<int32_t> order(S);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return lc.label[a] != lc.label[b] ? lc.label[a] < lc.label[b] : a < b;
    });
    struct Comp {
        std::vector<int32_t> v;
        Rational dens;
    };
    std::vector<Comp> comps;
    for (int32_t i = 0; i < S;) {
        int32_t j = i;
        Comp c;
        while (j < S && lc.label[order[j]] == lc.label[order[i]]) c.v.push_back(order[j++]);
        i = j;
        if (c.v.size() < 2) continue;
        comps.push_back(std::move(c));
    }
    // every component's h-cliques, from the GPU's counts when the caller has
    // them: a component whose network would pass the limit is refused before
    // anything is built, and the components are searched densest first
    auto gpu_mu = [&](int32_t label, uint64_t *mu) {
        auto it = std::lower_bound(lc.comp_mu.begin(), lc.comp_mu.end(), std::make_pair(label, (uint64_t)0));
        if (it == lc.comp_mu.end() || it->first != label) return false;
        *mu = it->second;
        return true;
    };
    for (Comp &c : comps) {
        uint64_t mu = 0;
        if (!gpu_mu(lc.label[c.v[0]], &mu)) {
            if (comps.size() == 1) continue;   // one component needs no order
            mu = count_cliques(lc, h, c.v);
        }
        if (h >= 4 && mu > max_host_cliques()) too_many_cliques();
        c.dens = reduced(mu, c.v.size());
    }
    if (comps.size() > 1)
        std::stable_sort(comps.begin(), comps.end(),
                         [](const Comp &a, const Comp &b) { return frac_less(b.dens, a.dens); });
    bool improved = false;
    std::vector<int32_t> found, cur, built;
    for (const Comp &c : comps) {
        Rational lc_l = l;
        std::vector<int32_t> U;
        std::unique_ptr<CompNet> net;
        while (true) {
            // Lemma 7: anything denser than l lies in the ceil(l)-clique-core
            uint64_t floor_k = std::max<uint64_t>(kpp, ceil_div_u(lc_l.num, lc_l.den));
            cur.clear();
            for (int32_t v : c.v)
                if (lc.core[v] >= floor_k) cur.push_back(v);
            if (cur.size() < 2) break;
            auto t0 = std::chrono::steady_clock::now();
            if (!net || cur != built) {
                net.reset(new CompNet(lc, h, cur));
                built = cur;
                st.gpu_networks += net->built_on_device();
            }
            auto t1 = std::chrono::steady_clock::now();
            st.max_nodes = std::max<int64_t>(st.max_nodes, net->nodes());
            st.flow_calls++;
            const int64_t g0 = net->gpu_calls();
            const double s0 = net->setup_ms();
            bool denser = net->denser_than(lc_l.num, lc_l.den, found);
            st.gpu_flow_calls += net->gpu_calls() - g0;
            st.setup_ms += net->setup_ms() - s0;
            auto t2 = std::chrono::steady_clock::now();
            st.build_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
            st.flow_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
            if (!denser) break;
            U = found;
            lc_l = reduced(count_cliques(lc, h, U), U.size());
        }
        if (!U.empty() && frac_less(l, lc_l)) {
            l = lc_l;
            best = U;
            improved = true;
        }
    }
    return improved;
}

bool exact_search_query(const LocatedCore &lc, int h, uint64_t x, const std::vector<int32_t> &q, Rational &l,
                        std::vector<int32_t> &best, ExactStats &st) {
    const int32_t S = (int32_t)lc.rank.size();
    bool improved = false;
    std::vector<int32_t> cur, built, found;
    std::unique_ptr<CompNet> net;
    while (true) {
        // the densest set containing q lies in R_k for k = min(x, ceil(l))
        const uint64_t floor_k = std::min<uint64_t>(x, ceil_div_u(l.num, l.den));
        cur.clear();
        for (int32_t v = 0; v < S; v++)
            if (lc.core[v] >= floor_k) cur.push_back(v);
        auto t0 = std::chrono::steady_clock::now();
        if (!net || cur != built) {
            net.reset(new CompNet(lc, h, cur));
            net->force(q);
            built = cur;
            st.gpu_networks += net->built_on_device();
        }
        auto t1 = std::chrono::steady_clock::now();
        st.max_nodes = std::max<int64_t>(st.max_nodes, net->nodes());
        st.flow_calls++;
        const int64_t g0 = net->gpu_calls();
        const double s0 = net->setup_ms();
        const bool denser = net->denser_than(l.num, l.den, found);
        st.gpu_flow_calls += net->gpu_calls() - g0;
        st.setup_ms += net->setup_ms() - s0;
        auto t2 = std::chrono::steady_clock::now();
        st.build_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
        st.flow_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
        if (!denser) break;
        const Rational d = reduced(count_cliques(lc, h, found), found.size());
        if (!frac_less(l, d)) break;
        l = d;
        best = found;
        improved = true;
    }
    return improved;
}

}  // namespace dsd
