// The graph handle behind the C ABI and the driver helpers shared by the
// single-graph entry points, the batch and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dsd.h"
#include "exact.hpp"
#include "graph.hpp"

namespace dsd {

// A full (k, Psi)-core decomposition, kept on the handle: the graph never
// changes, so later calls with the same h reuse it.
struct Decomp {
    bool valid = false;
    u64 mu = 0;
    u64 *core = nullptr;            // device, rank space, length n
    PeelResult levels;              // level table
    double t_enum_ms = 0, t_peel_ms = 0;
    KernelTimes kt;
};

}  // namespace dsd

struct dsd_graph_s {
    dsd::DevGraph g;
    hipStream_t stream = nullptr;
    dsd::Scratch sc;
    dsd::Scratch keep{(size_t)1 << 20};   // the handle's own arrays: CSR, triangle lists, core numbers
    dsd_stats stats{};
    dsd::Decomp dec[7];             // by h
    dsd::TriList tl;                // triangle lists, built by the first h = 3 decomposition that wants them
    bool tl_tried = false;
    bool time_main = false;         // dsd_set_kernel_timing
    ~dsd_graph_s() {
        (void)hipStreamSynchronize(stream);
        dsd::free_tri_list(tl);
        dsd::free_graph(g);
        // the stream is idle: the next handle reuses the chunks (the core
        // numbers, lists and CSR live in keep)
        sc.recycle();
        keep.recycle();
    }
};

namespace dsd {

// A call's scratch goes back to the shared chunk pool when the call returns
// (error or not), once the handle's stream is idle: an idle handle holds only
// its own arrays (keep), so thousands of handles cost their CSRs, not a
// scratch chunk each.
struct ScratchRelease {
    dsd_graph_s *G;
    ~ScratchRelease() {
        (void)hipStreamSynchronize(G->stream);
        G->sc.recycle();
    }
};

// records the message for dsd_last_error and returns the status
dsd_status fail(int st, const std::string &msg);

#define DSD_TRY(...)                                                      \
    try {                                                                 \
        __VA_ARGS__                                                       \
    } catch (const dsd::Error &e) {                                       \
        return dsd::fail(e.status, e.what());                             \
    } catch (const std::bad_alloc &) {                                    \
        return dsd::fail(DSD_ENOMEM, "host allocation failed");           \
    } catch (const std::exception &e) {                                   \
        return dsd::fail(DSD_EDEVICE, e.what());                          \
    }

// HIP-event timer on one stream
struct Timer {
    hipStream_t s;
    hipEvent_t a, b;
    explicit Timer(hipStream_t st) : s(st) {
        DSD_HIP(hipEventCreate(&a));
        DSD_HIP(hipEventCreate(&b));
        DSD_HIP(hipEventRecord(a, s));
    }
    double stop() {
        DSD_HIP(hipEventRecord(b, s));
        DSD_HIP(hipEventSynchronize(b));
        float ms = 0;
        DSD_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

void check_device();
void check_h(int h);
void check_out(const void *p, int mem);
dsd_rational make_rational(u64 num, u64 den);
bool rat_gt(u64 a, u64 b, u64 c, u64 d);   // a/b > c/d
u64 ceil_div_u(u64 a, u64 b);
void begin_stats(dsd_graph_s *G);
void end_stats(dsd_graph_s *G, const KernelTimes &kt);
// clique-degrees (rank space) inside mask and their total mu; throws on overflow
u64 degrees_and_mu(dsd_graph_s *G, int h, const uint8_t *mask, u64 *deg, KernelTimes *kt = nullptr);
// the handle's triangle lists, built on first use (deg: whole-graph triangle
// degrees, mu triangles) if they fit; nullptr if not
const TriList *tri_lists(dsd_graph_s *G, const u64 *deg, u64 mu);
// the cached decomposition for h, computed on first use
const Decomp &decompose(dsd_graph_s *G, int h);
void decomp_stats(dsd_graph_s *G, const Decomp &D);
// rank-space device array -> caller ids, into host or device memory
void write_u64(dsd_graph_s *G, const u64 *rank_space, uint64_t *out, int mem);
void write_u8(dsd_graph_s *G, const uint8_t *rank_space, uint8_t *out, int mem);
// CoreApp (Algorithm 6) on a handle: best (device, rank space, length n)
// receives the (k_max, Psi)-core; returns k_max, *density its density
u64 core_app_run(dsd_graph_s *G, int h, uint8_t *best, dsd_rational *density);
// PeelApp (Algorithm 2, all minimum-degree vertices per round) on a handle:
// best (device, rank space, length n) receives the densest residual graph;
// returns its density; *rounds / *best_round as dsd_peel_app reports them
dsd_rational peel_app_run(dsd_graph_s *G, int h, uint8_t *best, int64_t *rounds, int64_t *best_round);
// densest subgraph containing the query vertices q (caller ids, at least
// one) on a handle: res (device, rank space, length n) receives it; returns
// its density
dsd_rational core_exact_query_run(dsd_graph_s *G, int h, const std::vector<int32_t> &q, uint8_t *res);
// CoreExact on a handle: res (device, rank space, length n) receives the
// members of one densest subgraph; returns rho_opt
dsd_rational core_exact_run(dsd_graph_s *G, int h, uint8_t *res);

}  // namespace dsd
