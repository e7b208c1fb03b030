// Host exact step of CoreExact (Algorithm 4) over the GPU-located core.
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

namespace dsd {

// A located core handed over by the GPU: vertices (local ids 0..s-1) with
// their induced adjacency, clique-core numbers and component labels.
struct LocatedCore {
    std::vector<int32_t> rank;      // local -> rank-space id
    std::vector<int64_t> off;       // local CSR, rows sorted ascending
    std::vector<int32_t> adj;
    std::vector<uint64_t> core;     // clique-core number
    std::vector<int32_t> label;     // component label (any id, equal within a component)
    // (label, h-cliques) of every component, counted on the GPU, sorted by
    // label; empty when the caller did not count them
    std::vector<std::pair<int32_t, uint64_t>> comp_mu;
};

struct Rational {
    uint64_t num = 0, den = 1;
};

struct ExactStats {
    int64_t flow_calls = 0;
    int64_t max_nodes = 0;
    int64_t gpu_flow_calls = 0;          // minimum cuts computed on the GPU
    int64_t gpu_networks = 0;            // networks built on the device
    double build_ms = 0, flow_ms = 0;   // network construction / maximum flow
    double setup_ms = 0;                // part of flow_ms: moving a network to the device (arcs, residual CSR)
};

// Searches every component for a subgraph denser than `l` (the density of
// the best set found by the GPU, which `best` holds as local ids; may be
// empty when the caller keeps its own copy).  kpp = k'' (the components are
// those of the (k'', Psi)-core).  Returns true and overwrites best / l when
// a denser subgraph exists; best then lists local ids of a densest subgraph
// of the located core.  Throws Error(EOVERFLOW) when a scaled capacity would
// not fit in 63 bits.
bool exact_search(const LocatedCore &lc, int h, uint64_t kpp, Rational &l, std::vector<int32_t> &best,
                  ExactStats &st);

// The densest subgraph of the located core that contains every vertex of q
// (local ids).  x = the smallest clique-core number over q; l enters as the
// density of a set containing q (the caller's (x, Psi)-core) and the search
// runs over R_k, k = min(x, ceil(l)), which holds every such set at least
// that dense.  Returns true and overwrites best (local ids) / l when a denser
// set containing q exists.
bool exact_search_query(const LocatedCore &lc, int h, uint64_t x, const std::vector<int32_t> &q, Rational &l,
                        std::vector<int32_t> &best, ExactStats &st);

// h-cliques of the subgraph of lc induced by `verts` (local ids)
uint64_t count_cliques_host(const LocatedCore &lc, int h, const std::vector<int32_t> &verts);

}  // namespace dsd
