// Device graph layout and the internal launchers of every kernel family.
//
// All kernels work in *rank space*: vertex r is the vertex of rank r in the
// degree order (deg, id) ascending.  Row r of the CSR lists N(r) sorted by
// rank; its tail from dag_off[r] on is N+(r), the out-neighbours of r in the
// degree-ordered DAG (every h-clique is reached once from its lowest-rank
// member).  Outputs are mapped back to the caller's ids through orig_of /
// rank_of.
#pragma once

#include <vector>

#include "exact.hpp"
#include "primitives.hpp"

namespace dsd {

struct DevGraph {
    int32_t n = 0;
    int64_t m = 0;            // undirected edges
    int bits = 1;             // bits needed to hold n (ids < 2^bits - 1)
    int64_t *row_ptr = nullptr;  // [n+1]
    int32_t *col = nullptr;      // [2m]
    int64_t *dag_off = nullptr;  // [n]
    int32_t *orig_of = nullptr;  // [n] rank -> caller id
    int32_t *rank_of = nullptr;  // [n] caller id -> rank
    int32_t maxdeg = 0, maxdout = 0;
    u64 w2 = 0;   // sum_v d-(v) d+(v): directed 2-paths of the DAG (pairs the enumeration probes)
    u64 s2 = 0;   // sum_v deg(v) d+(v): out-list entries the peel probes over all removed vertices
    bool owned = true;   // the arrays were hipMalloc'd (else they live in a handle's scratch)
};

// HIP-event timing of the two kernel families, accumulated per call
struct KernelTimes {
    double k3_ms = 0, k4_ms = 0;
    u64 k3_launches = 0, k4_launches = 0;
    // the peel's main kernel (h = 3: the triangle probe; h = 2: the edge
    // pass), every launch timed on its own; pairs: out-list entries probed
    // (h = 3) or adjacency entries walked (h = 2); nbrs: neighbours expanded
    // (h = 3) or frontier vertices (h = 2)
    double main_ms = 0;
    u64 main_launches = 0, main_pairs = 0, main_nbrs = 0;
    u64 main_entries = 0;   // h >= 4 root mode: row entries scanned for the frontier vertices' C_v
    double main2_ms = 0;    // h >= 4 root mode: the counting kernel, timed like the main kernel
    u64 main2_launches = 0;
    u64 main2_words = 0;    // h >= 4 root mode: 64-bit bitmap words the counting kernel ANDed and counted (first level)
    int main_kind = 0;   // 1 edge pass, 2 triangle probe, 3 triangle lists, 4 x-star frontier pass, 5 4-loop pass,
                        // 6 h >= 4 root-mode block kernel
    bool time_main = false;   // bracket every main-kernel launch with HIP events (main_ms)
    // the tail engine (h = 3 with triangle lists, h = 2): its time (HIP
    // events around every launch, with time_main), launches (one per peel
    // that reaches it, plus one per grid round), the row pairs it walked and
    // the tail vertices it peeled; and the rounds it handed to the grid, their
    // time (with time_main) and pairs
    double tail_ms = 0;
    u64 tail_launches = 0, tail_pairs = 0, tail_vertices = 0;
    double tail_grid_ms = 0;
    u64 tail_grid_rounds = 0, tail_grid_pairs = 0;
};

// ---- K1 + K2: CSR build and degree-ordered orientation ----
// src/dst: device arrays of num_pairs raw pairs.  Throws Error(EINVAL) on an
// id outside [0, n).  t_orient receives the time of the orientation part.
// keep: where the graph's arrays live (nullptr: hipMalloc, freed by free_graph)
void build_graph(int32_t n, int64_t num_pairs, const int32_t *src, const int32_t *dst, DevGraph &g,
                 hipStream_t s, Scratch &sc, float *t_orient_ms, Scratch *keep = nullptr);
void free_graph(DevGraph &g);

// ---- K3: clique-degrees ----
// deg[r] (rank space, length n) = number of h-cliques containing r inside the
// subgraph induced by mask (mask == nullptr: whole graph).  deg is
// overwritten.  Returns false if the counts could overflow 64 bits.
// gs_blocks caps the grid of the class whose bitmaps live in global scratch
// (gs_blocks * 1280 * 20 words of sc).
bool clique_degrees(const DevGraph &g, int h, const uint8_t *mask, u64 *deg, hipStream_t s, Scratch &sc,
                    KernelTimes *kt = nullptr, int gs_blocks = 512);

// ---- launch-grid tuning of the clique enumeration ----
// One class's measurement: its roots, the default and the chosen grid cap
// (workgroups), and the time of one launch at each (ms).
struct TuneResult {
    int cls;
    int32_t roots;
    int cap_default, cap_best;
    double ms_default, ms_best;
};
// times every class of g's roots at h under a set of grid caps and keeps the
// fastest in the process-wide table (key: architecture, h, class)
std::vector<TuneResult> autotune(const DevGraph &g, int h, hipStream_t s, Scratch &sc);
// replaces the table with the JSON file's entries (nullptr: back to the defaults)
void tune_load(const char *path);
// writes the table, merged over the file's existing entries, to path
void tune_write(const char *path);

// ---- triangle lists (h = 3) ----
// Row v is pairs[2 voff[v] .. 2 voff[v+1]): a pair (a, b) for every triangle
// {v, a, b}, once, with a ranked below b, grouped by a: 3 mu pairs in all.
struct TriList {
    int64_t *voff = nullptr;   // [n + 1]
    int32_t *pairs = nullptr;  // [2 * entries]
    int64_t entries = 0;
    u64 mu = 0;
    bool owned = true;         // hipMalloc'd (else in a handle's scratch)
};
// whether the lists of a graph with mu triangles fit (positions in int32,
// out-degree within the listing kernels, at most a quarter of free device
// memory); the environment variable DSD_TRI_LIST=0 turns them off
bool tri_list_wanted(const DevGraph &g, u64 mu);
// The first pass of the listing alone: the size of every arc's segment (the
// triangles it will hold), and from them the clique-degrees (the sum over a
// vertex's segments) and mu.  The arrays live in the scratch until its next
// reset.
struct TlCounts {
    int64_t *rev = nullptr;   // [2m] reverse arc of every arc
    uint32_t *cnt = nullptr;  // [2m] segment sizes
    uint32_t *top = nullptr;  // [2m] triangles with the arc's head on top (forward arcs)
    int32_t *big = nullptr, *nbig = nullptr;
    int64_t *mid = nullptr;
    u64 mu = 0;
};
// whether the segment sizes can be counted (out-degrees within the listing
// kernels, room on the device; DSD_TRI_LIST=0 turns them off)
bool tri_counts_possible(const DevGraph &g);
// deg (length n) = clique-degrees (h = 3); returns mu
u64 tri_counts(const DevGraph &g, u64 *deg, TlCounts &w, hipStream_t s, Scratch &sc);
// the second pass: every triangle written out through per-arc cursors into
// the segments the counts give.  Allocates tl's arrays (released by
// free_tri_list).
// keep: where the lists live (nullptr: hipMalloc, freed by free_tri_list).
void build_tri_list(const DevGraph &g, TlCounts &w, TriList &tl, hipStream_t s, Scratch &sc,
                    Scratch *keep = nullptr);
// both passes for a graph with mu triangles (deg unused)
void build_tri_list(const DevGraph &g, const u64 *deg, u64 mu, TriList &tl, hipStream_t s, Scratch &sc,
                    Scratch *keep = nullptr);
// clique-degrees read off finished lists (one pair per triangle at a vertex)
void tri_list_degrees(const TriList &tl, int32_t n, u64 *deg, hipStream_t s);
void free_tri_list(TriList &tl);

// ---- K4: round-synchronous peel ----
// Once at most this many vertices of a single graph are alive (h = 2, or
// h = 3 with triangle lists), one workgroup finishes the peel in one launch
// (the tail engine); a peel that starts at or below it never launches a
// round kernel.
constexpr int64_t TAIL_ENGINE_VERTICES = 16384;
// A batch of graphs is peeled as one disjoint union in which every graph
// keeps its own level: a round moves every graph on by one step, so the
// batch takes as many rounds as its slowest graph.
struct PeelGroups {
    int32_t G = 1;
    const int32_t *gid = nullptr;      // [n] graph of every rank-space vertex
    const u64 *mu = nullptr;           // [G] cliques inside each graph's alive set (device)
    const int64_t *lv_base = nullptr;  // [G] first entry of each graph's level table (device)
    int64_t lv_total = 0;              // entries of all tables together (graph g needs n_g + 1)
};
struct PeelResult {
    int64_t rounds = 0;
    int64_t levels = 0;                // summed over the graphs
    std::vector<u64> level_k, level_size, level_mu;  // R_k for every level k reached (batch: every
                                                      // graph's table at its base)
    std::vector<int32_t> graph_levels; // batch: levels of each graph
    u64 kmax = 0;                      // single graph
};
// alive0 (nullable): vertices taking part (others are ignored).  deg: clique
// degrees inside the alive set (consumed).  mu: cliques inside the alive set
// (single graph; grp->mu for a batch).  k_floor: every vertex of degree <=
// k_floor goes in the first level (CoreApp starts its peel there); 0 for a
// full decomposition.  core: rank space.
// min_degree: PeelApp's order instead (Algorithm 2, all minimum-degree
// vertices of a graph per round; k_floor must be 0): core[] receives the
// round that removed each vertex, and the level table one entry per round of
// each graph: the smallest degree, |S| and mu(S) of the residual graph S
// before that round (entry j of a graph is round j).
// tl (h = 3, nullable): the graph's triangle lists; the rounds then walk the
// removed vertices' rows of triangles instead of intersecting neighbourhoods.
// pattern 1 (x-stars with px tails) or 2 (4-loops): peel pattern-degrees
// instead (deg: the pattern-degrees of the whole graph; alive0 must be
// nullptr; h, tl and min_degree unused).  Throws Error(-5) when a 2-hop
// neighbourhood is too large for the 4-loop tables.
PeelResult peel(const DevGraph &g, int h, const uint8_t *alive0, u64 *deg, u64 mu, u64 k_floor, u64 *core,
                hipStream_t s, Scratch &sc, KernelTimes *kt = nullptr, const PeelGroups *grp = nullptr,
                bool min_degree = false, const TriList *tl = nullptr, int pattern = 0, int px = 0);

// ---- special patterns ----
// deg[r] = x-star pattern-degree of r (closed form of the appendix on special
// patterns); false if a value could exceed 64 bits
bool star_degrees(const DevGraph &g, int x, u64 *deg, hipStream_t s, Scratch &sc);
// deg[r] = 4-loops through r (one workgroup per vertex with a table of its
// 2-hop neighbours); throws Error(-5) when a table would be too large
void loop4_degrees(const DevGraph &g, u64 *deg, hipStream_t s, Scratch &sc);

// ---- K5: connected components of the subgraph induced by mask ----
// label[r] = smallest rank of r's component for r in mask, -1 outside.
void components(const DevGraph &g, const uint8_t *mask, int32_t *label, hipStream_t s, Scratch &sc);

// ---- small kernels used by the drivers ----
void mask_core_at_least(const u64 *core, int32_t n, u64 k, uint8_t *mask, hipStream_t s);
void mask_from_order_prefix(const u64 *order, int32_t n, int64_t w, int bits, uint8_t *mask, hipStream_t s);
// out[id] = in[rank_of[id]]
void gather_to_orig_u64(const DevGraph &g, const u64 *in, u64 *out, hipStream_t s);
void gather_to_orig_u8(const DevGraph &g, const uint8_t *in, uint8_t *out, hipStream_t s);
void mask_core_equal(const u64 *core, int32_t n, u64 k, uint8_t *mask, hipStream_t s);
// per-component (size, sum of deg) keyed by label root; out arrays length n
void component_sums(const int32_t *label, const u64 *deg, int32_t n, u64 *size, u64 *dsum, hipStream_t s);
// max of a u64 array over mask (mask nullable) -> out[0] (device)
void masked_max_u64(const u64 *a, const uint8_t *mask, int32_t n, u64 *out, hipStream_t s);
void masked_min_u64(const u64 *a, const uint8_t *mask, int32_t n, u64 *out, hipStream_t s);
void mask_label_equal(const int32_t *label, int32_t n, int32_t l, uint8_t *mask, hipStream_t s);

// ---- hand-over of a located core to the host exact step ----
void extract_induced(const DevGraph &g, const uint8_t *mask, const int32_t *label, const u64 *core,
                     LocatedCore &out, hipStream_t s, Scratch &sc);
struct CompInfo {
    int32_t root;
    u64 size, dsum;   // |C| and the sum of clique-degrees inside C (= h * mu(C))
};
void collect_components(const int32_t *label, const u64 *size, const u64 *dsum, int32_t n,
                        std::vector<CompInfo> &out, hipStream_t s, Scratch &sc);

}  // namespace dsd
