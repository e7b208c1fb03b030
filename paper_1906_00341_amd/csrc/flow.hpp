// Maximum preflow and minimum cut on the GPU (the exact step's networks).
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

namespace dsd {

// Arc classes of the exact step's networks (Algorithm 1; Goldberg's network
// for h = 2): capacities follow from the class, the test density alpha = a/b
// and the arc's vertex.
enum FlowArc : uint8_t { ARC_SRC = 0, ARC_SNK = 1, ARC_INF = 2, ARC_MID = 3 };

// Capacities of one test.  h >= 3: s->v b*deg(v), v->t h*a, psi->v inf,
// v->psi b.  h = 2: s->v b*m, v->t b*m + 2a - b*deg(v), u<->v b both ways.
// Every value has been checked to fit by the caller.
struct FlowTest {
    int h;
    int64_t a, b, m, inf;
};

// A network resident on the device: its arcs (node 0 = s, node 1 = t, node
// 2 + i = vertex i of the component) are uploaded once and the residual CSR
// (every arc and its reverse) is built there; capacities are set per test by
// a kernel.  Owns a stream of its own.
class GpuFlow {
public:
    // E arcs eu[i] -> ev[i] of class cls[i]; deg: clique-degree of each of
    // the nv component vertices
    GpuFlow(int n, int64_t E, const int *eu, const int *ev, const uint8_t *cls, int nv, const uint64_t *deg);
    ~GpuFlow();
    GpuFlow(const GpuFlow &) = delete;
    GpuFlow &operator=(const GpuFlow &) = delete;
    // Algorithm 1's network for h = 3 over a component of nv vertices (at
    // most TRI_NET_MAX_NV), built on the device.  so/sa (host): the
    // component's adjacency in local ids, rows sorted ascending; fwd[i]: the
    // first entry of row i above i.  Nodes: s = 0, t = 1, vertex i -> 2 + i,
    // then one node per edge, numbered row by row over the rows' parts from
    // fwd on.  Arcs: the nv source arcs first, the nv sink arcs next, then
    // two infinite arcs per edge, then three arcs per triangle.  deg receives
    // the triangles through each vertex, *tri their number.  Throws
    // Error(-5) when the arcs would not fit int indices.
    static std::unique_ptr<GpuFlow> triangles(int nv, const int64_t *so, const int32_t *sa, const int64_t *fwd,
                                              std::vector<uint64_t> &deg, uint64_t *tri);
    int nodes() const;
    int64_t arcs() const;
    // the arcs' ends as built (arrays of arcs() entries, host)
    void download_arcs(int *eu, int *ev) const;
    // networks from triangles(): the source arcs of the vertices flagged in
    // forced (one flag per vertex) become infinite, the others finite again
    void force_sources(const std::vector<char> &forced);
    // Maximum s-t flow value at the test's capacities; reach_t[v] = 1 iff v
    // reaches t in the final residual network.  Gives up after max_passes
    // push/relabel passes (*converged = false).
    int64_t maxflow(const FlowTest &test, std::vector<char> &reach_t, int64_t max_passes, bool *converged);
    struct Impl;

private:
    GpuFlow();
    std::unique_ptr<Impl> p_;
};

// largest component triangles() takes (its LDS bitmap has one bit per vertex)
constexpr int TRI_NET_MAX_NV = 1 << 17;

// Triangles of a vertex set given as for GpuFlow::triangles (nv <=
// TRI_NET_MAX_NV), counted on the device with the same listing.
uint64_t count_triangles_device(int nv, const int64_t *so, const int32_t *sa, const int64_t *fwd);

}  // namespace dsd
