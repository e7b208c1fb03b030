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
    // Maximum s-t flow value at the test's capacities; reach_t[v] = 1 iff v
    // reaches t in the final residual network.  Gives up after max_passes
    // push/relabel passes (*converged = false).
    int64_t maxflow(const FlowTest &test, std::vector<char> &reach_t, int64_t max_passes, bool *converged);
    struct Impl;

private:
    std::unique_ptr<Impl> p_;
};

}  // namespace dsd
