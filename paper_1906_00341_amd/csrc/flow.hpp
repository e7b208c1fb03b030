// Maximum preflow and minimum cut on the GPU (the exact step's networks).
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

namespace dsd {

// A residual network (CSR of every arc and its reverse, as the host
// push-relabel builds it) resident on the device; its capacities change per
// test.  Owns a stream of its own.
class GpuFlow {
public:
    // first: n + 1 row offsets; to, rev: A entries (head of every residual
    // arc, index of its reverse)
    GpuFlow(int n, int64_t A, const int *first, const int *to, const int *rev);
    ~GpuFlow();
    GpuFlow(const GpuFlow &) = delete;
    GpuFlow &operator=(const GpuFlow &) = delete;
    // Maximum s-t flow value for the A residual capacities cap (host
    // memory); reach_t[v] = 1 iff v reaches t in the final residual network.
    // Gives up after max_passes push/relabel passes (*converged = false).
    int64_t maxflow(const int64_t *cap, int s, int t, std::vector<char> &reach_t, int64_t max_passes,
                    bool *converged);
    struct Impl;

private:
    std::unique_ptr<Impl> p_;
};

}  // namespace dsd
