// dsd_clique_degrees_noalloc: clique-degrees (Definition 3) without any
// device or pinned-host allocation.
//
// The enumeration's working memory (the rank-space degrees, the root lists
// of the out-degree classes, the class counters, the global bitmaps of the
// largest class, the partial sums of the total and, for host outputs, the
// staging of the gathered result) comes from one file-scope device array of
// NOALLOC_SCRATCH_BYTES, not from the handle's scratch.  Every GPU the
// library runs on holds its own copy of the array until the process ends;
// its address on a device is taken once, with that device current, by
// hipGetSymbolAddress, and only that address is handed to kernels and
// copies.  Calls on one GPU share the array, so calls that overlap on one
// GPU race; every counter the enumeration reads is cleared by a fill kernel
// at the start of a call.
#include <mutex>

#include "handle.hpp"
#include "primitives.hpp"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)112 << 20;
constexpr int32_t NOALLOC_MAX_N = 1 << 22;
// grid of the global-bitmap classes: 32 * (1280 * 20 + 2048 * 32) words = 22.5 MiB
constexpr int NOALLOC_GS_BLOCKS = 32;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on the current device, taken on the first
// call on that device
void *scratch_on_current_device() {
    int dev = 0;
    DSD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) throw dsd::Error(DSD_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw dsd::Error(DSD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

using namespace dsd;

extern "C" dsd_status dsd_clique_degrees_noalloc(dsd_graph G, int h, int out_mem, uint64_t *deg,
                                                 uint64_t *num_cliques) {
    if (!G) return fail(DSD_EINVAL, "NULL graph");
    DSD_TRY({
        check_h(h);
        const int32_t n = G->g.n;
        if (n > 0) check_out(deg, out_mem);
        if (n > NOALLOC_MAX_N)
            throw Error(DSD_EINVAL, "graph has more than 2^22 vertices, beyond the fixed scratch of the allocation-free "
                                    "entry point");
        hipStream_t s = G->stream;
        begin_stats(G);
        Scratch arena(scratch_on_current_device(), NOALLOC_SCRATCH_BYTES);
        u64 mu = 0;
        if (n > 0) {
            u64 *d = arena.get_n<u64>(n);
            if (!clique_degrees(G->g, h, nullptr, d, s, arena, nullptr, NOALLOC_GS_BLOCKS))
                throw Error(DSD_EOVERFLOW, "clique counts could exceed 64 bits");
            u64 *sum = arena.get_n<u64>(2);
            sum_u64_128(d, n, sum, s, arena);
            u64 hs[2] = {0, 0};
            DSD_HIP(hipMemcpyAsync(hs, sum, sizeof(hs), hipMemcpyDeviceToHost, s));
            DSD_HIP(hipStreamSynchronize(s));
            if (hs[1] != 0) throw Error(DSD_EOVERFLOW, "sum of clique-degrees exceeds 64 bits");
            if (hs[0] % (u64)h != 0) throw Error(DSD_EDEVICE, "clique-degree sum not divisible by h");
            mu = hs[0] / (u64)h;
            if (out_mem == DSD_MEM_DEVICE) {
                gather_to_orig_u64(G->g, d, (u64 *)deg, s);
            } else {
                u64 *stage = arena.get_n<u64>(n);
                gather_to_orig_u64(G->g, d, stage, s);
                DSD_HIP(hipMemcpyAsync(deg, stage, (size_t)n * sizeof(u64), hipMemcpyDeviceToHost, s));
            }
            DSD_HIP(hipStreamSynchronize(s));
        }
        if (num_cliques) *num_cliques = mu;
        G->stats.num_cliques = mu;
        return DSD_OK;
    })
}
