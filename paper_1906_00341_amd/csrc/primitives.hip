// Scans, reductions and a stable LSD radix sort of 64-bit keys for gfx950.
#include <map>
#include <mutex>

#include "primitives.hpp"

namespace dsd {

// ---------------------------------------------------------------- Scratch

namespace {

// recycled scratch chunks, by device and size
struct ChunkPool {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, char *> free;
    size_t bytes = 0;
};
ChunkPool &chunk_pool() {
    static ChunkPool *p = new ChunkPool();   // never destroyed: handles may outlive static destruction
    return *p;
}
constexpr size_t POOL_MAX = (size_t)16 << 30;

}  // namespace

Scratch::~Scratch() {
    if (external_) return;
    for (auto &c : chunks_) (void)hipFree(c.first);
}

void release_chunk_pool() {
    ChunkPool &P = chunk_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto &e : P.free) {
        if (have) (void)hipSetDevice(e.first.first);
        (void)hipFree(e.second);
    }
    if (have) (void)hipSetDevice(cur);
    P.free.clear();
    P.bytes = 0;
}

void *thread_pinned() {
    thread_local void *p = nullptr;
    if (!p && hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) {
        p = nullptr;
        throw Error(-2, "pinned host allocation failed");
    }
    return p;
}

void Scratch::recycle() {
    if (external_) {
        cur_ = 0;
        off_ = 0;
        return;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    ChunkPool &P = chunk_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto &c : chunks_) {
        if (dev >= 0 && P.bytes + c.second <= POOL_MAX) {
            P.free.emplace(std::make_pair(dev, c.second), c.first);
            P.bytes += c.second;
        } else {
            (void)hipFree(c.first);
        }
    }
    chunks_.clear();
    cur_ = 0;
    off_ = 0;
}

size_t Scratch::capacity() const {
    size_t t = 0;
    for (auto &c : chunks_) t += c.second;
    return t;
}

void *Scratch::get(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    while (cur_ < chunks_.size()) {
        if (off_ + bytes <= chunks_[cur_].second) {
            void *p = chunks_[cur_].first + off_;
            off_ += bytes;
            return p;
        }
        cur_++;
        off_ = 0;
    }
    if (external_) {
        cur_ = 0;
        off_ = 0;
        throw Error(-2, "the request needs more than the fixed scratch buffer holds");
    }
    size_t sz = bytes > min_chunk_ ? bytes : min_chunk_;
    char *p = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        // the smallest recycled chunk of this device that is large enough
        ChunkPool &P = chunk_pool();
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.free.lower_bound(std::make_pair(dev, sz));
        if (it != P.free.end() && it->first.first == dev) {
            p = it->second;
            sz = it->first.second;
            P.bytes -= sz;
            P.free.erase(it);
        }
    }
    if (!p && hipMalloc(&p, sz) != hipSuccess) throw Error(-2, "device allocation of scratch failed");
    chunks_.push_back({p, sz});
    cur_ = chunks_.size() - 1;
    off_ = bytes;
    return p;
}

// ---------------------------------------------------------------- fills

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u64(u64 *p, u64 v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<u64><<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(p, v, n);
}
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<int32_t><<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(p, v, n);
}
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<uint8_t><<<grid_for(n, BLOCK, 4096), BLOCK, 0, s>>>(p, v, n);
}

// ---------------------------------------------------------------- scan

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;   // 2048 elements per block

// exclusive scan of one tile; block total to sums[blockIdx.x]
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_scan_tile(const T *in, T *out, T *sums, int64_t n) {
    __shared__ T wsum[WAVES_PER_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        T x = (base + i < n) ? in[base + i] : (T)0;
        v[i] = acc;
        acc += x;
    }
    T incl = wave_incl_scan(acc);
    int w = threadIdx.x / WAVE;
    if (lane() == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    T woff = 0;
    for (int i = 0; i < w; i++) woff += wsum[i];
    T excl = woff + incl - acc;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++)
        if (base + i < n) out[base + i] = excl + v[i];
    if (threadIdx.x == BLOCK - 1) {
        T tot = 0;
        for (int i = 0; i < WAVES_PER_BLOCK; i++) tot += wsum[i];
        sums[blockIdx.x] = tot;
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_scan_add(T *out, const T *offs, int64_t n) {
    T o = offs[blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++)
        if (base + i < n) out[base + i] += o;
}

template <typename T>
static void scan_exclusive(const T *in, T *out, int64_t n, hipStream_t s, Scratch &sc) {
    if (n <= 0) return;
    int64_t tiles = ceil_div(n, SCAN_TILE);
    T *sums = sc.get_n<T>(tiles);
    k_scan_tile<T><<<(unsigned)tiles, BLOCK, 0, s>>>(in, out, sums, n);
    if (tiles > 1) {
        scan_exclusive<T>(sums, sums, tiles, s, sc);
        k_scan_add<T><<<(unsigned)tiles, BLOCK, 0, s>>>(out, sums, n);
    }
}

void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, Scratch &sc) {
    scan_exclusive<int64_t>(in, out, n, s, sc);
}
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s, Scratch &sc) {
    scan_exclusive<uint32_t>(in, out, n, s, sc);
}

// ---------------------------------------------------------------- 128-bit sum

__global__ __launch_bounds__(BLOCK) void k_sum128_partial(const u64 *in, int64_t n, u64 *part) {
    u64 lo = 0, hi = 0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        u64 x = in[i];
        lo += x;
        hi += (lo < x);
    }
    __shared__ u64 slo[BLOCK], shi[BLOCK];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 a = 0, b = 0;
        for (int i = 0; i < BLOCK; i++) {
            a += slo[i];
            b += shi[i] + (a < slo[i]);
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void k_sum128_final(const u64 *part, int nb, u64 *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        u64 a = 0, b = 0;
        for (int i = 0; i < nb; i++) {
            a += part[2 * i];
            b += part[2 * i + 1] + (a < part[2 * i]);
        }
        out[0] = a;
        out[1] = b;
    }
}

void sum_u64_128(const u64 *in, int64_t n, u64 *out2, hipStream_t s, Scratch &sc) {
    int nb = grid_for(n, BLOCK * 8, 1024);
    u64 *part = sc.get_n<u64>(2 * nb);
    k_sum128_partial<<<nb, BLOCK, 0, s>>>(in, n, part);
    k_sum128_final<<<1, 64, 0, s>>>(part, nb, out2);
}

// ---------------------------------------------------------------- radix sort
//
// LSD, 8-bit digits.  A tile is 4096 keys handled by 4 waves; wave w owns
// keys [w*1024, (w+1)*1024) of the tile in 16 rounds of 64 consecutive keys,
// so the order of keys inside a wave is (round, lane) -- the original order.
// Within a round, lanes with equal digits find each other with 8 ballots; a
// per-wave digit counter in LDS carries ranks across rounds, and per-wave
// counts are combined in wave order, which makes the scatter stable.

constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = BLOCK * RS_ITEMS;      // 4096
constexpr int RS_WAVE_KEYS = WAVE * RS_ITEMS;  // 1024

__global__ __launch_bounds__(BLOCK) void k_radix_hist(const u64 *keys, int64_t n, int shift, uint32_t *counts,
                                                      int64_t tiles) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    int64_t tile_base = (int64_t)blockIdx.x * RS_TILE;
    int w = threadIdx.x / WAVE;
#pragma unroll 4
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t idx = tile_base + (int64_t)w * RS_WAVE_KEYS + r * WAVE + lane();
        if (idx < n) atomicAdd(&hist[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * tiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(BLOCK) void k_radix_scatter(const u64 *keys, u64 *out, int64_t n, int shift,
                                                         const uint32_t *offsets, int64_t tiles) {
    __shared__ uint32_t wcnt[WAVES_PER_BLOCK][256];
    __shared__ uint32_t base[256];
    for (int i = threadIdx.x; i < WAVES_PER_BLOCK * 256; i += BLOCK) (&wcnt[0][0])[i] = 0;
    base[threadIdx.x] = offsets[(int64_t)threadIdx.x * tiles + blockIdx.x];
    __syncthreads();
    int64_t tile_base = (int64_t)blockIdx.x * RS_TILE;
    int w = threadIdx.x / WAVE;
    u64 key[RS_ITEMS];
    uint32_t rank[RS_ITEMS];
    const u64 lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t idx = tile_base + (int64_t)w * RS_WAVE_KEYS + r * WAVE + lane();
        bool valid = idx < n;
        u64 k = valid ? keys[idx] : 0;
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1u;
            u64 m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = valid ? wcnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        bool leader = valid && ((peers & lt) == 0);
        if (leader) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        key[r] = k;
        rank[r] = valid ? before + (uint32_t)__popcll(peers & lt) : 0xffffffffu;
    }
    __syncthreads();
    // wcnt[w][d] <- sum over earlier waves (exclusive, in wave order)
    {
        int d = threadIdx.x;
        uint32_t acc = 0;
        for (int i = 0; i < WAVES_PER_BLOCK; i++) {
            uint32_t c = wcnt[i][d];
            wcnt[i][d] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        if (rank[r] != 0xffffffffu) {
            uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            out[(int64_t)base[d] + wcnt[w][d] + rank[r]] = key[r];
        }
    }
}

void radix_sort_u64(u64 *keys, u64 *tmp, int64_t n, int bits, hipStream_t s, Scratch &sc) {
    if (n <= 1 || bits <= 0) return;
    int64_t tiles = ceil_div(n, RS_TILE);
    uint32_t *counts = sc.get_n<uint32_t>(256 * tiles);
    u64 *a = keys, *b = tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        k_radix_hist<<<(unsigned)tiles, BLOCK, 0, s>>>(a, n, shift, counts, tiles);
        scan_exclusive_u32(counts, counts, 256 * tiles, s, sc);
        k_radix_scatter<<<(unsigned)tiles, BLOCK, 0, s>>>(a, b, n, shift, counts, tiles);
        u64 *t = a; a = b; b = t;
    }
    if (a != keys) DSD_HIP(hipMemcpyAsync(keys, a, (size_t)n * sizeof(u64), hipMemcpyDeviceToDevice, s));
}

}  // namespace dsd
