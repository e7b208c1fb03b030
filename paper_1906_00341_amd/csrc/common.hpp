// Shared device helpers for libdsd (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace dsd {

typedef unsigned long long u64;
typedef long long i64;

constexpr int WAVE = 64;
constexpr int BLOCK = 256;               // 4 waves
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;
constexpr int32_t ALIVE = 0x7fffffff;    // stamp of a vertex not yet removed by the peel

// ---- error handling (host) -------------------------------------------------

struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define DSD_HIP(x)                                                                          \
    do {                                                                                    \
        hipError_t _e = (x);                                                                \
        if (_e != hipSuccess)                                                               \
            throw ::dsd::Error(-3, std::string(#x) + ": " + hipGetErrorString(_e));         \
    } while (0)

// ---- device helpers ----------------------------------------------------------

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ u64 lanemask_lt() { return (1ull << lane()) - 1ull; }

// inclusive scan across the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T o = __shfl_up(v, d, WAVE);
        if (lane() >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, WAVE);
        v = o < v ? o : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// global 64-bit atomics
__device__ __forceinline__ u64 atomic_add_u64(u64 *p, u64 v) { return atomicAdd(p, v); }
__device__ __forceinline__ u64 atomic_sub_u64(u64 *p, u64 v) { return atomicAdd(p, (u64)0 - v); }

// smallest index i in [0, n) with pre[i] > p (pre is inclusive-scanned, pre[n-1] > p)
__device__ __forceinline__ int upper_bound_i32(const int32_t *pre, int n, int32_t p) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] > p) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// index of x in the sorted array a[lo, hi), or -1
__device__ __forceinline__ i64 bsearch_i32(const int32_t *a, i64 lo, i64 hi, int32_t x) {
    while (lo < hi) {
        i64 mid = (lo + hi) >> 1;
        int32_t v = a[mid];
        if (v == x) return mid;
        if (v < x) lo = mid + 1; else hi = mid;
    }
    return -1;
}

// multiplicative hash of a vertex id into 2^bits slots
__device__ __forceinline__ uint32_t hash_slot(int32_t x, int bits) {
    return ((uint32_t)x * 2654435761u) >> (32 - bits);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
    int64_t g = ceil_div(work > 0 ? work : 1, per_block);
    return (int)(g > cap ? cap : g);
}

}  // namespace dsd
