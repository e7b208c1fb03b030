// Scans, reductions, compaction and a radix sort of 64-bit keys (host launchers).
#pragma once

#include <vector>

#include "common.hpp"

namespace dsd {

// Bump allocator over device chunks; reset() recycles everything (stream-ordered reuse).
// Device scratch: a bump allocator over chunks of at least min_chunk bytes
// (64 MiB unless given).  A new
// chunk comes from a process-wide pool of recycled chunks (per device, at
// most 16 GiB kept) before hipMalloc is asked; recycle() hands the chunks to
// that pool, and the caller promises that no work still uses them (its
// stream is idle).  Chunks not recycled are freed with the scratch.
class Scratch {
public:
    explicit Scratch(size_t min_chunk = (size_t)64 << 20) : min_chunk_(min_chunk) {}
    // a scratch over a caller-owned device buffer: it never allocates, frees
    // or recycles the buffer; a request beyond it throws DSD_ENOMEM
    Scratch(void *buf, size_t bytes) : min_chunk_(0), external_(true) { chunks_.push_back({(char *)buf, bytes}); }
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    ~Scratch();
    void *get(size_t bytes);
    void recycle();
    template <typename T> T *get_n(int64_t n) { return (T *)get((size_t)(n > 0 ? n : 1) * sizeof(T)); }
    void reset() { cur_ = 0; off_ = 0; }
    size_t capacity() const;

private:
    std::vector<std::pair<char *, size_t>> chunks_;
    size_t cur_ = 0, off_ = 0;
    size_t min_chunk_;
    bool external_ = false;
};

// out[i] = sum_{j<i} in[j]; returns nothing, total = out[n-1] + in[n-1].  in == out allowed.
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, Scratch &sc);
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s, Scratch &sc);

// Sort n 64-bit keys ascending on their low `bits` bits (higher bits must be 0).
// The result is in *keys; tmp has room for n keys.
void radix_sort_u64(u64 *keys, u64 *tmp, int64_t n, int bits, hipStream_t s, Scratch &sc);

// sum of a u64 array as a 128-bit (lo, hi) pair written to out[0], out[1] (device)
void sum_u64_128(const u64 *in, int64_t n, u64 *out2, hipStream_t s, Scratch &sc);

// free every recycled chunk of every device
void release_chunk_pool();

// a 64-byte pinned host buffer of the calling thread, for reading counters
// back; allocated on first use and kept until the process ends
void *thread_pinned();

// fill helpers (kernels, usable under stream capture)
void fill_u64(u64 *p, u64 v, int64_t n, hipStream_t s);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);

}  // namespace dsd
