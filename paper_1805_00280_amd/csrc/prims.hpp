// prims.hpp -- device-wide building blocks used while building graphs.
#pragma once

#include "common.hpp"

namespace n2v {

// Scratch bytes exclusive_scan_u64 needs for n elements.
size_t scan_scratch_bytes(uint64_t n);
// In-place exclusive prefix sum of data[0, n) (uint64, wrap-around arithmetic).
int exclusive_scan_u64(uint64_t *data, uint64_t n, void *scratch, hipStream_t st);

// Carves 256-byte aligned pieces out of a workspace.
struct Carver {
    char *base;
    size_t size, used;
    explicit Carver(void *b, size_t s) : base((char *)b), size(s), used(0) {}
    template <class T>
    T *take(uint64_t count)
    {
        size_t bytes = (size_t)count * sizeof(T);
        size_t at = (used + 255) & ~(size_t)255;
        used = at + bytes;
        if (!base) return nullptr;
        return used <= size ? (T *)(base + at) : nullptr;
    }
    size_t total() const { return (used + 255) & ~(size_t)255; }
};

}  // namespace n2v
