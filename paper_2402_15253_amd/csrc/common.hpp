// Shared device helpers and host plumbing of the k-core library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pico.h"

namespace pico {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kBlock = 256;   // threads per workgroup (4 waves)
constexpr int kWavesPerBlock = kBlock / kWave;

// Thread-mapping cut-offs of the frontier kernels (edges per frontier vertex).
// A vertex of degree <= kSmallDeg is expanded by one lane; up to kHeavyDeg by
// one whole wave; above that it is split into kChunk-edge pieces that any wave
// may take (the load balancing the paper delegates to Tigr, Section V-A).
constexpr int kSmallDeg = 16;
constexpr int kHeavyDeg = 4096;
constexpr int kChunk = 2048;

// LDS histogram capacity per wave for InitHisto (int32 buckets).
constexpr int kLdsBuckets = 2048;

// Upper bound on heavy-chunk descriptors that one pass can emit for a graph
// with m directed entries: a vertex is heavy only above kLdsBuckets (<=
// kHeavyDeg) edges, and contributes ceil(deg / kChunk) <= deg / kChunk + 1 <
// deg / kChunk + deg / kLdsBuckets pieces.
inline int64_t heavy_capacity(int64_t m) { return m / kChunk + m / kLdsBuckets + 16; }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ unsigned lane_rank(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Wave-aggregated append: lanes with `pred` reserve consecutive slots of a
// queue with one atomic per wave.  Returns the lane's slot, or -1.
__device__ __forceinline__ long long wave_append(bool pred, unsigned long long *tail) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(tail, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    return pred ? (long long)(base + lane_rank(mask)) : -1ll;
}

__device__ __forceinline__ int wave_min(int x) {
    for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off));
    return x;
}

__device__ __forceinline__ long long wave_sum64(long long x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Host side --------------------------------------------------------------

void set_error(const char *fmt, ...);
void clear_error();

#define PICO_HIP_TRY(expr)                                                         \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) {                                                    \
            ::pico::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                              __FILE__, __LINE__);                                 \
            return PICO_EHIP;                                                      \
        }                                                                          \
    } while (0)

#define PICO_LAUNCH_CHECK() PICO_HIP_TRY(hipGetLastError())

// Bump allocator over a caller-provided device workspace.
struct Carve {
    char *base;
    size_t used;
    size_t cap;
    template <typename T>
    T *take(int64_t count) {
        size_t bytes = ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
        if (used + bytes > cap) return nullptr;
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
};

inline size_t carve_bytes(int64_t count, size_t elem) {
    return ((size_t)count * elem + 255) & ~(size_t)255;
}

// Small pinned host buffer for counter read-back (one per host thread).
void *host_scratch(size_t bytes);

// Optional per-launch HIP-event timing (pico_profile_enable).  prof_begin
// returns a record index, or -1 when profiling is off on this host thread.
int prof_begin(const char *name, hipStream_t s);
void prof_end(int rec, hipStream_t s);

#define PICO_LAUNCH(name, kernel, grid, block, stream, ...)                    \
    do {                                                                     \
        int _pico_rec = ::pico::prof_begin(name, stream);                    \
        kernel<<<(grid), (block), 0, (stream)>>>(__VA_ARGS__);               \
        ::pico::prof_end(_pico_rec, stream);                                 \
    } while (0)

size_t peelone_ws_bytes(int64_t n, int64_t m);
size_t histocore_ws_bytes(int64_t n, int64_t m);

template <typename Off>
int run_peelone(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out,
                void *ws, size_t ws_bytes, pico_stats *st, hipStream_t stream);

template <typename Off>
int run_histocore(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out,
                  void *ws, size_t ws_bytes, pico_stats *st, hipStream_t stream);

inline int grid_for(int64_t items_per_block_units, int cap) {
    int64_t g = items_per_block_units;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace pico
