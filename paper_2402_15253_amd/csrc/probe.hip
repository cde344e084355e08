// Rates of the two random-access operations the decomposition kernels are
// built from -- 4-byte gathers and 4-byte device-scope atomic adds at
// uniformly random word indexes of one array -- so that a kernel's time can be
// set against what those operations alone cost on this device (a roofline for
// random access, where the HBM roofline of streamed bytes says little).
// Indexes come from the SplitMix64 output function (Steele, Lea and Flood,
// OOPSLA 2014) of the operation number, reduced modulo the word count.
#include <climits>

#include "common.hpp"

namespace pico {
namespace {

constexpr int kProbeInFlight = 8;  // independent operations per thread per step
constexpr int kProbePerCu = 8;     // workgroups per compute unit

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

template <bool kAtomic>
__global__ __launch_bounds__(kBlock) void probe_kernel(unsigned *buf, unsigned long long words, long long ops,
                                                       unsigned long long seed) {
    unsigned acc = 0;
    const long long stride = (long long)gridDim.x * kBlock * kProbeInFlight;
    for (long long base = ((long long)blockIdx.x * kBlock + threadIdx.x) * kProbeInFlight; base < ops;
         base += stride) {
        unsigned v[kProbeInFlight];
#pragma unroll
        for (int r = 0; r < kProbeInFlight; ++r) {
            v[r] = 0u;
            if (base + r < ops) {
                unsigned *p = buf + splitmix64(seed + (unsigned long long)(base + r)) % words;
                v[r] = kAtomic ? atomicAdd(p, 1u) : *p;
            }
        }
#pragma unroll
        for (int r = 0; r < kProbeInFlight; ++r) acc += v[r];
    }
    // keeps every load and returned value live; the test practically never holds
    if (acc == 0x9e3779b9u) buf[0] = acc;
}

template <bool kAtomic>
int time_probe(unsigned *buf, unsigned long long words, long long ops, hipStream_t stream, unsigned grid,
               double *per_s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PICO_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("hipEventCreate failed");
        return PICO_EHIP;
    }
    int rc = PICO_OK;
    float ms = 0.f;
    // one untimed run (first-touch of the pages and the code), then the timed one
    hipLaunchKernelGGL(probe_kernel<kAtomic>, dim3(grid), dim3(kBlock), 0, stream, buf, words, ops, 1ull);
    if (hipEventRecord(e0, stream) != hipSuccess) rc = PICO_EHIP;
    hipLaunchKernelGGL(probe_kernel<kAtomic>, dim3(grid), dim3(kBlock), 0, stream, buf, words, ops,
                       0x5eedull);
    if (rc == PICO_OK && hipEventRecord(e1, stream) != hipSuccess) rc = PICO_EHIP;
    if (rc == PICO_OK && hipGetLastError() != hipSuccess) rc = PICO_EHIP;
    if (rc == PICO_OK && hipEventSynchronize(e1) != hipSuccess) rc = PICO_EHIP;
    if (rc == PICO_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = PICO_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PICO_OK) {
        set_error("random-access probe failed: %s", hipGetErrorString(hipGetLastError()));
        return rc;
    }
    *per_s = ms > 0.f ? (double)ops / ((double)ms * 1e-3) : 0.0;
    return PICO_OK;
}

}  // namespace
}  // namespace pico

using namespace pico;

extern "C" int pico_probe_random_access(void *buf, size_t bytes, int64_t ops, double *gathers_per_s,
                                        double *atomics_per_s, void *stream) {
    clear_error();
    if (!buf || bytes < 4 || ops <= 0 || !gathers_per_s || !atomics_per_s) {
        set_error("pico_probe_random_access: need a buffer of at least 4 bytes, ops > 0 and both outputs");
        return PICO_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    PICO_HIP_TRY(hipGetDevice(&dev));
    PICO_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)(cus > 0 ? cus : 1) * kProbePerCu;
    unsigned *w = static_cast<unsigned *>(buf);
    const unsigned long long words = (unsigned long long)(bytes / 4);
    int rc = time_probe<false>(w, words, (long long)ops, s, grid, gathers_per_s);
    if (rc) return rc;
    return time_probe<true>(w, words, (long long)ops, s, grid, atomics_per_s);
}
