// Choice between PeelOne and HistoCore for one graph (PICO_ALGO_AUTO).
//
// The paper finds that neither paradigm wins everywhere (Section V, Table VII:
// HistoCore ahead where its round count l2 is far below PeelOne's level count
// l1) and leaves a hybrid to future work (Section VII).  PeelOne's cost on
// this GPU grows with its level count (each level costs grid barriers) and
// HistoCore's with its rounds and histogram traffic.  Two cheap features,
// measured before the run, predict which dominates:
//
//   H  -- the degree h-index: the largest h such that at least h vertices
//         have degree >= h.  A k-core needs k + 1 vertices of degree >= k, so
//         k_max <= H, and PeelOne's level count l1 <= k_max (Table V).
//   f  -- the share of sampled vertices already in HistoCore's first
//         frontier, cnt(v) < deg(v) (Theorem 2, with core = deg).  f == 0
//         means the degrees are already the coreness for the sample (cliques,
//         regular components): HistoCore's InitHisto alone finishes.
//
// The rule (constants from a sweep of 47 graphs on MI355X: ER, R-MAT with
// edge factors 4 to 48 and scales 10 to 21, planted blocks, clique unions):
//   m < 2^16                        -> PeelOne (launch-bound either way)
//   f < 1/64                        -> HistoCore
//   m < 2^23 and H >= 4 m / n       -> HistoCore (skewed, many levels,
//                                      histogram traffic still small)
//   otherwise                       -> PeelOne
#include <climits>

#include "common.hpp"

namespace pico {
namespace {

constexpr int kFeatLds = 2048;       // LDS histogram bins per workgroup
constexpr int kSamples = 1024;       // vertices sampled for f
constexpr int kSampleMaxDeg = 1024;  // sampled vertices of larger degree are skipped

// Degree histogram, bins 0..B (degrees above B counted in bin B).
template <typename Off>
__global__ __launch_bounds__(kBlock) void feat_hist(const Off *off, long long n, int B, unsigned *hist) {
    __shared__ unsigned lh[kFeatLds];
    for (int i = threadIdx.x; i < kFeatLds; i += kBlock) lh[i] = 0;
    __syncthreads();
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock) {
        const long long d = (long long)off[v + 1] - (long long)off[v];
        const int b = d < B ? (int)d : B;
        if (b < kFeatLds) atomicAdd(&lh[b], 1u);
        else atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kFeatLds && i <= B; i += kBlock)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// One wave per sampled vertex v_j = floor(j n / S): is cnt(v) < deg(v)?
template <typename Off>
__global__ __launch_bounds__(kBlock) void feat_sample(const Off *off, const int32_t *cols, long long n, int S,
                                                      unsigned *counts /* [0] valid, [1] in frontier */) {
    const int j = (int)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (j >= S) return;
    const long long v = (long long)j * n / S;
    const long long e0 = (long long)off[v];
    const long long d = (long long)off[v + 1] - e0;
    if (d == 0 || d > kSampleMaxDeg) return;
    int cnt = 0;
    for (long long e = lane_id(); e < d; e += kWave) {
        const int u = cols[e0 + e];
        cnt += ((long long)off[u + 1] - (long long)off[u]) >= d ? 1 : 0;
    }
    cnt = (int)wave_sum64(cnt);
    if (lane_id() == 0) {
        atomicAdd(&counts[0], 1u);
        if (cnt < d) atomicAdd(&counts[1], 1u);
    }
}

// H = the largest h with sum_{d >= h} hist[d] >= h, by one workgroup: each
// thread owns a contiguous run of bins, the runs' totals are suffix-summed,
// and each thread walks its run downwards.
__global__ __launch_bounds__(kBlock) void feat_hindex(const unsigned *hist, int B, long long *H_out) {
    __shared__ long long tot[kBlock];
    __shared__ long long best;
    const int per = (B + 1 + kBlock - 1) / kBlock;
    const int lo = threadIdx.x * per, hi = lo + per - 1 < B ? lo + per - 1 : B;
    long long s = 0;
    for (int b = lo; b <= hi; ++b) s += hist[b];
    tot[threadIdx.x] = s;
    if (threadIdx.x == 0) best = 0;
    __syncthreads();
    long long above = 0;  // vertices in the bins above this thread's run
    for (int t = threadIdx.x + 1; t < kBlock; ++t) above += tot[t];
    long long h = 0;
    for (int b = hi; b >= lo && b >= 1; --b) {
        above += hist[b];
        if (above >= b) {
            h = b;
            break;
        }
    }
    if (h) atomicMax((unsigned long long *)&best, (unsigned long long)h);
    __syncthreads();
    if (threadIdx.x == 0) *H_out = best;
}

__global__ void feat_clear(unsigned *p, long long words) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int feat_bins(int64_t n, int64_t m) {
    // H <= sqrt(m): H vertices of degree >= H hold at least H^2 entries
    long long r = 1;
    while ((r + 1) * (r + 1) <= m) ++r;
    long long B = r + 1;
    if (B > n) B = n;
    return (int)(B < 1 ? 1 : B);
}

}  // namespace

size_t select_ws_bytes(int64_t n, int64_t m) {
    return carve_bytes((int64_t)feat_bins(n, m) + 1, 4) + carve_bytes(4, 8);
}

int choose_algo(int64_t n, int64_t m, int64_t H, int64_t sampled, int64_t in_frontier) {
    if (m < (1ll << 16)) return PICO_ALGO_PEELONE;
    if (sampled > 0 && in_frontier * 64 < sampled) return PICO_ALGO_HISTOCORE;
    if (m < (1ll << 23) && n > 0 && H * n >= 4 * m) return PICO_ALGO_HISTOCORE;
    return PICO_ALGO_PEELONE;
}

template <typename Off>
int select_features(const Off *off, const int32_t *cols, int64_t n, int64_t m, void *ws, size_t ws_bytes,
                    hipStream_t stream, int64_t feat[3]) {
    feat[0] = feat[1] = feat[2] = 0;
    if (n <= 0) return PICO_OK;
    const int B = feat_bins(n, m);
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    unsigned *hist = cv.take<unsigned>((int64_t)B + 1);
    long long *res = cv.take<long long>(4);  // [0] H, [1] counts (two unsigned)
    if (!hist || !res) {
        set_error("workspace too small for the algorithm choice (%zu bytes given, %zu needed)", ws_bytes,
                  select_ws_bytes(n, m));
        return PICO_ENOMEM;
    }
    unsigned *counts = reinterpret_cast<unsigned *>(res + 1);
    PICO_LAUNCH("feat_clear", feat_clear, dim3(64), dim3(256), stream, hist, (long long)B + 1);
    PICO_LAUNCH("feat_clear", feat_clear, dim3(1), dim3(64), stream, reinterpret_cast<unsigned *>(res), 8ll);
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    PICO_LAUNCH("feat_hist", feat_hist<Off>, dim3((unsigned)blocks), dim3(kBlock), stream, off, (long long)n, B,
                hist);
    const int S = n < kSamples ? (int)n : kSamples;
    PICO_LAUNCH("feat_sample", feat_sample<Off>, dim3((unsigned)((S + kWavesPerBlock - 1) / kWavesPerBlock)),
                dim3(kBlock), stream, off, cols, (long long)n, S, counts);
    PICO_LAUNCH("feat_hindex", feat_hindex, dim3(1), dim3(kBlock), stream, hist, B, res);
    PICO_LAUNCH_CHECK();
    long long *h = static_cast<long long *>(host_scratch(4 * sizeof(long long)));
    if (!h) return PICO_EHIP;
    PICO_HIP_TRY(hipMemcpyAsync(h, res, 2 * sizeof(long long), hipMemcpyDeviceToHost, stream));
    PICO_HIP_TRY(hipStreamSynchronize(stream));
    const unsigned *c = reinterpret_cast<const unsigned *>(h + 1);
    feat[0] = h[0];
    feat[1] = c[0];
    feat[2] = c[1];
    return PICO_OK;
}

template int select_features<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, void *, size_t,
                                      hipStream_t, int64_t[3]);
template int select_features<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, void *, size_t,
                                      hipStream_t, int64_t[3]);

}  // namespace pico
