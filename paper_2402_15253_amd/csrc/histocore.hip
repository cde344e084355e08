// HistoCore (paper Section IV-B, Alg. 6) for gfx950.
//
// Index2core (Section II-A, Alg. 2): every vertex starts at its degree and
// repeatedly replaces its estimate by the h-index of its neighbours'
// estimates; the fixed point is the coreness.  HistoCore keeps, per vertex,
// a histogram of the neighbours' current estimates, so a vertex that changes
// many times never re-reads its adjacency to recompute the h-index.
//
// Histogram layout: bucket b (1 <= b <= deg(v)) of vertex v lives at
// histo[off[v] + b - 1], so the histograms of all vertices form one int32
// array of m entries aligned with the adjacency array.  For b < core[v] the
// bucket counts neighbours whose estimate is exactly b; bucket core[v] counts
// neighbours whose estimate is >= core[v], which is cnt(v) of Theorem 2;
// buckets above core[v] are dead.
//
// Phases (separate kernels, so each round sees the previous round's values):
//   InitHisto   bucket min(core[u], core[v]) of v counts neighbour u, with
//               core = deg; the first frontier is {v : cnt(v) < core(v)}.
//   SumHisto    for each frontier vertex, sum buckets from its old value
//               downwards and stop at the first k whose running sum reaches k
//               (Step II of Fig. 6); that k is the new estimate and the sum is
//               its cnt, stored in bucket k.
//   UpdateHisto for each vertex v that changed and each neighbour u valued
//               above v's new value (neighbour types N1 and N3 of Section
//               IV-B-1): move v from bucket min(oldcore[v], core[u]) of u to
//               bucket core[v].  When that takes u's top bucket from exactly
//               core[u] to core[u] - 1, u's cnt has just fallen below its
//               value, so u is the unique trigger that enqueues it for the
//               next round (the top bucket only decreases within the phase).
// The loop stops when a round enqueues nobody.  By Theorem 2 each round's
// frontier is exactly the set of vertices whose h-index changes in that
// synchronous round.
#include "common.hpp"

namespace pico {
namespace {

struct HcCounters {
    unsigned long long fcount[2];  // frontier sizes, by round parity
    unsigned long long heavy_n;    // heavy edge-chunk descriptors
    unsigned long long hv_n;       // heavy vertices (InitHisto) / heavy sums (SumHisto)
    unsigned long long upd_edges;  // statistics: adjacency entries read by UpdateHisto
    unsigned long long upd_moves;  // statistics: histogram moves (two atomics each)
    unsigned long long buckets;    // statistics: buckets summed by SumHisto
};

// SumHisto: a wave handles values up to this size; above, a workgroup does.
constexpr int kSumWaveMax = 8192;
constexpr int kGridCap = 4096;

int blocks_for(long long items) { return grid_for((items + kBlock - 1) / kBlock, kGridCap); }

__global__ void hc_reset(HcCounters *c) {
    c->fcount[0] = 0;
    c->fcount[1] = 0;
    c->heavy_n = 0;
    c->hv_n = 0;
    c->upd_edges = 0;
    c->upd_moves = 0;
    c->buckets = 0;
}

__device__ __forceinline__ void flush_count(long long x, unsigned long long *dst) {
    long long t = wave_sum64(x);
    if (lane_id() == 0 && t) atomicAdd(dst, (unsigned long long)t);
}

__global__ void hc_reset_round(HcCounters *c, int nxt) {
    c->fcount[nxt] = 0;
    c->heavy_n = 0;
    c->hv_n = 0;
}

__device__ __forceinline__ int wave_max_i(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_init_core(const Off *__restrict__ off, long long n,
                                                       int32_t *__restrict__ core) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
        core[v] = (int)(off[v + 1] - off[v]);
}

// InitHisto for light and medium vertices; heavy ones are listed and their
// segments handled by the chunk kernels below.
template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_init_histo(const Off *__restrict__ off,
                                                        const int32_t *__restrict__ cols, long long n,
                                                        const int32_t *__restrict__ core,
                                                        int32_t *__restrict__ histo,
                                                        int32_t *__restrict__ F,
                                                        HcCounters *__restrict__ cnt,
                                                        long long *__restrict__ heavy,
                                                        int32_t *__restrict__ hverts) {
    __shared__ int lds_all[kWavesPerBlock][kLdsBuckets];
    int *lds = lds_all[threadIdx.x >> 6];
    const int lane = lane_id();
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < n;
         base += stride) {
        long long v = base + lane;
        bool valid = v < n;
        int d = valid ? core[v] : 0;
        long long e0 = valid ? (long long)off[v] : 0;
        bool push = false;
        if (valid && d > 0 && d <= kSmallDeg) {
            // one lane owns v's segment: plain read-modify-write, no atomics
            for (int j = 0; j < d; ++j) histo[e0 + j] = 0;
            for (int j = 0; j < d; ++j) {
                int u = cols[e0 + j];
                int b = min(max(core[u], 1), d);  // core[u] >= 1 on a symmetric graph
                histo[e0 + b - 1] += 1;
            }
            push = histo[e0 + d - 1] < d;
        }
        unsigned long long mm = __ballot(valid && d > kSmallDeg && d <= kLdsBuckets);
        while (mm) {
            int l = __ffsll(mm) - 1;
            mm &= mm - 1;
            int dd = __shfl(d, l);
            long long a = __shfl(e0, l);
            for (int j = lane; j < dd; j += kWave) lds[j] = 0;
            wave_lds_sync();
            for (int j = lane; j < dd; j += kWave) {
                int u = cols[a + j];
                atomicAdd(&lds[min(max(core[u], 1), dd) - 1], 1);
            }
            wave_lds_sync();
            for (int j = lane; j < dd; j += kWave) histo[a + j] = lds[j];
            int top = lds[dd - 1];
            wave_lds_sync();
            if (lane == l) push = top < dd;
        }
        long long s = wave_append(push, &cnt->fcount[0]);
        if (push) F[s] = (int)v;
        bool hv = valid && d > kLdsBuckets;
        long long t = wave_append(hv, &cnt->hv_n);
        if (hv) {
            hverts[t] = (int)v;
            long long nch = ((long long)d + kChunk - 1) / kChunk;
            unsigned long long c0 = atomicAdd(&cnt->heavy_n, (unsigned long long)nch);
            for (long long j = 0; j < nch; ++j) heavy[c0 + j] = (v << 32) | j;
        }
    }
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_init_heavy_zero(const long long *__restrict__ heavy,
                                                             const HcCounters *__restrict__ cnt,
                                                             const Off *__restrict__ off,
                                                             int32_t *__restrict__ histo) {
    const long long nh = (long long)cnt->heavy_n;
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    for (long long h = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); h < nh; h += nw) {
        long long desc = heavy[h];
        int v = (int)(desc >> 32);
        long long j = desc & 0xffffffffll;
        long long vb = (long long)off[v], ve = (long long)off[v + 1];
        long long e0 = vb + j * kChunk, e1 = e0 + kChunk < ve ? e0 + kChunk : ve;
        for (long long e = e0 + lane_id(); e < e1; e += kWave) histo[e] = 0;
    }
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_init_heavy_count(const long long *__restrict__ heavy,
                                                              const HcCounters *__restrict__ cnt,
                                                              const Off *__restrict__ off,
                                                              const int32_t *__restrict__ cols,
                                                              const int32_t *__restrict__ core,
                                                              int32_t *histo) {
    const long long nh = (long long)cnt->heavy_n;
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    for (long long h = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); h < nh; h += nw) {
        long long desc = heavy[h];
        int v = (int)(desc >> 32);
        long long j = desc & 0xffffffffll;
        long long vb = (long long)off[v], ve = (long long)off[v + 1];
        int d = (int)(ve - vb);
        long long e0 = vb + j * kChunk, e1 = e0 + kChunk < ve ? e0 + kChunk : ve;
        for (long long e = e0 + lane_id(); e < e1; e += kWave) {
            int u = cols[e];
            atomicAdd(&histo[vb + min(max(core[u], 1), d) - 1], 1);
        }
    }
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_init_heavy_check(const int32_t *__restrict__ hverts,
                                                              const Off *__restrict__ off,
                                                              const int32_t *__restrict__ core,
                                                              const int32_t *__restrict__ histo,
                                                              int32_t *__restrict__ F,
                                                              HcCounters *__restrict__ cnt) {
    const long long nv = (long long)cnt->hv_n;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < nv;
         base += stride) {
        long long i = base + lane_id();
        bool push = false;
        int v = 0;
        if (i < nv) {
            v = hverts[i];
            int d = core[v];
            push = histo[(long long)off[v] + d - 1] < d;
        }
        long long s = wave_append(push, &cnt->fcount[0]);
        if (push) F[s] = v;
    }
}

// Reverse summation by one wave over buckets top, top-1, ..., floor (Step II
// of Fig. 6), starting from running sum `carry`, never below bucket `lowb`.
// Returns the first bucket b with carry + sum(b..top) >= b, with that sum,
// or b = 0 if none.
__device__ __forceinline__ void wave_reverse_sum(const int32_t *seg, int top, int lowb, int carry,
                                                 int &h, int &s) {
    const int lane = lane_id();
    h = 0;
    s = carry;
    while (top >= lowb) {
        int b = top - lane;
        int val = (b >= lowb) ? seg[b - 1] : 0;
        int S = carry + wave_incl_scan(val);
        unsigned long long mk = __ballot(b >= lowb && S >= b);
        if (mk) {
            int l = __ffsll(mk) - 1;
            h = top - l;
            s = __shfl(S, l);
            return;
        }
        carry = __shfl(S, kWave - 1);
        top -= kWave;
    }
    s = carry;
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_sum(const int32_t *__restrict__ F, long long nf,
                                                 const Off *__restrict__ off, int32_t *core,
                                                 int32_t *__restrict__ oldcore, int32_t *histo,
                                                 int32_t *__restrict__ hlist,
                                                 HcCounters *__restrict__ cnt) {
    const int lane = lane_id();
    const long long stride = (long long)gridDim.x * kBlock;
    long long nb = 0;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < nf;
         base += stride) {
        long long i = base + lane;
        bool valid = i < nf;
        int v = 0, c_old = 0;
        long long e0 = 0;
        if (valid) {
            v = F[i];
            c_old = core[v];
            e0 = (long long)off[v];
        }
        if (valid && c_old <= kSmallDeg) {
            int s = 0, k = c_old;
            for (; k >= 1; --k) {
                s += histo[e0 + k - 1];
                if (s >= k) break;
            }
            if (k < 1) k = 0;  // unreachable for a symmetric simple graph
            core[v] = k;
            oldcore[v] = c_old;
            if (k >= 1) histo[e0 + k - 1] = s;
            nb += c_old - max(k, 1) + 1;
        }
        unsigned long long mm = __ballot(valid && c_old > kSmallDeg && c_old <= kSumWaveMax);
        while (mm) {
            int l = __ffsll(mm) - 1;
            mm &= mm - 1;
            int vv = __shfl(v, l), cc = __shfl(c_old, l);
            long long a = __shfl(e0, l);
            int h, s;
            wave_reverse_sum(histo + a, cc, 1, 0, h, s);
            if (lane == 0) {
                core[vv] = h;
                oldcore[vv] = cc;
                if (h >= 1) histo[a + h - 1] = s;
                nb += cc - max(h, 1) + 1;
            }
        }
        bool hv = valid && c_old > kSumWaveMax;
        long long t = wave_append(hv, &cnt->hv_n);
        if (hv) hlist[t] = v;
    }
    flush_count(nb, &cnt->buckets);
}

// SumHisto for vertices with very large old values: a workgroup per vertex.
// Each thread sums one slice of the bucket range; the slices' running sums
// locate the slice holding the answer (carry + sum(b..top) - b decreases
// strictly as b grows), and one wave finishes inside that slice.
template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_sum_heavy(const int32_t *__restrict__ hlist,
                                                       HcCounters *__restrict__ cnt,
                                                       const Off *__restrict__ off, int32_t *core,
                                                       int32_t *__restrict__ oldcore,
                                                       int32_t *histo) {
    __shared__ int part[kBlock];
    __shared__ int first_ok;
    const int t = threadIdx.x;
    const long long nh = (long long)cnt->hv_n;
    for (long long j = blockIdx.x; j < nh; j += gridDim.x) {
        int v = hlist[j];
        int c_old = core[v];
        long long e0 = (long long)off[v];
        const int32_t *seg = histo + e0;
        int L = (c_old + kBlock - 1) / kBlock;
        int hi_b = c_old - t * L;          // slice t covers buckets [lo_b, hi_b]
        int lo_b = max(1, hi_b - L + 1);
        int sum = 0;
        for (int b = hi_b; b >= lo_b; --b) sum += seg[b - 1];
        if (hi_b < 1) sum = 0;
        part[t] = sum;
        if (t == 0) first_ok = kBlock;
        __syncthreads();
        // inclusive running sum over slices 0..t (highest buckets first)
        for (int o = 1; o < kBlock; o <<= 1) {
            int y = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += y;
            __syncthreads();
        }
        bool ok = hi_b >= 1 && part[t] >= lo_b;
        if (ok) atomicMin(&first_ok, t);
        __syncthreads();
        int ts = first_ok;
        if (ts < kBlock && (t >> 6) == 0) {
            int top = c_old - ts * L;
            int lowb = max(1, top - L + 1);
            int carry = ts > 0 ? part[ts - 1] : 0;
            int h, s;
            wave_reverse_sum(seg, top, lowb, carry, h, s);
            if (t == 0) {
                core[v] = h;
                oldcore[v] = c_old;
                if (h >= 1) histo[e0 + h - 1] = s;
                atomicAdd(&cnt->buckets, (unsigned long long)(c_old - max(h, 1) + 1));
            }
        } else if (ts >= kBlock && t == 0) {
            core[v] = 0;  // unreachable for a symmetric simple graph
            oldcore[v] = c_old;
        }
        __syncthreads();
    }
}

// UpdateHisto for one edge (v, u); every lane of the wave calls it together.
template <typename Off>
__device__ __forceinline__ void hc_relax(bool active, int u, int cv, int ov,
                                         const Off *__restrict__ off,
                                         const int32_t *__restrict__ core, int32_t *histo,
                                         int32_t *__restrict__ Fn, unsigned long long *fcnt,
                                         long long &nmove) {
    bool push = false;
    if (active) {
        int cu = core[u];
        if (cu > cv && cv >= 1) {
            long long hb = (long long)off[u] - 1;
            int b = min(ov, cu);
            int c = atomicSub(&histo[hb + b], 1);
            atomicAdd(&histo[hb + cv], 1);
            push = (ov >= cu) && (c == cu);
            ++nmove;
        }
    }
    long long s = wave_append(push, fcnt);
    if (push) Fn[s] = u;
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_update(const int32_t *__restrict__ F, long long nf,
                                                    const Off *__restrict__ off,
                                                    const int32_t *__restrict__ cols,
                                                    const int32_t *__restrict__ core,
                                                    const int32_t *__restrict__ oldcore,
                                                    int32_t *histo, int32_t *__restrict__ Fn,
                                                    HcCounters *__restrict__ cnt, int nxt,
                                                    long long *__restrict__ heavy) {
    const int lane = lane_id();
    unsigned long long *fcnt = &cnt->fcount[nxt];
    const long long stride = (long long)gridDim.x * kBlock;
    long long nmove = 0, nedge = 0;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < nf;
         base += stride) {
        long long i = base + lane;
        bool valid = i < nf;
        int v = 0, cv = 0, ov = 0;
        long long e0 = 0, e1 = 0;
        if (valid) {
            v = F[i];
            cv = core[v];
            ov = oldcore[v];
            e0 = (long long)off[v];
            e1 = (long long)off[v + 1];
        }
        long long d = e1 - e0;
        nedge += d;
        bool small = d <= kSmallDeg;
        int dj = small ? (int)d : 0;
        int maxd = wave_max_i(dj);
        for (int j = 0; j < maxd; ++j) {
            bool act = j < dj;
            int u = act ? cols[e0 + j] : 0;
            hc_relax<Off>(act, u, cv, ov, off, core, histo, Fn, fcnt, nmove);
        }
        unsigned long long mm = __ballot(!small && d <= kHeavyDeg);
        while (mm) {
            int l = __ffsll(mm) - 1;
            mm &= mm - 1;
            long long a = __shfl(e0, l), b = __shfl(e1, l);
            int cvv = __shfl(cv, l), ovv = __shfl(ov, l);
            for (long long e = a; e < b; e += kWave) {
                long long ee = e + lane;
                bool act = ee < b;
                int u = act ? cols[ee] : 0;
                hc_relax<Off>(act, u, cvv, ovv, off, core, histo, Fn, fcnt, nmove);
            }
        }
        if (d > kHeavyDeg) {
            long long nch = (d + kChunk - 1) / kChunk;
            unsigned long long s = atomicAdd(&cnt->heavy_n, (unsigned long long)nch);
            for (long long j = 0; j < nch; ++j) heavy[s + j] = ((long long)v << 32) | j;
        }
    }
    flush_count(nmove, &cnt->upd_moves);
    flush_count(nedge, &cnt->upd_edges);
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_update_heavy(const long long *__restrict__ heavy,
                                                          const Off *__restrict__ off,
                                                          const int32_t *__restrict__ cols,
                                                          const int32_t *__restrict__ core,
                                                          const int32_t *__restrict__ oldcore,
                                                          int32_t *histo, int32_t *__restrict__ Fn,
                                                          HcCounters *__restrict__ cnt, int nxt) {
    const long long nh = (long long)cnt->heavy_n;
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    long long nmove = 0;
    for (long long h = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); h < nh; h += nw) {
        long long desc = heavy[h];
        int v = (int)(desc >> 32);
        long long j = desc & 0xffffffffll;
        int cv = core[v], ov = oldcore[v];
        long long vb = (long long)off[v], ve = (long long)off[v + 1];
        long long e0 = vb + j * kChunk, e1 = e0 + kChunk < ve ? e0 + kChunk : ve;
        for (long long e = e0; e < e1; e += kWave) {
            long long ee = e + lane_id();
            bool act = ee < e1;
            int u = act ? cols[ee] : 0;
            hc_relax<Off>(act, u, cv, ov, off, core, histo, Fn, &cnt->fcount[nxt], nmove);
        }
    }
    flush_count(nmove, &cnt->upd_moves);
}

}  // namespace

size_t histocore_ws_bytes(int64_t n, int64_t m) {
    return carve_bytes(m, 4) + carve_bytes(n, 4) * 4 + carve_bytes(heavy_capacity(m), 8) +
           carve_bytes(1, sizeof(HcCounters));
}

template <typename Off>
int run_histocore(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out, void *ws,
                  size_t ws_bytes, pico_stats *st, hipStream_t stream) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    int32_t *histo = cv.take<int32_t>(m);
    int32_t *oldcore = cv.take<int32_t>(n);
    int32_t *F[2] = {cv.take<int32_t>(n), cv.take<int32_t>(n)};
    int32_t *hlist = cv.take<int32_t>(n);
    long long *heavy = cv.take<long long>(heavy_capacity(m));
    HcCounters *cnt = cv.take<HcCounters>(1);
    if (!histo || !oldcore || !F[0] || !F[1] || !hlist || !heavy || !cnt) {
        set_error("HistoCore workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  histocore_ws_bytes(n, m));
        return PICO_ENOMEM;
    }
    HcCounters *h = static_cast<HcCounters *>(host_scratch(sizeof(HcCounters)));
    if (!h) return PICO_EHIP;
    int32_t *core = out;  // the estimates converge in place to the coreness

    PICO_LAUNCH("hc_reset", hc_reset, dim3(1), dim3(1), stream, cnt);
    PICO_LAUNCH("hc_init_core", hc_init_core<Off>, dim3(blocks_for(n)), dim3(kBlock), stream, off,
                (long long)n, core);
    PICO_LAUNCH("hc_init_histo", hc_init_histo<Off>, dim3(blocks_for(n)), dim3(kBlock), stream, off,
                cols, (long long)n, core, histo, F[0], cnt, heavy, hlist);
    PICO_LAUNCH("hc_init_heavy", hc_init_heavy_zero<Off>, dim3(kGridCap), dim3(kBlock), stream,
                heavy, cnt, off, histo);
    PICO_LAUNCH("hc_init_heavy", hc_init_heavy_count<Off>, dim3(kGridCap), dim3(kBlock), stream,
                heavy, cnt, off, cols, core, histo);
    PICO_LAUNCH("hc_init_heavy", hc_init_heavy_check<Off>, dim3(64), dim3(kBlock), stream, hlist,
                off, core, histo, F[0], cnt);
    PICO_LAUNCH_CHECK();
    PICO_HIP_TRY(hipMemcpyAsync(h, cnt, sizeof(HcCounters), hipMemcpyDeviceToHost, stream));
    PICO_HIP_TRY(hipStreamSynchronize(stream));

    long long nf = (long long)h->fcount[0];
    const long long first_frontier = nf;
    int cur = 0;
    int64_t rounds = 0, frontier_total = 0;
    while (nf > 0) {
        // Every round lowers the value of each frontier vertex, so there are
        // at most sum(deg) = m rounds; more means a malformed graph.
        if (rounds > m) {
            set_error("HistoCore made no progress after %lld rounds (malformed graph?)",
                      (long long)rounds);
            return PICO_EINVAL;
        }
        ++rounds;
        frontier_total += nf;
        int nxt = cur ^ 1;
        PICO_LAUNCH("hc_reset", hc_reset_round, dim3(1), dim3(1), stream, cnt, nxt);
        PICO_LAUNCH("hc_sum", hc_sum<Off>, dim3(blocks_for(nf)), dim3(kBlock), stream, F[cur], nf, off,
                    core, oldcore, histo, hlist, cnt);
        PICO_LAUNCH("hc_sum_heavy", hc_sum_heavy<Off>, dim3(256), dim3(kBlock), stream, hlist, cnt, off,
                    core, oldcore, histo);
        PICO_LAUNCH("hc_update", hc_update<Off>, dim3(blocks_for(nf)), dim3(kBlock), stream, F[cur],
                    nf, off, cols, core, oldcore, histo, F[nxt], cnt, nxt, heavy);
        PICO_LAUNCH("hc_update_heavy", hc_update_heavy<Off>, dim3(kGridCap), dim3(kBlock), stream,
                    heavy, off, cols, core, oldcore, histo, F[nxt], cnt, nxt);
        PICO_LAUNCH_CHECK();
        PICO_HIP_TRY(hipMemcpyAsync(h, cnt, sizeof(HcCounters), hipMemcpyDeviceToHost, stream));
        PICO_HIP_TRY(hipStreamSynchronize(stream));
        nf = (long long)h->fcount[nxt];
        cur = nxt;
    }
    if (st) {
        st->iterations = rounds;
        st->sub_rounds = rounds;
        st->scans = 0;
        st->frontier_total = frontier_total;
        st->k_max = 0;
        st->edges_scanned = (int64_t)h->upd_edges;
        st->atomics = (int64_t)h->upd_moves;
        st->buckets_scanned = (int64_t)h->buckets;
        st->pushes_dynamic = frontier_total - first_frontier;
    }
    return PICO_OK;
}

template int run_histocore<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                    void *, size_t, pico_stats *, hipStream_t);
template int run_histocore<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                    void *, size_t, pico_stats *, hipStream_t);

}  // namespace pico
