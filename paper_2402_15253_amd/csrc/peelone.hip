// PeelOne with the assertion decrement and the dynamic in-level frontier
// (paper Section III, Alg. 4), for gfx950.
//
// Level k peels every residual vertex whose residual degree has reached k.
// The working array `core` holds residual degrees; by Corollary 1 every
// residual vertex has core >= k while level k runs, so the level's scan
// frontier is simply {v residual : core[v] == k} (no removal flag).
//
// Assertion decrement (Section III-B).  The paper's atomicSub_{>=k} stores
// max(old - 1, k).  gfx950 has no clamped-decrement atomic, so the scatter
// filters on core[u] > k (the test the paper puts before the atomic) and then
// issues a plain fetch-and-subtract; the thread whose fetch returns exactly
// k + 1 is the unique one that lowers u to k, so it alone asserts u into the
// level's queue and records out[u] = k.  A racing decrement that lands below
// k only touches a vertex already asserted at level k, whose final value is
// held in `out`, and no vertex receives more than deg(u) decrements, so the
// counter never underflows.  The vector produced is the one the clamped atomic
// gives, without compare-and-swap retry loops under hub contention.
//
// Dynamic frontier (Section III-C, step 3).  Asserted vertices are appended to
// the same queue and drained in the same level, batch after batch, so the
// level count equals the number of distinct coreness values.  A level whose
// scan finds no vertex jumps k straight to the smallest surviving value.
//
// Every vertex enters the queue exactly once over the whole run, so the queue
// is one array of n entries holding the peel order.
#include <climits>

#include "common.hpp"

namespace pico {
namespace {

struct PoCounters {
    unsigned long long qtail;    // vertices asserted into the peel queue so far
    unsigned long long na_next;  // survivors written by the current scan
    unsigned long long heavy_n;  // heavy edge-chunk descriptors of the current batch
    unsigned long long atomics;  // decrements issued (statistics)
    int minnext;                 // smallest surviving value above k seen by the scan
    int pad;
};

__global__ void po_reset_scan(PoCounters *c) {
    c->na_next = 0;
    c->minnext = INT_MAX;
}

__global__ void po_reset_all(PoCounters *c) {
    c->qtail = 0;
    c->na_next = 0;
    c->heavy_n = 0;
    c->atomics = 0;
    c->minnext = INT_MAX;
}

__global__ void po_reset_heavy(PoCounters *c) { c->heavy_n = 0; }

__device__ __forceinline__ void scan_one(bool valid, int v, int c, int k, int32_t *__restrict__ out,
                                         int32_t *__restrict__ Q, int32_t *__restrict__ A_next,
                                         PoCounters *__restrict__ cnt, int &local_min) {
    bool fr = valid && c == k;
    bool sv = valid && c > k;
    long long s = wave_append(fr, &cnt->qtail);
    if (fr) {
        Q[s] = v;
        out[v] = k;
    }
    long long t = wave_append(sv, &cnt->na_next);
    if (sv) {
        A_next[t] = v;
        local_min = min(local_min, c);
    }
}

// First scan over all vertex ids: core[v] = deg(v) (Alg. 4, initial step),
// isolated vertices get coreness 0, frontier = {deg == k}, survivors listed.
template <typename Off>
__global__ __launch_bounds__(kBlock) void po_first_scan(const Off *__restrict__ off, long long n,
                                                        int32_t *__restrict__ core,
                                                        int32_t *__restrict__ out, int k,
                                                        int32_t *__restrict__ Q,
                                                        int32_t *__restrict__ A_next,
                                                        PoCounters *__restrict__ cnt) {
    const long long stride = (long long)gridDim.x * kBlock;
    int local_min = INT_MAX;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < n;
         base += stride) {
        long long i = base + lane_id();
        bool valid = i < n;
        int c = -1;
        if (valid) {
            c = (int)(off[i + 1] - off[i]);
            core[i] = c;
            if (c == 0) out[i] = 0;
        }
        scan_one(valid && c > 0, (int)i, c, k, out, Q, A_next, cnt, local_min);
    }
    local_min = wave_min(local_min);
    if (lane_id() == 0 && local_min != INT_MAX) atomicMin(&cnt->minnext, local_min);
}

// Level scan over the survivor list of the previous scan (Alg. 4, scan
// kernel).  Entries peeled since then hold values below k and drop out.
__global__ __launch_bounds__(kBlock) void po_scan(const int32_t *__restrict__ A, long long nA,
                                                  const int32_t *__restrict__ core,
                                                  int32_t *__restrict__ out, int k,
                                                  int32_t *__restrict__ Q,
                                                  int32_t *__restrict__ A_next,
                                                  PoCounters *__restrict__ cnt) {
    const long long stride = (long long)gridDim.x * kBlock;
    int local_min = INT_MAX;
    for (long long base = (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < nA;
         base += stride) {
        long long i = base + lane_id();
        bool valid = i < nA;
        int v = 0, c = -1;
        if (valid) {
            v = A[i];
            c = core[v];
        }
        scan_one(valid, v, c, k, out, Q, A_next, cnt, local_min);
    }
    local_min = wave_min(local_min);
    if (lane_id() == 0 && local_min != INT_MAX) atomicMin(&cnt->minnext, local_min);
}

// One edge of the scatter (Alg. 4, graph operator): neighbour u of a peeled
// vertex.  Called by every lane of a wave together (`active` masks lanes out).
__device__ __forceinline__ void po_relax(bool active, int u, int k, int32_t *core,
                                         int32_t *__restrict__ out, int32_t *__restrict__ Q,
                                         PoCounters *__restrict__ cnt, int &natom) {
    bool push = false;
    if (active) {
        int cu = core[u];
        if (cu > k) {
            int old = atomicSub(&core[u], 1);
            push = (old == k + 1);
            ++natom;
        }
    }
    long long s = wave_append(push, &cnt->qtail);
    if (push) {
        Q[s] = u;
        out[u] = k;
    }
}

__device__ __forceinline__ int wave_max_i(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ void flush_count(int natom, unsigned long long *dst) {
    long long t = wave_sum64(natom);
    if (lane_id() == 0 && t) atomicAdd(dst, (unsigned long long)t);
}

// Scatter of queue batch Q[lo, hi): a lane per low-degree vertex, a wave per
// medium vertex, and fixed-size edge chunks for heavy vertices (emitted as
// descriptors for po_heavy).
template <typename Off>
__global__ __launch_bounds__(kBlock) void po_scatter(long long lo, long long hi,
                                                     const Off *__restrict__ off,
                                                     const int32_t *__restrict__ cols,
                                                     int32_t *core, int32_t *__restrict__ out,
                                                     int k, int32_t *Q,
                                                     PoCounters *__restrict__ cnt,
                                                     long long *__restrict__ heavy) {
    const long long stride = (long long)gridDim.x * kBlock;
    int natom = 0;
    for (long long base = lo + (long long)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < hi;
         base += stride) {
        long long i = base + lane_id();
        bool valid = i < hi;
        int v = 0;
        long long e0 = 0, e1 = 0;
        if (valid) {
            v = Q[i];
            e0 = (long long)off[v];
            e1 = (long long)off[v + 1];
        }
        long long d = e1 - e0;
        bool small = d <= kSmallDeg;
        int dj = small ? (int)d : 0;
        int maxd = wave_max_i(dj);
        for (int j = 0; j < maxd; ++j) {
            bool act = j < dj;
            int u = act ? cols[e0 + j] : 0;
            po_relax(act, u, k, core, out, Q, cnt, natom);
        }
        unsigned long long mm = __ballot(!small && d <= kHeavyDeg);
        while (mm) {
            int l = __ffsll(mm) - 1;
            mm &= mm - 1;
            long long a = __shfl(e0, l), b = __shfl(e1, l);
            for (long long e = a; e < b; e += kWave) {
                long long ee = e + lane_id();
                bool act = ee < b;
                int u = act ? cols[ee] : 0;
                po_relax(act, u, k, core, out, Q, cnt, natom);
            }
        }
        if (d > kHeavyDeg) {
            long long nch = (d + kChunk - 1) / kChunk;
            unsigned long long s = atomicAdd(&cnt->heavy_n, (unsigned long long)nch);
            for (long long j = 0; j < nch; ++j) heavy[s + j] = ((long long)v << 32) | j;
        }
    }
    flush_count(natom, &cnt->atomics);
}

// Heavy-vertex edge chunks of the current batch, one wave per chunk.
template <typename Off>
__global__ __launch_bounds__(kBlock) void po_heavy(const long long *__restrict__ heavy,
                                                   const Off *__restrict__ off,
                                                   const int32_t *__restrict__ cols,
                                                   int32_t *core, int32_t *__restrict__ out,
                                                   int k, int32_t *Q,
                                                   PoCounters *__restrict__ cnt) {
    const long long nh = (long long)cnt->heavy_n;
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    int natom = 0;
    for (long long h = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); h < nh; h += nw) {
        long long desc = heavy[h];
        int v = (int)(desc >> 32);
        long long j = desc & 0xffffffffll;
        long long vb = (long long)off[v], ve = (long long)off[v + 1];
        long long e0 = vb + j * kChunk;
        long long e1 = e0 + kChunk < ve ? e0 + kChunk : ve;
        for (long long e = e0; e < e1; e += kWave) {
            long long ee = e + lane_id();
            bool act = ee < e1;
            int u = act ? cols[ee] : 0;
            po_relax(act, u, k, core, out, Q, cnt, natom);
        }
    }
    flush_count(natom, &cnt->atomics);
}

constexpr int kGridCap = 4096;

int blocks_for(long long items) { return grid_for((items + kBlock - 1) / kBlock, kGridCap); }

}  // namespace

size_t peelone_ws_bytes(int64_t n, int64_t m) {
    return carve_bytes(n, 4) * 4 + carve_bytes(heavy_capacity(m), 8) + carve_bytes(1, sizeof(PoCounters));
}

template <typename Off>
int run_peelone(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out, void *ws,
                size_t ws_bytes, pico_stats *st, hipStream_t stream) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    int32_t *core = cv.take<int32_t>(n);
    int32_t *A[2] = {cv.take<int32_t>(n), cv.take<int32_t>(n)};
    int32_t *Q = cv.take<int32_t>(n);
    long long *heavy = cv.take<long long>(heavy_capacity(m));
    PoCounters *cnt = cv.take<PoCounters>(1);
    if (!core || !A[0] || !A[1] || !Q || !heavy || !cnt) {
        set_error("PeelOne workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  peelone_ws_bytes(n, m));
        return PICO_ENOMEM;
    }
    PoCounters *h = static_cast<PoCounters *>(host_scratch(sizeof(PoCounters)));
    if (!h) return PICO_EHIP;

    auto readback = [&]() -> int {
        PICO_HIP_TRY(hipMemcpyAsync(h, cnt, sizeof(PoCounters), hipMemcpyDeviceToHost, stream));
        PICO_HIP_TRY(hipStreamSynchronize(stream));
        return PICO_OK;
    };

    int k = 1;
    int cur = 0;  // A[cur] receives the survivors of the next scan
    PICO_LAUNCH("po_reset", po_reset_all, dim3(1), dim3(1), stream, cnt);
    PICO_LAUNCH("po_scan", po_first_scan<Off>, dim3(blocks_for(n)), dim3(kBlock), stream, off,
                (long long)n, core, out, k, Q, A[cur], cnt);
    PICO_LAUNCH_CHECK();
    int rc = readback();
    if (rc) return rc;
    const unsigned long long peelable = h->qtail + h->na_next;
    long long nA = (long long)h->na_next;
    unsigned long long level_lo = 0;
    int64_t levels = 0, batches = 0, scans = 1, dynamic = 0;
    int kmax = 0;

    while (true) {
        // Each pass either peels a level (k grows by one) or jumps k to a
        // larger surviving value, so there are fewer than 2n + 2 passes.
        if (scans > 2 * n + 2) {
            set_error("PeelOne made no progress after %lld scans", (long long)scans);
            return PICO_EINVAL;
        }
        unsigned long long lo = level_lo, hi = h->qtail;
        if (hi == lo) {
            // Empty level: every residual value exceeds k; jump to the smallest.
            if (nA == 0) break;
            k = h->minnext;
        } else {
            ++levels;
            kmax = k;
            unsigned long long level_scan_end = hi;
            while (lo < hi) {
                ++batches;
                PICO_LAUNCH("po_reset", po_reset_heavy, dim3(1), dim3(1), stream, cnt);
                PICO_LAUNCH("po_scatter", po_scatter<Off>, dim3(blocks_for((long long)(hi - lo))),
                            dim3(kBlock), stream, (long long)lo, (long long)hi, off, cols, core, out,
                            k, Q, cnt, heavy);
                PICO_LAUNCH("po_heavy", po_heavy<Off>, dim3(kGridCap), dim3(kBlock), stream, heavy,
                            off, cols, core, out, k, Q, cnt);
                PICO_LAUNCH_CHECK();
                rc = readback();
                if (rc) return rc;
                lo = hi;
                hi = h->qtail;
            }
            dynamic += (int64_t)(h->qtail - level_scan_end);
            if (h->qtail >= peelable) break;
            k += 1;
        }
        // Scan the survivors of the previous scan at the new level.
        const int32_t *src = A[cur];
        cur ^= 1;
        level_lo = h->qtail;
        PICO_LAUNCH("po_reset", po_reset_scan, dim3(1), dim3(1), stream, cnt);
        PICO_LAUNCH("po_scan", po_scan, dim3(blocks_for(nA)), dim3(kBlock), stream, src, nA, core,
                    out, k, Q, A[cur], cnt);
        PICO_LAUNCH_CHECK();
        ++scans;
        rc = readback();
        if (rc) return rc;
        nA = (long long)h->na_next;
    }
    if (st) {
        st->iterations = levels;
        st->sub_rounds = batches;
        st->scans = scans;
        st->frontier_total = (int64_t)h->qtail;
        st->k_max = kmax;
        st->edges_scanned = m;  // every peeled vertex scans its whole row once
        st->atomics = (int64_t)h->atomics;
        st->buckets_scanned = 0;
        st->pushes_dynamic = dynamic;
    }
    return PICO_OK;
}

template int run_peelone<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                  void *, size_t, pico_stats *, hipStream_t);
template int run_peelone<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                  void *, size_t, pico_stats *, hipStream_t);

}  // namespace pico
