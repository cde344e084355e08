// Batched decomposition of many independent graphs in one launch.
//
// Work items are graphs.  Each workgroup claims whole graphs from a device
// counter (in the order given, normally largest first) and runs the complete
// decomposition of a graph by itself -- PeelOne (paper Section III, Alg. 4)
// or HistoCore (Section IV-B, Alg. 6) -- with only workgroup barriers between
// phases, so thousands of graphs cost one launch and no grid-wide step.
// Graphs whose vertex values fit in the workgroup's LDS keep them there (LDS
// atomics); larger ones keep them in global memory, where a graph's working
// set stays within the L2 of the XCD running it.
//
// Two ways in: a packed multi-CSR (graph g owns global vertices
// [vptr[g], vptr[g+1]) and graph-local column ids), and a list of task
// descriptors, one per graph, each with its own CSR, output and scratch.
// Both are turned into the same device task table by a small kernel.
//
// Per graph the algorithms are those of peelone.hip and histocore.hip:
// PeelOne peels level by level with the filtered fetch-and-subtract
// assertion (the decrement returning k + 1 asserts the vertex, exactly once)
// and drains each level's queue, including vertices asserted on the way,
// before the next level; HistoCore runs synchronous SumHisto / UpdateHisto
// rounds over maintained histograms (bucket b of vertex v at position
// off[v] + b - 1 of the graph's histogram array) until no cnt falls below its
// value.
#include <climits>

#include "common.hpp"

namespace pico {
namespace {

constexpr int kBatchRounds = 4;  // edges per thread per expansion step
constexpr int kSumWaveMinDefault = 64;

struct BatchState {
    Line next;  // graph claim counter
    Line levels, atomics, lds_graphs, frontier, edges, buckets, pushes, bad;
};

// One graph of a batch, as the kernel sees it.  `off` holds positions into
// `cols` (not necessarily starting at 0); `histo` is indexed by position - e0.
struct Task {
    const long long *off;
    const int32_t *cols;
    long long e0;
    int32_t *out, *core, *L0, *L1, *L2, *oldcore, *histo;
    int n;
    int pad;
};

struct BatchArgs {
    const Task *tasks;
    long long T;
    int algo;
    int lds_cap;       // vertices whose values fit in dynamic LDS
    int sum_wave_min;  // SumHisto: larger values scan with a whole wave
    BatchState *st;
};

// Scratch layout of one public task: core, L0, L1, L2 (n each), then for
// HistoCore oldcore (n) and the histogram (m), each 256-byte aligned.
__host__ __device__ inline long long task_al(long long count) { return (count + 63) & ~63ll; }

// Per-thread event counts, summed once per workgroup at exit.
struct Counts {
    long long levels = 0, atomics = 0, lds = 0, frontier = 0, edges = 0, buckets = 0, pushes = 0;
};

extern __shared__ int dyn_lds[];

// Vertex values of the current graph: in LDS or in global memory.
template <bool kLds>
struct Vals {
    int32_t *g;
    __device__ __forceinline__ int get(int i) const {
        if constexpr (kLds) return dyn_lds[i];
        else return g[i];
    }
    __device__ __forceinline__ void set(int i, int v) const {
        if constexpr (kLds) dyn_lds[i] = v;
        else g[i] = v;
    }
    __device__ __forceinline__ int fetch_sub1(int i) const {
        if constexpr (kLds) return atomicSub(&dyn_lds[i], 1);
        else return atomicSub(&g[i], 1);
    }
};

// Workgroup-uniform counters in LDS.
struct WgCounters {
    unsigned a, b, c;
    int mn;
};

// Workgroup append of one item per thread (pred) to list[*cnt ...]; one LDS
// atomic per wave.  Every lane of the wave must call it.
__device__ __forceinline__ void wg_append(bool pred, int item, int32_t *list, unsigned *cnt) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt, (unsigned)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) list[base + lane_rank(mask)] = item;
}

// ---------------------------------------------------------------- PeelOne

template <bool kLds>
__device__ void peel_graph(const Task &t, WgCounters &w, ExpandLds &X, Counts &c) {
    const int nv = t.n;
    const long long *off = t.off;
    Vals<kLds> cv{t.core};
    int32_t *out = t.out;
    int32_t *A[2] = {t.L0, t.L1};
    int32_t *Q = t.L2;

    if (threadIdx.x == 0) {
        w.a = 0;
        w.b = 0;
        w.mn = INT_MAX;
    }
    __syncthreads();
    // core = deg; isolated vertices are done (coreness 0); the rest survive
    for (int i = threadIdx.x; i - (int)threadIdx.x < nv; i += kBlock) {
        bool live = false;
        if (i < nv) {
            const int d = (int)(off[i + 1] - off[i]);
            cv.set(i, d);
            if (d == 0) out[i] = 0;
            live = d > 0;
            if (live) atomicMin(&w.mn, d);
        }
        wg_append(live, i, A[0], &w.a);
    }
    __syncthreads();
    const int peelable = (int)w.a;
    int na = peelable, k = w.mn;
    int cur = 0, qtail = 0;
    __syncthreads();
    while (qtail < peelable) {
        // level scan: survivors at value k open the level's queue, the rest
        // (value > k) survive to the next scan
        if (threadIdx.x == 0) {
            w.b = 0;
            w.c = (unsigned)qtail;
            w.mn = INT_MAX;
        }
        __syncthreads();
        const int32_t *src = A[cur];
        int32_t *dst = A[cur ^ 1];
        for (int i = threadIdx.x; i - (int)threadIdx.x < na; i += kBlock) {
            int v = -1, cval = -1;
            if (i < na) {
                v = src[i];
                cval = cv.get(v);
                if (cval > k) atomicMin(&w.mn, cval);
                if (cval == k) out[v] = k;
            }
            wg_append(cval == k, v, Q, &w.c);
            wg_append(cval > k, v, dst, &w.b);
        }
        __syncthreads();
        const int lo0 = qtail, hi0 = (int)w.c;
        na = (int)w.b;
        cur ^= 1;
        if (hi0 == lo0) {  // empty level: jump to the smallest value left
            k = w.mn;
            __syncthreads();
            if (na == 0) break;  // nothing left (unreachable for a symmetric graph)
            continue;
        }
        // drain the level's queue, including vertices asserted on the way;
        // block_expand opens with a workgroup barrier, so every wave has read
        // w.c above before any append below moves it
        int lo = lo0, hi = hi0;
        while (lo < hi) {
            for (int base = lo; base < hi; base += kBlock) {
                const int i = base + (int)threadIdx.x;
                const int v = i < hi ? Q[i] : -1;
                long long rs = 0;
                int d = 0;
                if (v >= 0) {
                    rs = off[v];
                    d = (int)(off[v + 1] - rs);
                }
                c.edges += d;
                block_expand<kBatchRounds>(
                    d, rs, 0, 0, t.cols, X,
                    [&](const bool (&act)[kBatchRounds], const int (&u)[kBatchRounds],
                        const int (&)[kBatchRounds]) {
                        int cu[kBatchRounds], old[kBatchRounds];
#pragma unroll
                        for (int r = 0; r < kBatchRounds; ++r) cu[r] = act[r] ? cv.get(u[r]) : 0;
#pragma unroll
                        for (int r = 0; r < kBatchRounds; ++r) {
                            old[r] = 0;
                            if (act[r] && cu[r] > k) {
                                old[r] = cv.fetch_sub1(u[r]);
                                ++c.atomics;
                            }
                        }
#pragma unroll
                        for (int r = 0; r < kBatchRounds; ++r) {
                            const bool push = act[r] && cu[r] > k && old[r] == k + 1;
                            if (push) {
                                out[u[r]] = k;
                                ++c.pushes;
                            }
                            wg_append(push, u[r], Q, &w.c);
                        }
                    });
            }
            __syncthreads();
            lo = hi;
            hi = (int)w.c;
            __syncthreads();
        }
        qtail = hi;
        ++c.levels;
        k += 1;
    }
    c.frontier += peelable;
    __syncthreads();
}

// ---------------------------------------------------------------- HistoCore

template <bool kLds>
__device__ void histo_graph(const Task &t, int sum_wave_min, WgCounters &w, ExpandLds &X,
                            Counts &c) {
    const int nv = t.n;
    const long long *off = t.off;
    const long long e0 = t.e0;
    Vals<kLds> cv{t.core};
    int32_t *out = t.out;
    int32_t *oldc = t.oldcore;
    int32_t *F[2] = {t.L0, t.L1};
    int32_t *histo = t.histo;  // bucket b of v at histo[off[v] - e0 + b - 1]
    const long long m = off[nv] - e0;

    if (threadIdx.x == 0) {
        w.a = 0;
        w.b = 0;
    }
    for (int i = threadIdx.x; i < nv; i += kBlock) cv.set(i, (int)(off[i + 1] - off[i]));
    for (long long e = threadIdx.x; e < m; e += kBlock) histo[e] = 0;
    __syncthreads();
    // InitHisto: bucket min(core[u], core[v]) of v counts neighbour u
    for (int base = 0; base < nv; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        long long rs = 0;
        int d = 0;
        if (i < nv) {
            rs = off[i];
            d = (int)(off[i + 1] - rs);
        }
        block_expand<kBatchRounds>(
            d, rs, d, 0, t.cols, X,
            [&](const bool (&act)[kBatchRounds], const int (&u)[kBatchRounds],
                const int (&own)[kBatchRounds]) {
#pragma unroll
                for (int r = 0; r < kBatchRounds; ++r) {
                    if (!act[r]) continue;
                    const int dv = X.p0[own[r]];
                    const int b = min(max(cv.get(u[r]), 1), dv);
                    atomicAdd(&histo[X.e0[own[r]] - e0 + b - 1], 1);
                }
            });
    }
    __syncthreads();
    // first frontier: vertices whose top bucket (cnt) is below their value
    for (int i = threadIdx.x; i - (int)threadIdx.x < nv; i += kBlock) {
        bool push = false;
        if (i < nv) {
            const int d = cv.get(i);
            push = d > 0 && histo[off[i] - e0 + d - 1] < d;
        }
        wg_append(push, i, F[0], &w.a);
    }
    __syncthreads();
    int nf = (int)w.a, cur = 0;
    __syncthreads();
    while (nf > 0) {
        ++c.levels;
        c.frontier += nf;
        const int32_t *Fc = F[cur];
        int32_t *Fn = F[cur ^ 1];
        if (threadIdx.x == 0) w.b = 0;
        // SumHisto: each frontier vertex scans its buckets downwards from its
        // old value to the first k whose running sum reaches k; new value k,
        // and bucket k keeps the running sum (the new cnt).  A wave takes the
        // long scans together.
        for (int base = 0; base < nf; base += kBlock) {
            const int i = base + (int)threadIdx.x;
            int v = -1, c_old = 0;
            long long rs = 0;
            if (i < nf) {
                v = Fc[i];
                c_old = cv.get(v);
                rs = off[v] - e0;
            }
            if (v >= 0 && c_old <= sum_wave_min) {
                int s = 0, kk = c_old;
                for (; kk >= 1; --kk) {
                    s += histo[rs + kk - 1];
                    if (s >= kk) break;
                }
                if (kk < 1) kk = 0;
                c.buckets += c_old - max(kk, 1) + 1;
                cv.set(v, kk);
                oldc[v] = c_old;
                if (kk >= 1) histo[rs + kk - 1] = s;
            }
            unsigned long long mm = __ballot(v >= 0 && c_old > sum_wave_min);
            while (mm) {
                const int l = __ffsll(mm) - 1;
                mm &= mm - 1;
                const int vv = __shfl(v, l), cc = __shfl(c_old, l);
                const long long ra = __shfl(rs, l);
                int top = cc, carry = 0, h = 0, s = 0;
                while (top >= 1) {
                    const int bb = top - lane_id();
                    const int val = bb >= 1 ? histo[ra + bb - 1] : 0;
                    const int S = carry + wave_incl_scan(val);
                    const unsigned long long mk = __ballot(bb >= 1 && S >= bb);
                    if (mk) {
                        const int l2 = __ffsll(mk) - 1;
                        h = top - l2;
                        s = __shfl(S, l2);
                        break;
                    }
                    carry = __shfl(S, kWave - 1);
                    top -= kWave;
                }
                if (lane_id() == 0) {
                    c.buckets += cc - max(h, 1) + 1;
                    cv.set(vv, h);
                    oldc[vv] = cc;
                    if (h >= 1) histo[ra + h - 1] = s;
                }
            }
        }
        __syncthreads();
        // UpdateHisto: for each changed v and neighbour u valued above v's new
        // value, move v's count in u's histogram from bucket min(old, core[u])
        // to the new value; u joins the next frontier when its top bucket
        // falls from exactly its value (once per round)
        for (int base = 0; base < nf; base += kBlock) {
            const int i = base + (int)threadIdx.x;
            int v = -1, c_new = 0, c_old = 0, d = 0;
            long long rs = 0;
            if (i < nf) {
                v = Fc[i];
                c_new = cv.get(v);
                c_old = oldc[v];
                rs = off[v];
                d = (int)(off[v + 1] - rs);
            }
            c.edges += d;
            block_expand<kBatchRounds>(
                d, rs, c_new, c_old, t.cols, X,
                [&](const bool (&act)[kBatchRounds], const int (&u)[kBatchRounds],
                    const int (&own)[kBatchRounds]) {
                    int cu[kBatchRounds];
#pragma unroll
                    for (int r = 0; r < kBatchRounds; ++r) cu[r] = act[r] ? cv.get(u[r]) : 0;
                    bool push[kBatchRounds];
#pragma unroll
                    for (int r = 0; r < kBatchRounds; ++r) {
                        push[r] = false;
                        const int cvv = X.p0[own[r]], ov = X.p1[own[r]];
                        if (act[r] && cu[r] > cvv && cvv >= 1) {
                            const long long hb = off[u[r]] - e0 - 1;
                            if (ov >= cu[r]) {
                                push[r] = atomicSub(&histo[hb + cu[r]], 1) == cu[r];
                            } else {
                                atomicSub(&histo[hb + ov], 1);
                            }
                            atomicAdd(&histo[hb + cvv], 1);
                            ++c.atomics;
                            c.pushes += push[r] ? 1 : 0;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kBatchRounds; ++r) wg_append(push[r], u[r], Fn, &w.b);
                });
        }
        __syncthreads();
        nf = (int)w.b;
        cur ^= 1;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nv; i += kBlock) out[i] = cv.get(i);
    __syncthreads();
}

// One graph, by the workgroup: LDS tier if its values fit.
__device__ __forceinline__ void decompose(const Task &t, int algo, int lds_cap, int sum_wave_min,
                                          WgCounters &w, ExpandLds &X, Counts &c) {
    if (t.n <= 0) return;
    const bool lds = t.n <= lds_cap;
    c.lds += lds ? 1 : 0;
    if (algo == PICO_ALGO_PEELONE) {
        if (lds) peel_graph<true>(t, w, X, c);
        else peel_graph<false>(t, w, X, c);
    } else {
        if (lds) histo_graph<true>(t, sum_wave_min, w, X, c);
        else histo_graph<false>(t, sum_wave_min, w, X, c);
    }
}

__global__ __launch_bounds__(kBlock) void batched_kernel(BatchArgs a) {
    __shared__ WgCounters w;
    __shared__ ExpandLds X;
    __shared__ long long claim;
    Counts c;
    while (true) {
        if (threadIdx.x == 0) claim = (long long)atomicAdd(&a.st->next.v, 1ull);
        __syncthreads();
        const long long j = claim;
        __syncthreads();
        if (j >= a.T) break;
        const Task t = a.tasks[j];
        decompose(t, a.algo, a.lds_cap, a.sum_wave_min, w, X, c);
    }
    // per-thread counts: atomics, edges, buckets, pushes; per-workgroup
    // (uniform, thread 0's): levels, frontier, lds graphs
    const long long s_atom = wave_sum64(c.atomics), s_edges = wave_sum64(c.edges);
    const long long s_buck = wave_sum64(c.buckets), s_push = wave_sum64(c.pushes);
    if (lane_id() == 0) {
        if (s_atom) atomicAdd(&a.st->atomics.v, (unsigned long long)s_atom);
        if (s_edges) atomicAdd(&a.st->edges.v, (unsigned long long)s_edges);
        if (s_buck) atomicAdd(&a.st->buckets.v, (unsigned long long)s_buck);
        if (s_push) atomicAdd(&a.st->pushes.v, (unsigned long long)s_push);
    }
    if (threadIdx.x == 0) {
        if (c.levels) atomicAdd(&a.st->levels.v, (unsigned long long)c.levels);
        if (c.frontier) atomicAdd(&a.st->frontier.v, (unsigned long long)c.frontier);
        if (c.lds) atomicAdd(&a.st->lds_graphs.v, (unsigned long long)c.lds);
    }
}

__global__ void batch_state_init(BatchState *st) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(st);
    const int words = (int)(sizeof(BatchState) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0ull;
}

struct PackedArrays {
    const long long *vptr, *off;
    const int32_t *cols, *order;
    long long G;
    int32_t *out, *core, *L0, *L1, *L2, *oldcore, *histo;
};

// Task j of a packed batch: graph order[j] (or j), its rows and columns in
// place, its scratch at its global vertex / position range.
__global__ void packed_tasks(PackedArrays p, Task *tasks, BatchState *st) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.G) return;
    const long long g = p.order ? (long long)p.order[j] : j;
    Task t;
    const long long x0 = p.vptr[g];
    long long n = p.vptr[g + 1] - x0;
    if (n < 0 || n > INT_MAX) {
        atomicAdd(&st->bad.v, 1ull);
        n = 0;
    }
    t.off = p.off + x0;
    t.cols = p.cols;
    t.e0 = p.off[x0];
    t.n = (int)n;
    t.pad = 0;
    t.out = p.out + x0;
    t.core = p.core + x0;
    t.L0 = p.L0 + x0;
    t.L1 = p.L1 + x0;
    t.L2 = p.L2 + x0;
    t.oldcore = p.oldcore ? p.oldcore + x0 : nullptr;
    t.histo = p.histo ? p.histo + t.e0 : nullptr;
    tasks[j] = t;
}


__global__ void public_tasks(const pico_task *pt, long long T, int histocore, Task *tasks) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= T) return;
    const pico_task p = pt[j];
    Task t;
    const long long n = p.n;
    t.off = reinterpret_cast<const long long *>(p.offsets);
    t.cols = p.cols;
    t.e0 = n > 0 ? t.off[0] : 0;
    t.n = (int)n;
    t.pad = 0;
    t.out = p.out_core;
    int32_t *s = static_cast<int32_t *>(p.scratch);
    const long long an = task_al(n);
    t.core = s;
    t.L0 = s + an;
    t.L1 = s + 2 * an;
    t.L2 = s + 3 * an;
    t.oldcore = histocore ? s + 4 * an : nullptr;
    t.histo = histocore ? s + 5 * an : nullptr;
    tasks[j] = t;
}

struct Launch {
    int lds_bytes, blocks_per_cu;
    long long blocks;
};

int launch_config(const void *kernel, const pico_batch_tune *tune, long long T, Launch *L) {
    int lds_bytes = tune && tune->lds_bytes >= 0 ? tune->lds_bytes : 64 * 1024;
    int dev = 0, cus = 0, max_dyn = 0;
    PICO_HIP_TRY(hipGetDevice(&dev));
    PICO_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PICO_HIP_TRY(hipDeviceGetAttribute(&max_dyn, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int static_bytes = (int)(sizeof(WgCounters) + sizeof(ExpandLds) + 64);
    if (lds_bytes > max_dyn - static_bytes) lds_bytes = max_dyn - static_bytes;
    if (lds_bytes < 0) lds_bytes = 0;
    lds_bytes &= ~3;
    if (lds_bytes > 48 * 1024)
        PICO_HIP_TRY(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes));
    int per_cu = tune && tune->blocks_per_cu > 0 ? tune->blocks_per_cu : 0;
    int occ = 0;
    PICO_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kBlock, lds_bytes));
    if (occ < 1) occ = 1;
    if (per_cu == 0 || per_cu > occ) per_cu = occ;
    long long blocks = (long long)per_cu * cus;
    if (blocks > T) blocks = T > 0 ? T : 1;
    L->lds_bytes = lds_bytes;
    L->blocks_per_cu = per_cu;
    L->blocks = blocks;
    return PICO_OK;
}

int launch_tasks(const Task *tasks, long long T, int algo, const pico_batch_tune *tune,
                 BatchState *st, pico_batch_stats *stats, hipStream_t stream) {
    Launch L;
    int rc = launch_config(reinterpret_cast<const void *>(batched_kernel), tune, T, &L);
    if (rc) return rc;
    BatchArgs a;
    a.tasks = tasks;
    a.T = T;
    a.algo = algo;
    a.lds_cap = L.lds_bytes / 4;
    a.sum_wave_min = tune && tune->sum_wave_min > 0 ? tune->sum_wave_min : kSumWaveMinDefault;
    a.st = st;
    int rec = prof_begin("batched_kernel", stream);
    hipLaunchKernelGGL(batched_kernel, dim3((unsigned)L.blocks), dim3(kBlock), L.lds_bytes, stream, a);
    prof_end(rec, stream);
    PICO_LAUNCH_CHECK();
    if (stats) {
        BatchState *h = static_cast<BatchState *>(host_scratch(sizeof(BatchState)));
        if (!h) return PICO_EHIP;
        PICO_HIP_TRY(hipMemcpyAsync(h, st, sizeof(BatchState), hipMemcpyDeviceToHost, stream));
        PICO_HIP_TRY(hipStreamSynchronize(stream));
        stats->graphs = T;
        stats->iterations = (int64_t)h->levels.v;
        stats->atomics = (int64_t)h->atomics.v;
        stats->frontier_total = (int64_t)h->frontier.v;
        stats->edges_scanned = (int64_t)h->edges.v;
        stats->buckets_scanned = (int64_t)h->buckets.v;
        stats->pushes = (int64_t)h->pushes.v;
        stats->lds_graphs = (int64_t)h->lds_graphs.v;
        stats->workgroups = L.blocks;
        stats->lds_bytes = L.lds_bytes;
        stats->blocks_per_cu = L.blocks_per_cu;
        if (h->bad.v) {
            set_error("%llu graphs of the batch have a vertex count outside [0, 2^31)",
                      (unsigned long long)h->bad.v);
            return PICO_EINVAL;
        }
    }
    return PICO_OK;
}

}  // namespace

size_t batched_ws_bytes(int64_t G, int64_t total_n, int64_t total_m, int algo) {
    size_t b = carve_bytes(total_n, 4) * 4 + carve_bytes(1, sizeof(BatchState)) +
               carve_bytes(G, sizeof(Task));
    if ((algo & PICO_ALGO_MASK) == PICO_ALGO_HISTOCORE) b += carve_bytes(total_m, 4) + carve_bytes(total_n, 4);
    return b;
}

size_t task_scratch_bytes(int64_t n, int64_t m, int algo) {
    long long words = 4 * task_al(n);
    if ((algo & PICO_ALGO_MASK) == PICO_ALGO_HISTOCORE) words += task_al(n) + task_al(m);
    return (size_t)words * 4;
}

size_t tasks_ws_bytes(int64_t T) {
    return carve_bytes(T, sizeof(Task)) + carve_bytes(T, sizeof(pico_task)) +
           carve_bytes(1, sizeof(BatchState));
}

int run_batched(const long long *vptr, const long long *off, const int32_t *cols, int64_t G,
                int64_t total_n, int64_t total_m, int algo, const int32_t *order, int32_t *out,
                void *ws, size_t ws_bytes, const pico_batch_tune *tune, pico_batch_stats *stats,
                hipStream_t stream) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    PackedArrays p;
    p.vptr = vptr;
    p.off = off;
    p.cols = cols;
    p.order = order;
    p.G = G;
    p.out = out;
    p.core = cv.take<int32_t>(total_n);
    p.L0 = cv.take<int32_t>(total_n);
    p.L1 = cv.take<int32_t>(total_n);
    p.L2 = cv.take<int32_t>(total_n);
    p.histo = nullptr;
    p.oldcore = nullptr;
    const bool hc = algo == PICO_ALGO_HISTOCORE;
    if (hc) {
        p.histo = cv.take<int32_t>(total_m);
        p.oldcore = cv.take<int32_t>(total_n);
    }
    BatchState *st = cv.take<BatchState>(1);
    Task *tasks = cv.take<Task>(G);
    if (!p.core || !p.L0 || !p.L1 || !p.L2 || !st || !tasks ||
        (hc && ((total_m > 0 && !p.histo) || !p.oldcore))) {
        set_error("batched workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  batched_ws_bytes(G, total_n, total_m, algo));
        return PICO_ENOMEM;
    }
    PICO_LAUNCH("batch_state_init", batch_state_init, dim3(1), dim3(kBlock), stream, st);
    PICO_LAUNCH("packed_tasks", packed_tasks, dim3((unsigned)((G + 255) / 256)), dim3(256), stream, p,
                tasks, st);
    return launch_tasks(tasks, G, algo, tune, st, stats, stream);
}

int run_tasks_device(const pico_task *dev_tasks, int64_t T, int algo, void *ws, size_t ws_bytes,
                     const pico_batch_tune *tune, pico_batch_stats *stats, hipStream_t stream) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    Task *tasks = cv.take<Task>(T);
    cv.take<pico_task>(T);
    BatchState *st = cv.take<BatchState>(1);
    if (!tasks || !st) {
        set_error("tasks workspace too small (%zu bytes given, %zu needed)", ws_bytes, tasks_ws_bytes(T));
        return PICO_ENOMEM;
    }
    PICO_LAUNCH("batch_state_init", batch_state_init, dim3(1), dim3(kBlock), stream, st);
    PICO_LAUNCH("public_tasks", public_tasks, dim3((unsigned)((T + 255) / 256)), dim3(256), stream,
                dev_tasks, (long long)T, algo == PICO_ALGO_HISTOCORE ? 1 : 0, tasks);
    return launch_tasks(tasks, T, algo, tune, st, stats, stream);
}

// Device copy of a host task array inside the tasks workspace (second slot).
pico_task *tasks_table(void *ws, size_t ws_bytes, int64_t T) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    cv.take<Task>(T);
    return cv.take<pico_task>(T);
}

}  // namespace pico
