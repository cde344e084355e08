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
#include <cstddef>
#include <cstdlib>
#include <mutex>

#include "common.hpp"

namespace pico {
namespace {

constexpr int kBatchRounds = 4;  // edges per thread per expansion step
constexpr int kSumWaveMinDefault = 64;
constexpr long long kSmallMaxEdgesDefault = 1ll << 14;  // one-workgroup path, single graphs

// ------------------------------------------------------------ helping
//
// A graph too large for one workgroup to finish quickly (values in global
// memory, at least help_min vertices) is decomposed by the workgroup that
// claimed it -- its leader -- with the help of workgroups that have no graph
// left to claim.  The leader runs the algorithm's outer loop; each phase of
// it is a parallel loop over an index range, cut into chunks: for PeelOne
// the initialisation, a level's scan and each round of the level's drain;
// for HistoCore clearing the histogram, core = deg, InitHisto, the first
// frontier, and per round SumHisto and then UpdateHisto (separate phases, so
// the rounds stay synchronous), and the final copy to the output.  For a phase worth
// sharing the leader publishes it in its job record and lists the record on
// an open board; any idle workgroup claims chunks with one compare-and-swap
// on the record's packed (sequence, chunk count, next chunk) word, runs them
// exactly as the leader would, and counts them done.  The leader takes
// chunks too, then waits until every chunk is done and closes the phase.
// Nobody waits for a workgroup that is not running: the leader waits only
// for chunks already claimed by running helpers, and helpers wait for
// nothing but new work (they leave once every graph of the launch is
// finished).  Every wait is bounded.  Appends and the level minimum use
// global counters in the job record.
constexpr int kMaxGrid = 2048;        // workgroups per launch (job records)
constexpr int kOpen = 64;             // board entries
constexpr int kChunkItems = 1024;     // vertices / survivors per chunk
constexpr int kChunkQueue = 256;      // queue entries per drain chunk
constexpr long long kChunkEdges = 1 << 16;  // histogram positions per clearing chunk
constexpr int kHelpMinDefault = 32768;

enum {
    PH_INIT = 0, PH_SCAN = 1, PH_DRAIN = 2,                      // PeelOne
    PH_HZERO = 3, PH_HINIT = 4, PH_HHIST = 5, PH_HFRONT = 6,     // HistoCore set-up
    PH_HSUM = 7, PH_HUPD = 8, PH_HOUT = 9                        // HistoCore rounds, output
};

// Items per chunk of each phase (leader and helpers cut phases alike).
__host__ __device__ inline long long chunk_of(int phase) {
    return phase == PH_DRAIN || phase == PH_HUPD ? kChunkQueue : phase == PH_HZERO ? kChunkEdges : kChunkItems;
}

struct alignas(128) JobCtl {
    unsigned long long ctl;   // seq (16) | chunks (24) | next chunk (24); odd seq = open
    unsigned long long done;  // chunks completed in the open phase
};
struct alignas(128) JobParams {
    long long task, lo, hi;
    int phase, k, cur, pad;
};
struct alignas(128) JobCnt {
    unsigned a, b, c;
    int mn;
};
struct Job {
    JobCtl x;
    JobParams p;
    JobCnt n;
};

__host__ __device__ constexpr unsigned long long job_word(unsigned long long seq, unsigned long long nch,
                                                          unsigned long long next) {
    return (seq << 48) | (nch << 24) | next;
}

struct BatchState {
    Line next;  // graph claim counter
    Line levels, atomics, lds_graphs, frontier, edges, buckets, pushes, bad;
    Line finished;  // graphs done (helpers leave when it reaches the graph count)
    Line helped;    // graphs decomposed with the board open to helpers
    Line helpchunks;
    Line stuck;     // phases whose helpers did not finish within the wait bound
    Line chose_hc;  // PICO_ALGO_AUTO: graphs the choice gave to HistoCore
    unsigned long long open[kOpen];  // board: job index + 1, or 0
    Job jobs[kMaxGrid];
};

// One graph of a batch, as the kernel sees it.  `off` holds positions into
// `cols` (not necessarily starting at 0); `histo` is indexed by position - e0.
// Batches use 64-bit offsets; a single small graph may come with 32-bit ones.
template <typename Off>
struct TaskT {
    const Off *off;
    const int32_t *cols;
    long long e0;
    int32_t *out, *core, *L0, *L1, *L2, *oldcore, *histo;
    int n;
    int slot;  // index of the graph's status word, or -1 (no status: a hole or a single graph)
};
using Task = TaskT<long long>;

struct BatchArgs {
    const Task *tasks;
    long long T;
    int lds_cap;       // vertices whose values fit in dynamic LDS
    int sum_wave_min;  // SumHisto: larger values scan with a whole wave
    int help_min;      // graphs of at least this many vertices (global tier) take helpers; 0 = never
    unsigned long long limit;  // bound on every wait (wall-clock ticks)
    BatchState *st;
    int32_t *status;  // per graph: PICO_EHIP until it is finished, then PICO_OK (PICO_EINVAL stays)
};

// Scratch layout of one public task: core, L0, L1, L2 (n each), then for
// HistoCore oldcore (n) and the histogram (m), each 256-byte aligned.
__host__ __device__ inline long long task_al(long long count) { return (count + 63) & ~63ll; }

// Per-thread event counts, summed once per workgroup at exit.
struct Counts {
    long long levels = 0, atomics = 0, lds = 0, frontier = 0, edges = 0, buckets = 0, pushes = 0;
    long long scans = 0, drains = 0, kmax = 0;  // PeelOne schedule (uniform in the workgroup)
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

template <bool kLds, typename Off>
__device__ void peel_graph(const TaskT<Off> &t, WgCounters &w, ExpandLds &X, Counts &c) {
    const int nv = t.n;
    const Off *off = t.off;
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
        ++c.scans;
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
            ++c.drains;
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
        c.kmax = k;
        k += 1;
    }
    c.frontier += peelable;
    __syncthreads();
}

// ---------------------------------------------------------------- HistoCore

// warm: upper bounds of the coreness to start from, plus warm_add (nullptr:
// start from the degrees).
template <bool kLds, typename Off>
__device__ void histo_graph(const TaskT<Off> &t, int sum_wave_min, WgCounters &w, ExpandLds &X,
                            Counts &c, const int32_t *warm = nullptr, int warm_add = 0) {
    const int nv = t.n;
    const Off *off = t.off;
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
    for (int i = threadIdx.x; i < nv; i += kBlock) {
        const int d = (int)(off[i + 1] - off[i]);
        int v0 = d;
        if (warm && d > 0) {
            const long long b = (long long)warm[i] + warm_add;
            v0 = (int)(b < 1 ? 1 : (b > d ? d : b));
        }
        cv.set(i, v0);
    }
    for (long long e = threadIdx.x; e < m; e += kBlock) histo[e] = 0;
    __syncthreads();
    // InitHisto: bucket min(core[u], core[v]) of v counts neighbour u
    for (int base = 0; base < nv; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        long long rs = 0;
        int d = 0, nb = 0;  // neighbours, buckets (the starting value)
        if (i < nv) {
            rs = off[i];
            d = (int)(off[i + 1] - rs);
            nb = cv.get(i);
        }
        block_expand<kBatchRounds>(
            d, rs, nb, 0, t.cols, X,
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
                int h, s;
                wave_reverse_sum_wide(histo + ra, cc, h, s);
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

// ------------------------------------------------ PeelOne with helpers

// Wave-aggregated append to a list with a global counter.  Every lane of the
// wave must call it.
__device__ __forceinline__ void g_append(bool pred, int item, int32_t *list, unsigned *cnt) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt, (unsigned)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) list[base + lane_rank(mask)] = item;
}

__device__ __forceinline__ void g_min(bool pred, int x, int *mn) {
    const int m = wave_min(pred ? x : INT_MAX);
    if (lane_id() == 0 && m != INT_MAX) atomicMin(mn, m);
}

// One chunk [c0, c1) of a HistoCore phase of graph t (values in t.core, the
// frontier lists in t.L0 / t.L1 by round parity), run by the whole
// workgroup; the same steps as histo_graph, with global counters.
__device__ void run_chunk_histo(const Task &t, const JobParams &p, JobCnt *n, long long c0, long long c1,
                                ExpandLds &X, Counts &c) {
    const long long *off = t.off;
    const long long e0 = t.e0;
    int32_t *core = t.core;
    int32_t *histo = t.histo;
    if (p.phase == PH_HZERO) {  // histogram positions [c0, c1)
        for (long long e = c0 + threadIdx.x; e < c1; e += kBlock) histo[e] = 0;
    } else if (p.phase == PH_HINIT) {
        for (long long i = c0 + threadIdx.x; i < c1; i += kBlock) core[i] = (int)(off[i + 1] - off[i]);
    } else if (p.phase == PH_HHIST) {  // InitHisto of vertices [c0, c1)
        for (long long base = c0; base < c1; base += kBlock) {
            const long long i = base + threadIdx.x;
            long long rs = 0;
            int d = 0;
            if (i < c1) {
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
                        const int b = min(max(core[u[r]], 1), dv);
                        atomicAdd(&histo[X.e0[own[r]] - e0 + b - 1], 1);
                    }
                });
        }
    } else if (p.phase == PH_HFRONT) {  // the first frontier: top bucket below the value
        for (long long i = c0 + threadIdx.x; i - (long long)threadIdx.x < c1; i += kBlock) {
            bool push = false;
            if (i < c1) {
                const int d = core[i];
                push = d > 0 && histo[off[i] - e0 + d - 1] < d;
            }
            g_append(push, (int)i, t.L0, &n->a);
        }
    } else if (p.phase == PH_HSUM) {  // SumHisto of frontier entries [c0, c1); p.k: wave threshold
        const int32_t *Fc = p.cur ? t.L1 : t.L0;
        const int sum_wave_min = p.k;
        for (long long base = c0; base < c1; base += kBlock) {
            const long long i = base + threadIdx.x;
            int v = -1, c_old = 0;
            long long rs = 0;
            if (i < c1) {
                v = Fc[i];
                c_old = core[v];
                rs = off[v] - e0;
            }
            if (v >= 0 && c_old <= sum_wave_min) {
                int sum = 0, kk = c_old;
                for (; kk >= 1; --kk) {
                    sum += histo[rs + kk - 1];
                    if (sum >= kk) break;
                }
                if (kk < 1) kk = 0;
                c.buckets += c_old - max(kk, 1) + 1;
                core[v] = kk;
                t.oldcore[v] = c_old;
                if (kk >= 1) histo[rs + kk - 1] = sum;
            }
            unsigned long long mm = __ballot(v >= 0 && c_old > sum_wave_min);
            while (mm) {
                const int l = __ffsll(mm) - 1;
                mm &= mm - 1;
                const int vv = __shfl(v, l), cc = __shfl(c_old, l);
                const long long ra = __shfl(rs, l);
                int h, sum;
                wave_reverse_sum_wide(histo + ra, cc, h, sum);
                if (lane_id() == 0) {
                    c.buckets += cc - max(h, 1) + 1;
                    core[vv] = h;
                    t.oldcore[vv] = cc;
                    if (h >= 1) histo[ra + h - 1] = sum;
                }
            }
        }
    } else if (p.phase == PH_HUPD) {  // UpdateHisto of frontier entries [c0, c1)
        const int32_t *Fc = p.cur ? t.L1 : t.L0;
        int32_t *Fn = p.cur ? t.L0 : t.L1;
        for (long long base = c0; base < c1; base += kBlock) {
            const long long i = base + threadIdx.x;
            int v = -1, c_new = 0, c_old = 0, d = 0;
            long long rs = 0;
            if (i < c1) {
                v = Fc[i];
                c_new = core[v];
                c_old = t.oldcore[v];
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
                    for (int r = 0; r < kBatchRounds; ++r) cu[r] = act[r] ? core[u[r]] : 0;
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
                    for (int r = 0; r < kBatchRounds; ++r) g_append(push[r], u[r], Fn, &n->b);
                });
        }
    } else {  // PH_HOUT
        for (long long i = c0 + threadIdx.x; i < c1; i += kBlock) t.out[i] = core[i];
    }
}

// One chunk [c0, c1) of a phase of graph t, run by the whole workgroup.
// kAlgo: the launch's algorithm (each its own kernel, so neither carries the
// other's registers).
template <int kAlgo>
__device__ void run_chunk(const Task &t, const JobParams &p, JobCnt *n, long long c0, long long c1,
                          ExpandLds &X, Counts &c) {
    if constexpr (kAlgo == PICO_ALGO_HISTOCORE) {
        run_chunk_histo(t, p, n, c0, c1, X, c);
        return;
    }
    const long long *off = t.off;
    int32_t *core = t.core;
    const int k = p.k;
    if (p.phase == PH_INIT) {
        for (long long i = c0 + threadIdx.x; i - (long long)threadIdx.x < c1; i += kBlock) {
            int d = 0;
            const bool in = i < c1;
            if (in) {
                d = (int)(off[i + 1] - off[i]);
                core[i] = d;
                if (d == 0) t.out[i] = 0;
            }
            g_append(in && d > 0, (int)i, t.L0, &n->a);
            g_min(in && d > 0, d, &n->mn);
        }
    } else if (p.phase == PH_SCAN) {
        const int32_t *src = p.cur ? t.L1 : t.L0;
        int32_t *dst = p.cur ? t.L0 : t.L1;
        for (long long i = c0 + threadIdx.x; i - (long long)threadIdx.x < c1; i += kBlock) {
            int v = -1, cv = -1;
            if (i < c1) {
                v = src[i];
                cv = core[v];
                if (cv == k) t.out[v] = k;
            }
            g_append(cv == k, v, t.L2, &n->c);
            g_append(cv > k, v, dst, &n->b);
            g_min(cv > k, cv, &n->mn);
        }
    } else {  // PH_DRAIN: expand queue entries [c0, c1)
        for (long long base = c0; base < c1; base += kBlock) {
            const long long i = base + threadIdx.x;
            const int v = i < c1 ? t.L2[i] : -1;
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
                    for (int r = 0; r < kBatchRounds; ++r) cu[r] = act[r] ? core[u[r]] : 0;
#pragma unroll
                    for (int r = 0; r < kBatchRounds; ++r) {
                        old[r] = 0;
                        if (act[r] && cu[r] > k) {
                            old[r] = atomicSub(&core[u[r]], 1);
                            ++c.atomics;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kBatchRounds; ++r) {
                        const bool push = act[r] && cu[r] > k && old[r] == k + 1;
                        if (push) {
                            t.out[u[r]] = k;
                            ++c.pushes;
                        }
                        g_append(push, u[r], t.L2, &n->c);
                    }
                });
        }
    }
}

struct LeadLds {
    long long chunk;  // claimed chunk index, or -1
    unsigned a, b, c;
    int mn;
    int err;
};

// Claim the next chunk of an open job whose control word reads x (thread 0).
__device__ __forceinline__ long long claim_chunk(Job *job, unsigned long long x) {
    while (true) {
        const unsigned long long seq = x >> 48, nch = (x >> 24) & 0xffffffull, nx = x & 0xffffffull;
        if ((seq & 1ull) == 0 || nx >= nch) return -1;
        const unsigned long long y = atomicCAS(&job->x.ctl, x, x + 1);
        if (y == x) return (long long)nx;
        x = y;
    }
}

// The leader runs phase p over `items` items in chunks of `chunk`, opening
// it to helpers when there is more than one chunk and the board took the
// job.  On return every chunk is done and the job's counters are in `sh`.
template <int kAlgo>
__device__ void run_phase(const BatchArgs &a, const Task &t, Job *job, bool shared, JobParams p,
                          long long items, long long chunk, LeadLds &sh, ExpandLds &X, Counts &c) {
    const long long nch = (items + chunk - 1) / chunk;
    const bool open = shared && nch > 1;
    if (threadIdx.x == 0) {
        st_rlx(&job->p.task, p.task);
        st_rlx(&job->p.lo, p.lo);
        st_rlx(&job->p.hi, p.hi);
        st_rlx(&job->p.phase, p.phase);
        st_rlx(&job->p.k, p.k);
        st_rlx(&job->p.cur, p.cur);
        if (open) {
            st_rlx(&job->x.done, 0ull);
            // 16-bit sequence; 2^16 is even, so the parity survives the wrap
            const unsigned long long seq = ((ld_rlx(&job->x.ctl) >> 48) + 1) & 0xffffull;  // odd: open
            // parameters and counters before the control word
            st_rel(&job->x.ctl, job_word(seq, (unsigned long long)nch, 0));
        }
        // The counters this thread reset between phases must be in place
        // before any wave of the workgroup adds to them: the barrier below
        // does not wait for the stores.
        wave_mem_drain();
    }
    __syncthreads();
    long long own = 0;
    for (long long q = 0;; ++q) {
        if (threadIdx.x == 0) sh.chunk = open ? claim_chunk(job, ld_rlx(&job->x.ctl)) : (q < nch ? q : -1);
        __syncthreads();
        const long long ci = sh.chunk;
        __syncthreads();
        if (ci < 0) break;
        const long long c0 = p.lo + ci * chunk, c1 = c0 + chunk < p.hi ? c0 + chunk : p.hi;
        run_chunk<kAlgo>(t, p, &job->n, c0, c1, X, c);
        ++own;
    }
    // every wave's stores and atomics performed before the count below (the
    // workgroup barrier does not wait for other waves' vector-memory traffic)
    wave_mem_drain();
    __syncthreads();
    if (threadIdx.x == 0) {
        if (open) {
            // (no release here: only this thread reads the count, and the next
            // phase's control word publishes what this workgroup wrote)
            unsigned long long d = atomicAdd(&job->x.done, (unsigned long long)own) + own;
            const unsigned long long t0 = wall_clock64();
            while (d < (unsigned long long)nch) {  // chunks still being run by helpers
                if (wall_clock64() - t0 > a.limit) {
                    sh.err = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                d = ld_acq(&job->x.done);
            }
            const unsigned long long seq = ((ld_rlx(&job->x.ctl) >> 48) + 1) & 0xffffull;  // even: closed
            st_rlx(&job->x.ctl, job_word(seq, 0, 0));  // publishes nothing
            fence_acquire();
        }
        sh.a = ld_rlx(&job->n.a);
        sh.b = ld_rlx(&job->n.b);
        sh.c = ld_rlx(&job->n.c);
        sh.mn = ld_rlx(&job->n.mn);
    }
    __syncthreads();
}

// The leader lists its job on the board (no helpers if the board is full)
// and clears the job's counters.  Returns the board slot, or -1.
__device__ int board_enter(const BatchArgs &a, Job *job, LeadLds &sh) {
    if (threadIdx.x == 0) {
        sh.err = 0;
        sh.chunk = -1;
        for (int q = 0; q < kOpen; ++q) {
            const int s = (int)((blockIdx.x + q) % kOpen);
            if (atomicCAS(&a.st->open[s], 0ull, (unsigned long long)blockIdx.x + 1) == 0ull) {
                sh.chunk = s;
                break;
            }
        }
        st_rlx(&job->n.a, 0u);
        st_rlx(&job->n.b, 0u);
        st_rlx(&job->n.c, 0u);
        st_rlx(&job->n.mn, INT_MAX);
    }
    __syncthreads();
    const int slot = (int)sh.chunk;
    __syncthreads();
    return slot;
}

// The leader takes its job off the board and records how the graph went.
__device__ void board_leave(const BatchArgs &a, int slot, const LeadLds &sh) {
    if (threadIdx.x == 0) {
        if (slot >= 0) st_rlx(&a.st->open[slot], 0ull);
        if (sh.err) atomicAdd(&a.st->stuck.v, 1ull);
        atomicAdd(&a.st->helped.v, slot >= 0 ? 1ull : 0ull);
    }
    __syncthreads();
}

// PeelOne of a global-tier graph by its leader, phases shared with helpers.
__device__ void peel_graph_helped(const BatchArgs &a, const Task &t, long long task, LeadLds &sh,
                                  ExpandLds &X, Counts &c) {
    Job *job = &a.st->jobs[blockIdx.x];
    const int slot = board_enter(a, job, sh);
    const bool shared = slot >= 0;
    JobParams p;
    p.task = task;
    p.pad = 0;
    p.phase = PH_INIT;
    p.k = 0;
    p.cur = 0;
    p.lo = 0;
    p.hi = t.n;
    run_phase<PICO_ALGO_PEELONE>(a, t, job, shared, p, t.n, kChunkItems, sh, X, c);
    const int peelable = (int)sh.a;
    int k = sh.mn, cur = 0, qtail = 0, na = peelable;
    while (qtail < peelable && !sh.err) {
        if (threadIdx.x == 0) {
            st_rlx(&job->n.b, 0u);
            st_rlx(&job->n.c, (unsigned)qtail);
            st_rlx(&job->n.mn, INT_MAX);
        }
        p.phase = PH_SCAN;
        p.k = k;
        p.cur = cur;
        p.lo = 0;
        p.hi = na;
        run_phase<PICO_ALGO_PEELONE>(a, t, job, shared, p, na, kChunkItems, sh, X, c);
        const int hi0 = (int)sh.c;
        na = (int)sh.b;
        cur ^= 1;
        if (hi0 == qtail) {  // empty level: jump to the smallest value left
            k = sh.mn;
            if (na == 0) break;
            continue;
        }
        int lo = qtail, hi = hi0;
        while (lo < hi && !sh.err) {
            p.phase = PH_DRAIN;
            p.lo = lo;
            p.hi = hi;
            run_phase<PICO_ALGO_PEELONE>(a, t, job, shared, p, hi - lo, kChunkQueue, sh, X, c);
            lo = hi;
            hi = (int)sh.c;
        }
        qtail = hi;
        ++c.levels;
        k += 1;
    }
    c.frontier += peelable;
    board_leave(a, slot, sh);
}

// HistoCore of a global-tier graph by its leader, phases shared with helpers
// (the steps of histo_graph; the rounds stay synchronous because SumHisto
// and UpdateHisto are separate phases).
__device__ void histo_graph_helped(const BatchArgs &a, const Task &t, long long task, LeadLds &sh,
                                   ExpandLds &X, Counts &c) {
    Job *job = &a.st->jobs[blockIdx.x];
    const int slot = board_enter(a, job, sh);
    const bool shared = slot >= 0;
    const long long m = t.off[t.n] - t.e0;
    JobParams p;
    p.task = task;
    p.pad = 0;
    p.k = a.sum_wave_min;
    p.cur = 0;
    p.lo = 0;
    const int setup[4] = {PH_HZERO, PH_HINIT, PH_HHIST, PH_HFRONT};
    for (int ph : setup) {
        p.phase = ph;
        p.hi = ph == PH_HZERO ? m : t.n;
        run_phase<PICO_ALGO_HISTOCORE>(a, t, job, shared, p, p.hi, chunk_of(ph), sh, X, c);
        if (sh.err) break;
    }
    long long nf = sh.a;
    int cur = 0;
    while (nf > 0 && !sh.err) {
        ++c.levels;
        c.frontier += nf;
        p.cur = cur;
        p.hi = nf;
        p.phase = PH_HSUM;
        run_phase<PICO_ALGO_HISTOCORE>(a, t, job, shared, p, nf, chunk_of(PH_HSUM), sh, X, c);
        if (threadIdx.x == 0) st_rlx(&job->n.b, 0u);
        p.phase = PH_HUPD;
        run_phase<PICO_ALGO_HISTOCORE>(a, t, job, shared, p, nf, chunk_of(PH_HUPD), sh, X, c);
        nf = sh.b;
        cur ^= 1;
    }
    p.phase = PH_HOUT;
    p.hi = t.n;
    if (!sh.err) run_phase<PICO_ALGO_HISTOCORE>(a, t, job, shared, p, t.n, chunk_of(PH_HOUT), sh, X, c);
    board_leave(a, slot, sh);
}

// A workgroup with no graph left helps open jobs until every graph of the
// launch is finished.
template <int kAlgo>
__device__ void help(const BatchArgs &a, LeadLds &sh, ExpandLds &X, Counts &c) {
    __shared__ long long job_ix;
    const unsigned long long t0 = wall_clock64();
    unsigned nap = 1;
    while (true) {
        if (threadIdx.x == 0) {
            sh.chunk = -1;
            job_ix = -1;
            for (int q = 0; q < kOpen && sh.chunk < 0; ++q) {
                const unsigned long long w = ld_rlx(&a.st->open[(blockIdx.x + q) % kOpen]);
                if (w == 0ull) continue;
                Job *job = &a.st->jobs[w - 1];
                const long long ci = claim_chunk(job, ld_rlx(&job->x.ctl));
                if (ci >= 0) {
                    sh.chunk = ci;
                    job_ix = (long long)(w - 1);
                }
            }
            if (sh.chunk >= 0) {
                fence_acquire();  // the phase's parameters and what earlier phases wrote
                nap = 1;
            } else if ((long long)ld_acq(&a.st->finished.v) >= a.T || wall_clock64() - t0 > a.limit) {
                job_ix = -2;  // every graph is done: leave
            } else {
                for (unsigned q = 0; q < nap; ++q) __builtin_amdgcn_s_sleep(8);
                nap = nap < 32 ? nap * 2 : 32;
            }
        }
        __syncthreads();
        const long long jx = job_ix, ci = sh.chunk;
        __syncthreads();
        if (jx == -2) break;
        if (ci < 0) continue;
        Job *job = &a.st->jobs[jx];
        // The record is rewritten every phase: read it with atomic loads, never
        // from a line this XCD's L2 may still hold from an earlier phase.
        JobParams p;
        p.task = ld_rlx(&job->p.task);
        p.lo = ld_rlx(&job->p.lo);
        p.hi = ld_rlx(&job->p.hi);
        p.phase = ld_rlx(&job->p.phase);
        p.k = ld_rlx(&job->p.k);
        p.cur = ld_rlx(&job->p.cur);
        p.pad = 0;
        const Task t = a.tasks[p.task];
        const long long chunk = chunk_of(p.phase);
        const long long c0 = p.lo + ci * chunk, c1 = c0 + chunk < p.hi ? c0 + chunk : p.hi;
        run_chunk<kAlgo>(t, p, &job->n, c0, c1, X, c);
        // every wave's stores and atomics performed before the chunk is counted
        // (the workgroup barrier does not wait for vector-memory traffic)
        wave_mem_drain();
        __syncthreads();
        if (threadIdx.x == 0) {
            fence_release();
            atomicAdd(&job->x.done, 1ull);
            atomicAdd(&a.st->helpchunks.v, 1ull);
        }
    }
}

// One graph, by the workgroup: LDS tier if its values fit.
template <int kAlgo, typename Off>
__device__ __forceinline__ void decompose(const TaskT<Off> &t, int lds_cap, int sum_wave_min,
                                          WgCounters &w, ExpandLds &X, Counts &c) {
    if (t.n <= 0) return;
    const bool lds = t.n <= lds_cap;
    c.lds += lds ? 1 : 0;
    if constexpr (kAlgo == PICO_ALGO_PEELONE) {
        if (lds) peel_graph<true>(t, w, X, c);
        else peel_graph<false>(t, w, X, c);
    } else {
        if (lds) histo_graph<true>(t, sum_wave_min, w, X, c);
        else histo_graph<false>(t, sum_wave_min, w, X, c);
    }
}

// kAlgo: PICO_ALGO_PEELONE or PICO_ALGO_HISTOCORE, one kernel each.
template <int kAlgo>
__global__ __launch_bounds__(kBlock) void batched_kernel(BatchArgs a) {
    __shared__ WgCounters w;
    __shared__ ExpandLds X;
    __shared__ LeadLds sh;
    __shared__ long long claim;
    Counts c;
    bool stop = false;
    while (true) {
        if (threadIdx.x == 0) claim = (long long)atomicAdd(&a.st->next.v, 1ull);
        __syncthreads();
        const long long j = claim;
        __syncthreads();
        if (j >= a.T) break;
        const Task t = a.tasks[j];
        const bool helped = a.help_min > 0 && t.n > a.lds_cap && t.n >= a.help_min;
        if (helped) {
            if constexpr (kAlgo == PICO_ALGO_PEELONE) peel_graph_helped(a, t, j, sh, X, c);
            else histo_graph_helped(a, t, j, sh, X, c);
        } else {
            decompose<kAlgo>(t, a.lds_cap, a.sum_wave_min, w, X, c);
        }
        __syncthreads();
        // A leader that gave up waiting for a helper left its graph unfinished
        // (status stays PICO_EHIP).  It takes no further graph and does not
        // help: helpers still inside a chunk of its last phase may yet add to
        // its job record's counters, which no later phase may then use.
        const bool stuck = helped && sh.err;
        if (threadIdx.x == 0) {
            atomicAdd(&a.st->finished.v, 1ull);
            if (!stuck && t.slot >= 0) atomicCAS(&a.status[t.slot], (int)PICO_EHIP, (int)PICO_OK);
        }
        if (stuck) {
            stop = true;
            break;
        }
    }
    if (a.help_min > 0 && !stop) help<kAlgo>(a, sh, X, c);
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

// ------------------------------------------------ one small graph
//
// A graph whose vertex values fit in one workgroup's LDS is decomposed by a
// single workgroup: the same per-graph code as a batch, launched alone, with
// workgroup barriers where the grid-wide kernels need grid barriers (a few
// microseconds each on a full device, which decide small graphs).

enum { SM_LEVELS = 0, SM_SCANS, SM_DRAINS, SM_KMAX, SM_FRONTIER, SM_ATOMICS, SM_EDGES, SM_BUCKETS,
       SM_PUSHES, SM_WORDS };

// The workgroup's counts into stats[SM_*] (plain stores by thread 0).
__device__ void small_stats(const Counts &c, unsigned long long *stats) {
    __shared__ long long part[kBlock / kWave][4];
    const long long s_atom = wave_sum64(c.atomics), s_edges = wave_sum64(c.edges);
    const long long s_buck = wave_sum64(c.buckets), s_push = wave_sum64(c.pushes);
    if (lane_id() == 0) {
        const int wv = (int)threadIdx.x / kWave;
        part[wv][0] = s_atom;
        part[wv][1] = s_edges;
        part[wv][2] = s_buck;
        part[wv][3] = s_push;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t[4] = {0, 0, 0, 0};
        for (int wv = 0; wv < kBlock / kWave; ++wv)
            for (int j = 0; j < 4; ++j) t[j] += part[wv][j];
        stats[SM_LEVELS] = (unsigned long long)c.levels;
        stats[SM_SCANS] = (unsigned long long)c.scans;
        stats[SM_DRAINS] = (unsigned long long)c.drains;
        stats[SM_KMAX] = (unsigned long long)c.kmax;
        stats[SM_FRONTIER] = (unsigned long long)c.frontier;
        stats[SM_ATOMICS] = (unsigned long long)t[0];
        stats[SM_EDGES] = (unsigned long long)t[1];
        stats[SM_BUCKETS] = (unsigned long long)t[2];
        stats[SM_PUSHES] = (unsigned long long)t[3];
    }
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void po_small(TaskT<Off> t, unsigned long long *stats) {
    __shared__ WgCounters w;
    __shared__ ExpandLds X;
    Counts c;
    peel_graph<true>(t, w, X, c);
    small_stats(c, stats);
}

template <typename Off>
__global__ __launch_bounds__(kBlock) void hc_small(TaskT<Off> t, int sum_wave_min, const int32_t *warm,
                                                    int warm_add, unsigned long long *stats) {
    __shared__ WgCounters w;
    __shared__ ExpandLds X;
    Counts c;
    histo_graph<true>(t, sum_wave_min, w, X, c, warm, warm_add);
    small_stats(c, stats);
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
__global__ void packed_tasks(PackedArrays p, Task *tasks, BatchState *st, int32_t *status) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.G) return;
    const long long g = p.order ? (long long)p.order[j] : j;
    Task t;
    const long long x0 = p.vptr[g];
    long long n = p.vptr[g + 1] - x0;
    int32_t s0 = PICO_EHIP;  // not finished (yet)
    if (n < 0 || n > INT_MAX) {
        atomicAdd(&st->bad.v, 1ull);
        n = 0;
        s0 = PICO_EINVAL;
    }
    status[g] = s0;
    t.off = p.off + x0;
    t.cols = p.cols;
    t.e0 = p.off[x0];
    t.n = (int)n;
    t.slot = (int)g;
    t.out = p.out + x0;
    t.core = p.core + x0;
    t.L0 = p.L0 + x0;
    t.L1 = p.L1 + x0;
    t.L2 = p.L2 + x0;
    t.oldcore = p.oldcore ? p.oldcore + x0 : nullptr;
    t.histo = p.histo ? p.histo + t.e0 : nullptr;
    tasks[j] = t;
}


__global__ void public_tasks(const pico_task *pt, long long T, int histocore, Task *tasks, int32_t *status) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= T) return;
    status[j] = PICO_EHIP;  // not finished (yet)
    const pico_task p = pt[j];
    Task t;
    const long long n = p.n;
    t.off = reinterpret_cast<const long long *>(p.offsets);
    t.cols = p.cols;
    t.e0 = n > 0 ? t.off[0] : 0;
    t.n = (int)n;
    t.slot = (int)j;
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

// PICO_ALGO_AUTO over a task table: per graph, PeelOne or HistoCore.  With
// one workgroup per graph PeelOne's levels cost only workgroup barriers, and
// it was the faster algorithm on all but a few hundred-vertex graphs of the
// 4,096-graph mixed batch (by tens of microseconds); HistoCore wins where its
// first frontier is (nearly) empty -- the degrees are then (nearly) the
// coreness and InitHisto all but finishes, while PeelOne still walks every
// level (regular components, unions of cliques; Table VII's cases where l2
// is far below l1).  One workgroup per graph samples up to kChooseSamples
// evenly spaced vertices of degree 1..kChooseMaxDeg, a wave each, and counts
// those with cnt(v) < deg(v) (Theorem 2 with core = deg); fewer than 1/64 in
// the frontier gives HistoCore.
constexpr int kChooseSamples = 64;
constexpr int kChooseMaxDeg = 1024;

__global__ __launch_bounds__(kBlock) void choose_tasks(const Task *tasks, long long T, int32_t *choice,
                                                       BatchState *st) {
    __shared__ unsigned cnt[2];
    for (long long j = blockIdx.x; j < T; j += gridDim.x) {
        const Task t = tasks[j];
        if (threadIdx.x == 0) cnt[0] = cnt[1] = 0u;
        __syncthreads();
        const int S = t.n < kChooseSamples ? t.n : kChooseSamples;
        for (int q = (int)(threadIdx.x >> 6); q < S; q += kWavesPerBlock) {
            const long long v = (long long)q * t.n / S;
            const long long e0 = t.off[v], d = t.off[v + 1] - e0;
            if (d == 0 || d > kChooseMaxDeg) continue;  // uniform across the wave
            long long ge = 0;
            for (long long e = lane_id(); e < d; e += kWave) {
                const int u = t.cols[e0 + e];
                ge += (t.off[u + 1] - t.off[u]) >= d ? 1 : 0;
            }
            ge = wave_sum64(ge);
            if (lane_id() == 0) {
                atomicAdd(&cnt[0], 1u);
                if (ge < d) atomicAdd(&cnt[1], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const bool hc = cnt[0] > 0u && cnt[1] * 64u < cnt[0];
            choice[j] = hc ? PICO_ALGO_HISTOCORE : PICO_ALGO_PEELONE;
            if (hc) atomicAdd(&st->chose_hc.v, 1ull);
        }
        __syncthreads();
    }
}

// The two per-algorithm tables of an AUTO launch: each keeps the caller's
// order, with the other algorithm's graphs as empty holes (no status word).
__global__ void split_tasks(const Task *all, long long T, const int32_t *choice, Task *po, Task *hc) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= T) return;
    const Task t = all[j];
    Task hole = t;
    hole.n = 0;
    hole.slot = -1;
    const bool h = choice[j] == PICO_ALGO_HISTOCORE;
    po[j] = h ? hole : t;
    hc[j] = h ? t : hole;
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

int help_min_of(const pico_batch_tune *tune) {
    if (!tune || tune->help_min_vertices == 0) return kHelpMinDefault;
    return tune->help_min_vertices < 0 ? 0 : tune->help_min_vertices;
}

constexpr long long kHelpersPerBig = 32;  // extra workgroups per large task in a task-list launch

// want: workgroups wanted (the task count, plus helpers for large tasks);
// the grid is the smaller of that and what the device holds.
// chose_hc (optional): with stats, receives the AUTO choice count the state
// holds.
int launch_tasks(const Task *tasks, long long T, int algo, const pico_batch_tune *tune,
                 BatchState *st, int32_t *status, pico_batch_stats *stats, hipStream_t stream,
                 long long want, long long *chose_hc = nullptr) {
    Launch L;
    const int help_min = help_min_of(tune);
    const bool hc = algo == PICO_ALGO_HISTOCORE;
    const void *kernel = hc ? reinterpret_cast<const void *>(batched_kernel<PICO_ALGO_HISTOCORE>)
                            : reinterpret_cast<const void *>(batched_kernel<PICO_ALGO_PEELONE>);
    int rc = launch_config(kernel, tune, want, &L);
    if (rc) return rc;
    if (L.blocks > kMaxGrid) L.blocks = kMaxGrid;
    BatchArgs a;
    a.tasks = tasks;
    a.T = T;
    a.lds_cap = L.lds_bytes / 4;
    a.sum_wave_min = tune && tune->sum_wave_min > 0 ? tune->sum_wave_min : kSumWaveMinDefault;
    a.help_min = help_min;
    // every wait gives up after a minute (PICO_BATCH_WAIT_US: a shorter bound,
    // for tests of the give-up path)
    const int wait_us = tune_int("PICO_BATCH_WAIT_US", 0);
    a.limit = wait_us > 0 ? wall_ticks(wait_us * 1e-6) : wall_ticks(60.0);
    a.st = st;
    a.status = status;
    int rec = prof_begin("batched_kernel", stream);
    if (hc)
        hipLaunchKernelGGL(batched_kernel<PICO_ALGO_HISTOCORE>, dim3((unsigned)L.blocks), dim3(kBlock),
                           L.lds_bytes, stream, a);
    else
        hipLaunchKernelGGL(batched_kernel<PICO_ALGO_PEELONE>, dim3((unsigned)L.blocks), dim3(kBlock),
                           L.lds_bytes, stream, a);
    prof_end(rec, stream);
    PICO_LAUNCH_CHECK();
    if (stats) {
        BatchState *h = static_cast<BatchState *>(host_scratch(sizeof(BatchState)));
        if (!h) return PICO_EHIP;
        // the counters only, not the job board
        PICO_HIP_TRY(hipMemcpyAsync(h, st, offsetof(BatchState, open), hipMemcpyDeviceToHost, stream));
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
        stats->helped_graphs = (int64_t)h->helped.v;
        stats->help_chunks = (int64_t)h->helpchunks.v;
        stats->histocore_graphs = algo == PICO_ALGO_HISTOCORE ? (int64_t)T : 0;
        if (chose_hc) *chose_hc = (long long)h->chose_hc.v;
        if (h->stuck.v) {
            set_error("%llu helped phases did not finish within the wait bound", (unsigned long long)h->stuck.v);
            return PICO_EHIP;
        }
        if (h->bad.v) {
            set_error("%llu graphs of the batch have a vertex count outside [0, 2^31)",
                      (unsigned long long)h->bad.v);
            return PICO_EINVAL;
        }
    }
    return PICO_OK;
}

}  // namespace

// ------------------------------------------------ one small graph (host)

namespace {

// Dynamic LDS one workgroup of `kernel` may take (bytes), its launch limit
// raised to that once per kernel.
int small_lds_cap(const void *kernel, int *cap) {
    static std::mutex mu;
    static const void *keys[4] = {nullptr, nullptr, nullptr, nullptr};
    static int caps[4] = {0, 0, 0, 0};
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < 4; ++i)
        if (keys[i] == kernel) {
            *cap = caps[i];
            return PICO_OK;
        }
    int dev = 0, max_dyn = 0;
    PICO_HIP_TRY(hipGetDevice(&dev));
    PICO_HIP_TRY(hipDeviceGetAttribute(&max_dyn, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    hipFuncAttributes fa;
    PICO_HIP_TRY(hipFuncGetAttributes(&fa, kernel));
    int c = (max_dyn - (int)fa.sharedSizeBytes) & ~255;
    if (c < 0) c = 0;
    if (c > 48 * 1024) PICO_HIP_TRY(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, c));
    for (int i = 0; i < 4; ++i)
        if (!keys[i]) {
            keys[i] = kernel;
            caps[i] = c;
            break;
        }
    *cap = c;
    return PICO_OK;
}

template <typename Off>
const void *small_kernel(int algo) {
    return (algo & PICO_ALGO_MASK) == PICO_ALGO_HISTOCORE ? reinterpret_cast<const void *>(hc_small<Off>)
                                                          : reinterpret_cast<const void *>(po_small<Off>);
}

// Largest m the one-workgroup path takes by default (PICO_SMALL_MAX_EDGES
// overrides; 0 turns the default path off).
long long small_max_edges() {
    static long long v = -1;
    if (v < 0) {
        const char *e = getenv("PICO_SMALL_MAX_EDGES");
        v = (e && *e && atoll(e) >= 0) ? atoll(e) : kSmallMaxEdgesDefault;
    }
    return v;
}

}  // namespace

size_t small_ws_bytes(int64_t n, int64_t m, int algo) {
    size_t b = carve_bytes(n, 4) * 4 + carve_bytes(SM_WORDS, 8);
    if ((algo & PICO_ALGO_MASK) == PICO_ALGO_HISTOCORE) b += carve_bytes(n, 4) + carve_bytes(m, 4);
    return b;
}

int small_path(int64_t n, int64_t m, int algo, bool *use) {
    *use = false;
    if (algo & (PICO_PATH_GRID | PICO_PO_STATIC | PICO_PO_ROLLBACK | PICO_PO_GPP)) return PICO_OK;
    const bool forced = (algo & PICO_PATH_WG) != 0;
    if (!forced && m > small_max_edges()) return PICO_OK;
    int cap = 0;
    const bool i64 = (algo & PICO_OFFSETS_I64) != 0;
    int rc = small_lds_cap(i64 ? small_kernel<int64_t>(algo) : small_kernel<int32_t>(algo), &cap);
    if (rc) return rc;
    if (n * 4 > (int64_t)cap) {
        if (forced) {
            set_error("PICO_PATH_WG: %lld vertex values need %lld bytes of LDS, %d available",
                      (long long)n, (long long)n * 4, cap);
            return PICO_ENOTSUP;
        }
        return PICO_OK;
    }
    *use = true;
    return PICO_OK;
}

template <typename Off>
int run_small(const Off *off, const int32_t *cols, int64_t n, int64_t m, int algo, int32_t *out,
              void *ws, size_t ws_bytes, pico_stats *stats, hipStream_t stream, const int32_t *warm,
              int warm_add) {
    const bool hc = (algo & PICO_ALGO_MASK) == PICO_ALGO_HISTOCORE;
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    TaskT<Off> t;
    t.off = off;
    t.cols = cols;
    t.e0 = 0;
    t.n = (int)n;
    t.slot = -1;
    t.out = out;
    t.core = cv.take<int32_t>(n);  // values live in LDS; unused
    t.L0 = cv.take<int32_t>(n);
    t.L1 = cv.take<int32_t>(n);
    t.L2 = cv.take<int32_t>(n);
    t.oldcore = hc ? cv.take<int32_t>(n) : nullptr;
    t.histo = hc ? cv.take<int32_t>(m) : nullptr;
    unsigned long long *sm = cv.take<unsigned long long>(SM_WORDS);
    if (!t.core || !t.L0 || !t.L1 || !t.L2 || !sm || (hc && (!t.oldcore || !t.histo))) {
        set_error("workspace too small for the one-workgroup path (%zu bytes given, %zu needed)", ws_bytes,
                  small_ws_bytes(n, m, algo));
        return PICO_ENOMEM;
    }
    const size_t lds = (size_t)n * 4;
    int rec = prof_begin(hc ? "hc_small" : "po_small", stream);
    if (hc)
        hipLaunchKernelGGL(hc_small<Off>, dim3(1), dim3(kBlock), lds, stream, t, kSumWaveMinDefault, warm,
                           warm_add, sm);
    else
        hipLaunchKernelGGL(po_small<Off>, dim3(1), dim3(kBlock), lds, stream, t, sm);
    prof_end(rec, stream);
    PICO_LAUNCH_CHECK();
    if (stats) {
        unsigned long long *h = static_cast<unsigned long long *>(host_scratch(SM_WORDS * 8));
        if (!h) return PICO_EHIP;
        PICO_HIP_TRY(hipMemcpyAsync(h, sm, SM_WORDS * 8, hipMemcpyDeviceToHost, stream));
        PICO_HIP_TRY(hipStreamSynchronize(stream));
        stats->iterations = (int64_t)h[SM_LEVELS];
        stats->sub_rounds = hc ? (int64_t)h[SM_LEVELS] : (int64_t)h[SM_DRAINS];
        stats->scans = hc ? 0 : (int64_t)h[SM_SCANS];
        stats->frontier_total = (int64_t)h[SM_FRONTIER];
        stats->k_max = hc ? 0 : (int32_t)h[SM_KMAX];
        stats->edges_scanned = (int64_t)h[SM_EDGES];
        stats->atomics = (int64_t)h[SM_ATOMICS];
        stats->buckets_scanned = (int64_t)h[SM_BUCKETS];
        stats->pushes_dynamic = (int64_t)h[SM_PUSHES];
    }
    return PICO_OK;
}

template int run_small<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, int, int32_t *, void *,
                                size_t, pico_stats *, hipStream_t, const int32_t *, int);
template int run_small<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, int, int32_t *, void *,
                                size_t, pico_stats *, hipStream_t, const int32_t *, int);

// Workspace of a packed batch: the per-graph status words first (where
// pico_batch_status finds them), then the working arrays.  PICO_ALGO_AUTO
// holds HistoCore's arrays plus a second state and two more task tables.
size_t batched_ws_bytes(int64_t G, int64_t total_n, int64_t total_m, int algo) {
    const int a = algo & PICO_ALGO_MASK;
    size_t b = carve_bytes(G, 4) + carve_bytes(total_n, 4) * 4 + carve_bytes(1, sizeof(BatchState)) +
               carve_bytes(G, sizeof(Task));
    if (a == PICO_ALGO_HISTOCORE || a == PICO_ALGO_AUTO) b += carve_bytes(total_m, 4) + carve_bytes(total_n, 4);
    if (a == PICO_ALGO_AUTO) b += carve_bytes(1, sizeof(BatchState)) + carve_bytes(G, sizeof(Task)) * 2 + carve_bytes(G, 4);
    return b;
}

int help_min_large(const pico_batch_tune *tune, int algo) {
    (void)algo;  // both algorithms take helpers
    return help_min_of(tune);
}

size_t task_scratch_bytes(int64_t n, int64_t m, int algo) {
    const int a = algo & PICO_ALGO_MASK;
    long long words = 4 * task_al(n);
    if (a == PICO_ALGO_HISTOCORE || a == PICO_ALGO_AUTO) words += task_al(n) + task_al(m);
    return (size_t)words * 4;
}

// Task-list workspace: status words first, the task table, the host list's
// device copy, the state; then what PICO_ALGO_AUTO adds (a second state, two
// per-algorithm tables, the choices).
size_t tasks_ws_bytes(int64_t T) {
    return carve_bytes(T, 4) + carve_bytes(T, sizeof(Task)) + carve_bytes(T, sizeof(pico_task)) +
           carve_bytes(1, sizeof(BatchState)) + carve_bytes(1, sizeof(BatchState)) +
           carve_bytes(T, sizeof(Task)) * 2 + carve_bytes(T, 4);
}

namespace {

void merge_stats(pico_batch_stats *into, const pico_batch_stats &x) {
    into->iterations += x.iterations;
    into->atomics += x.atomics;
    into->frontier_total += x.frontier_total;
    into->edges_scanned += x.edges_scanned;
    into->buckets_scanned += x.buckets_scanned;
    into->pushes += x.pushes;
    into->lds_graphs += x.lds_graphs;
    into->workgroups += x.workgroups;
    into->helped_graphs += x.helped_graphs;
    into->help_chunks += x.help_chunks;
    into->histocore_graphs += x.histocore_graphs;
}

// PICO_ALGO_AUTO over a built task table `all`: choose per graph, split into
// two tables with holes, one launch per algorithm on the stream (PeelOne
// first).  With stats, each launch waits and the two are merged.
int launch_auto(Task *all, Task *po, Task *hc, int32_t *choice, long long T, const pico_batch_tune *tune,
                BatchState *st_po, BatchState *st_hc, int32_t *status, pico_batch_stats *stats,
                hipStream_t stream, long long want) {
    long long cb = T < 4096 ? T : 4096;
    PICO_LAUNCH("choose_tasks", choose_tasks, dim3((unsigned)(cb > 0 ? cb : 1)), dim3(kBlock), stream, all, T,
                choice, st_hc);
    PICO_LAUNCH("split_tasks", split_tasks, dim3((unsigned)((T + 255) / 256)), dim3(256), stream, all, T, choice,
                po, hc);
    pico_batch_stats s_po, s_hc;
    int rc = launch_tasks(po, T, PICO_ALGO_PEELONE, tune, st_po, status, stats ? &s_po : nullptr, stream, want);
    if (rc) return rc;
    long long chose = 0;
    rc = launch_tasks(hc, T, PICO_ALGO_HISTOCORE, tune, st_hc, status, stats ? &s_hc : nullptr, stream, want,
                      &chose);
    if (rc) return rc;
    if (stats) {
        *stats = s_po;
        merge_stats(stats, s_hc);
        stats->graphs = T;
        stats->histocore_graphs = chose;
        if (s_hc.lds_bytes > stats->lds_bytes) stats->lds_bytes = s_hc.lds_bytes;
    }
    return PICO_OK;
}

}  // namespace

int run_batched(const long long *vptr, const long long *off, const int32_t *cols, int64_t G,
                int64_t total_n, int64_t total_m, int algo, const int32_t *order, int32_t *out,
                void *ws, size_t ws_bytes, const pico_batch_tune *tune, pico_batch_stats *stats,
                hipStream_t stream) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    int32_t *status = cv.take<int32_t>(G);
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
    const bool hc = algo == PICO_ALGO_HISTOCORE || algo == PICO_ALGO_AUTO;
    if (hc) {
        p.histo = cv.take<int32_t>(total_m);
        p.oldcore = cv.take<int32_t>(total_n);
    }
    BatchState *st = cv.take<BatchState>(1);
    Task *tasks = cv.take<Task>(G);
    const bool aut = algo == PICO_ALGO_AUTO;
    BatchState *st2 = aut ? cv.take<BatchState>(1) : nullptr;
    Task *po = aut ? cv.take<Task>(G) : nullptr;
    Task *hct = aut ? cv.take<Task>(G) : nullptr;
    int32_t *choice = aut ? cv.take<int32_t>(G) : nullptr;
    if (!status || !p.core || !p.L0 || !p.L1 || !p.L2 || !st || !tasks ||
        (hc && ((total_m > 0 && !p.histo) || !p.oldcore)) || (aut && (!st2 || !po || !hct || !choice))) {
        set_error("batched workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  batched_ws_bytes(G, total_n, total_m, algo));
        return PICO_ENOMEM;
    }
    PICO_LAUNCH("batch_state_init", batch_state_init, dim3(1), dim3(kBlock), stream, st);
    if (aut) PICO_LAUNCH("batch_state_init", batch_state_init, dim3(1), dim3(kBlock), stream, st2);
    PICO_LAUNCH("packed_tasks", packed_tasks, dim3((unsigned)((G + 255) / 256)), dim3(256), stream, p,
                tasks, st, status);
    // a packed batch fills the device: its tail is helped by whoever is idle
    const long long want = G > kMaxGrid ? G : kMaxGrid;
    if (aut) return launch_auto(tasks, po, hct, choice, G, tune, st, st2, status, stats, stream, want);
    return launch_tasks(tasks, G, algo, tune, st, status, stats, stream, want);
}

int run_tasks_device(const pico_task *dev_tasks, int64_t T, int algo, void *ws, size_t ws_bytes,
                     const pico_batch_tune *tune, pico_batch_stats *stats, hipStream_t stream,
                     int64_t n_large) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    int32_t *status = cv.take<int32_t>(T);
    Task *tasks = cv.take<Task>(T);
    cv.take<pico_task>(T);
    BatchState *st = cv.take<BatchState>(1);
    BatchState *st2 = cv.take<BatchState>(1);
    Task *po = cv.take<Task>(T);
    Task *hct = cv.take<Task>(T);
    int32_t *choice = cv.take<int32_t>(T);
    if (!status || !tasks || !st || !st2 || !po || !hct || !choice) {
        set_error("tasks workspace too small (%zu bytes given, %zu needed)", ws_bytes, tasks_ws_bytes(T));
        return PICO_ENOMEM;
    }
    const bool aut = algo == PICO_ALGO_AUTO;
    PICO_LAUNCH("batch_state_init", batch_state_init, dim3(1), dim3(kBlock), stream, st);
    if (aut) PICO_LAUNCH("batch_state_init", batch_state_init, dim3(1), dim3(kBlock), stream, st2);
    PICO_LAUNCH("public_tasks", public_tasks, dim3((unsigned)((T + 255) / 256)), dim3(256), stream,
                dev_tasks, (long long)T, algo == PICO_ALGO_PEELONE ? 0 : 1, tasks, status);
    // a few helpers per large task, so that a launch holding one large graph
    // leaves room on the device for the launches beside it
    const long long want = T + kHelpersPerBig * n_large;
    if (aut) return launch_auto(tasks, po, hct, choice, T, tune, st, st2, status, stats, stream, want);
    return launch_tasks(tasks, T, algo, tune, st, status, stats, stream, want);
}

// The status words at the start of a batched or task-list workspace.
const int32_t *status_words(const void *ws) { return static_cast<const int32_t *>(ws); }

// Device copy of a host task array inside the tasks workspace (third slot).
pico_task *tasks_table(void *ws, size_t ws_bytes, int64_t T) {
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    cv.take<int32_t>(T);
    cv.take<Task>(T);
    return cv.take<pico_task>(T);
}

}  // namespace pico
