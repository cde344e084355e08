// PeelOne with the assertion decrement and the dynamic in-level frontier
// (paper Section III, Alg. 4), for gfx950, as one persistent cooperative
// kernel per decomposition.
//
// Level k peels every residual vertex whose residual degree has reached k.
// The working array `core` holds residual degrees; by Corollary 1 every
// residual vertex has core >= k while level k runs, so the level's scan
// frontier is simply {v residual : core[v] == k} (no removal flag).
//
// Assertion decrement (Section III-B).  The paper's atomicSub_{>=k} stores
// max(old - 1, k).  gfx950 has no clamped-decrement atomic, so the scatter
// filters on core[u] > k (the test the paper puts before the atomic; batches
// expanded locally skip it, see "Local links") and then issues a plain
// fetch-and-subtract; the thread whose fetch returns exactly k + 1 is the
// unique one that lowers u to k, so it alone asserts u into the level's
// frontier and records out[u] = k.  A racing decrement that lands
// below k only touches a vertex already asserted at level k, whose final value
// is held in `out`, and no vertex receives more than deg(u) decrements, so the
// counter never underflows.  The vector produced is the one the clamped atomic
// gives, without compare-and-swap retry loops under hub contention.  The
// filter may read a stale (larger) value cached before a concurrent
// decrement; that only costs a wasted atomic, never a missed one.
//
// Claims.  A level's scan and its scatter overlap (a workgroup expands what
// its own scan found while others still scan), so each vertex is claimed by
// exactly one thread with a compare-and-swap of out[v] from -1 to k: the
// scanner that reads core[v] == k, or the decrementer whose fetch returns
// k + 1 (it lowered v to k) or k (an unfiltered local decrement, or a stale
// filter read, lowered a not-yet-claimed level-k vertex below k).  Every
// vertex whose value reaches k or less during level k meets one of these, so
// none is lost, and the compare-and-swap lets only one expand it.  Once the
// level's scan phase has ended (a grid barrier), every vertex valued k or
// less is claimed, so in the level's rounds the one decrement whose fetch
// returns k + 1 claims its vertex alone, with a plain store.
//
// Dynamic frontier (Section III-C, step 3).  An asserted vertex is processed
// in the same level.  While the work it brings is small, the workgroup that
// asserted it expands it at once from an LDS queue, so peel chains advance
// without any grid-wide step; larger bursts go to the global frontier list,
// which the whole grid shares out in the level's next round, one grid
// barrier later.  The level ends at the first barrier after which the global
// list has nothing new.  A level whose scan finds nobody jumps k straight to
// the smallest surviving value.
//
// Local links.  A peel cascade followed through the LDS queue is a chain of
// dependent memory round trips per link, so each link takes as few as it
// can: the claim's compare-and-swap is issued together with the loads of the
// claimed vertex's row bounds, which travel in the queue beside its id, and
// a batch expanded locally decrements every neighbour without first reading
// its value (a neighbour already peeled holds a value below k, so the fetch
// returns less than k and claims nothing; every entry still decrements at
// most once).  The edge-balanced rounds keep the filter read: they are
// bound by throughput, and the read spares a memory-side atomic for every
// peeled neighbour.
//
// Edge balance.  Each global frontier entry records where its adjacency row
// starts in the concatenation of the round's rows, reserved together with the
// entry's slot through one packed counter, so a round hands every workgroup
// an equal slice of the round's edges however skewed the degrees are (the
// load balancing the paper takes from Tigr, Section V-A).  Every thread keeps
// eight edges in flight to hide memory latency.
//
// Every vertex enters a frontier exactly once over the whole run, so the
// global list needs at most n entries.
#include <climits>

#include "common.hpp"

namespace pico {
namespace {

constexpr int kLq = 2048;          // LDS continuation queue per workgroup
constexpr int kLocalMax = 4096;    // an LDS batch is expanded locally up to this many edges (default)
// Survivors per thread per scan step.  16 was measured too: 156 VGPRs
// instead of 125, the same scan time and slower drains (RMAT-26 131 -> 134
// ms, RMAT-22 19.1 -> 21.0 ms).
constexpr int kScanR = 8;
constexpr int kTile = kBlock * kScanR;  // scan items per block step

// Ablations of Alg. 4 (the variants the paper measures against):
//   kStatic   -- no dynamic frontier (Table IV): a decrement never claims;
//                vertices brought down to k wait for the next scan at the same
//                level, which takes every survivor at or below k.  Scanned
//                vertices always go to the global list, so no decrement of an
//                iteration overlaps its scan and the iteration count is the
//                serial one.
//   kRollback -- the decrement of PP-dyn style methods (Section III-B): a
//                fetch-and-subtract that lands at or below k is undone with a
//                fetch-and-add, each counted as an atomic.
//   kGpp      -- General Parallel Peel (Alg. 3, Section II-C; the GPP
//                baseline of Section V): as kStatic, but every neighbour not
//                yet removed is decremented (the removal flag is the filter,
//                not the value), and k advances by one at a time.  Alg. 3
//                raises k at the head of a while-loop iteration, when no
//                residual vertex is at or below k, and scans with the raised
//                k in the same iteration; here that test is a scan that finds
//                nobody, so such a scan right after a scan that removed
//                vertices opens the next iteration instead of being one.
//                Isolated vertices, removed at k = 0 in Alg. 3's first
//                iteration, are written at initialisation and counted as
//                that iteration.
enum { kDynamic = 0, kStatic = 1, kRollback = 2, kGpp = 3 };

// Cumulative counters of the grid state.  QET packs (edges << 31) | slots of
// the global frontier list.
enum { QET = 0, N_DYN, N_ATOM };
constexpr int kSnap = 1;  // counters read at barriers: QET

struct PoState {
    GridState g;
    Line na[3];  // survivors listed by scan j, in slot j % 3
    Line mn[3];  // smallest surviving value seen by scan j
    Line nf[3];  // vertices claimed by scan j
    Line dynl[3];  // vertices asserted by decrements in the level of scan j (schedule only)
    Line levels, scans, kmax, rounds, peelable, gpp_iters;
    Line phase[kNumPhases];
};

template <typename Off>
struct PoArgs {
    const Off *off;
    const int32_t *cols;
    long long n;
    int32_t *core;
    int32_t *out;
    int32_t *A0;
    int32_t *A1;
    int32_t *Q;      // global frontier list: vertex ids
    long long *QE;   // ... start of each entry's row in the concatenated edge space
    long long *QR;   // ... first CSR position of each entry's row
    PoState *st;
    unsigned long long limit;  // wall-clock ticks any single wait may last
    pico_step *sched;          // optional per-level schedule record (device), or null
    long long sched_cap;
    double ns_per_tick;        // device wall clock period
    int mode;                  // kDynamic, or an ablation: kStatic, kRollback
    int local_max;             // LDS batches up to this many edges are expanded locally
};

__global__ void po_state_init(PoState *st) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(st);
    const int words = (int)(sizeof(PoState) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0ull;
    __syncthreads();
    if (threadIdx.x < 3) st->mn[threadIdx.x].v = (unsigned long long)INT_MAX;
}

// The workgroup's LDS continuation queue: a ring of kLq vertex ids.  `take`
// is the next entry to hand out; `keep` the oldest entry still being read
// (entries are consumed in workgroup-wide batches).
struct LdsQueue {
    int *buf;
    long long *rs;  // each entry's first CSR position
    int *d;         // ... and its row length
    unsigned *take;
    unsigned *tail;
    unsigned *keep;
};

template <typename Off>
struct PoCtx {
    const Off *off;
    int32_t *core;
    int32_t *out;
    int32_t *Q;
    long long *QE;
    long long *QR;
    unsigned long long *qet;  // packed global frontier counter
    LdsQueue lq;
    int k;
    int natom;
    int ndyn;
    int mode;
    bool scanning;  // the level's scan phase: scanners claim too, so claims need a compare-and-swap
};

// Append the lanes' vertices to the global frontier list (one atomic per
// wave), with their row starts in the concatenated edge space.
template <typename Off>
__device__ __forceinline__ void push_global(bool pred, int u, long long rs, long long d, PoCtx<Off> &c) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    if (!pred) rs = d = 0;
    long long dpre = wave_incl_scan64(d) - d;
    long long dtot = __shfl(dpre + d, kWave - 1);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long old = 0;
    if (lane_id() == leader)
        old = atomicAdd(c.qet, ((unsigned long long)dtot << kSlotBits) | (unsigned long long)__popcll(mask));
    old = __shfl(old, leader);
    if (pred) {
        unsigned long long slot = (old & kSlotMask) + lane_rank(mask);
        c.Q[slot] = u;
        c.QE[slot] = (long long)(old >> kSlotBits) + dpre;
        c.QR[slot] = rs;
    }
}

// Assert the lanes' vertices into the level's frontier: the workgroup's LDS
// queue while it has room, else the global list for the next round.
template <typename Off>
__device__ __forceinline__ void enqueue(bool pred, int u, long long rs, int d, PoCtx<Off> &c) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    const unsigned cnt = (unsigned)__popcll(mask);
    int global = 0;
    unsigned base = 0;
    if (lane_id() == leader) {
        while (true) {
            unsigned t = *(volatile unsigned *)c.lq.tail;
            if (t + cnt - *(volatile unsigned *)c.lq.keep > (unsigned)kLq) {
                global = 1;
                break;
            }
            if (atomicCAS(c.lq.tail, t, t + cnt) == t) {
                base = t;
                break;
            }
        }
    }
    global = __shfl(global, leader);
    base = __shfl(base, leader);
    c.ndyn += pred ? 1 : 0;
    if (global) {
        push_global(pred, u, rs, (long long)d, c);
    } else if (pred) {
        const unsigned i = (base + lane_rank(mask)) % kLq;
        c.lq.buf[i] = u;
        c.lq.rs[i] = rs;
        c.lq.d[i] = d;
    }
}

__device__ __forceinline__ bool claim_vertex(int32_t *out, int v, int k) {
    return atomicCAS(&out[v], -1, k) == -1;
}

// kEbR edges per thread of the scatter (Alg. 4, graph operator): the filter
// reads and the decrements of all edges are issued before any result is used.
// kMode: the variant this kernel is compiled for (each its own kernel, so
// Alg. 4's carries none of the ablations' code).
template <typename Off, int kMode>
__device__ __forceinline__ void relax(const bool (&act)[kEbR], const int (&u)[kEbR], PoCtx<Off> &c,
                                      bool filter = true) {
    constexpr int mode = kMode;
    const bool gpp = mode == kGpp;
    int cu[kEbR];
    if (mode == kDynamic && !filter) {
        // a local batch: every neighbour is decremented, without the filter read
#pragma unroll
        for (int r = 0; r < kEbR; ++r) cu[r] = act[r] ? INT_MAX : 0;
    } else {
#pragma unroll
        for (int r = 0; r < kEbR; ++r) cu[r] = act[r] ? (gpp ? c.out[u[r]] : c.core[u[r]]) : 0;
    }
    int old[kEbR];
#pragma unroll
    for (int r = 0; r < kEbR; ++r) {
        old[r] = 0;
        if (act[r] && (gpp ? cu[r] == -1 : cu[r] > c.k)) {
            old[r] = atomicSub(&c.core[u[r]], 1);
            ++c.natom;
        }
    }
    if (mode == kStatic || gpp) return;  // lowered vertices wait for the next scan
    if (mode == kRollback) {
#pragma unroll
        for (int r = 0; r < kEbR; ++r) {
            if (act[r] && cu[r] > c.k && old[r] <= c.k) {
                atomicAdd(&c.core[u[r]], 1);
                ++c.natom;
            }
        }
    }
    int got[kEbR];
    long long rs[kEbR], re[kEbR];
    if (mode == kDynamic && !c.scanning) {
        // after the level's scan every vertex at or below k is claimed, so the
        // one decrement that takes u from k + 1 to k claims it alone
#pragma unroll
        for (int r = 0; r < kEbR; ++r) {
            got[r] = act[r] && cu[r] > c.k && old[r] == c.k + 1 ? 1 : 0;
            rs[r] = re[r] = 0;
            if (got[r]) {
                c.out[u[r]] = c.k;
                rs[r] = (long long)c.off[u[r]];
                re[r] = (long long)c.off[u[r] + 1];
            }
        }
    } else {
        // a candidate's claim and its row bounds in one round trip
#pragma unroll
        for (int r = 0; r < kEbR; ++r) {
            got[r] = 0;
            rs[r] = re[r] = 0;
            if (act[r] && cu[r] > c.k && (old[r] == c.k + 1 || old[r] == c.k)) {
                got[r] = atomicCAS(&c.out[u[r]], -1, c.k) == -1 ? 1 : 0;
                rs[r] = (long long)c.off[u[r]];
                re[r] = (long long)c.off[u[r] + 1];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kEbR; ++r) enqueue(got[r] != 0, u[r], rs[r], (int)(re[r] - rs[r]), c);
}

// Expand the workgroup's LDS queue until it is empty: a batch of up to 256
// queued vertices at a time, expanded here when its rows hold at most
// local_max edges, otherwise sent to the global list for the next round.
template <typename Off, int kMode>
__device__ void drain_lds(const PoArgs<Off> &a, PoCtx<Off> &c, ExpandLds &X) {
    while (true) {
        __syncthreads();
        const unsigned tk = *c.lq.take, tl = *c.lq.tail;
        if (tl == tk) break;
        const unsigned cnt = tl - tk < (unsigned)kBlock ? tl - tk : (unsigned)kBlock;
        __syncthreads();
        if (threadIdx.x == 0) {
            *c.lq.keep = tk;
            *c.lq.take = tk + cnt;
        }
        __syncthreads();
        int v = -1;
        long long rs = 0, d = 0;
        if (threadIdx.x < cnt) {
            const unsigned i = (tk + threadIdx.x) % kLq;
            v = c.lq.buf[i];
            rs = c.lq.rs[i];
            d = c.lq.d[i];
        }
        long long tot = 0;
        (void)block_excl_scan64(d, tot, X.scan_l);
        if (tot > a.local_max) {
            push_global(v >= 0, v, rs, d, c);  // a burst: share it out next round
        } else {
            block_expand<kEbR>((int)d, rs, 0, 0, a.cols, X,
                               [&](const bool (&act)[kEbR], const int (&u)[kEbR], const int (&)[kEbR]) {
                                   relax<Off, kMode>(act, u, c, false);
                               });
        }
        __syncthreads();
        if (threadIdx.x == 0) *c.lq.keep = *c.lq.take;
    }
}

// First pass over all ids: core = deg, out = 0 for isolated vertices and -1
// (unclaimed) for the others, which are listed; smallest positive degree.
template <typename Off>
__device__ void po_init(const PoArgs<Off> &a, unsigned long long *na_ctr, unsigned long long *mn_ctr,
                        int *lds, unsigned long long *lds64) {
    int lmin = INT_MAX;
    const long long step = (long long)gridDim.x * kTile;
    for (long long tile = (long long)blockIdx.x * kTile; tile < a.n; tile += step) {
        unsigned sv = 0;
#pragma unroll
        for (int r = 0; r < kScanR; ++r) {
            long long i = tile + r * kBlock + threadIdx.x;
            if (i < a.n) {
                int c = (int)(a.off[i + 1] - a.off[i]);
                a.core[i] = c;
                a.out[i] = c == 0 ? 0 : -1;
                if (c > 0) {
                    sv |= 1u << r;
                    lmin = min(lmin, c);
                }
            }
        }
        int ts = 0;
        int ps = block_excl_scan(__popc(sv), ts, lds);
        unsigned long long bs = block_reserve(ts, na_ctr, lds64);
#pragma unroll
        for (int r = 0; r < kScanR; ++r)
            if (sv >> r & 1u) a.A0[bs + ps++] = (int)(tile + r * kBlock + threadIdx.x);
    }
    int bm = block_min(lmin, lds);
    if (threadIdx.x == 0 && bm != INT_MAX) atomicMin(mn_ctr, (unsigned long long)bm);
}

// Scan of the survivor list at level k (Alg. 4, scan kernel), block-
// aggregated: vertices with core == k are claimed and become frontier,
// survivors (core > k) go to the next list, and the smallest surviving value
// is recorded.  A tile's claimed frontier stays in the workgroup's LDS queue
// while the workgroup's share is small (expanded right after the scan);
// otherwise it goes to the global list for an edge-balanced round.
template <typename Off, int kMode>
__device__ void po_scan(const PoArgs<Off> &a, PoCtx<Off> &c, const int32_t *__restrict__ src,
                        long long nsrc, int32_t *__restrict__ dst, unsigned long long *na_ctr,
                        unsigned long long *mn_ctr, unsigned long long *nf_ctr, int *lds,
                        long long *lds_l, unsigned long long *lds64) {
    GridState *gs = &a.st->g;
    const int k = c.k;
    int lmin = INT_MAX;
    long long local_edges = 0;  // block-uniform
    int claimed = 0;
    const long long step = (long long)gridDim.x * kTile;
    for (long long tile = (long long)blockIdx.x * kTile; tile < nsrc; tile += step) {
        int vv[kScanR];
        long long vrs[kScanR];
        int vd[kScanR];
        unsigned fr = 0, sv = 0, cand = 0;
        long long dsum = 0;
#pragma unroll
        for (int r = 0; r < kScanR; ++r) {
            long long i = tile + r * kBlock + threadIdx.x;
            int v = -1, cv = -1;
            if (i < nsrc) {
                v = src[i];
                cv = c.core[v];
            }
            vv[r] = v;
            if (cv > k) {
                sv |= 1u << r;
                lmin = min(lmin, cv);
            }
            if (cv == k || ((kMode == kStatic || kMode == kGpp) && v >= 0 && cv < k)) cand |= 1u << r;
        }
        // a candidate's claim and its row bounds in one round trip
        bool won[kScanR];
        long long vre[kScanR];
#pragma unroll
        for (int r = 0; r < kScanR; ++r) {
            const int v = vv[r];
            won[r] = false;
            vrs[r] = vre[r] = 0;
            if (cand >> r & 1u) {
                won[r] = claim_vertex(c.out, v, k);
                vrs[r] = (long long)a.off[v];
                vre[r] = (long long)a.off[v + 1];
            }
        }
#pragma unroll
        for (int r = 0; r < kScanR; ++r) {
            vd[r] = 0;
            if (won[r]) {
                fr |= 1u << r;
                vd[r] = (int)(vre[r] - vrs[r]);
                dsum += vd[r];
            }
        }
        int ts = 0;
        int ps = block_excl_scan(__popc(sv), ts, lds);
        unsigned long long bs = block_reserve(ts, na_ctr, lds64);
#pragma unroll
        for (int r = 0; r < kScanR; ++r)
            if (sv >> r & 1u) dst[bs + ps++] = vv[r];
        int tf = 0;
        long long te = 0;
        int pf = block_excl_scan(__popc(fr), tf, lds);
        long long pe = block_excl_scan64(dsum, te, lds_l);
        if (tf == 0) continue;
        claimed += tf;
        const unsigned tail = *c.lq.tail, keep = *c.lq.keep;
        const bool local = kMode != kStatic && kMode != kGpp && local_edges + te <= a.local_max &&
                           tail + tf - keep <= (unsigned)kLq;
        if (local) {
            local_edges += te;
#pragma unroll
            for (int r = 0; r < kScanR; ++r)
                if (fr >> r & 1u) {
                    const unsigned i = (tail + pf++) % kLq;
                    c.lq.buf[i] = vv[r];
                    c.lq.rs[i] = vrs[r];
                    c.lq.d[i] = vd[r];
                }
            __syncthreads();
            if (threadIdx.x == 0) *c.lq.tail = tail + tf;
            __syncthreads();
        } else {
            if (threadIdx.x == 0)
                lds64[0] = atomicAdd(&gs->ctr[QET].v,
                                     ((unsigned long long)te << kSlotBits) | (unsigned long long)tf);
            __syncthreads();
            const unsigned long long old = lds64[0];
            __syncthreads();
            const unsigned long long bq = old & kSlotMask;
            const long long be = (long long)(old >> kSlotBits);
#pragma unroll
            for (int r = 0; r < kScanR; ++r) {
                if (fr >> r & 1u) {
                    a.Q[bq + pf] = vv[r];
                    a.QE[bq + pf] = be + pe;
                    a.QR[bq + pf] = vrs[r];
                    ++pf;
                    pe += vd[r];
                }
            }
        }
    }
    int bm = block_min(lmin, lds);
    if (threadIdx.x == 0) {
        if (bm != INT_MAX) atomicMin(mn_ctr, (unsigned long long)bm);
        if (claimed) atomicAdd(nf_ctr, (unsigned long long)claimed);
    }
}

// One edge-balanced round of level k over global frontier entries [q0, q1)
// (edge space [e0, e1)), then this workgroup's LDS queue.
template <typename Off, int kMode>
__device__ void po_round(const PoArgs<Off> &a, PoCtx<Off> &c, unsigned long long q0,
                         unsigned long long q1, unsigned long long e0, unsigned long long e1,
                         EbLds &E, ExpandLds &X) {
    edge_balanced(a.Q, a.QE, a.QR, nullptr, nullptr, (long long)q0, (long long)q1, (long long)e0,
                  (long long)e1, a.cols, nullptr, E,
                  [&](const bool (&act)[kEbR], const int (&u)[kEbR], const int (&)[kEbR], EbLds &,
                      const int (&)[kEbR]) { relax<Off, kMode>(act, u, c); });
    drain_lds<Off, kMode>(a, c, X);
}

template <typename Off, int kMode>
__global__ __launch_bounds__(kBlock) void po_persistent(PoArgs<Off> a) {
    constexpr int mode = kMode;
    __shared__ int lds[kWavesPerBlock];
    __shared__ long long lds_l[kWavesPerBlock];
    __shared__ unsigned long long lds64[1];
    __shared__ unsigned long long snap[kNumCtr + 1];
    __shared__ int lq_buf[kLq];
    __shared__ long long lq_rs[kLq];
    __shared__ int lq_d[kLq];
    __shared__ unsigned lq_take, lq_tail, lq_keep;
    __shared__ EbLds eb;
    __shared__ ExpandLds xl;
    PoState *st = a.st;
    GridState *gs = &st->g;
    const unsigned nb = gridDim.x;
    unsigned long long bar = 0;
    if (threadIdx.x == 0) lq_take = lq_tail = lq_keep = 0;
    PoCtx<Off> c{a.off, a.core, a.out, a.Q, a.QE, a.QR, &gs->ctr[QET].v,
                 LdsQueue{lq_buf, lq_rs, lq_d, &lq_take, &lq_tail, &lq_keep}, 0, 0, 0, mode, true};

    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    PhaseClock clk;
    if (timer) clk.start();
    // Phase 0: core = deg, claims cleared, list of non-isolated vertices.
    po_init<Off>(a, &st->na[0].v, &st->mn[0].v, lds, lds64);
    if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
    if (timer) clk.lap(&st->phase[0].v);
    const unsigned long long peelable = ld_rlx(&st->na[0].v);
    long long nprev = (long long)peelable;
    c.k = mode == kGpp ? 1 : (int)ld_rlx(&st->mn[0].v);
    unsigned long long q_end = 0, e_end = 0;  // global list consumed so far
    long long levels = 0, scans = 0, rounds = 0;
    int kmax = 0;
    // GPP's while-loop iterations (Alg. 3): the isolated vertices' k = 0
    // iteration, then every scan except an empty one that follows a scan
    // that removed vertices (that one is the test opening the next iteration)
    long long gpp_iters = (long long)peelable < a.n ? 1 : 0;
    bool gpp_prev_removed = false;
    // Schedule record: the vertices the decrements assert during the level
    // of scan j are added to dynl[j % 3] before each of the level's barriers.
    int ndyn_flushed = 0;
    auto flush_dyn = [&](int slot) {
        if (!a.sched) return;
        const long long t = wave_sum64(c.ndyn - ndyn_flushed);
        ndyn_flushed = c.ndyn;
        if (lane_id() == 0 && t) atomicAdd(&st->dynl[slot].v, (unsigned long long)t);
    };

    for (int j = 1; peelable > 0; ++j) {
        const int32_t *src = (j & 1) ? a.A0 : a.A1;
        int32_t *dst = (j & 1) ? a.A1 : a.A0;
        const unsigned long long t_level = timer ? wall_clock64() : 0ull;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_rlx(&st->na[(j + 1) % 3].v, 0ull);
            st_rlx(&st->mn[(j + 1) % 3].v, (unsigned long long)INT_MAX);
            st_rlx(&st->nf[(j + 1) % 3].v, 0ull);
            st_rlx(&st->dynl[(j + 1) % 3].v, 0ull);
        }
        c.scanning = true;
        po_scan<Off, kMode>(a, c, src, nprev, dst, &st->na[j % 3].v, &st->mn[j % 3].v, &st->nf[j % 3].v,
                     lds, lds_l, lds64);
        drain_lds<Off, kMode>(a, c, xl);
        ++scans;
        flush_dyn(j % 3);
        if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
        const unsigned long long t_scan = wall_clock64();
        if (timer) clk.lap(&st->phase[1].v);
        const long long nsurv_in = nprev;
        nprev = (long long)ld_rlx(&st->na[j % 3].v);
        if (ld_rlx(&st->nf[j % 3].v) == 0ull) {  // empty level: jump to the smallest value left
            if (mode == kGpp) {
                gpp_iters += gpp_prev_removed ? 0 : 1;
                gpp_prev_removed = false;
            }
            if (nprev == 0) break;
            c.k = mode == kGpp ? c.k + 1 : (int)ld_rlx(&st->mn[j % 3].v);
            continue;
        }
        if (mode == kGpp) {
            ++gpp_iters;
            gpp_prev_removed = true;
        }
        const long long rounds_before = rounds;
        unsigned long long q0 = q_end, e0 = e_end;
        unsigned long long q1 = snap[QET] & kSlotMask, e1 = snap[QET] >> kSlotBits;
        c.scanning = false;
        while (q0 < q1) {
            po_round<Off, kMode>(a, c, q0, q1, e0, e1, eb, xl);
            ++rounds;
            flush_dyn(j % 3);
            if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
            q0 = q1;
            e0 = e1;
            q1 = snap[QET] & kSlotMask;
            e1 = snap[QET] >> kSlotBits;
        }
        if (timer) clk.lap(&st->phase[2].v);
        if (timer && a.sched && levels < a.sched_cap) {
            pico_step *sp = a.sched + levels;
            sp->key = c.k;
            sp->vertices = (long long)(ld_rlx(&st->nf[j % 3].v) + ld_rlx(&st->dynl[j % 3].v));
            sp->work = nsurv_in;
            sp->edges = (long long)(e1 - e_end);
            sp->rounds = rounds - rounds_before;
            sp->ns = (long long)((double)(wall_clock64() - t_level) * a.ns_per_tick);
            sp->scan_ns = (long long)((double)(t_scan - t_level) * a.ns_per_tick);
            sp->kind = 0;
        }
        q_end = q1;
        e_end = e1;
        ++levels;
        kmax = c.k;
        if (nprev == 0) break;  // no survivor left after this level's scan: all claimed
        if (mode != kStatic && mode != kGpp) c.k += 1;  // static, GPP: rescan the same level
    }
    long long t = wave_sum64(c.natom);
    if (lane_id() == 0 && t) atomicAdd(&gs->ctr[N_ATOM].v, (unsigned long long)t);
    t = wave_sum64(c.ndyn);
    if (lane_id() == 0 && t) atomicAdd(&gs->ctr[N_DYN].v, (unsigned long long)t);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->levels.v = (unsigned long long)levels;
        st->scans.v = (unsigned long long)scans;
        st->kmax.v = (unsigned long long)kmax;
        st->rounds.v = (unsigned long long)rounds;
        st->peelable.v = peelable;
        st->gpp_iters.v = (unsigned long long)gpp_iters;
    }
}

}  // namespace

size_t peelone_ws_bytes(int64_t n, int64_t m) {
    return carve_bytes(n, 4) * 4 + carve_bytes(n, 8) * 2 + carve_bytes(1, sizeof(PoState));
}

template <typename Off>
int run_peelone(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out, void *ws,
                size_t ws_bytes, pico_stats *stats, hipStream_t stream, int mode, pico_step *sched,
                int64_t sched_cap, int64_t *sched_len) {
    if ((unsigned long long)m >= (1ull << (64 - kSlotBits))) {
        set_error("m=%lld too large for the packed frontier counter", (long long)m);
        return PICO_ENOTSUP;
    }
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    PoArgs<Off> a;
    a.off = off;
    a.cols = cols;
    a.n = n;
    a.core = cv.take<int32_t>(n);
    a.out = out;
    a.A0 = cv.take<int32_t>(n);
    a.A1 = cv.take<int32_t>(n);
    a.Q = cv.take<int32_t>(n);
    a.QE = cv.take<long long>(n);
    a.QR = cv.take<long long>(n);
    a.st = cv.take<PoState>(1);
    if (!a.core || !a.A0 || !a.A1 || !a.Q || !a.QE || !a.QR || !a.st) {
        set_error("PeelOne workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  peelone_ws_bytes(n, m));
        return PICO_ENOMEM;
    }
    a.limit = wall_ticks(20.0);
    a.sched = sched;
    a.sched_cap = sched ? sched_cap : 0;
    a.ns_per_tick = 1e9 / (double)wall_ticks(1.0);
    a.mode = mode;
    a.local_max = tune_int_nonneg("PICO_PO_LOCAL_EDGES", kLocalMax);
    int blocks = 0;
    // One workgroup per CU keeps the grid barriers cheap, which decides small
    // graphs (RMAT-22: 21.4 ms at one, 23.1 at two); on graphs with billions
    // of edges the edge rounds dominate and a second workgroup per CU hides
    // more gather latency (RMAT-26: 142 ms at one, 133.5 at two, 137.7 at four).
    const int per_cu_default = m >= (1ll << 28) ? 2 : 1;
    const void *kernel = mode == kStatic     ? reinterpret_cast<const void *>(po_persistent<Off, kStatic>)
                         : mode == kRollback ? reinterpret_cast<const void *>(po_persistent<Off, kRollback>)
                         : mode == kGpp      ? reinterpret_cast<const void *>(po_persistent<Off, kGpp>)
                                             : reinterpret_cast<const void *>(po_persistent<Off, kDynamic>);
    int rc = persistent_grid(kernel, kBlock,
                             tune_int("PICO_PO_BLOCKS_PER_CU", per_cu_default), grid_want_peelone(m), &blocks);
    if (rc) return rc;
    PICO_LAUNCH("po_state_init", po_state_init, dim3(1), dim3(kBlock), stream, a.st);
    PICO_LAUNCH_CHECK();
    void *args[] = {&a};
    int rec = prof_begin("po_persistent", stream);
    PICO_HIP_TRY(hipLaunchCooperativeKernel(kernel,
                                            dim3(blocks), dim3(kBlock), args, 0, stream));
    prof_end(rec, stream);

    PoState *h = static_cast<PoState *>(host_scratch(sizeof(PoState)));
    if (!h) return PICO_EHIP;
    PICO_HIP_TRY(hipMemcpyAsync(h, a.st, sizeof(PoState), hipMemcpyDeviceToHost, stream));
    PICO_HIP_TRY(hipStreamSynchronize(stream));
    if (h->g.error.v) {
        set_error("PeelOne kernel stopped (error %llu; grid of %d blocks)",
                  (unsigned long long)h->g.error.v, blocks);
        return PICO_EHIP;
    }
    if (sched_len) *sched_len = (int64_t)h->levels.v;
    if (stats) {
        stats->iterations = (int64_t)(mode == kGpp ? h->gpp_iters.v : h->levels.v);  // GPP: Alg. 3's loop
        stats->sub_rounds = (int64_t)h->rounds.v;
        stats->scans = (int64_t)h->scans.v;
        stats->frontier_total = (int64_t)h->peelable.v;
        stats->k_max = (int32_t)h->kmax.v;
        stats->edges_scanned = m;  // every peeled vertex scans its whole row once
        stats->atomics = (int64_t)h->g.ctr[N_ATOM].v;
        stats->buckets_scanned = 0;
        stats->pushes_dynamic = (int64_t)h->g.ctr[N_DYN].v;
        const double tick_ms = 1.0 / (double)wall_ticks(1e-3);
        for (int i = 0; i < kNumPhases; ++i) stats->phase_ms[i] = (double)h->phase[i].v * tick_ms;
    }
    return PICO_OK;
}

template int run_peelone<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                  void *, size_t, pico_stats *, hipStream_t, int, pico_step *, int64_t,
                                  int64_t *);
template int run_peelone<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                  void *, size_t, pico_stats *, hipStream_t, int, pico_step *, int64_t,
                                  int64_t *);

}  // namespace pico
