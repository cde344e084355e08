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

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// SumHisto's reverse summation (Step II of Fig. 6) by one wave, from bucket
// `top` of a vertex's histogram `seg` (bucket b at seg[b - 1]) down to bucket
// 1: the first b with sum(b..top) >= b, and that sum (h = 0 if none).  A first
// pass of 64 buckets (one per lane; the answer is usually near the top),
// then passes of 64 * kSumSlice buckets in which each lane loads its own
// contiguous slice at once.  Running sums only grow as b falls, so sum(b..top)
// - b rises strictly as b falls: the answer lies in the first slice (from the
// top) whose lowest bucket already meets the test, and that slice's lane
// finishes it from the values it holds.
constexpr int kSumSlice = 8;
__device__ __forceinline__ void wave_reverse_sum_wide(const int32_t *seg, int top, int &h, int &s) {
    const int lane = lane_id();
    int carry = 0;
    {
        const int b = top - lane;
        const int val = b >= 1 ? seg[b - 1] : 0;
        const int S = wave_incl_scan(val);
        const unsigned long long mk = __ballot(b >= 1 && S >= b);
        if (mk) {
            const int l = __ffsll(mk) - 1;
            h = top - l;
            s = __shfl(S, l);
            return;
        }
        carry = __shfl(S, kWave - 1);
        top -= kWave;
    }
    while (top >= 1) {
        const int hi = top - lane * kSumSlice;  // this lane's slice: hi down to hi - kSumSlice + 1
        int v[kSumSlice];
        int ls = 0;
#pragma unroll
        for (int j = 0; j < kSumSlice; ++j) {
            v[j] = hi - j >= 1 ? seg[hi - j - 1] : 0;
            ls += v[j];
        }
        const int S = carry + wave_incl_scan(ls);  // carry + sum(lowest bucket of the slice .. top)
        const int lo = hi - kSumSlice + 1 < 1 ? 1 : hi - kSumSlice + 1;
        const unsigned long long mk = __ballot(hi >= 1 && S >= lo);
        if (mk) {
            const int l = __ffsll(mk) - 1;
            int hh = 0, ss = 0;
            if (lane == l) {
                int run = S - ls;  // carry + the buckets above this slice
                bool done = false;
#pragma unroll
                for (int j = 0; j < kSumSlice; ++j) {
                    run += v[j];
                    if (!done && hi - j >= 1 && run >= hi - j) {
                        hh = hi - j;
                        ss = run;
                        done = true;
                    }
                }
            }
            h = __shfl(hh, l);
            s = __shfl(ss, l);
            return;
        }
        carry = __shfl(S, kWave - 1);
        top -= kWave * kSumSlice;
    }
    h = 0;
    s = carry;
}

__device__ __forceinline__ int wave_max_int(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

// Index of the lane owning position t of a wave-wide concatenation whose
// exclusive prefix sums are `pre` (non-decreasing across lanes, pre of lane 0
// is 0): the last lane j with pre_j <= t.  Binary lifting over lanes.
__device__ __forceinline__ int wave_owner(int pre, int t) {
    int pos = 0;
    for (int s = 64; s > 0; s >>= 1) {
        int idx = pos + s - 1;
        int pm = __shfl(pre, idx < kWave ? idx : kWave - 1);
        if (idx < kWave && pm <= t) pos += s;
    }
    return pos - 1;
}

// Agent-scope atomics with explicit ordering (HIP's atomicAdd & co. are
// relaxed at agent scope).
template <typename T>
__device__ __forceinline__ T ld_acq(T *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_rlx(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_rlx(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_rel(T *p, T v);  // release fence, then a relaxed store

// A counter alone on its cache lines, so hot counters do not share a line.
struct alignas(128) Line {
    unsigned long long v;
    unsigned long long pad[15];
};

// Grid-wide state of a persistent cooperative kernel: a two-level barrier,
// an error flag and cumulative counters.  At every barrier the releasing
// block copies all counters into snap[generation & 1], so every block takes
// control decisions from the same values even though fast blocks resume
// updating the counters before slow ones have left the barrier.
constexpr int kNumCtr = 8;
constexpr int kBarGroups = 8;  // one arrival counter per XCD (blocks go round-robin)
struct GridState {
    Line group_arrivals[kBarGroups];
    Line top_arrivals;
    Line gen;
    Line error;
    Line ctr[kNumCtr];
    unsigned long long snap[2][kNumCtr];
};

// Phase timing: block 0 stamps the wall clock at phase boundaries.
constexpr int kNumPhases = 8;
struct PhaseClock {
    unsigned long long last;
    __device__ void start() { last = wall_clock64(); }
    __device__ void lap(unsigned long long *acc) {
        unsigned long long now = wall_clock64();
        *acc += now - last;
        last = now;
    }
};

// Bounded wait: every spin loop gives up after `limit` wall-clock ticks and
// raises the grid error flag, so no input can leave waves spinning forever.
struct Waiter {
    unsigned long long t0, limit;
    unsigned n;
    __device__ explicit Waiter(unsigned long long lim) : t0(wall_clock64()), limit(lim), n(0) {}
    // true when the wait must stop (time limit hit or error raised elsewhere)
    __device__ bool stop(GridState *gs) {
        __builtin_amdgcn_s_sleep(1);
        if ((++n & 63u) != 0) return false;
        if (ld_rlx(&gs->error.v) != 0) return true;
        if (wall_clock64() - t0 > limit) {
            st_rlx(&gs->error.v, 1ull);
            return true;
        }
        return false;
    }
};

struct NoRelease {
    __device__ void operator()(GridState *) const {}
};

// Wait until this wave's outstanding memory operations (vector loads,
// stores and atomics; scalar and LDS traffic) have completed.
__device__ __forceinline__ void wave_mem_drain() { __builtin_amdgcn_s_waitcnt(0); }

// Agent-scope release: the fence writes back this XCD's L2 (buffer_wbl2),
// and the explicit wait makes the write-back complete before whatever
// follows.  The compiler's own wait after the write-back is dropped when the
// wave has no other memory operation outstanding (it does not count the
// write-back as one), and then the signal after the fence could reach memory
// before the data it publishes.
__device__ __forceinline__ void fence_release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
}
template <typename T>
__device__ __forceinline__ void st_rel(T *p, T v) {
    fence_release();
    st_rlx(p, v);
}
__device__ __forceinline__ void fence_acquire() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Grid barrier for a cooperative grid (all blocks co-resident).  Two levels:
// blocks arrive on the counter of their group (blockIdx % kBarGroups, i.e.
// their XCD), the last of each group on the top counter, so no counter sees
// more than about nblocks / 8 serialised atomics.  Counters only grow: the
// b-th barrier completes when a counter reaches (b + 1) times its group
// size, so nothing is ever reset.  Waiting blocks poll the generation word
// with relaxed loads and fence once on the way out.
//
// `bar_no` counts the barriers this block has passed (the same sequence in
// every block).  Only the first NSNAP counters are snapshotted.  `on_release(gs)` runs on the releasing block after all have
// arrived and before any is let go.  snap_out (LDS, kNumCtr + 1 entries)
// receives the counters as they stood then, and the error flag.  Returns
// false if the grid is in error.
template <int NSNAP = kNumCtr, typename Rel = NoRelease>
__device__ __forceinline__ bool grid_sync(GridState *gs, unsigned nblocks, unsigned long long limit,
                                          unsigned long long *snap_out, unsigned long long &bar_no,
                                          Rel on_release = Rel()) {
    // every wave's stores and atomics are performed before the block arrives
    // (the workgroup barrier waits for LDS traffic only); thread 0's release
    // fence below then writes them back from this XCD's L2
    wave_mem_drain();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned ngroups = nblocks < (unsigned)kBarGroups ? nblocks : (unsigned)kBarGroups;
        const unsigned grp = blockIdx.x % ngroups;
        const unsigned gsize = nblocks / ngroups + (grp < nblocks % ngroups ? 1u : 0u);
        const unsigned long long b = bar_no;
        fence_release();
        unsigned long long a =
            __hip_atomic_fetch_add(&gs->group_arrivals[grp].v, 1ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) + 1;
        bool released = false;
        if (a == (b + 1) * gsize) {
            fence_acquire();
            fence_release();
            unsigned long long t =
                __hip_atomic_fetch_add(&gs->top_arrivals.v, 1ull, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT) + 1;
            if (t == (b + 1) * ngroups) {
                fence_acquire();
                on_release(gs);
                unsigned long long c[NSNAP > 0 ? NSNAP : 1];
#pragma unroll
                for (int i = 0; i < NSNAP; ++i) c[i] = ld_rlx(&gs->ctr[i].v);
#pragma unroll
                for (int i = 0; i < NSNAP; ++i) {
                    st_rlx(&gs->snap[b & 1][i], c[i]);
                    snap_out[i] = c[i];
                }
                fence_release();
                st_rlx(&gs->gen.v, b + 1);
                released = true;
            }
        }
        if (!released) {
            Waiter w(limit);
            while (ld_rlx(&gs->gen.v) < b + 1) {
                if (w.stop(gs)) break;
            }
            fence_acquire();
#pragma unroll
            for (int i = 0; i < NSNAP; ++i) snap_out[i] = ld_rlx(&gs->snap[b & 1][i]);
        }
        snap_out[kNumCtr] = ld_rlx(&gs->error.v);
    }
    ++bar_no;
    __syncthreads();
    return snap_out[kNumCtr] == 0;
}

// Block-wide exclusive scan of one int per thread; `lds` holds
// kWavesPerBlock ints.  Returns the thread's prefix; `total` = block sum.
__device__ __forceinline__ int block_excl_scan(int x, int &total, int *lds) {
    const int w = threadIdx.x >> 6;
    int incl = wave_incl_scan(x);
    if (lane_id() == kWave - 1) lds[w] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
        int s = lds[i];
        before += i < w ? s : 0;
        total += s;
    }
    __syncthreads();
    return before + incl - x;
}

// Largest index o in [0, kBlock) with pre[o] <= t, for a non-decreasing LDS
// array pre with pre[0] = 0 (the item owning position t of a concatenation).
__device__ __forceinline__ int block_owner(const int *pre, int t) {
    int lo = 0;
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1)
        if (pre[lo + s] <= t) lo += s;
    return lo;
}

// LDS staging of one workgroup-wide row expansion.
struct ExpandLds {
    int pre[kBlock];
    long long e0[kBlock];
    int p0[kBlock];
    int p1[kBlock];
    int scan[kWavesPerBlock];
    long long scan_l[kWavesPerBlock];
};

// Workgroup-wide load-balanced expansion of up to kBlock adjacency rows, one
// per thread (length d, first entry e0, two ints of payload): a prefix sum of
// the lengths, then every thread takes R edges per step, each located by a
// binary search over the prefix sums.  f(act[R], u[R], owner[R]) is called
// by all threads together for each step; owner indexes the LDS payload.
template <int R, typename F>
__device__ __forceinline__ void block_expand(int d, long long e0, int p0, int p1,
                                             const int32_t *__restrict__ cols, ExpandLds &L, F &&f) {
    int total = 0;
    int pre = block_excl_scan(d, total, L.scan);
    L.pre[threadIdx.x] = pre;
    L.e0[threadIdx.x] = e0;
    L.p0[threadIdx.x] = p0;
    L.p1[threadIdx.x] = p1;
    __syncthreads();
    for (int t0 = 0; t0 < total; t0 += kBlock * R) {
        bool act[R];
        int u[R], own[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int t = t0 + r * kBlock + (int)threadIdx.x;
            act[r] = t < total;
            int o = block_owner(L.pre, act[r] ? t : total - 1);
            own[r] = o;
            u[r] = act[r] ? cols[L.e0[o] + (t - L.pre[o])] : 0;
        }
        f(act, u, own);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Edge-balanced rounds.  A frontier list holds, per entry i, a vertex id, the
// entry's start es[i] in the concatenation of the entries' adjacency rows
// (non-decreasing in i) and the row's first CSR position rs[i].  A round
// gives every workgroup an equal contiguous slice of the concatenated edges,
// whatever the row lengths; each step loads the entries covering the next
// kBlock * R edges into LDS and locates every edge's entry by binary search.

constexpr int kEbR = 8;                   // edges per thread per step
constexpr int kEbWin = kBlock * kEbR;     // edges per step
constexpr int kEbEnt = 1024;              // frontier entries per LDS window
struct EbLds {
    int id[kEbEnt + 1];
    long long es[kEbEnt + 1];  // es[w]: start of the first entry past the window
    long long rs[kEbEnt + 1];
    int p0[kEbEnt + 1];
    int p1[kEbEnt + 1];
    long long next;
};

// Largest j in [0, w) with es[j] <= x (es non-decreasing, es[0] <= x).
__device__ __forceinline__ int lds_owner(const long long *es, int w, long long x) {
    int lo = 0, hi = w;  // invariant: es[lo] <= x, answer in [lo, hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (es[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Process edges [e_lo, e_hi) of the concatenation of entries [q0, q1), this
// workgroup's share being an equal slice.  P0/P1 (may be null) are per-entry
// payloads copied to LDS; aux (may be null) is a per-edge array read beside
// cols.  f(act[kEbR], u[kEbR], own[kEbR], L, aux[kEbR]) is called by all
// threads together for each step; own indexes L's entry arrays.
template <typename F>
__device__ __forceinline__ void edge_balanced(const int32_t *__restrict__ ids,
                                              const long long *__restrict__ es,
                                              const long long *__restrict__ rs,
                                              const int32_t *__restrict__ P0,
                                              const int32_t *__restrict__ P1, long long q0, long long q1,
                                              long long e_lo, long long e_hi,
                                              const int32_t *__restrict__ cols,
                                              const int32_t *__restrict__ aux, EbLds &L, F &&f) {
    const long long span = e_hi - e_lo;
    const long long lo = e_lo + span * (long long)blockIdx.x / (long long)gridDim.x;
    const long long hi = e_lo + span * (long long)(blockIdx.x + 1) / (long long)gridDim.x;
    if (lo >= hi) return;  // uniform across the workgroup
    {
        // largest i in [q0, q1) with es[i] <= lo, by the whole workgroup: each
        // pass reads kBlock evenly spaced entries of the bracket [a, b) at once
        // and keeps the gap between the last sample <= lo and the next one, so
        // a list of up to 2^24 entries takes three dependent reads, not 24
        long long a = q0, b = q1;
        while (b - a > 1) {
            const long long span = b - a;
            const long long p = a + span * (long long)threadIdx.x / kBlock;
            const int below = __syncthreads_count(es[p] <= lo);  // samples <= lo: a prefix, sample 0 is a
            const long long na = a + span * (long long)(below - 1) / kBlock;
            if (below < kBlock) b = a + span * (long long)below / kBlock;
            a = na;
        }
        if (threadIdx.x == 0) L.next = a;
    }
    __syncthreads();
    // Window size: about twice the entries one step of kEbWin edges covers at
    // the round's mean row length.  A step ends at the window's end, so any
    // size is correct; with long rows a short window saves most of the loads
    // (UpdateHisto on RMAT-22 averages about 430 edges per entry).
    int wcap = kEbEnt;
    if (q1 > q0 && e_hi > e_lo) {
        const long long want = 2 * (long long)kEbWin * (q1 - q0) / (e_hi - e_lo) + 32;
        wcap = want < (long long)kEbEnt ? (int)want : kEbEnt;
    }
    long long i0 = L.next;
    for (long long s0 = lo; s0 < hi;) {
        // the window: up to wcap entries from the one holding s0, and the
        // start of the entry after them, which bounds the edges this step
        // may take (every entry holds at least one edge, so it lies past s0)
        const int w = (int)(q1 - i0 < (long long)wcap ? q1 - i0 : (long long)wcap);
        for (int j = threadIdx.x; j <= w; j += kBlock) {
            long long i = i0 + j;
            if (j < w) {
                L.id[j] = ids[i];
                L.es[j] = es[i];
                L.rs[j] = rs[i];
                L.p0[j] = P0 ? P0[i] : 0;
                L.p1[j] = P1 ? P1[i] : 0;
            } else {
                L.es[j] = i < q1 ? es[i] : LLONG_MAX;
            }
        }
        __syncthreads();
        long long we = s0 + kEbWin < hi ? s0 + kEbWin : hi;
        if (L.es[w] < we) we = L.es[w];
        bool act[kEbR];
        int u[kEbR], own[kEbR], ax[kEbR];
#pragma unroll
        for (int r = 0; r < kEbR; ++r) {
            long long x = s0 + r * kBlock + threadIdx.x;
            act[r] = x < we;
            int j = lds_owner(L.es, w, act[r] ? x : s0);
            own[r] = j;
            long long e = L.rs[j] + (x - L.es[j]);
            u[r] = act[r] ? cols[e] : 0;
            ax[r] = (act[r] && aux) ? aux[e] : 0;
        }
        f(act, u, own, L, ax);
        __syncthreads();
        if (threadIdx.x == 0 && we < hi) L.next = i0 + lds_owner(L.es, w + 1, we);
        __syncthreads();
        i0 = L.next;
        s0 = we;
    }
}

__device__ __forceinline__ long long wave_incl_scan64(long long x) {
    const int lane = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// 64-bit block-wide exclusive scan; `lds` holds kWavesPerBlock long longs.
__device__ __forceinline__ long long block_excl_scan64(long long x, long long &total, long long *lds) {
    const int w = threadIdx.x >> 6;
    long long incl = wave_incl_scan64(x);
    if (lane_id() == kWave - 1) lds[w] = incl;
    __syncthreads();
    long long before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
        long long s = lds[i];
        before += i < w ? s : 0;
        total += s;
    }
    __syncthreads();
    return before + incl - x;
}

// Frontier lists whose slot and edge-space reservations must stay in the same
// order share one 64-bit counter: (edges << kSlotBits) | slots.
constexpr int kSlotBits = 31;
constexpr unsigned long long kSlotMask = (1ull << kSlotBits) - 1;

// Wave-aggregated append of (id, row start rs, row length d) to a frontier
// list with a packed counter; entries land at index (slot - slot_base).
__device__ __forceinline__ void wave_push_packed(bool pred, int id, long long rs, long long d,
                                                 unsigned long long *ctr,
                                                 unsigned long long slot_base, int32_t *ids,
                                                 long long *es, long long *rsa) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    if (!pred) d = 0;
    long long dpre = wave_incl_scan64(d) - d;
    long long dtot = __shfl(dpre + d, kWave - 1);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long old = 0;
    if (lane_id() == leader)
        old = atomicAdd(ctr, ((unsigned long long)dtot << kSlotBits) | (unsigned long long)__popcll(mask));
    old = __shfl(old, leader);
    if (pred) {
        unsigned long long i = (old & kSlotMask) + lane_rank(mask) - slot_base;
        ids[i] = id;
        es[i] = (long long)(old >> kSlotBits) + dpre;
        rsa[i] = rs;
    }
}

// One atomic per block: reserve `total` slots of a counter; all threads get
// the base.  `lds64` is one LDS word.
__device__ __forceinline__ unsigned long long block_reserve(int total, unsigned long long *ctr,
                                                            unsigned long long *lds64) {
    if (threadIdx.x == 0) lds64[0] = total ? atomicAdd(ctr, (unsigned long long)total) : 0ull;
    __syncthreads();
    unsigned long long b = lds64[0];
    __syncthreads();
    return b;
}

__device__ __forceinline__ int block_min(int x, int *lds) {
    x = wave_min(x);
    if (lane_id() == 0) lds[threadIdx.x >> 6] = x;
    __syncthreads();
    int r = lds[0];
#pragma unroll
    for (int i = 1; i < kWavesPerBlock; ++i) r = min(r, lds[i]);
    __syncthreads();
    return r;
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

// Cooperative launch of a persistent kernel: the largest co-resident grid
// (capped at `max_per_cu` blocks per compute unit), or `want` blocks if that
// is smaller (want <= 0: no cap).  Returns the grid size used in *blocks.
int persistent_grid(const void *kernel, int block, int max_per_cu, long long want, int *blocks);

// Workgroups a persistent launch asks for on a graph of m entries (0: the
// whole device).  Below a few million entries the grid barriers, not the
// edge work, decide the time, and a smaller grid makes each barrier cheaper.
// The bounds come from a sweep of grid sizes on MI355X over ER and R-MAT
// graphs of 8 thousand to 7.6 million entries (PeelOne best at 16-64
// workgroups there, HistoCore at about m / 2048 up to one per CU).
inline long long clamp_ll(long long x, long long lo, long long hi) { return x < lo ? lo : (x > hi ? hi : x); }
inline long long grid_want_peelone(int64_t m) { return m >= (1ll << 23) ? 0 : clamp_ll(m >> 14, 16, 64); }
inline long long grid_want_histocore(int64_t m) { return m >= (1ll << 23) ? 0 : clamp_ll(m >> 11, 8, 256); }

// Wall-clock ticks for `seconds` (device wall clock rate).
unsigned long long wall_ticks(double seconds);

// Integer tuning knob read once from the environment (default if unset).
int tune_int(const char *name, int dflt);
// The same for knobs where 0 is meaningful (default if unset or negative).
int tune_int_nonneg(const char *name, int dflt);

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

// mode: 0 = Alg. 4 (assertion, dynamic frontier); 1 = no dynamic frontier;
// 2 = fetch-and-add rollback decrement; 3 = General Parallel Peel (the
// paper's comparison variants).
// sched (optional, device): one record per non-empty level, the first
// sched_cap of them; *sched_len (optional, host) gets the level count.
template <typename Off>
int run_peelone(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out,
                void *ws, size_t ws_bytes, pico_stats *st, hipStream_t stream, int mode = 0,
                pico_step *sched = nullptr, int64_t sched_cap = 0, int64_t *sched_len = nullptr);

size_t batched_ws_bytes(int64_t G, int64_t total_n, int64_t total_m, int algo);

// Choice between PeelOne and HistoCore (PICO_ALGO_AUTO): features measured on
// the device -- feat[0] the degree h-index, feat[1] vertices sampled,
// feat[2] of those in HistoCore's first frontier -- and the rule over them.
size_t select_ws_bytes(int64_t n, int64_t m);
template <typename Off>
int select_features(const Off *off, const int32_t *cols, int64_t n, int64_t m, void *ws, size_t ws_bytes,
                    hipStream_t stream, int64_t feat[3]);
int choose_algo(int64_t n, int64_t m, int64_t H, int64_t sampled, int64_t in_frontier);

// One graph by one workgroup, vertex values in LDS (graphs small enough that
// grid barriers would dominate).  small_path decides from n, m and the path
// flags of algo; run_small runs it.
size_t small_ws_bytes(int64_t n, int64_t m, int algo);
int small_path(int64_t n, int64_t m, int algo, bool *use);
template <typename Off>
int run_small(const Off *off, const int32_t *cols, int64_t n, int64_t m, int algo, int32_t *out,
              void *ws, size_t ws_bytes, pico_stats *stats, hipStream_t stream,
              const int32_t *warm = nullptr, int warm_add = 0);
size_t task_scratch_bytes(int64_t n, int64_t m, int algo);
size_t tasks_ws_bytes(int64_t T);
pico_task *tasks_table(void *ws, size_t ws_bytes, int64_t T);
// The per-graph status words at the start of a batched or task-list
// workspace (PICO_EHIP until finished, then PICO_OK; PICO_EINVAL for an
// invalid packed graph).
const int32_t *status_words(const void *ws);
// n_large: how many tasks will take helpers (help_min_large); the grid gets a
// few extra workgroups for each.
int run_tasks_device(const pico_task *dev_tasks, int64_t T, int algo, void *ws, size_t ws_bytes,
                     const pico_batch_tune *tune, pico_batch_stats *stats, hipStream_t stream,
                     int64_t n_large);
// vertex count from which a PeelOne task takes helpers (0 = never)
int help_min_large(const pico_batch_tune *tune, int algo);
int check_device();
size_t ws_bytes_for(int64_t n, int64_t m, int algo);


int run_batched(const long long *vptr, const long long *off, const int32_t *cols, int64_t G,
                int64_t total_n, int64_t total_m, int algo, const int32_t *order, int32_t *out,
                void *ws, size_t ws_bytes, const pico_batch_tune *tune, pico_batch_stats *stats,
                hipStream_t stream);

// CntCore (cnt_mode 1) or NbrCore (0): Index2core with every h-index rebuilt
// from the neighbours' values, the baselines of the paper's Table VI.
size_t index2core_ws_bytes(int64_t n, int64_t m);
template <typename Off>
int run_index2core(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out, void *ws,
                   size_t ws_bytes, pico_stats *stats, hipStream_t stream, int cnt_mode);

// warm (optional): start from these upper bounds of the coreness, plus
// warm_add, instead of the degrees.
// sched / sched_cap / sched_len: as run_peelone, one record per round.
template <typename Off>
int run_histocore(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out,
                  void *ws, size_t ws_bytes, pico_stats *st, hipStream_t stream,
                  const int32_t *warm = nullptr, int warm_add = 0, pico_step *sched = nullptr,
                  int64_t sched_cap = 0, int64_t *sched_len = nullptr);

inline int grid_for(int64_t items_per_block_units, int cap) {
    int64_t g = items_per_block_units;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace pico
