// HistoCore (paper Section IV-B, Alg. 6) for gfx950, as one persistent
// cooperative kernel per decomposition.
//
// Index2core (Section II-A, Alg. 2): every vertex starts at its degree and
// repeatedly replaces its estimate by the h-index of its neighbours'
// estimates; the fixed point is the coreness.  HistoCore keeps, per vertex,
// a histogram of the neighbours' current estimates, so a vertex that changes
// many times never re-reads its adjacency to recompute its h-index.
//
// Histogram layout: bucket b (1 <= b <= deg(v)) of vertex v lives at
// histo[off[v] + b - 1], so all histograms form one int32 array of m entries
// aligned with the adjacency array.  For b < core[v] the bucket counts
// neighbours whose estimate is exactly b; bucket core[v] counts neighbours
// whose estimate is >= core[v], which is cnt(v) of Theorem 2; buckets above
// core[v] are dead.  Every bucket index used is in [1, core[v]] with
// core[v] <= deg(v), so all accesses stay inside v's segment.
//
// Phases, separated by grid barriers so that each round sees the previous
// round's values (synchronous rounds):
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
//
// Edge balance.  Frontier entries record where their rows start in the
// concatenation of the round's rows (reserved with the entry's slot through
// one packed counter), so UpdateHisto gives every workgroup an equal slice of
// the round's edges, whatever the degrees.
#include <climits>

#include "common.hpp"

namespace pico {
namespace {

constexpr int kSmall = 16;     // lane-serial work up to this many items
constexpr int kLdsCap = 2048;  // InitHisto: LDS histogram per wave up to this degree
constexpr int kInitCh = 1024;  // InitHisto: edges per heavy piece
constexpr int kSumWave = 4096;  // SumHisto: one wave up to this value, a workgroup above
// Rounds whose frontier rows hold at least this share of m (in 1/1000)
// rebuild the histograms instead of running UpdateHisto.  Measured on
// MI355X: a rebuild costs about one InitHisto pass over the current values
// (RMAT-26: 41 ms, RMAT-22: 1.9 ms), an UpdateHisto round about 115 ps per
// histogram move, and moves run at 0.25-0.47 of a round's frontier edges;
// rebuilding paid in the rounds whose frontier rows held at least 0.65 of
// the entries (the first six or seven on RMAT-22 and RMAT-26) and lost in
// the next ones.
constexpr int kRebuildPermille = 640;

// Cumulative counters.  FET packs (edges << 31) | slots of the frontier lists.
enum { FET = 0, H_TAIL, HS_TAIL, N_MOVES, N_EDGES, N_BUCKETS };
constexpr int kSnap = 3;  // counters read at barriers: FET, H_TAIL, HS_TAIL

struct HcState {
    GridState g;
    Line rounds, first_frontier, frontier_total;
    Line moves_sched;  // histogram moves so far, flushed every round (schedule only)
    Line rebuilds;     // rounds that rebuilt the histograms instead of UpdateHisto
    Line phase[kNumPhases];
};

template <typename Off>
struct HcArgs {
    const Off *off;
    const int32_t *cols;
    long long n;
    int32_t *core;  // the caller's output array: estimates converge in place
    int32_t *histo;
    int32_t *ndeg;     // per adjacency entry: degree of the neighbour (written by InitHisto)
    int32_t *oldcore;
    int32_t *F[2];     // frontier ids, by round parity
    long long *FE[2];  // ... row start in the round's concatenated edge space
    long long *FR[2];  // ... first CSR position of the row
    int32_t *P0;       // per entry of the current round: new value
    int32_t *P1;       // ... old value
    int32_t *HS;       // ring of n: heavy InitHisto rows (vertex ids) / heavy sums (entries)
    long long *H;      // ring of hcap heavy InitHisto pieces (v << 32 | piece)
    long long hcap;
    HcState *st;
    unsigned long long limit;
    long long m;
    const int32_t *warm;  // upper bounds of the coreness to start from (nullptr: the degrees)
    int warm_add;         // added to every bound
    int rebuild_permille; // a round whose frontier rows hold >= this share of m (in 1/1000)
                          // rebuilds the histograms instead of UpdateHisto
    pico_step *sched;     // optional per-round schedule record (device), or null
    long long sched_cap;
    double ns_per_tick;   // device wall clock period
};

inline long long pieces_cap(int64_t m) { return m / kInitCh + m / kLdsCap + 64; }

__global__ void hc_state_init(HcState *st) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(st);
    const int words = (int)(sizeof(HcState) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0ull;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void flush_count(long long x, unsigned long long *dst) {
    long long t = wave_sum64(x);
    if (lane_id() == 0 && t) atomicAdd(dst, (unsigned long long)t);
}

__device__ __forceinline__ long long wave_id_global() {
    return (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
}

// Reverse summation by one wave over buckets top, top-1, ..., lowb (Step II
// of Fig. 6), starting from running sum `carry`.  Returns the first bucket b
// with carry + sum(b..top) >= b, with that sum, or h = 0 if none.
__device__ __forceinline__ void wave_reverse_sum(const int32_t *seg, int top, int lowb, int carry,
                                                 int &h, int &s) {
    const int lane = lane_id();
    h = 0;
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

// ---------------------------------------------------------------- InitHisto

// One wave counts entries [e0, e0 + d) of the adjacency into a histogram of
// c buckets (bucket min(core[u], c)) and records each neighbour's value in
// ndeg; four entries per lane in flight: their columns, then their values,
// then the counts.  Buckets up to `cap` are counted in the LDS array `lds`,
// higher ones (c > cap: hub rows at the start, valued by their degree) with
// atomics on the row's histogram `hrow` in memory.
template <typename Off>
__device__ __forceinline__ void count_row_lds(const HcArgs<Off> &a, long long e0, int d, int c, int *lds,
                                              int cap, int32_t *hrow) {
    constexpr int kR = 4;
    const int lane = lane_id();
    for (int j0 = 0; j0 < d; j0 += kR * kWave) {
        int x[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int j = j0 + r * kWave + lane;
            x[r] = j < d ? a.cols[e0 + j] : 0;
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int j = j0 + r * kWave + lane;
            x[r] = j < d ? a.core[x[r]] : 0;
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int j = j0 + r * kWave + lane;
            if (j < d) {
                a.ndeg[e0 + j] = x[r];
                const int b = min(max(x[r], 1), c);
                if (b <= cap) atomicAdd(&lds[b - 1], 1);
                else atomicAdd(&hrow[b - 1], 1);
            }
        }
    }
}

// Builds every vertex's histogram from its neighbours' current values and
// pushes {v : cnt(v) < core(v)} to frontier buffer `buf`.  At the start
// (rebuild false) a vertex's value is its degree, or its given bound; in a
// rebuild round (Jacobi round after SumHisto, in place of UpdateHisto) the
// values are the current estimates, below the degrees.
template <typename Off>
__device__ void init_histo(const HcArgs<Off> &a, int *lds, int *lds_scan, long long *lds_scan_l,
                           unsigned long long *lds64, int buf, bool rebuild) {
    GridState *gs = &a.st->g;
    const int lane = lane_id();
    // Block-uniform tiles of kBlock vertices (a wave takes 64 of them), so the
    // frontier pushes of a tile cost one atomic.
    for (long long tile = (long long)blockIdx.x * kBlock; tile < a.n;
         tile += (long long)gridDim.x * kBlock) {
        long long v = tile + threadIdx.x;
        bool valid = v < a.n;
        // c: v's value, its number of buckets; d: its neighbours (equal at a
        // cold start)
        int c = valid ? a.core[v] : 0;
        long long e0 = valid ? (long long)a.off[v] : 0;
        int d = valid && (a.warm || rebuild) ? (int)((long long)a.off[v + 1] - e0) : c;
        bool push = false;
        if (valid && d > 0 && d <= kSmall) {
            // one lane owns v's segment: all its columns, then all their
            // values, each group of loads in flight at once; the counts in
            // the lane's own LDS slots (no atomics), written out once
            int *h = lds + lane * (kSmall + 1);
            for (int j = 0; j < c; ++j) h[j] = 0;
            int x[kSmall];
#pragma unroll
            for (int j = 0; j < kSmall; ++j) x[j] = j < d ? a.cols[e0 + j] : 0;
#pragma unroll
            for (int j = 0; j < kSmall; ++j) x[j] = j < d ? a.core[x[j]] : 0;
#pragma unroll
            for (int j = 0; j < kSmall; ++j) {
                if (j < d) {
                    a.ndeg[e0 + j] = x[j];
                    h[min(max(x[j], 1), c) - 1] += 1;  // core[u] >= 1 on a symmetric graph
                }
            }
            for (int j = 0; j < c; ++j) a.histo[e0 + j] = h[j];
            push = h[c - 1] < c;
        }
        wave_lds_sync();  // the lanes' slots are done before the rows below reuse them
        unsigned long long mm = __ballot(valid && d > kSmall && d <= kLdsCap);
        while (mm) {
            int l = __ffsll(mm) - 1;
            mm &= mm - 1;
            int dd = __shfl(d, l), cc = __shfl(c, l);
            long long ea = __shfl(e0, l);
            for (int j = lane; j < cc; j += kWave) lds[j] = 0;
            wave_lds_sync();
            count_row_lds(a, ea, dd, cc, lds, cc, a.histo + ea);
            wave_lds_sync();
            for (int j = lane; j < cc; j += kWave) a.histo[ea + j] = lds[j];
            int top = lds[cc - 1];
            wave_lds_sync();
            if (lane == l) push = top < cc;
        }
        int tot = 0;
        long long etot = 0;
        int pre = block_excl_scan(push ? 1 : 0, tot, lds_scan);
        long long epre = block_excl_scan64(push ? (long long)d : 0ll, etot, lds_scan_l);
        if (threadIdx.x == 0)
            lds64[0] = tot ? atomicAdd(&gs->ctr[FET].v, ((unsigned long long)etot << kSlotBits) |
                                                            (unsigned long long)tot)
                           : 0ull;
        __syncthreads();
        const unsigned long long old = lds64[0];
        __syncthreads();
        if (push) {
            unsigned long long i = (old & kSlotMask) + pre;
            a.F[buf][i] = (int)v;
            a.FE[buf][i] = (long long)(old >> kSlotBits) + epre;
            a.FR[buf][i] = e0;
        }
        bool hv = valid && d > kLdsCap;
        long long t = wave_append(hv, &gs->ctr[HS_TAIL].v);
        if (hv) {
            a.HS[t % a.n] = (int)v;  // a ring: the counter runs on over rounds
            long long np = ((long long)d + kInitCh - 1) / kInitCh;
            unsigned long long b = atomicAdd(&gs->ctr[H_TAIL].v, (unsigned long long)np);
            for (long long j = 0; j < np; ++j) a.H[(b + j) % a.hcap] = (v << 32) | j;
        }
    }
}

// Heavy InitHisto rows, piece by piece: zero (pass 0) or count (pass 1).
// A piece's buckets up to kLdsCap are counted in the wave's LDS histogram
// and added to the row with one atomic per non-empty bucket (in rebuild
// rounds a hub's value, hence every bucket, is usually below kLdsCap; at the
// start its value is its degree but most of its neighbours' are small); the
// buckets above, one atomic per entry.
template <typename Off>
__device__ void init_heavy(const HcArgs<Off> &a, unsigned long long h0, unsigned long long h1,
                           int pass, int *lds) {
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    const int lane = lane_id();
    for (long long p = (long long)h0 + wave_id_global(); p < (long long)h1; p += nw) {
        long long desc = a.H[p % a.hcap];
        int v = (int)(desc >> 32);
        long long j = desc & 0xffffffffll;
        long long vb = (long long)a.off[v], ve = (long long)a.off[v + 1];
        const int c = a.core[v];  // buckets (the degree unless started from bounds)
        long long e0 = vb + j * kInitCh, e1 = e0 + kInitCh < ve ? e0 + kInitCh : ve;
        if (pass == 0) {
            for (long long e = e0 + lane; e < e1; e += kWave) a.histo[e] = 0;
        } else {
            const int cap = c < kLdsCap ? c : kLdsCap;
            for (int b = lane; b < cap; b += kWave) lds[b] = 0;
            wave_lds_sync();
            count_row_lds(a, e0, (int)(e1 - e0), c, lds, cap, a.histo + vb);
            wave_lds_sync();
            for (int b = lane; b < cap; b += kWave) {
                const int x = lds[b];
                if (x) atomicAdd(&a.histo[vb + b], x);
            }
            wave_lds_sync();
        }
    }
}

template <typename Off>
__device__ void init_heavy_check(const HcArgs<Off> &a, unsigned long long s0, unsigned long long s1, int buf) {
    GridState *gs = &a.st->g;
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    for (long long base = (long long)s0 + wave_id_global() * kWave; base < (long long)s1;
         base += nw * kWave) {
        long long i = base + lane_id();
        bool push = false;
        int v = 0, d = 0;
        long long rs = 0;
        if (i < (long long)s1) {
            v = a.HS[i % a.n];
            const int c = a.core[v];
            rs = (long long)a.off[v];
            d = (int)((long long)a.off[v + 1] - rs);  // the row, for the round's edge space
            push = a.histo[rs + c - 1] < c;
        }
        wave_push_packed(push, v, rs, d, &gs->ctr[FET].v, 0, a.F[buf], a.FE[buf], a.FR[buf]);
    }
}

// ---------------------------------------------------------------- SumHisto

// Entry i of the round's frontier: the new value goes to core and P0[i], the
// old one to oldcore and P1[i].
template <typename Off>
__device__ void sum_histo(const HcArgs<Off> &a, const int32_t *F, const long long *FR, long long nf,
                          long long &nb) {
    GridState *gs = &a.st->g;
    const int lane = lane_id();
    const long long nw = (long long)gridDim.x * kWavesPerBlock;
    // Entries per wave per step: 64, or fewer when the frontier would leave
    // waves idle, so that the values a wave scans one after another (below)
    // are spread over every wave of the grid.
    const int per = nf >= nw * kWave ? kWave : (int)((nf + nw - 1) / nw);
    for (long long base = wave_id_global() * per; base < nf; base += nw * per) {
        long long i = base + lane;
        bool valid = lane < per && i < nf;
        int v = 0, c_old = 0;
        long long e0 = 0;
        if (valid) {
            v = F[i];
            c_old = a.core[v];
            e0 = FR[i];
        }
        if (valid && c_old <= kSmall) {
            int s = 0, k = c_old;
            for (; k >= 1; --k) {
                s += a.histo[e0 + k - 1];
                if (s >= k) break;
            }
            if (k < 1) k = 0;  // unreachable for a symmetric simple graph
            a.core[v] = k;
            a.oldcore[v] = c_old;
            a.P0[i] = k;
            a.P1[i] = c_old;
            if (k >= 1) a.histo[e0 + k - 1] = s;
            nb += c_old - max(k, 1) + 1;
        }
        unsigned long long mm = __ballot(valid && c_old > kSmall && c_old <= kSumWave);
        while (mm) {
            int l = __ffsll(mm) - 1;
            mm &= mm - 1;
            int vv = __shfl(v, l), cc = __shfl(c_old, l);
            long long ea = __shfl(e0, l);
            long long ii = __shfl(i, l);
            int h, s;
            wave_reverse_sum_wide(a.histo + ea, cc, h, s);
            if (lane == 0) {
                a.core[vv] = h;
                a.oldcore[vv] = cc;
                a.P0[ii] = h;
                a.P1[ii] = cc;
                if (h >= 1) a.histo[ea + h - 1] = s;
                nb += cc - max(h, 1) + 1;
            }
        }
        bool hv = valid && c_old > kSumWave;
        long long t = wave_append(hv, &gs->ctr[HS_TAIL].v);
        if (hv) a.HS[t % a.n] = (int)i;
    }
}

// SumHisto for large old values: a workgroup per frontier entry.  Each
// thread sums one slice of the bucket range; carry + sum(b..top) - b falls
// strictly as b grows, so the running sums at slice bottoms locate the slice
// holding the answer, and one wave finishes inside it.
template <typename Off>
__device__ void sum_heavy(const HcArgs<Off> &a, const int32_t *F, const long long *FR,
                          unsigned long long s0, unsigned long long s1, int *part, int *first_ok) {
    GridState *gs = &a.st->g;
    const int t = threadIdx.x;
    for (long long j = (long long)s0 + blockIdx.x; j < (long long)s1; j += gridDim.x) {
        const int i = a.HS[j % a.n];
        int v = F[i];
        int c_old = a.core[v];
        long long e0 = FR[i];
        const int32_t *seg = a.histo + e0;
        int L = (c_old + kBlock - 1) / kBlock;
        int hi_b = c_old - t * L;
        int lo_b = max(1, hi_b - L + 1);
        int sum = 0;
        for (int b = hi_b; b >= lo_b; --b) sum += seg[b - 1];
        part[t] = sum;
        if (t == 0) *first_ok = kBlock;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            int y = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += y;
            __syncthreads();
        }
        if (hi_b >= 1 && part[t] >= lo_b) atomicMin(first_ok, t);
        __syncthreads();
        int ts = *first_ok;
        if (ts < kBlock && (t >> 6) == 0) {
            int top = c_old - ts * L;
            int lowb = max(1, top - L + 1);
            int carry = ts > 0 ? part[ts - 1] : 0;
            int h, s;
            wave_reverse_sum(seg, top, lowb, carry, h, s);
            if (t == 0) {
                a.core[v] = h;
                a.oldcore[v] = c_old;
                a.P0[i] = h;
                a.P1[i] = c_old;
                if (h >= 1) a.histo[e0 + h - 1] = s;
                atomicAdd(&gs->ctr[N_BUCKETS].v, (unsigned long long)(c_old - max(h, 1) + 1));
            }
        } else if (ts >= kBlock && t == 0) {
            a.core[v] = 0;  // unreachable for a symmetric simple graph
            a.oldcore[v] = c_old;
            a.P0[i] = 0;
            a.P1[i] = c_old;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- UpdateHisto

// kEbR edges (v, u) of UpdateHisto per thread, all threads together: the
// neighbour values, then the offsets of the neighbours that move, then the
// histogram updates, each for all edges before any result is used.  A
// neighbour whose cnt falls below its value joins the next frontier.
template <typename Off>
__device__ __forceinline__ void hc_relax(const bool (&act0)[kEbR], const int (&u)[kEbR],
                                         const int (&cv)[kEbR], const int (&ov)[kEbR],
                                         const int (&du)[kEbR], const HcArgs<Off> &a, int nxt,
                                         unsigned long long fbase, long long &nmove) {
    GridState *gs = &a.st->g;
    // A neighbour of degree <= cv has core[u] <= deg(u) <= cv: never moved.
    bool act[kEbR];
#pragma unroll
    for (int r = 0; r < kEbR; ++r) act[r] = act0[r] && du[r] > cv[r];
    int cu[kEbR];
#pragma unroll
    for (int r = 0; r < kEbR; ++r) cu[r] = act[r] ? a.core[u[r]] : 0;
    bool mv[kEbR];
    long long hb[kEbR];
#pragma unroll
    for (int r = 0; r < kEbR; ++r) {
        mv[r] = act[r] && cu[r] > cv[r] && cv[r] >= 1;
        hb[r] = mv[r] ? (long long)a.off[u[r]] - 1 : 0;
    }
    bool push[kEbR];
#pragma unroll
    for (int r = 0; r < kEbR; ++r) {
        push[r] = false;
        if (mv[r]) {
            // v moves from bucket src = min(oldcore[v], core[u]) of u to bucket
            // cv.  When the two are neighbours in one aligned 8-byte word (in
            // the rounds after the rebuild rounds values fall by one per
            // round, so every move is between neighbouring buckets, half of
            // them so aligned), one 64-bit add of +1 to the low half and -1
            // to the high half does both: the low count cannot carry out and
            // the high one is >= 1 (v is counted there).  The old high half
            // is the old count of src, which the crossing test needs.
            const bool top = ov[r] >= cu[r];
            const int src = top ? cu[r] : ov[r];
            const long long lo = hb[r] + cv[r];  // bucket cv's position
            if (src == cv[r] + 1 && (lo & 1) == 0) {
                const unsigned long long old =
                    atomicAdd(reinterpret_cast<unsigned long long *>(a.histo + lo), 0xffffffff00000001ull);
                push[r] = top && (int)(old >> 32) == cu[r];
            } else {
                if (top) {
                    // v leaves u's top bucket: the only case whose old count matters
                    int c = atomicSub(&a.histo[hb[r] + cu[r]], 1);
                    push[r] = c == cu[r];
                } else {
                    atomicSub(&a.histo[hb[r] + ov[r]], 1);  // no return value needed
                }
                atomicAdd(&a.histo[lo], 1);
            }
            ++nmove;
        }
    }
#pragma unroll
    for (int r = 0; r < kEbR; ++r) {
        long long rs = hb[r] + 1, d = 0;
        if (push[r]) d = (long long)a.off[u[r] + 1] - rs;
        wave_push_packed(push[r], u[r], rs, d, &gs->ctr[FET].v, fbase, a.F[nxt], a.FE[nxt],
                         a.FR[nxt]);
    }
}

// InitHisto's per-wave histograms and UpdateHisto's edge window are used in
// different phases: one LDS block serves both.
union HcLds {
    int hist[kWavesPerBlock][kLdsCap];
    EbLds eb;
};

// At most 128 VGPRs, so that four workgroups share a compute unit: the
// histogram moves are memory-side atomics, and more waves in flight raise
// their rate (RMAT-26: 891 ms at two workgroups per CU, 792 at three, 769 at
// four).
template <typename Off>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void hc_persistent(HcArgs<Off> a) {
    __shared__ HcLds U;
    __shared__ int part[kBlock];
    __shared__ int first_ok;
    __shared__ int lds_scan[kWavesPerBlock];
    __shared__ long long lds_scan_l[kWavesPerBlock];
    __shared__ unsigned long long lds64[1];
    __shared__ unsigned long long snap[kNumCtr + 1];
    EbLds &eb = U.eb;
    HcState *st = a.st;
    GridState *gs = &st->g;
    const unsigned nb = gridDim.x;
    long long nmove = 0, nedge = 0, nbuck = 0;
    unsigned long long bar = 0;
    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    PhaseClock clk;
    if (timer) clk.start();

    // core = deg, or the given upper bound capped by the degree (at least 1
    // on a vertex with neighbours, whose coreness is at least 1)
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < a.n;
         v += (long long)gridDim.x * kBlock) {
        const int d = (int)(a.off[v + 1] - a.off[v]);
        int c = d;
        if (a.warm && d > 0) {
            const long long w = (long long)a.warm[v] + a.warm_add;
            c = (int)(w < 1 ? 1 : (w > d ? d : w));
        }
        a.core[v] = c;
    }
    if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
    if (timer) clk.lap(&st->phase[0].v);
    // InitHisto, and in rebuild rounds the same pass over current values:
    // rows up to kLdsCap in this pass, longer ones in pieces after it
    // (cleared, then counted), then their frontier test.  Heavy-row lists are
    // rings indexed by running counters, so every pass starts where the
    // previous one ended.
    auto build_histograms = [&](int buf, bool rebuild) -> bool {
        const unsigned long long h0 = snap[H_TAIL], hs0 = snap[HS_TAIL];
        init_histo<Off>(a, U.hist[threadIdx.x >> 6], lds_scan, lds_scan_l, lds64, buf, rebuild);
        if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return false;
        const unsigned long long h1 = snap[H_TAIL], hs1 = snap[HS_TAIL];
        init_heavy<Off>(a, h0, h1, 0, U.hist[threadIdx.x >> 6]);
        if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return false;
        init_heavy<Off>(a, h0, h1, 1, U.hist[threadIdx.x >> 6]);
        if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return false;
        init_heavy_check<Off>(a, hs0, hs1, buf);
        return grid_sync<kSnap>(gs, nb, a.limit, snap, bar);
    };
    if (!build_histograms(0, false)) return;
    if (timer) clk.lap(&st->phase[1].v);

    // Round r's frontier: entries [0, nf) of buffer r & 1, edge space [0, e1).
    // The packed counter restarts from zero every round (block 0 clears it
    // before SumHisto; the next pushes come after two more barriers), so its
    // fields hold one round's slots (<= n) and edges (<= m), not running sums
    // over all rounds, which would outgrow the edge field on large graphs.
    long long nf = (long long)(snap[FET] & kSlotMask);
    unsigned long long e1 = snap[FET] >> kSlotBits;
    const long long first = nf;
    long long rounds = 0, ftotal = 0, nrebuild = 0;
    long long nmove_flushed = 0;          // this thread's moves already in moves_sched
    unsigned long long moves_seen = 0;    // block 0: moves_sched at the last record
    for (int r = 0; nf > 0; ++r) {
        const int cur = r & 1, nxt = cur ^ 1;
        const unsigned long long t_round = timer ? wall_clock64() : 0ull;
        const long long e_round = (long long)e1;
        ++rounds;
        ftotal += nf;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(&gs->ctr[FET].v, 0ull);
        const unsigned long long hs0 = snap[HS_TAIL];
        sum_histo<Off>(a, a.F[cur], a.FR[cur], nf, nbuck);
        if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
        if (timer) clk.lap(&st->phase[2].v);
        sum_heavy<Off>(a, a.F[cur], a.FR[cur], hs0, snap[HS_TAIL], part, &first_ok);
        if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
        if (timer) clk.lap(&st->phase[3].v);
        const unsigned long long t_sum = timer ? wall_clock64() : 0ull;
        const unsigned long long fnext = snap[FET] & kSlotMask;  // 0: cleared this round
        // A round whose frontier rows cover a large share of the adjacency
        // rebuilds every histogram from the current values instead (one
        // InitHisto pass: a gather per entry and LDS counting, against two
        // memory-side atomics per moved entry).  It leaves the histograms
        // UpdateHisto would (bucket b < core[u] counts neighbours valued b,
        // bucket core[u] those valued >= core[u]) and the same next frontier:
        // every vertex has cnt >= core when UpdateHisto starts and cnt only
        // falls during it, so the vertices it would push are exactly those
        // with cnt < core after it.
        const bool rebuild = (unsigned long long)e_round * 1000ull >= (unsigned long long)a.rebuild_permille *
                                                                           (unsigned long long)a.m;
        if (rebuild) {
            nedge += (blockIdx.x == 0 && threadIdx.x == 0) ? a.m : 0;
            if (!build_histograms(nxt, true)) return;
            ++nrebuild;
            if (timer) clk.lap(&st->phase[5].v);
        } else {
            nedge += (blockIdx.x == 0 && threadIdx.x == 0) ? (long long)e1 : 0;
            edge_balanced(a.F[cur], a.FE[cur], a.FR[cur], a.P0, a.P1, 0, nf, 0ll, (long long)e1,
                          a.cols, a.ndeg, eb,
                          [&](const bool (&act)[kEbR], const int (&u)[kEbR], const int (&own)[kEbR],
                              EbLds &L, const int (&du)[kEbR]) {
                              int cvr[kEbR], ovr[kEbR];
#pragma unroll
                              for (int q = 0; q < kEbR; ++q) {
                                  cvr[q] = L.p0[own[q]];
                                  ovr[q] = L.p1[own[q]];
                              }
                              hc_relax<Off>(act, u, cvr, ovr, du, a, nxt, fnext, nmove);
                          });
            if (a.sched) {  // this round's moves, for the schedule record
                flush_count(nmove - nmove_flushed, &st->moves_sched.v);
                nmove_flushed = nmove;
            }
            if (!grid_sync<kSnap>(gs, nb, a.limit, snap, bar)) return;
            if (timer) clk.lap(&st->phase[4].v);
        }
        if (timer && a.sched && r < a.sched_cap) {
            pico_step *sp = a.sched + r;
            sp->key = r + 1;
            sp->vertices = nf;
            const unsigned long long mv = ld_rlx(&st->moves_sched.v);
            sp->work = (long long)(mv - moves_seen);
            moves_seen = mv;
            sp->edges = e_round;
            sp->rounds = 1;
            sp->ns = (long long)((double)(wall_clock64() - t_round) * a.ns_per_tick);
            sp->scan_ns = (long long)((double)(t_sum - t_round) * a.ns_per_tick);
            sp->kind = rebuild ? 1 : 0;
        }
        nf = (long long)((snap[FET] & kSlotMask) - fnext);
        e1 = snap[FET] >> kSlotBits;
    }
    flush_count(nmove, &gs->ctr[N_MOVES].v);
    flush_count(nedge, &gs->ctr[N_EDGES].v);
    flush_count(nbuck, &gs->ctr[N_BUCKETS].v);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rounds.v = (unsigned long long)rounds;
        st->first_frontier.v = (unsigned long long)first;
        st->frontier_total.v = (unsigned long long)ftotal;
        st->rebuilds.v = (unsigned long long)nrebuild;
    }
}


// ---------------------------------------------------------------- CntCore / NbrCore
//
// The Index2core baselines the paper measures HistoCore against (Section
// IV-A, Alg. 5, and Section V, Table VI), in synchronous rounds from the
// degrees, with every h-index rebuilt from the neighbours' values (Step I
// and Step II of Fig. 6 each time; no histogram carried between rounds):
//   CntCore -- round t counts, for each vertex of the active set A (all
//     vertices in the first round, afterwards the neighbours of the previous
//     frontier), cnt(v) = |{u in nbr(v) : core[u] >= core[v]}|; the frontier
//     is {v in A : cnt(v) < core[v]} (Theorem 2), and only it recomputes.
//   NbrCore -- every vertex of A recomputes; A is then the neighbours of the
//     vertices whose value changed.
// Per round: [cnt scan] -> frontier (+ clear its histogram rows) -> Step I
// -> Step II (SumHisto, shared with HistoCore) -> mark the neighbours of the
// changed vertices into the next active list.  All passes over adjacency are
// edge-balanced.

// Counter slots: the frontier list (FET) and heavy sums (HS_TAIL) and the
// bucket count (N_BUCKETS) keep HistoCore's positions, which SumHisto uses.
enum { IC_AET = H_TAIL, IC_ATOM = N_MOVES, IC_EDGES = N_EDGES };

template <typename Off>
struct IcArgs {
    HcArgs<Off> h;     // core (the output), histo, oldcore, frontier lists F[0]/FE[0]/FR[0], P0, P1, HS, st
    int32_t *cnt;      // per vertex
    int32_t *mark;     // per vertex: the round that last put it in the next active list
    int32_t *A[2];     // active lists, by round parity
    long long *AE[2];  // ... row start in the list's concatenated edge space
    long long *AR[2];  // ... first CSR position of the row
    int cnt_mode;      // 1: CntCore, 0: NbrCore
};

template <typename Off>
__global__ __launch_bounds__(kBlock) void ic_persistent(IcArgs<Off> a) {
    __shared__ int part[kBlock];
    __shared__ int first_ok;
    __shared__ unsigned long long snap[kNumCtr + 1];
    __shared__ EbLds eb;
    const HcArgs<Off> &h = a.h;
    HcState *st = h.st;
    GridState *gs = &st->g;
    const unsigned nb = gridDim.x;
    unsigned long long bar = 0;
    long long natom = 0, nbuck = 0, nedge = 0;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;

    // core = deg; every vertex with neighbours is active in the first round
    for (long long base = (long long)blockIdx.x * kBlock; base < h.n; base += (long long)gridDim.x * kBlock) {
        const long long v = base + threadIdx.x;
        int d = 0;
        long long rs = 0;
        if (v < h.n) {
            rs = (long long)h.off[v];
            d = (int)((long long)h.off[v + 1] - rs);
            h.core[v] = d;
            a.cnt[v] = 0;
            a.mark[v] = 0;
        }
        wave_push_packed(v < h.n && d > 0, (int)v, rs, d, &gs->ctr[IC_AET].v, 0, a.A[0], a.AE[0], a.AR[0]);
    }
    if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
    long long na = (long long)(snap[IC_AET] & kSlotMask);
    long long ea = (long long)(snap[IC_AET] >> kSlotBits);
    long long rounds_changed = 0, rounds_run = 0, active = 0, hidx = 0, activations = 0;
    for (int t = 1; na > 0; ++t) {
        const int cur = (t - 1) & 1, nxt = cur ^ 1;
        active += na;
        if (lead) {
            atomicExch(&gs->ctr[FET].v, 0ull);
            atomicExch(&gs->ctr[IC_AET].v, 0ull);  // the next list fills in the marking pass
        }
        if (a.cnt_mode) {  // cnt of every active vertex
            nedge += lead ? ea : 0;
            edge_balanced(a.A[cur], a.AE[cur], a.AR[cur], nullptr, nullptr, 0, na, 0ll, ea, h.cols, nullptr, eb,
                          [&](const bool (&act)[kEbR], const int (&u)[kEbR], const int (&own)[kEbR], EbLds &L,
                              const int (&)[kEbR]) {
#pragma unroll
                              for (int r = 0; r < kEbR; ++r) {
                                  if (!act[r]) continue;
                                  const int v = L.id[own[r]];
                                  if (h.core[u[r]] >= h.core[v]) {
                                      atomicAdd(&a.cnt[v], 1);
                                      ++natom;
                                  }
                              }
                          });
        }
        if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
        // the frontier, with its histogram rows (buckets 1..core[v]) cleared
        const int lane = lane_id();
        for (long long base = (long long)blockIdx.x * kBlock; base < na; base += (long long)gridDim.x * kBlock) {
            const long long i = base + threadIdx.x;
            int v = 0, c = 0;
            long long rs = 0, d = 0;
            bool in = false;
            if (i < na) {
                v = a.A[cur][i];
                rs = a.AR[cur][i];
                d = (long long)h.off[v + 1] - rs;
                c = h.core[v];
                in = a.cnt_mode ? a.cnt[v] < c : true;
            }
            if (in && c <= kSmall)
                for (int b = 0; b < c; ++b) h.histo[rs + b] = 0;
            unsigned long long mm = __ballot(in && c > kSmall);
            while (mm) {
                const int l = __ffsll(mm) - 1;
                mm &= mm - 1;
                const int cc = __shfl(c, l);
                const long long ra = __shfl(rs, l);
                for (int b = lane; b < cc; b += kWave) h.histo[ra + b] = 0;
            }
            wave_push_packed(in, v, rs, d, &gs->ctr[FET].v, 0, h.F[0], h.FE[0], h.FR[0]);
        }
        if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
        const long long nf = (long long)(snap[FET] & kSlotMask);
        const long long ef = (long long)(snap[FET] >> kSlotBits);
        if (nf == 0) break;  // CntCore: nobody changes
        ++rounds_run;
        hidx += nf;
        // Step I: bucket min(core[u], core[v]) of v counts neighbour u
        nedge += lead ? ef : 0;
        edge_balanced(h.F[0], h.FE[0], h.FR[0], nullptr, nullptr, 0, nf, 0ll, ef, h.cols, nullptr, eb,
                      [&](const bool (&act)[kEbR], const int (&u)[kEbR], const int (&own)[kEbR], EbLds &L,
                          const int (&)[kEbR]) {
                          int cu[kEbR];
#pragma unroll
                          for (int r = 0; r < kEbR; ++r) cu[r] = act[r] ? h.core[u[r]] : 0;
#pragma unroll
                          for (int r = 0; r < kEbR; ++r) {
                              if (!act[r]) continue;
                              const int cv = h.core[L.id[own[r]]];
                              const int b = min(max(cu[r], 1), cv);
                              atomicAdd(&h.histo[L.rs[own[r]] + b - 1], 1);
                              ++natom;
                          }
                      });
        if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
        // Step II: the new values (core, P0) and the old ones (oldcore, P1)
        const unsigned long long hs0 = snap[HS_TAIL];
        sum_histo<Off>(h, h.F[0], h.FR[0], nf, nbuck);
        if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
        sum_heavy<Off>(h, h.F[0], h.FR[0], hs0, snap[HS_TAIL], part, &first_ok);
        if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
        // the neighbours of the vertices that changed form the next active list
        long long emark = 0;
        edge_balanced(h.F[0], h.FE[0], h.FR[0], h.P0, h.P1, 0, nf, 0ll, ef, h.cols, nullptr, eb,
                      [&](const bool (&act)[kEbR], const int (&u)[kEbR], const int (&own)[kEbR], EbLds &L,
                          const int (&)[kEbR]) {
#pragma unroll
                          for (int r = 0; r < kEbR; ++r) {
                              bool first = false;
                              if (act[r] && L.p0[own[r]] != L.p1[own[r]]) {
                                  ++emark;
                                  first = atomicExch(&a.mark[u[r]], t) != t;
                                  if (first) a.cnt[u[r]] = 0;
                              }
                              long long rs = 0, d = 0;
                              if (first) {
                                  rs = (long long)h.off[u[r]];
                                  d = (long long)h.off[u[r] + 1] - rs;
                              }
                              wave_push_packed(first, u[r], rs, d, &gs->ctr[IC_AET].v, 0, a.A[nxt], a.AE[nxt],
                                               a.AR[nxt]);
                          }
                      });
        nedge += emark;
        if (!grid_sync<kSnap>(gs, nb, h.limit, snap, bar)) return;
        na = (long long)(snap[IC_AET] & kSlotMask);
        ea = (long long)(snap[IC_AET] >> kSlotBits);
        if (na > 0) ++rounds_changed;
        activations += na;
    }
    flush_count(natom, &gs->ctr[IC_ATOM].v);
    flush_count(nbuck, &gs->ctr[N_BUCKETS].v);
    flush_count(nedge, &gs->ctr[IC_EDGES].v);
    if (lead) {
        st->rounds.v = (unsigned long long)rounds_changed;
        st->first_frontier.v = (unsigned long long)rounds_run;
        st->frontier_total.v = (unsigned long long)hidx;
        st->phase[0].v = (unsigned long long)active;
        st->phase[1].v = (unsigned long long)activations;
    }
}
}  // namespace

size_t histocore_ws_bytes(int64_t n, int64_t m) {
    return carve_bytes(m, 4) * 2 + carve_bytes(n, 4) * 6 + carve_bytes(n, 8) * 4 +
           carve_bytes(pieces_cap(m), 8) + carve_bytes(1, sizeof(HcState));
}

template <typename Off>
int run_histocore(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out, void *ws,
                  size_t ws_bytes, pico_stats *stats, hipStream_t stream, const int32_t *warm,
                  int warm_add, pico_step *sched, int64_t sched_cap, int64_t *sched_len) {
    if ((unsigned long long)m >= (1ull << (64 - kSlotBits))) {
        set_error("m=%lld too large for the packed frontier counter", (long long)m);
        return PICO_ENOTSUP;
    }
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    HcArgs<Off> a;
    a.off = off;
    a.cols = cols;
    a.n = n;
    a.core = out;
    a.histo = cv.take<int32_t>(m);
    a.ndeg = cv.take<int32_t>(m);
    a.oldcore = cv.take<int32_t>(n);
    for (int b = 0; b < 2; ++b) {
        a.F[b] = cv.take<int32_t>(n);
        a.FE[b] = cv.take<long long>(n);
        a.FR[b] = cv.take<long long>(n);
    }
    a.P0 = cv.take<int32_t>(n);
    a.P1 = cv.take<int32_t>(n);
    a.HS = cv.take<int32_t>(n);
    a.hcap = pieces_cap(m);
    a.H = cv.take<long long>(a.hcap);
    a.st = cv.take<HcState>(1);
    if ((m > 0 && (!a.histo || !a.ndeg)) || !a.oldcore || !a.F[0] || !a.F[1] || !a.FE[0] || !a.FE[1] || !a.FR[0] ||
        !a.FR[1] || !a.P0 || !a.P1 || !a.HS || !a.H || !a.st) {
        set_error("HistoCore workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  histocore_ws_bytes(n, m));
        return PICO_ENOMEM;
    }
    a.limit = wall_ticks(20.0);
    a.m = m;
    a.warm = warm;
    a.warm_add = warm_add;
    a.rebuild_permille = tune_int("PICO_HC_REBUILD_PERMILLE", kRebuildPermille);
    a.sched = sched;
    a.sched_cap = sched ? sched_cap : 0;
    a.ns_per_tick = 1e9 / (double)wall_ticks(1.0);
    int blocks = 0;
    int rc = persistent_grid(reinterpret_cast<const void *>(hc_persistent<Off>), kBlock,
                             tune_int("PICO_HC_BLOCKS_PER_CU", 4), grid_want_histocore(m), &blocks);
    if (rc) return rc;
    PICO_LAUNCH("hc_state_init", hc_state_init, dim3(1), dim3(kBlock), stream, a.st);
    PICO_LAUNCH_CHECK();
    void *args[] = {&a};
    int rec = prof_begin("hc_persistent", stream);
    PICO_HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(hc_persistent<Off>),
                                            dim3(blocks), dim3(kBlock), args, 0, stream));
    prof_end(rec, stream);
    HcState *h = static_cast<HcState *>(host_scratch(sizeof(HcState)));
    if (!h) return PICO_EHIP;
    PICO_HIP_TRY(hipMemcpyAsync(h, a.st, sizeof(HcState), hipMemcpyDeviceToHost, stream));
    PICO_HIP_TRY(hipStreamSynchronize(stream));
    if (h->g.error.v) {
        set_error("HistoCore kernel stopped (error %llu; grid of %d blocks)",
                  (unsigned long long)h->g.error.v, blocks);
        return PICO_EHIP;
    }
    if (sched_len) *sched_len = (int64_t)h->rounds.v;
    if (stats) {
        stats->iterations = (int64_t)h->rounds.v;
        stats->sub_rounds = (int64_t)h->rounds.v;
        stats->scans = (int64_t)h->rebuilds.v;
        stats->frontier_total = (int64_t)h->frontier_total.v;
        stats->k_max = 0;
        stats->edges_scanned = (int64_t)h->g.ctr[N_EDGES].v;
        stats->atomics = (int64_t)h->g.ctr[N_MOVES].v;
        stats->buckets_scanned = (int64_t)h->g.ctr[N_BUCKETS].v;
        stats->pushes_dynamic = (int64_t)(h->frontier_total.v - h->first_frontier.v);
        const double tick_ms = 1.0 / (double)wall_ticks(1e-3);
        for (int i = 0; i < kNumPhases; ++i) stats->phase_ms[i] = (double)h->phase[i].v * tick_ms;
    }
    return PICO_OK;
}

template int run_histocore<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                    void *, size_t, pico_stats *, hipStream_t, const int32_t *, int,
                                    pico_step *, int64_t, int64_t *);
template int run_histocore<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, int32_t *,
                                    void *, size_t, pico_stats *, hipStream_t, const int32_t *, int,
                                    pico_step *, int64_t, int64_t *);

size_t index2core_ws_bytes(int64_t n, int64_t m) {
    return histocore_ws_bytes(n, m) + carve_bytes(n, 4) * 4 + carve_bytes(n, 8) * 4;
}

template <typename Off>
int run_index2core(const Off *off, const int32_t *cols, int64_t n, int64_t m, int32_t *out, void *ws,
                   size_t ws_bytes, pico_stats *stats, hipStream_t stream, int cnt_mode) {
    if ((unsigned long long)m >= (1ull << (64 - kSlotBits))) {
        set_error("m=%lld too large for the packed frontier counter", (long long)m);
        return PICO_ENOTSUP;
    }
    Carve cv{static_cast<char *>(ws), 0, ws_bytes};
    IcArgs<Off> a;
    HcArgs<Off> &h = a.h;
    h.off = off;
    h.cols = cols;
    h.n = n;
    h.core = out;
    h.histo = cv.take<int32_t>(m);
    h.ndeg = nullptr;
    h.oldcore = cv.take<int32_t>(n);
    h.F[0] = cv.take<int32_t>(n);
    h.FE[0] = cv.take<long long>(n);
    h.FR[0] = cv.take<long long>(n);
    h.F[1] = nullptr;
    h.FE[1] = nullptr;
    h.FR[1] = nullptr;
    h.P0 = cv.take<int32_t>(n);
    h.P1 = cv.take<int32_t>(n);
    h.HS = cv.take<int32_t>(n);
    h.hcap = 0;
    h.H = nullptr;
    h.st = cv.take<HcState>(1);
    h.limit = wall_ticks(20.0);
    h.m = m;
    h.warm = nullptr;
    h.warm_add = 0;
    h.rebuild_permille = 0;
    h.sched = nullptr;
    h.sched_cap = 0;
    h.ns_per_tick = 0.0;
    a.cnt = cv.take<int32_t>(n);
    a.mark = cv.take<int32_t>(n);
    for (int b = 0; b < 2; ++b) {
        a.A[b] = cv.take<int32_t>(n);
        a.AE[b] = cv.take<long long>(n);
        a.AR[b] = cv.take<long long>(n);
    }
    a.cnt_mode = cnt_mode;
    if ((m > 0 && !h.histo) || !h.oldcore || !h.F[0] || !h.FE[0] || !h.FR[0] || !h.P0 || !h.P1 || !h.HS ||
        !h.st || !a.cnt || !a.mark || !a.A[0] || !a.A[1] || !a.AE[0] || !a.AE[1] || !a.AR[0] || !a.AR[1]) {
        set_error("Index2core workspace too small (%zu bytes given, %zu needed)", ws_bytes,
                  index2core_ws_bytes(n, m));
        return PICO_ENOMEM;
    }
    int blocks = 0;
    int rc = persistent_grid(reinterpret_cast<const void *>(ic_persistent<Off>), kBlock,
                             tune_int("PICO_HC_BLOCKS_PER_CU", 2), grid_want_histocore(m), &blocks);
    if (rc) return rc;
    PICO_LAUNCH("hc_state_init", hc_state_init, dim3(1), dim3(kBlock), stream, h.st);
    PICO_LAUNCH_CHECK();
    void *args[] = {&a};
    int rec = prof_begin(cnt_mode ? "cntcore_persistent" : "nbrcore_persistent", stream);
    PICO_HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(ic_persistent<Off>), dim3(blocks),
                                            dim3(kBlock), args, 0, stream));
    prof_end(rec, stream);
    HcState *hs = static_cast<HcState *>(host_scratch(sizeof(HcState)));
    if (!hs) return PICO_EHIP;
    PICO_HIP_TRY(hipMemcpyAsync(hs, h.st, sizeof(HcState), hipMemcpyDeviceToHost, stream));
    PICO_HIP_TRY(hipStreamSynchronize(stream));
    if (hs->g.error.v) {
        set_error("Index2core kernel stopped (error %llu; grid of %d blocks)", (unsigned long long)hs->g.error.v,
                  blocks);
        return PICO_EHIP;
    }
    if (stats) {
        stats->iterations = (int64_t)hs->rounds.v;         // rounds that changed a value (l2)
        stats->sub_rounds = (int64_t)hs->first_frontier.v;  // rounds that computed h-indexes
        stats->scans = (int64_t)hs->phase[0].v;             // active vertices, summed over rounds
        stats->frontier_total = (int64_t)hs->frontier_total.v;  // h-indexes computed
        stats->k_max = 0;
        stats->edges_scanned = (int64_t)hs->g.ctr[IC_EDGES].v;
        stats->atomics = (int64_t)hs->g.ctr[IC_ATOM].v;
        stats->buckets_scanned = (int64_t)hs->g.ctr[N_BUCKETS].v;
        stats->pushes_dynamic = (int64_t)hs->phase[1].v;  // activations after the first round
    }
    return PICO_OK;
}

template int run_index2core<int32_t>(const int32_t *, const int32_t *, int64_t, int64_t, int32_t *, void *,
                                     size_t, pico_stats *, hipStream_t, int);
template int run_index2core<int64_t>(const int64_t *, const int32_t *, int64_t, int64_t, int32_t *, void *,
                                     size_t, pico_stats *, hipStream_t, int);

}  // namespace pico
