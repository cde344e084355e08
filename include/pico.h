/*
 * pico.h -- C ABI of the MI355X (gfx950) k-core decomposition library.
 *
 * Problem (paper, Section I and Table I): for an undirected simple graph
 * G = (V, E), compute core(v) for every vertex: the largest k such that v
 * belongs to the k-core, the maximal subgraph whose vertices all have degree
 * >= k.  A vertex of degree 0 has coreness 0.
 *
 * Two algorithms, both computing the same unique vector:
 *   PICO_ALGO_PEELONE   -- PeelOne with the assertion decrement and dynamic
 *                          in-level frontier (Section III, Alg. 4).
 *   PICO_ALGO_HISTOCORE -- HistoCore: h-index iteration over maintained
 *                          per-vertex histograms (Section IV-B, Alg. 6).
 *
 * Graph input (Section II-B, "Graph Storage"): CSR with both directions of
 * every undirected edge stored.
 *   csr_offsets  device pointer, n+1 entries, int32 by default or int64 when
 *                PICO_OFFSETS_I64 is OR-ed into `algo`; offsets[0] = 0,
 *                offsets[n] = m, non-decreasing.
 *   csr_cols     device pointer, int32[m], neighbour ids in [0, n).
 * Preconditions (not checked on the hot path; pico_validate_csr checks
 * them): symmetric, no self-loops, no duplicate entries, n < 2^31.
 * Rows need not be sorted.
 *
 * Ownership: the caller owns every buffer passed in.  Inputs are read only.
 * Stream: every device operation is enqueued on `stream` (a hipStream_t;
 * NULL means the null stream).  The calls return after the result is
 * complete on that stream (the host waits for the level / iteration loop),
 * so out_core may be read as soon as the call returns PICO_OK.
 * Errors never throw across this boundary; they are status codes, with a
 * thread-local detail string from pico_last_error().
 * Thread safety: calls on different streams may run concurrently from
 * different host threads if each uses its own workspace.
 *
 * Test and development overrides (environment variables; unset in
 * production, where the library picks launch shapes itself).  They are read
 * at each call and must be positive integers (anything else is ignored),
 * except where marked >= 0; PICO_SMALL_MAX_EDGES is read once per process:
 *   PICO_GRID_BLOCKS        workgroups of a grid-wide persistent launch
 *                           (capped at what is co-resident)
 *   PICO_PO_BLOCKS_PER_CU   PeelOne workgroups per compute unit (default 1,
 *                           2 from 2^28 entries)
 *   PICO_HC_BLOCKS_PER_CU   HistoCore workgroups per compute unit (default 4;
 *                           CntCore / NbrCore 2)
 *   PICO_PO_LOCAL_EDGES     PeelOne: a batch of vertices asserted within a
 *                           workgroup is expanded by that workgroup when its
 *                           rows hold at most this many edges (default 4096;
 *                           0 sends every asserted vertex to the shared
 *                           frontier of the next round); >= 0
 *   PICO_HC_REBUILD_PERMILLE HistoCore rounds whose frontier rows hold at least
 *                           this share of the m entries (in 1/1000; default
 *                           640, above 1000 never) rebuild the histograms
 *                           instead of running UpdateHisto
 *   PICO_BATCH_WAIT_US      bound, in microseconds, on each wait of the
 *                           multi-graph kernels for a graph's leader or
 *                           helpers (default one minute); a graph whose wait
 *                           runs out is left unfinished and its status word
 *                           stays PICO_EHIP
 *   PICO_SMALL_MAX_EDGES    entry bound of the one-workgroup path (default
 *                           2^14; 0 = never)
 * All but PICO_BATCH_WAIT_US change only the launch shape or the work, never
 * the result.
 */
#ifndef PICO_H
#define PICO_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PICO_API __attribute__((visibility("default")))
#else
#define PICO_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pico_status {
    PICO_OK = 0,
    PICO_EINVAL = -1,   /* bad argument: NULL with n > 0, n < 0, m < 0, bad algo,
                           int32 offsets with m >= 2^31, n >= 2^31 */
    PICO_ENOMEM = -2,   /* workspace too small, or device allocation failed */
    PICO_EHIP = -3,     /* a HIP runtime call failed; see pico_last_error() */
    PICO_ENOTSUP = -4,  /* unsupported device (not gfx950) or option */
    PICO_EBADCSR = -5   /* pico_validate_csr found a malformed graph */
} pico_status;

enum {
    PICO_ALGO_PEELONE = 0,
    PICO_ALGO_HISTOCORE = 1,
    PICO_ALGO_AUTO = 2,       /* single-graph calls: PeelOne or HistoCore, chosen per
                                 graph by pico_select_algorithm's rule */
    /* Index2core baselines HistoCore is measured against (Section IV-A,
     * Alg. 5; Section V, Table VI), single-graph calls on the grid path:
     * synchronous rounds from the degrees with every h-index rebuilt from
     * the neighbours' values.  CntCore recomputes only vertices whose cnt
     * (neighbours valued >= their own value) fell below their value
     * (Theorem 2); NbrCore recomputes every neighbour of a vertex that
     * changed.  Same coreness.  Their pico_stats: iterations = rounds that
     * changed a value (l2), sub_rounds = rounds that computed h-indexes,
     * scans = active vertices (cnt computed / recompute candidates) summed
     * over rounds, frontier_total = h-indexes computed, edges_scanned = all
     * adjacency entries read, atomics = histogram and cnt increments,
     * pushes_dynamic = activations after the first round. */
    PICO_ALGO_CNTCORE = 3,
    PICO_ALGO_NBRCORE = 4,
    PICO_ALGO_MASK = 0xff,
    PICO_OFFSETS_I64 = 0x100, /* OR-ed into algo: csr_offsets is int64[n+1] */
    /* Path selection, OR-ed into algo (single-graph calls only; at most one).
     * Without either flag a graph whose vertex values fit in one workgroup's
     * LDS (n * 4 bytes, about 160 KiB on gfx950) and whose m is at most
     * 2^14 (environment PICO_SMALL_MAX_EDGES overrides; 0 = never) is
     * decomposed by one workgroup, the rest by the grid-wide persistent
     * kernels.  Both paths compute the same coreness and statistics (the
     * per-phase times in phase_ms are grid-path only). */
    PICO_PATH_GRID = 0x200,   /* always the grid-wide persistent kernels */
    PICO_PATH_WG = 0x400,     /* always one workgroup; PICO_ENOTSUP if the
                                 values do not fit in its LDS */
    /* Ablations of PeelOne, OR-ed into PICO_ALGO_PEELONE (single-graph calls,
     * grid path; at most one).  Same coreness; they exist to measure what
     * Alg. 4's mechanisms save (Section III, Tables IV and V).
     *   PICO_PO_STATIC: no dynamic frontier -- a vertex lowered to k waits
     *     for the next scan at level k; stats.iterations then counts every
     *     iteration (Table IV's l1 for this variant).
     *   PICO_PO_ROLLBACK: the decrement of atomicAdd-rollback methods
     *     (Section III-B) -- a decrement landing at or below k is undone by an
     *     atomic add; stats.atomics counts both.
     *   PICO_PO_GPP: General Parallel Peel (Alg. 3, Section II-C), the
     *     GPP baseline of Section V -- no dynamic frontier, every neighbour not yet
     *     removed decremented, k advancing by one when no residual vertex is
     *     at or below it; stats.iterations counts Alg. 3's while-loop
     *     iterations (k is raised at the head of an iteration and scanned
     *     with in the same one; isolated vertices take the first, at k = 0),
     *     stats.scans every scan the kernel ran. */
    PICO_PO_STATIC = 0x800,
    PICO_PO_ROLLBACK = 0x1000,
    PICO_PO_GPP = 0x2000
};

/* Run statistics (all counts over the whole call). */
typedef struct pico_stats {
    int64_t iterations;     /* PeelOne: levels with a non-empty frontier (l1);
                               HistoCore: SumHisto/UpdateHisto rounds (l2) */
    int64_t sub_rounds;     /* PeelOne: frontier batches drained, all levels;
                               HistoCore: equal to iterations */
    int64_t scans;          /* PeelOne: level scans, including ones that found
                               an empty level and jumped k forward */
    int64_t frontier_total; /* PeelOne: vertices peeled (= non-isolated n);
                               HistoCore: sum over rounds of |V_cnt| */
    int32_t k_max;          /* largest coreness found (PeelOne; 0 for HistoCore) */
    int32_t algo_used;      /* the algorithm that ran (PICO_ALGO_PEELONE or
                               PICO_ALGO_HISTOCORE), also under PICO_ALGO_AUTO */
    double elapsed_ms;      /* host wall time of the call's device work */
    int64_t edges_scanned;  /* adjacency entries read by the frontier kernels:
                               PeelOne scatter (= m), HistoCore UpdateHisto */
    int64_t atomics;        /* PeelOne: decrements issued (each an atomic RMW);
                               HistoCore: edges whose histogram was updated
                               (two atomic RMWs each) */
    int64_t buckets_scanned;/* HistoCore: histogram buckets read by SumHisto */
    int64_t pushes_dynamic; /* PeelOne: vertices asserted by the scatter (the
                               dynamic frontier) rather than found by a scan
                               (on the grid path a vertex valued k when level k
                               starts may be claimed by a decrement before the
                               level's scan reaches it, so this split varies
                               between runs; the level's total does not);
                               HistoCore: frontier entries pushed by UpdateHisto */
    double phase_ms[8];     /* device wall time by phase, barrier waits included.
                               PeelOne: [0] initialisation, [1] level scans,
                               [2] level drains.  HistoCore: [0] core = deg,
                               [1] InitHisto, [2] SumHisto, [3] SumHisto of
                               large values, [4] UpdateHisto, [5] rounds that
                               rebuilt the histograms instead. */
} pico_stats;

/* One step of a decomposition's schedule (pico_coreness_schedule): a level
   of PeelOne or a round of HistoCore.  64 bytes. */
typedef struct pico_step {
    int64_t key;        /* PeelOne: the level's k; HistoCore: the round t = 1, 2, ... */
    int64_t vertices;   /* PeelOne: vertices peeled at level k, found by the level's
                           scan or asserted by a decrement (= |{v : core(v) = k}|,
                           Table V); HistoCore: |V_cnt| of round t, the vertices
                           whose h-index changes in synchronous round t (Theorem 2) */
    int64_t work;       /* PeelOne: survivor-list entries the level's scan read;
                           HistoCore: histogram moves of round t (N1 / N3 updates
                           of UpdateHisto, two atomics each) */
    int64_t edges;      /* PeelOne: adjacency entries of the level's edge-balanced
                           rounds (rows expanded from a workgroup's LDS queue are
                           not counted); HistoCore: sum of the frontier's degrees,
                           the edge space of round t's UpdateHisto */
    int64_t rounds;     /* PeelOne: edge-balanced rounds of the level; HistoCore: 1 */
    int64_t ns;         /* device wall time of the step (timing, not fixed by the graph) */
    int64_t scan_ns;    /* of which PeelOne's scan / HistoCore's SumHisto */
    int64_t kind;       /* HistoCore: 0 = UpdateHisto round, 1 = round that rebuilt
                           every histogram from the current values instead (same
                           histograms and next frontier); PeelOne: 0 */
} pico_step;

/* Accumulated HIP-event timing of one kernel over profiled calls. */
typedef struct pico_kernel_stat {
    const char *name;       /* static string owned by the library */
    int64_t launches;
    double total_ms;        /* sum over launches of (stop event - start event) */
} pico_kernel_stat;

/*
 * pico_coreness -- coreness of every vertex into out_core (device int32[n],
 * caller-owned).  Allocates its scratch space with the HIP stream-ordered
 * allocator and frees it before returning.  n == 0 is a no-op returning
 * PICO_OK.  Implements Alg. 4 (algo PICO_ALGO_PEELONE) or Alg. 6
 * (PICO_ALGO_HISTOCORE) of the paper.
 */
PICO_API int pico_coreness(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                  int algo, int32_t *out_core, void *stream);

/*
 * pico_coreness_noalloc -- as pico_coreness (same arguments, same result),
 * for callers that cannot allocate device or host memory during the call:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The workspace is a static device array of
 * PICO_NOALLOC_SCRATCH_BYTES held by the library on every GPU it runs on
 * until the process ends; the call allocates nothing (no hipMalloc, pinned
 * host memory or profiling events; pico_profile_enable does not apply).
 * Graphs whose workspace (pico_workspace_bytes for the same algo) exceeds
 * PICO_NOALLOC_SCRATCH_BYTES get PICO_ENOMEM before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on the
 * same GPU (several host threads, or streams not ordered with each other)
 * race and must be serialised by the caller.  The array keeps the previous
 * call's contents; the kernels initialise what they read.  Waits for the
 * result before returning.
 */
#define PICO_NOALLOC_SCRATCH_BYTES (64ull << 20)
PICO_API int pico_coreness_noalloc(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                                   int algo, int32_t *out_core, void *stream);

/*
 * pico_workspace_bytes -- bytes of device scratch that pico_coreness_ws needs
 * for a graph of n vertices and m directed entries.  Writes *bytes; returns
 * PICO_EINVAL on bad sizes or algo.
 */
PICO_API int pico_workspace_bytes(int64_t n, int64_t m, int algo, size_t *bytes);

/*
 * pico_coreness_ws -- as pico_coreness, with caller-provided device scratch
 * (`workspace`, at least pico_workspace_bytes() bytes, 256-byte aligned, owned
 * by the caller, contents need not be initialised and are clobbered).
 * `stats` (host pointer) may be NULL.  Returns PICO_ENOMEM if ws_bytes is too
 * small.
 */
PICO_API int pico_coreness_ws(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                     int algo, int32_t *out_core, void *workspace, size_t ws_bytes,
                     pico_stats *stats, void *stream);

/*
 * pico_coreness_schedule -- as pico_coreness_ws, and also records the run's
 * schedule: one pico_step per PeelOne level (Alg. 4: levels k with a
 * non-empty frontier, in order) or per HistoCore round (Alg. 6: the rounds
 * of SumHisto then UpdateHisto, in order).
 *   steps      device pico_step[cap], caller-owned; the first min(cap, count)
 *              records are written, the rest of the array is untouched.
 *   cap        >= 0 (0: nothing recorded, the count is still returned).
 *   num_steps  host int64 (may be NULL): the number of steps the run took
 *              (= stats->iterations).
 * `algo` is PICO_ALGO_PEELONE, PICO_ALGO_HISTOCORE or PICO_ALGO_AUTO (with
 * PICO_OFFSETS_I64 as needed); the schedule comes from the grid-wide
 * persistent kernels, which this call always uses (PICO_PATH_WG and the
 * ablation flags give PICO_EINVAL; PICO_PATH_GRID is accepted).  Other
 * arguments, the workspace size (pico_workspace_bytes) and errors as
 * pico_coreness_ws; a NULL `steps` with cap > 0 is PICO_EINVAL.
 */
PICO_API int pico_coreness_schedule(const void *csr_offsets, const int32_t *csr_cols, int64_t n,
                                    int64_t m, int algo, int32_t *out_core, void *workspace,
                                    size_t ws_bytes, pico_stats *stats, pico_step *steps, int64_t cap,
                                    int64_t *num_steps, void *stream);

/*
 * pico_coreness_update -- coreness of a graph that changed since a coreness
 * was last computed (core maintenance, the dynamic-graph use of the h-index
 * formulation that Section IV builds on): HistoCore (Alg. 6) started from
 * upper bounds instead of the degrees.  The h-index iteration converges to
 * the coreness from any vector of upper bounds, and a started run only
 * lowers what is too high, so a small change costs few rounds.
 *
 *   prev_core  device int32[n]: for each vertex of the new graph a value such
 *              that prev_core[v] + bound_add >= its new coreness.  Deleting
 *              edges never raises a coreness, so after deletions the old
 *              coreness with bound_add = 0 qualifies; inserting one edge raises
 *              any coreness by at most one, so after b insertions (and any
 *              deletions) the old coreness with bound_add = b does.  Vertices
 *              new to the graph take any value >= their degree.  Values are
 *              capped by the degree and raised to 1 on vertices with
 *              neighbours.  With a bound below the coreness the result is
 *              undefined.  May alias out_core (in-place update).
 *   bound_add  >= 0, added to every prev_core value.
 *   algo       PICO_ALGO_HISTOCORE (PeelOne cannot start from bounds:
 *              PICO_ENOTSUP), optionally | PICO_OFFSETS_I64 and a path flag.
 * Other arguments, workspace (pico_workspace_bytes for HistoCore) and errors
 * as pico_coreness_ws.
 */
PICO_API int pico_coreness_update(const void *csr_offsets, const int32_t *csr_cols, int64_t n,
                                  int64_t m, int algo, const int32_t *prev_core, int32_t bound_add,
                                  int32_t *out_core, void *workspace, size_t ws_bytes,
                                  pico_stats *stats, void *stream);

/*
 * pico_select_algorithm -- the algorithm PICO_ALGO_AUTO runs on this graph
 * (the hybrid the paper leaves to future work, Section VII; Table VII shows
 * each paradigm ahead on different graphs).  Two features are measured on
 * the device:
 *   features[0]  H, the degree h-index: the largest h with at least h
 *                vertices of degree >= h.  It bounds k_max, hence PeelOne's
 *                level count (Table V: l1 = k_max).
 *   features[1]  vertices sampled (1024 evenly spaced ids, those of degree 1
 *                to 1024 counted),
 *   features[2]  of those, the ones in HistoCore's first frontier, with
 *                fewer than deg(v) neighbours of degree >= deg(v) (Theorem 2).
 * Rule (constants from a sweep of 47 graphs on MI355X): m < 2^16 ->
 * PeelOne; fewer than 1/64 of the sample in the first frontier -> HistoCore;
 * m < 2^23 and H >= 4 m / n -> HistoCore; otherwise PeelOne.  For m < 2^16
 * nothing is measured (features all 0).
 *   algo         PICO_ALGO_AUTO, optionally | PICO_OFFSETS_I64.
 *   workspace    at least pico_workspace_bytes(n, m, algo) bytes (device).
 *   algo_out     host int: PICO_ALGO_PEELONE or PICO_ALGO_HISTOCORE.
 *   features     host int64[3] or NULL.
 * Synchronises `stream`.  Errors as pico_coreness_ws.
 */
PICO_API int pico_select_algorithm(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                                   int algo, void *workspace, size_t ws_bytes, int *algo_out,
                                   int64_t *features, void *stream);

/* Tuning of the batched kernel (NULL = defaults). */
typedef struct pico_batch_tune {
    int32_t lds_bytes;      /* dynamic LDS per workgroup for a graph's vertex values;
                               graphs with more than lds_bytes / 4 vertices keep them
                               in global memory.  -1 = default (64 KiB), clamped to the
                               device limit. */
    int32_t blocks_per_cu;  /* resident workgroups per compute unit; 0 = occupancy limit
                               (larger values are clamped to it) */
    int32_t sum_wave_min;   /* HistoCore SumHisto: a vertex whose value exceeds this
                               scans its buckets with a whole wave, smaller ones with
                               one thread; 0 = default (64) */
    int32_t help_min_vertices; /* graphs with at least this many vertices (and values
                               in global memory) are decomposed by their workgroup
                               with the help of idle workgroups of the same launch
                               (PeelOne and HistoCore); 0 = default (32768),
                               -1 = never */
} pico_batch_tune;

/* Statistics of one batched call (filled only if requested; the call then
   waits for the device). */
typedef struct pico_batch_stats {
    int64_t graphs;
    int64_t iterations;      /* PeelOne: non-empty levels summed over graphs;
                                HistoCore: rounds summed over graphs */
    int64_t atomics;         /* PeelOne: decrements; HistoCore: histogram moves
                                (two atomic RMWs each); summed over graphs */
    int64_t frontier_total;  /* PeelOne: vertices peeled; HistoCore: sum over
                                rounds of the frontier size */
    int64_t edges_scanned;   /* adjacency entries read by the frontier phases
                                (PeelOne drain, HistoCore UpdateHisto) */
    int64_t buckets_scanned; /* HistoCore: histogram buckets read by SumHisto */
    int64_t pushes;          /* PeelOne: vertices asserted during a level's drain;
                                HistoCore: next-frontier pushes by UpdateHisto */
    int64_t lds_graphs;      /* graphs whose vertex values lived in LDS */
    int64_t workgroups;      /* workgroups launched */
    int32_t lds_bytes;       /* dynamic LDS per workgroup used */
    int32_t blocks_per_cu;   /* resident workgroups per compute unit used */
    int64_t helped_graphs;   /* graphs decomposed with their phases open to helpers */
    int64_t help_chunks;     /* phase chunks run by helping workgroups */
    int64_t histocore_graphs;/* graphs decomposed by HistoCore (under PICO_ALGO_AUTO:
                                the ones the per-graph choice gave it) */
} pico_batch_stats;

/*
 * pico_batched_workspace_bytes -- device scratch for pico_coreness_batched
 * over num_graphs graphs totalling total_n vertices and total_m directed
 * entries.
 */
PICO_API int pico_batched_workspace_bytes(int64_t num_graphs, int64_t total_n, int64_t total_m,
                                          int algo, size_t *bytes);

/*
 * pico_coreness_batched -- coreness of many independent graphs in one launch
 * (each graph decomposed by Alg. 4 or Alg. 6 of the paper inside one
 * workgroup).  Packed multi-CSR, all device pointers:
 *   graph_vptr   int64[num_graphs + 1]: graph g owns global vertices
 *                [graph_vptr[g], graph_vptr[g+1]); graph_vptr[num_graphs] = total_n
 *   csr_offsets  int64[total_n + 1]: row of global vertex x is
 *                csr_cols[csr_offsets[x] .. csr_offsets[x+1]); csr_offsets[0] = 0,
 *                csr_offsets[total_n] = total_m
 *   csr_cols     int32[total_m]: graph-local neighbour ids in [0, n_g)
 *   order        int32[num_graphs] processing order (e.g. largest graph first),
 *                or NULL for 0..num_graphs-1
 *   out_core     int32[total_n], caller-owned
 * `algo` is PICO_ALGO_PEELONE, PICO_ALGO_HISTOCORE or PICO_ALGO_AUTO (offsets
 * are always int64 here; PICO_OFFSETS_I64 is accepted and ignored).
 * PICO_ALGO_AUTO chooses per graph on the device (the hybrid the paper leaves
 * to future work, Section VII): HistoCore for a graph in which fewer than
 * 1/64 of up to 64 evenly spaced sampled vertices are in HistoCore's first
 * frontier (cnt(v) < deg(v), Theorem 2: the degrees are then nearly the
 * coreness), PeelOne otherwise -- with one workgroup per graph PeelOne's
 * levels are cheap and it is the faster algorithm elsewhere; the two groups
 * run as two launches on `stream`.  Each graph must be a simple undirected
 * graph with fewer than 2^31 vertices and edges.  The workspace (>=
 * pico_batched_workspace_bytes for the same algo, 256-byte aligned) is
 * caller-owned; it begins with one int32 status word per graph (see
 * pico_batch_status).  The call only enqueues work on `stream` unless `stats`
 * is non-NULL, in which case it waits, fills it, and returns PICO_EHIP if a
 * graph was left unfinished (a wait bound expired) or PICO_EINVAL if a graph's
 * vertex range was invalid; out_core is valid once the stream has completed.
 */
PICO_API int pico_coreness_batched(const int64_t *graph_vptr, const int64_t *csr_offsets,
                                   const int32_t *csr_cols, int64_t num_graphs, int64_t total_n,
                                   int64_t total_m, int algo, const int32_t *order,
                                   int32_t *out_core, const pico_batch_tune *tune, void *workspace,
                                   size_t ws_bytes, pico_batch_stats *stats, void *stream);

/*
 * Task lists: the batched kernel over graphs that live anywhere in device
 * memory, each with its own output and scratch (the form a request server
 * needs).  One descriptor per graph:
 *   offsets   device int64[n+1]: positions into cols; offsets[0] need not be 0
 *   cols      device int32: the graph's rows at cols[offsets[v] .. offsets[v+1]),
 *             graph-local neighbour ids in [0, n)
 *   n, m      vertices (< 2^31) and directed entries (offsets[n] - offsets[0])
 *   out_core  device int32[n], caller-owned
 *   scratch   device, 256-byte aligned, scratch_bytes >= pico_task_scratch_bytes
 *             (n, m, algo), caller-owned; its contents are clobbered
 * Scratch of concurrently running tasks must not overlap.
 */
typedef struct pico_task {
    const int64_t *offsets;
    const int32_t *cols;
    int64_t n;
    int64_t m;
    int32_t *out_core;
    void *scratch;
    size_t scratch_bytes;
} pico_task;

/* pico_task_scratch_bytes -- per-task scratch for a graph of n vertices and m
   directed entries: 16 n bytes for PeelOne, 20 n + 4 m for HistoCore and for
   PICO_ALGO_AUTO (each array rounded up to 256 bytes). */
PICO_API int pico_task_scratch_bytes(int64_t n, int64_t m, int algo, size_t *bytes);

/* pico_tasks_workspace_bytes -- device workspace of pico_coreness_tasks for a
   list of num_tasks descriptors (status words first, then task tables and
   counters), for any algo. */
PICO_API int pico_tasks_workspace_bytes(int64_t num_tasks, size_t *bytes);

/*
 * pico_coreness_tasks -- coreness of every graph of a task list in one launch
 * of the batched kernel (each graph by Alg. 4 or Alg. 6 inside one workgroup;
 * tasks are claimed in list order, so put large graphs first).  `tasks` is a
 * HOST array, copied to the workspace on `stream` during the call and free to
 * reuse on return.  Arguments are checked on the host: n in [0, 2^31), m >= 0,
 * pointers present, scratch large enough and aligned (PICO_EINVAL /
 * PICO_ENOMEM).  `algo` as for pico_coreness_batched (PICO_ALGO_AUTO chooses
 * per task; its tasks need HistoCore-sized scratch).  Enqueues only, unless
 * `stats` is non-NULL (then waits, and reports unfinished tasks as
 * pico_coreness_batched does); per-task outcomes: pico_batch_status.
 */
PICO_API int pico_coreness_tasks(const pico_task *tasks, int64_t num_tasks, int algo,
                                 const pico_batch_tune *tune, void *workspace, size_t ws_bytes,
                                 pico_batch_stats *stats, void *stream);

/*
 * pico_batch_status -- outcome of every graph of the last pico_coreness_batched
 * or pico_coreness_tasks call on `workspace`: waits for `stream` (the stream
 * of that call), then copies `count` int32 status words into `status` (host
 * array; NULL to get only the summary), one per graph in the caller's
 * numbering (graph index of the packed batch, position in the task list):
 *   PICO_OK      decomposed; its out_core is the coreness
 *   PICO_EHIP    not finished: a wait inside the launch reached its bound
 *                (a minute) and the graph was left incomplete
 *   PICO_EINVAL  not decomposed: invalid vertex range (packed batches)
 * Returns PICO_OK if every word is PICO_OK, else the first other status, with
 * the counts in pico_last_error().  For callers that enqueue without stats.
 */
PICO_API int pico_batch_status(const void *workspace, size_t ws_bytes, int64_t count, int32_t *status,
                               void *stream);

/*
 * Request server: continuous batching of decomposition requests on one GPU.
 * Requests name a device-resident graph (int64 offsets, as in pico_task) and
 * a device output.  The server's algo may be PICO_ALGO_AUTO (a choice per
 * request, as in pico_coreness_batched; requests then reserve HistoCore-sized
 * scratch).  A request is admitted once its scratch
 * (pico_task_scratch_bytes) fits in the caller's HBM arena (first come,
 * first served within its size class); admitted requests are launched
 * together, largest first, as one batched-kernel call on a free launch slot
 * (one HIP stream each, up to max_inflight launches in flight), so requests
 * that arrive while others run start on a free slot at once and overlap with
 * them on the device.  A launch holds requests of one size class only
 * (vertex counts below class_bounds[0], below class_bounds[1], the rest), so
 * small requests never wait for a large graph in their launch; large requests
 * hold at most max_large_slots slots.  The caller drives it: submit queues,
 * progress reaps finished launches, launches what fits and returns
 * completions.  Single host thread per server.
 */
typedef struct pico_server pico_server;

typedef struct pico_server_config {
    int32_t algo;                  /* PICO_ALGO_PEELONE, PICO_ALGO_HISTOCORE or
                                      PICO_ALGO_AUTO */
    int32_t max_inflight;          /* launch slots (streams), 1..64 */
    int64_t max_tasks_per_launch;  /* requests per launch, >= 1 */
    void *arena;                   /* device, 256-byte aligned, caller-owned: the
                                      admission budget for request scratch */
    size_t arena_bytes;
    pico_batch_tune tune;          /* batched-kernel tuning (zeros / -1 = defaults) */
    int64_t class_bounds[2];       /* vertex-count bounds of the small and medium
                                      classes; 0 = 16384 and 131072 */
    int32_t max_large_slots;       /* slots the large class may hold; 0 = half */
    int32_t reserved;              /* must be 0 */
} pico_server_config;

typedef struct pico_request {
    const int64_t *offsets;  /* device int64[n+1], positions into cols */
    const int32_t *cols;     /* device int32, graph-local ids */
    int64_t n, m;
    int32_t *out_core;       /* device int32[n], caller-owned, valid on completion */
    int64_t tag;             /* caller's id, returned in the completion */
} pico_request;

typedef struct pico_completion {
    int64_t tag;
    int32_t status;          /* PICO_OK, or PICO_EHIP if the request's launch left
                                it unfinished (a wait bound expired); its
                                out_core is then not the coreness */
    int32_t reserved;
    uint64_t t_submit_ns;    /* host steady-clock times: submit, launch, and */
    uint64_t t_launch_ns;    /* when progress saw the launch complete */
    uint64_t t_done_ns;
} pico_completion;

typedef struct pico_server_status {
    int64_t waiting, inflight, ready, busy_slots, launches, completed, arena_used, arena_bytes;
} pico_server_status;

/* pico_server_create -- set up streams, events, pinned staging and per-slot
   device tables; the arena stays caller-owned and must outlive the server. */
PICO_API int pico_server_create(const pico_server_config *cfg, pico_server **server);
/* pico_server_submit -- queue one request (host-checked; PICO_ENOMEM if its
   scratch can never fit the arena).  Does not touch the device. */
PICO_API int pico_server_submit(pico_server *server, const pico_request *req);
/* pico_server_progress -- reap finished launches, launch what fits on free
   slots, and copy up to max_done completions into done (host array);
   *num_done gets the count.  Never blocks. */
PICO_API int pico_server_progress(pico_server *server, pico_completion *done, int max_done,
                                  int *num_done);
/* pico_server_query -- queue lengths, busy slots, launches so far and arena use. */
PICO_API int pico_server_query(const pico_server *server, pico_server_status *status);
/* pico_server_destroy -- wait for launches in flight, release everything the
   server allocated; requests still waiting are dropped. */
PICO_API int pico_server_destroy(pico_server *server);

/*
 * pico_validate_csr -- O(n + m) device check of the preconditions that are
 * cheap to verify in place: offsets[0] == 0, offsets[n] == m, offsets
 * non-decreasing, every column in [0, n) and no self-loop.  Symmetry and
 * duplicates are not checked.  Returns PICO_OK or PICO_EBADCSR.  Blocks until
 * the check is done.
 */
PICO_API int pico_validate_csr(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                      int algo, void *stream);

/*
 * pico_profile_enable -- on the calling host thread, bracket every kernel
 * launch of subsequent calls with HIP events on the call's stream (on != 0),
 * or stop doing so (on == 0).  Enabling clears the accumulated table.
 */
PICO_API int pico_profile_enable(int on);

/*
 * pico_profile_read -- copy up to `cap` accumulated per-kernel entries of the
 * calling host thread into `out` (host array) and the number available into
 * *count.  Entries accumulate over all profiled calls since enabling.
 */
PICO_API int pico_profile_read(pico_kernel_stat *out, int cap, int *count);

/*
 * pico_probe_random_access -- a measurement aid beside the method, against
 * which the kernels' times can be set: the rate at which this device
 * performs the two random-access operations both algorithms are built from
 * (the gather of a neighbour's value, Alg. 4 and Alg. 6; the decrement or
 * histogram update, Section III-B and Section IV-B), over an array of the
 * size the kernels touch, with nothing else running.
 *   buf, bytes     device array, caller-owned, at least 4 bytes; its contents
 *                  are overwritten.  Operations go to uniformly random 4-byte
 *                  words of it.
 *   ops            operations of each kind, > 0.
 *   gathers_per_s  host double: random 4-byte loads per second.
 *   atomics_per_s  host double: random 4-byte device-scope atomic adds
 *                  (returning the old value) per second.
 * Enqueues, on `stream`, an untimed and a timed launch of each kind, times
 * the timed ones with HIP events and waits for them.  Errors: PICO_EINVAL
 * for a null pointer, bytes < 4 or ops <= 0; PICO_EHIP for HIP failures.
 */
PICO_API int pico_probe_random_access(void *buf, size_t bytes, int64_t ops, double *gathers_per_s,
                                      double *atomics_per_s, void *stream);

/* Static description of a status code. */
PICO_API const char *pico_status_string(int status);

/* Detail of the last failure on the calling host thread ("" if none). */
PICO_API const char *pico_last_error(void);

/* Library version string. */
PICO_API const char *pico_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PICO_H */
