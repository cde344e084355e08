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
    PICO_ALGO_MASK = 0xff,
    PICO_OFFSETS_I64 = 0x100 /* OR-ed into algo: csr_offsets is int64[n+1] */
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
    int32_t reserved;
    double elapsed_ms;      /* host wall time of the call's device work */
    int64_t edges_scanned;  /* adjacency entries read by the frontier kernels:
                               PeelOne scatter (= m), HistoCore UpdateHisto */
    int64_t atomics;        /* PeelOne: decrements issued (each an atomic RMW);
                               HistoCore: edges whose histogram was updated
                               (two atomic RMWs each) */
    int64_t buckets_scanned;/* HistoCore: histogram buckets read by SumHisto */
    int64_t pushes_dynamic; /* PeelOne: vertices asserted by the scatter (the
                               dynamic frontier) rather than found by a scan;
                               HistoCore: frontier entries pushed by UpdateHisto */
    double phase_ms[8];     /* device wall time by phase, barrier waits included.
                               PeelOne: [0] initialisation, [1] level scans,
                               [2] level drains.  HistoCore: [0] core = deg,
                               [1] InitHisto, [2] SumHisto, [3] SumHisto of
                               large values, [4] UpdateHisto, [5] UpdateHisto
                               of long rows. */
} pico_stats;

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
