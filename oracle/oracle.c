/*
 * CPU oracle for k-core decomposition -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, obviously-correct reference routines that the tests,
 * the smoke check and the benchmark's CPU-baseline leg use to judge the GPU
 * library.  Nothing in the product path links, loads or calls this file, and
 * it shares no code, header or table with the GPU library.
 *
 * Graph input everywhere: an undirected simple graph in CSR with both
 * directions of every edge stored (paper, Section II-B "Graph Storage"),
 * offsets int64[n+1], neighbour ids int32[m].
 *
 *  - oracle_bz:            coreness by the Batagelj-Zaversnik O(n+m) bucket
 *                          peel (cited in the paper's related work, Section
 *                          VI-A); it computes exactly the definition of
 *                          Section I: core(v) = the largest k such that v lies
 *                          in the k-core, the maximal subgraph of minimum
 *                          degree >= k.
 *  - oracle_peel_gpp:      General Parallel Peel (Alg. 3), serially, counting
 *                          its while-loop iterations.
 *  - oracle_index2core:    CntCore (Alg. 5) and NbrCore, synchronous rounds,
 *                          with their work counts (Table VI's baselines).
 *  - oracle_peel_static:   PeelOne without the dynamic frontier (Table IV's
 *                          variant), serially, counting its iterations.
 *  - oracle_hindex_jacobi_from: the same iteration started from upper bounds
 *                          of the coreness (core maintenance on a changed
 *                          graph), never raising a value.
 *  - oracle_hindex_jacobi: the Index2core paradigm (Section II-A, Alg. 2) run
 *                          in synchronous rounds: x_0 = deg and
 *                          x_{t+1}(v) = H({x_t(u) : u in nbr(v)}), where H is
 *                          the h-index (largest h with at least h neighbours
 *                          valued >= h).  H is computed by sorting the
 *                          neighbour values, not by a histogram.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_bz(int64_t n, const int64_t *off, const int32_t *adj, int32_t *core)
{
    if (n < 0 || (n > 0 && (!off || !core))) return -1;
    if (n == 0) return 0;

    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = off[v + 1] - off[v];
        if (d < 0) return -1;
        if (d > maxdeg) maxdeg = d;
    }
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *bin = (int64_t *)calloc((size_t)maxdeg + 2, sizeof(int64_t));
    if (!deg || !pos || !vert || !bin) {
        free(deg); free(pos); free(vert); free(bin);
        return -2;
    }

    /* Bucket the vertices by degree: bin[d] = first slot of degree class d in
     * vert[], vert[] = vertices in non-decreasing degree order, pos[v] = slot
     * of v in vert[]. */
    for (int64_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(off[v + 1] - off[v]);
        bin[deg[v]]++;
    }
    int64_t start = 0;
    for (int64_t d = 0; d <= maxdeg; ++d) {
        int64_t cnt = bin[d];
        bin[d] = start;
        start += cnt;
    }
    for (int64_t v = 0; v < n; ++v) {
        pos[v] = bin[deg[v]];
        vert[pos[v]] = (int32_t)v;
        bin[deg[v]]++;
    }
    for (int64_t d = maxdeg; d >= 1; --d) bin[d] = bin[d - 1];
    bin[0] = 0;

    /* Peel in non-decreasing current-degree order.  When v is removed its
     * current degree is its coreness; every neighbour still ranked above v
     * loses one degree and moves to the front of its (lower) bucket. */
    for (int64_t i = 0; i < n; ++i) {
        int32_t v = vert[i];
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = adj[e];
            if (deg[u] > deg[v]) {
                int32_t du = deg[u];
                int64_t pu = pos[u];
                int64_t pw = bin[du];
                int32_t w = vert[pw];
                if (u != w) {
                    pos[u] = pw; vert[pu] = w;
                    pos[w] = pu; vert[pw] = u;
                }
                bin[du]++;
                deg[u]--;
            }
        }
    }
    memcpy(core, deg, sizeof(int32_t) * (size_t)n);
    free(deg); free(pos); free(vert); free(bin);
    return 0;
}

static int cmp_desc_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x < y) - (x > y);
}

/* h-index of a multiset: the largest h such that at least h of the values
 * are >= h.  With the values sorted in descending order s[0] >= s[1] >= ...,
 * that is the largest h with s[h-1] >= h. */
static int32_t h_index_sorted(int32_t *vals, int64_t cnt)
{
    qsort(vals, (size_t)cnt, sizeof(int32_t), cmp_desc_i32);
    int64_t h = 0;
    while (h < cnt && vals[h] >= h + 1) ++h;
    return (int32_t)h;
}

/*
 * Synchronous h-index iteration from x_0 = deg.
 *   max_rounds:      stop after this many rounds even if not converged
 *   x_out:           int32[n], the values after the last round executed
 *   changed_per_round: optional int64[max_rounds]; entry t-1 = number of
 *                    vertices whose value changed in round t
 *   changed_round_of: optional int32[n]; the last round in which v changed
 *                    (0 if never)
 * Returns the number of rounds in which at least one value changed (the
 * convergence round count when it converged), -1 on bad arguments, -2 on
 * allocation failure.
 */
int64_t oracle_hindex_jacobi(int64_t n, const int64_t *off, const int32_t *adj,
                             int64_t max_rounds, int32_t *x_out,
                             int64_t *changed_per_round, int32_t *changed_round_of)
{
    if (n < 0 || (n > 0 && (!off || !x_out)) || max_rounds < 0) return -1;
    if (n == 0) return 0;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = off[v + 1] - off[v];
        if (d > maxdeg) maxdeg = d;
    }
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *y = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    if (!x || !y || !buf) { free(x); free(y); free(buf); return -2; }
    for (int64_t v = 0; v < n; ++v) x[v] = (int32_t)(off[v + 1] - off[v]);
    if (changed_round_of) memset(changed_round_of, 0, sizeof(int32_t) * (size_t)n);

    int64_t rounds = 0;
    for (int64_t t = 1; t <= max_rounds; ++t) {
        int64_t changed = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t d = off[v + 1] - off[v];
            for (int64_t j = 0; j < d; ++j) buf[j] = x[adj[off[v] + j]];
            y[v] = h_index_sorted(buf, d);
            if (y[v] != x[v]) {
                ++changed;
                if (changed_round_of) changed_round_of[v] = (int32_t)t;
            }
        }
        if (changed == 0) break;
        if (changed_per_round) changed_per_round[t - 1] = changed;
        rounds = t;
        int32_t *tmp = x; x = y; y = tmp;
    }
    memcpy(x_out, x, sizeof(int32_t) * (size_t)n);
    free(x); free(y); free(buf);
    return rounds;
}

/*
 * The same synchronous iteration started from given upper bounds x0 of the
 * coreness instead of the degrees (core maintenance: after edge deletions
 * the old coreness is such a bound, after b insertions the old coreness
 * plus b).  The start is x_0(v) = min(deg(v), max(x0[v] + add, 1)) on
 * vertices with neighbours and 0 on isolated ones, and each round sets
 * x_{t+1}(v) = min(x_t(v), H(x_t)(v)): a value never rises.  (From the
 * degrees H never raises a value, so this is the iteration above.)  The
 * iterates stay >= the coreness and stop at a vector with x <= H(x), which
 * is at most the coreness, so they end at the coreness.
 * Arguments and return value as oracle_hindex_jacobi; x0 may not be NULL.
 */
int64_t oracle_hindex_jacobi_from(int64_t n, const int64_t *off, const int32_t *adj,
                                  const int32_t *x0, int64_t add, int64_t max_rounds,
                                  int32_t *x_out, int64_t *changed_per_round,
                                  int32_t *changed_round_of)
{
    if (n < 0 || (n > 0 && (!off || !x_out || !x0)) || max_rounds < 0) return -1;
    if (n == 0) return 0;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = off[v + 1] - off[v];
        if (d > maxdeg) maxdeg = d;
    }
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *y = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    if (!x || !y || !buf) { free(x); free(y); free(buf); return -2; }
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = off[v + 1] - off[v];
        int64_t b = (int64_t)x0[v] + add;
        if (b < 1) b = 1;
        x[v] = (int32_t)(d == 0 ? 0 : (b < d ? b : d));
    }
    if (changed_round_of) memset(changed_round_of, 0, sizeof(int32_t) * (size_t)n);

    int64_t rounds = 0;
    for (int64_t t = 1; t <= max_rounds; ++t) {
        int64_t changed = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t d = off[v + 1] - off[v];
            for (int64_t j = 0; j < d; ++j) buf[j] = x[adj[off[v] + j]];
            int32_t h = h_index_sorted(buf, d);
            y[v] = h < x[v] ? h : x[v];
            if (y[v] != x[v]) {
                ++changed;
                if (changed_round_of) changed_round_of[v] = (int32_t)t;
            }
        }
        if (changed == 0) break;
        if (changed_per_round) changed_per_round[t - 1] = changed;
        rounds = t;
        int32_t *tmp = x; x = y; y = tmp;
    }
    memcpy(x_out, x, sizeof(int32_t) * (size_t)n);
    free(x); free(y); free(buf);
    return rounds;
}

/*
 * PeelOne without the dynamic frontier (the variant the paper measures in
 * Table IV against Alg. 4's in-level frontier), executed serially: at level
 * k each iteration takes the residual vertices whose residual degree equals
 * k, removes them with coreness k, and decrements each residual neighbour
 * whose residual degree is above k; vertices brought down to k wait for the
 * next iteration at the same level.  A level ends when an iteration finds
 * nobody; k then jumps to the smallest residual degree (an empty level is
 * not an iteration).  Returns the number of iterations (Table IV's l1 for
 * this variant), -1 on bad arguments, -2 on allocation failure; core_out
 * gets the coreness.
 */
int64_t oracle_peel_static(int64_t n, const int64_t *off, const int32_t *adj, int32_t *core_out)
{
    if (n < 0 || (n > 0 && (!off || !core_out))) return -1;
    if (n == 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char *alive = (unsigned char *)malloc((size_t)n);
    int32_t *frontier = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !alive || !frontier) { free(deg); free(alive); free(frontier); return -2; }
    int64_t left = 0;
    for (int64_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(off[v + 1] - off[v]);
        alive[v] = deg[v] > 0;
        core_out[v] = 0;
        left += alive[v];
    }
    int64_t iterations = 0;
    int32_t k = 1;
    while (left > 0) {
        int64_t nf = 0;
        for (int64_t v = 0; v < n; ++v)
            if (alive[v] && deg[v] == k) frontier[nf++] = (int32_t)v;
        if (nf == 0) {  /* empty level: jump to the smallest residual degree */
            int32_t mn = INT32_MAX;
            for (int64_t v = 0; v < n; ++v)
                if (alive[v] && deg[v] < mn) mn = deg[v];
            k = mn;
            continue;
        }
        ++iterations;
        for (int64_t i = 0; i < nf; ++i) {
            alive[frontier[i]] = 0;
            core_out[frontier[i]] = k;
        }
        left -= nf;
        for (int64_t i = 0; i < nf; ++i) {
            int32_t v = frontier[i];
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                int32_t u = adj[e];
                if (alive[u] && deg[u] > k) deg[u]--;
            }
        }
    }
    free(deg); free(alive); free(frontier);
    return iterations;
}

/*
 * CntCore (Alg. 5) and NbrCore (the Index2core baseline the paper compares
 * with, Section V: a vertex whose value changed makes all its neighbours
 * recompute), in synchronous rounds from x = deg, the h-index recomputed
 * from scratch for every vertex that needs it (no maintained histogram).
 *   CntCore (mode 1): round t takes the active set A (all vertices in round
 *     1, afterwards the neighbours of the previous frontier), computes
 *     cnt(v) = |{u in nbr(v) : x(u) >= x(v)}| for v in A, and the frontier
 *     F = {v in A : cnt(v) < x(v)} (Theorem 2: exactly the vertices whose
 *     h-index drops); if F is empty it stops; each v in F takes the h-index
 *     of its neighbours' values; the next A is the union of F's neighbours.
 *   NbrCore (mode 0): every v in A takes the h-index of its neighbours'
 *     values (capped at x(v)); C = those that changed; if C is empty it stops;
 *     the next A is the union of C's neighbours.
 * out[0] rounds that changed a value, [1] rounds run, [2] sum |A|, [3] sum of
 * h-index computations (|F| or |A|), [4] adjacency entries read by cnt
 * scans, [5] by h-index computations, [6] by neighbour marking, [7] sum over
 * rounds of activations after round 1.  x_out gets the coreness.  Returns 0,
 * -1 on bad arguments, -2 on allocation failure.
 */
int oracle_index2core(int64_t n, const int64_t *off, const int32_t *adj, int mode, int32_t *x_out,
                      int64_t *out)
{
    if (n < 0 || (n > 0 && (!off || !x_out)) || !out || (mode != 0 && mode != 1)) return -1;
    for (int i = 0; i < 8; ++i) out[i] = 0;
    if (n == 0) return 0;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] - off[v] > maxdeg) maxdeg = off[v + 1] - off[v];
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *y = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *fr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    if (!x || !y || !act || !nxt || !fr || !mark || !buf) {
        free(x); free(y); free(act); free(nxt); free(fr); free(mark); free(buf);
        return -2;
    }
    int64_t na = 0;
    for (int64_t v = 0; v < n; ++v) {
        x[v] = (int32_t)(off[v + 1] - off[v]);
        mark[v] = 0;
        if (x[v] > 0) act[na++] = (int32_t)v;
    }
    for (int64_t t = 1; na > 0; ++t) {
        out[1] += 1;
        out[2] += na;
        int64_t nf = 0;
        if (mode == 1) {
            for (int64_t i = 0; i < na; ++i) {
                int32_t v = act[i];
                int64_t cnt = 0;
                for (int64_t e = off[v]; e < off[v + 1]; ++e) cnt += x[adj[e]] >= x[v];
                out[4] += off[v + 1] - off[v];
                if (cnt < x[v]) fr[nf++] = v;
            }
            if (nf == 0) { out[1] -= 1; break; }  /* an empty frontier ends the run before any h-index */
        } else {
            for (int64_t i = 0; i < na; ++i) fr[nf++] = act[i];
        }
        out[3] += nf;
        /* h-index from the previous round's values for every frontier vertex */
        int64_t nc = 0;
        for (int64_t i = 0; i < nf; ++i) {
            int32_t v = fr[i];
            int64_t d = off[v + 1] - off[v];
            for (int64_t j = 0; j < d; ++j) buf[j] = x[adj[off[v] + j]];
            out[5] += d;
            int32_t h = h_index_sorted(buf, d);
            y[v] = h < x[v] ? h : x[v];
        }
        for (int64_t i = 0; i < nf; ++i) {
            int32_t v = fr[i];
            if (y[v] != x[v]) fr[nc++] = v;
        }
        for (int64_t i = 0; i < nc; ++i) x[fr[i]] = y[fr[i]];
        if (nc == 0) break;
        out[0] += 1;
        int64_t nn = 0;
        for (int64_t i = 0; i < nc; ++i) {
            int32_t v = fr[i];
            out[6] += off[v + 1] - off[v];
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                int32_t u = adj[e];
                if (mark[u] != t) {
                    mark[u] = t;
                    nxt[nn++] = u;
                }
            }
        }
        out[7] += nn;
        int32_t *tmp = act; act = nxt; nxt = tmp;
        na = nn;
    }
    memcpy(x_out, x, sizeof(int32_t) * (size_t)n);
    free(x); free(y); free(act); free(nxt); free(fr); free(mark); free(buf);
    return 0;
}

/*
 * General Parallel Peel (Alg. 3, Section II-C; the GPP baseline of Section V),
 * serially, in the algorithm's own order.  k starts at 0 and every vertex,
 * isolated ones included, starts residual.  Each iteration of the while loop
 * first raises k by one if no residual vertex has residual degree <= k, then
 * scans: the residual vertices of degree <= k (which may be none, when even
 * the raised k finds nobody) are removed with coreness k, and every residual
 * neighbour of a removed vertex loses one degree.  On G1 this takes the three
 * iterations Section III-A states.  Returns the number of iterations, -1 on
 * bad arguments, -2 on allocation failure; *decrements gets the number of
 * degree decrements (one per edge from a removed vertex to a residual one).
 */
int64_t oracle_peel_gpp(int64_t n, const int64_t *off, const int32_t *adj, int32_t *core_out,
                        int64_t *decrements)
{
    if (n < 0 || (n > 0 && (!off || !core_out)) || !decrements) return -1;
    *decrements = 0;
    if (n == 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char *alive = (unsigned char *)malloc((size_t)n);
    int32_t *frontier = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !alive || !frontier) { free(deg); free(alive); free(frontier); return -2; }
    for (int64_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(off[v + 1] - off[v]);
        alive[v] = 1;
        core_out[v] = 0;
    }
    int64_t left = n;
    int64_t iterations = 0;
    int32_t k = 0;
    while (left > 0) {
        ++iterations;
        /* the test that precedes the scan: is any residual vertex at or below k? */
        int any = 0;
        for (int64_t v = 0; v < n && !any; ++v)
            if (alive[v] && deg[v] <= k) any = 1;
        if (!any) ++k;
        /* scan */
        int64_t nf = 0;
        for (int64_t v = 0; v < n; ++v)
            if (alive[v] && deg[v] <= k) frontier[nf++] = (int32_t)v;
        for (int64_t i = 0; i < nf; ++i) {
            alive[frontier[i]] = 0;
            core_out[frontier[i]] = k;
        }
        left -= nf;
        /* scatter: residual neighbours only (the rem flag of Alg. 3) */
        for (int64_t i = 0; i < nf; ++i) {
            int32_t v = frontier[i];
            for (int64_t e = off[v]; e < off[v + 1]; ++e)
                if (alive[adj[e]]) {
                    deg[adj[e]]--;
                    ++*decrements;
                }
        }
    }
    free(deg); free(alive); free(frontier);
    return iterations;
}
