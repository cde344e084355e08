// C ABI of the k-core library: argument checks, workspace, dispatch on the
// offsets width, status codes and error strings.  The problem solved is the
// one of the paper's Section I (coreness of every vertex of an undirected
// graph); the algorithms live in peelone.hip (Alg. 4) and histocore.hip
// (Alg. 6).
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace pico {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// Set while pico_coreness_noalloc runs on this host thread: read-backs go to
// a fixed thread-local buffer instead of pinned memory, and no profiling
// events are created.
static thread_local bool g_no_alloc = false;

void *host_scratch(size_t bytes) {
    if (g_no_alloc) {
        alignas(256) static thread_local unsigned char fixed[1 << 14];
        if (bytes > sizeof(fixed)) {
            set_error("read-back of %zu bytes exceeds the fixed host buffer (%zu)", bytes, sizeof(fixed));
            return nullptr;
        }
        return fixed;
    }
    static thread_local void *buf = nullptr;
    static thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        size_t want = bytes < 4096 ? 4096 : bytes;
        hipError_t e = hipHostMalloc(&buf, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            set_error("hipHostMalloc(%zu) failed: %s", want, hipGetErrorString(e));
            buf = nullptr;
            return nullptr;
        }
        cap = want;
    }
    return buf;
}

int persistent_grid(const void *kernel, int block, int max_per_cu, long long want, int *blocks) {
    int dev = 0;
    PICO_HIP_TRY(hipGetDevice(&dev));
    int cus = 0, coop = 0;
    PICO_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PICO_HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) {
        set_error("device %d does not support cooperative launches", dev);
        return PICO_ENOTSUP;
    }
    int per_cu = 0;
    PICO_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
    if (per_cu > max_per_cu) per_cu = max_per_cu;
    if (per_cu < 1) {
        set_error("persistent kernel does not fit on a compute unit");
        return PICO_ENOTSUP;
    }
    long long b = (long long)per_cu * cus;
    const int forced = tune_int("PICO_GRID_BLOCKS", 0);  // development override
    if (forced > 0) want = forced;
    if (want > 0 && want < b) b = want;
    *blocks = (int)b;
    return PICO_OK;
}

int tune_int(const char *name, int dflt) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    int x = atoi(v);
    return x > 0 ? x : dflt;
}

int tune_int_nonneg(const char *name, int dflt) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    int x = atoi(v);
    return x >= 0 ? x : dflt;
}

unsigned long long wall_ticks(double seconds) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;  // 100 MHz, the usual constant clock
    return (unsigned long long)(seconds * 1000.0 * (double)khz);
}

namespace {

struct ProfRec {
    const char *name;
    hipEvent_t start, stop;
};

struct ProfState {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<ProfRec> pending;
    std::vector<pico_kernel_stat> table;
};

thread_local ProfState g_prof;

hipEvent_t prof_event() {
    if (g_prof.used == g_prof.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof.pool.push_back(e);
    }
    return g_prof.pool[g_prof.used++];
}

// Fold the recorded launches of the finished call into the table.
int prof_resolve() {
    int rc = PICO_OK;
    for (const ProfRec &r : g_prof.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess ||
            hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            set_error("profiling events could not be resolved");
            rc = PICO_EHIP;
            continue;
        }
        pico_kernel_stat *slot = nullptr;
        for (auto &t : g_prof.table)
            if (strcmp(t.name, r.name) == 0) slot = &t;
        if (!slot) {
            g_prof.table.push_back(pico_kernel_stat{r.name, 0, 0.0});
            slot = &g_prof.table.back();
        }
        slot->launches += 1;
        slot->total_ms += ms;
    }
    g_prof.pending.clear();
    g_prof.used = 0;
    return rc;
}


int check_args(const void *off, const int32_t *cols, int64_t n, int64_t m, int algo,
               const int32_t *out) {
    int a = algo & PICO_ALGO_MASK;
    if (a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO && a != PICO_ALGO_CNTCORE &&
        a != PICO_ALGO_NBRCORE) {
        set_error("unknown algo %d", algo);
        return PICO_EINVAL;
    }
    if ((a == PICO_ALGO_CNTCORE || a == PICO_ALGO_NBRCORE) && (algo & PICO_PATH_WG)) {
        set_error("CntCore and NbrCore run on the grid path only");
        return PICO_ENOTSUP;
    }
    if ((algo & ~(PICO_ALGO_MASK | PICO_OFFSETS_I64 | PICO_PATH_GRID | PICO_PATH_WG | PICO_PO_STATIC |
                  PICO_PO_ROLLBACK | PICO_PO_GPP)) != 0) {
        set_error("unknown flag bits in algo 0x%x", algo);
        return PICO_EINVAL;
    }
    if ((algo & PICO_PATH_GRID) && (algo & PICO_PATH_WG)) {
        set_error("PICO_PATH_GRID and PICO_PATH_WG are exclusive");
        return PICO_EINVAL;
    }
    const int abl = algo & (PICO_PO_STATIC | PICO_PO_ROLLBACK | PICO_PO_GPP);
    if (abl) {
        if (a != PICO_ALGO_PEELONE || (abl & (abl - 1))) {
            set_error("PICO_PO_STATIC / PICO_PO_ROLLBACK / PICO_PO_GPP: one of them, with PeelOne only");
            return PICO_EINVAL;
        }
        if (algo & PICO_PATH_WG) {
            set_error("the PeelOne ablations run on the grid path only");
            return PICO_ENOTSUP;
        }
    }
    if (n < 0 || m < 0) {
        set_error("negative size (n=%lld, m=%lld)", (long long)n, (long long)m);
        return PICO_EINVAL;
    }
    if (n >= (int64_t)1 << 31) {
        set_error("n=%lld does not fit 32-bit vertex ids", (long long)n);
        return PICO_EINVAL;
    }
    if (!(algo & PICO_OFFSETS_I64) && m >= (int64_t)1 << 31) {
        set_error("m=%lld needs int64 offsets (PICO_OFFSETS_I64)", (long long)m);
        return PICO_EINVAL;
    }
    if (n > 0 && (!off || !out)) {
        set_error("NULL offsets or output with n=%lld", (long long)n);
        return PICO_EINVAL;
    }
    if (m > 0 && !cols) {
        set_error("NULL columns with m=%lld", (long long)m);
        return PICO_EINVAL;
    }
    return PICO_OK;
}


// warm / warm_add: HistoCore started from given upper bounds (nullptr: from
// the degrees).
// The algorithm PICO_ALGO_AUTO runs on this graph (features measured only
// when the rule needs them).
int pick_algo(const void *off, const int32_t *cols, int64_t n, int64_t m, int algo, void *ws,
              size_t ws_bytes, hipStream_t s, int *chosen, int64_t feat[3]) {
    feat[0] = feat[1] = feat[2] = 0;
    *chosen = PICO_ALGO_PEELONE;
    if (m < (1ll << 16)) return PICO_OK;  // the rule's first case needs no features
    const bool i64 = (algo & PICO_OFFSETS_I64) != 0;
    int rc = i64 ? select_features<int64_t>(static_cast<const int64_t *>(off), cols, n, m, ws, ws_bytes, s, feat)
                 : select_features<int32_t>(static_cast<const int32_t *>(off), cols, n, m, ws, ws_bytes, s, feat);
    if (rc) return rc;
    *chosen = choose_algo(n, m, feat[0], feat[1], feat[2]);
    return PICO_OK;
}

int dispatch(const void *off, const int32_t *cols, int64_t n, int64_t m, int algo, int32_t *out,
             void *ws, size_t ws_bytes, pico_stats *st, hipStream_t s, const int32_t *warm = nullptr,
             int warm_add = 0, pico_step *sched = nullptr, int64_t sched_cap = 0,
             int64_t *sched_len = nullptr) {
    const bool i64 = (algo & PICO_OFFSETS_I64) != 0;
    if ((algo & PICO_ALGO_MASK) == PICO_ALGO_AUTO) {
        int chosen = PICO_ALGO_PEELONE;
        int64_t feat[3];
        int rc = pick_algo(off, cols, n, m, algo, ws, ws_bytes, s, &chosen, feat);
        if (rc) return rc;
        algo = (algo & ~PICO_ALGO_MASK) | chosen;
    }
    if (st) st->algo_used = algo & PICO_ALGO_MASK;
    const int base = algo & PICO_ALGO_MASK;
    if (base == PICO_ALGO_CNTCORE || base == PICO_ALGO_NBRCORE) {
        const int mode = base == PICO_ALGO_CNTCORE ? 1 : 0;
        return i64 ? run_index2core<int64_t>(static_cast<const int64_t *>(off), cols, n, m, out, ws, ws_bytes, st,
                                             s, mode)
                   : run_index2core<int32_t>(static_cast<const int32_t *>(off), cols, n, m, out, ws, ws_bytes, st,
                                             s, mode);
    }
    bool small = false;
    int rc = small_path(n, m, algo, &small);
    if (rc) return rc;
    if (small)
        return i64 ? run_small<int64_t>(static_cast<const int64_t *>(off), cols, n, m, algo, out, ws,
                                        ws_bytes, st, s, warm, warm_add)
                   : run_small<int32_t>(static_cast<const int32_t *>(off), cols, n, m, algo, out, ws,
                                        ws_bytes, st, s, warm, warm_add);
    if ((algo & PICO_ALGO_MASK) == PICO_ALGO_PEELONE) {
        const int mode = (algo & PICO_PO_STATIC) ? 1 : (algo & PICO_PO_ROLLBACK) ? 2 : (algo & PICO_PO_GPP) ? 3 : 0;
        return i64 ? run_peelone<int64_t>(static_cast<const int64_t *>(off), cols, n, m, out, ws,
                                          ws_bytes, st, s, mode, sched, sched_cap, sched_len)
                   : run_peelone<int32_t>(static_cast<const int32_t *>(off), cols, n, m, out, ws,
                                          ws_bytes, st, s, mode, sched, sched_cap, sched_len);
    }
    return i64 ? run_histocore<int64_t>(static_cast<const int64_t *>(off), cols, n, m, out, ws,
                                        ws_bytes, st, s, warm, warm_add, sched, sched_cap, sched_len)
               : run_histocore<int32_t>(static_cast<const int32_t *>(off), cols, n, m, out, ws,
                                        ws_bytes, st, s, warm, warm_add, sched, sched_cap, sched_len);
}

template <typename Off>
__global__ void validate_kernel(const Off *__restrict__ off, const int32_t *__restrict__ cols,
                                long long n, long long m, int *__restrict__ bad) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        long long a = (long long)off[v], b = (long long)off[v + 1];
        if (v == 0 && a != 0) atomicOr(bad, 1);
        if (v == n - 1 && b != m) atomicOr(bad, 2);
        if (b < a || a < 0 || b > m) {
            atomicOr(bad, 4);
            continue;
        }
        for (long long e = a; e < b; ++e) {
            int u = cols[e];
            if (u < 0 || u >= n) atomicOr(bad, 8);
            else if (u == v) atomicOr(bad, 16);
        }
    }
}

}  // namespace

size_t ws_bytes_for(int64_t n, int64_t m, int algo) {
    const int a = algo & PICO_ALGO_MASK;
    if (a == PICO_ALGO_AUTO) {  // either algorithm, and the features before it
        size_t b = select_ws_bytes(n, m);
        for (int x : {PICO_ALGO_PEELONE, PICO_ALGO_HISTOCORE}) {
            const size_t w = ws_bytes_for(n, m, (algo & ~PICO_ALGO_MASK) | x);
            if (w > b) b = w;
        }
        return b;
    }
    if (a == PICO_ALGO_CNTCORE || a == PICO_ALGO_NBRCORE) return index2core_ws_bytes(n, m);
    // enough for either path, so the path may change without a new workspace
    const size_t grid = a == PICO_ALGO_PEELONE ? peelone_ws_bytes(n, m) : histocore_ws_bytes(n, m);
    const size_t small = small_ws_bytes(n, m, algo);
    return grid > small ? grid : small;
}

int check_device() {
    int dev = -1;
    PICO_HIP_TRY(hipGetDevice(&dev));
    static int checked[64] = {0};  // 0 unknown, 1 ok, -1 unsupported
    if (dev >= 0 && dev < 64 && checked[dev] != 0) return checked[dev] > 0 ? PICO_OK : PICO_ENOTSUP;
    hipDeviceProp_t prop;
    PICO_HIP_TRY(hipGetDeviceProperties(&prop, dev));
    bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev >= 0 && dev < 64) checked[dev] = ok ? 1 : -1;
    if (!ok) {
        set_error("device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
        return PICO_ENOTSUP;
    }
    return PICO_OK;
}

int prof_begin(const char *name, hipStream_t s) {
    if (!g_prof.on || g_no_alloc) return -1;
    ProfRec r{name, prof_event(), prof_event()};
    if (!r.start || !r.stop) return -1;
    if (hipEventRecord(r.start, s) != hipSuccess) return -1;
    g_prof.pending.push_back(r);
    return (int)g_prof.pending.size() - 1;
}

void prof_end(int rec, hipStream_t s) {
    if (rec >= 0) (void)hipEventRecord(g_prof.pending[rec].stop, s);
}

}  // namespace pico

using namespace pico;

// Workspace of pico_coreness_noalloc: one array per GPU, held until the
// process ends.  Host code never passes its name to a kernel (on the host it
// is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[PICO_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of `scratch`.
int scratch_for_current_device(void **out) {
    int dev = -1;
    PICO_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal %d out of range for the static scratch table", dev);
        return PICO_ENOTSUP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
            return PICO_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PICO_OK;
}

struct NoAllocScope {
    NoAllocScope() { g_no_alloc = true; }
    ~NoAllocScope() { g_no_alloc = false; }
};

}  // namespace

static bool tune_ok(const pico_batch_tune *tune) {
    if (tune && tune->help_min_vertices < -1) {
        set_error("pico_batch_tune.help_min_vertices must be -1, 0 or positive");
        return false;
    }
    return true;
}

extern "C" {

const char *pico_version(void) { return "pico-mi355x 0.1 (gfx950)"; }

const char *pico_last_error(void) { return g_err; }

const char *pico_status_string(int status) {
    switch (status) {
        case PICO_OK: return "ok";
        case PICO_EINVAL: return "invalid argument";
        case PICO_ENOMEM: return "out of memory or workspace too small";
        case PICO_EHIP: return "HIP runtime error";
        case PICO_ENOTSUP: return "unsupported device or option";
        case PICO_EBADCSR: return "malformed CSR graph";
        default: return "unknown status";
    }
}

int pico_profile_enable(int on) {
    clear_error();
    g_prof.on = on != 0;
    if (g_prof.on) g_prof.table.clear();
    return PICO_OK;
}

int pico_profile_read(pico_kernel_stat *out, int cap, int *count) {
    clear_error();
    if (!count || (cap > 0 && !out) || cap < 0) {
        set_error("bad profile_read arguments");
        return PICO_EINVAL;
    }
    *count = (int)g_prof.table.size();
    for (int i = 0; i < cap && i < (int)g_prof.table.size(); ++i) out[i] = g_prof.table[i];
    return PICO_OK;
}

int pico_workspace_bytes(int64_t n, int64_t m, int algo, size_t *bytes) {
    clear_error();
    int rc = check_args((const void *)1, (const int32_t *)1, n, m, algo, (const int32_t *)1);
    if (rc) return rc;
    if (!bytes) {
        set_error("NULL bytes pointer");
        return PICO_EINVAL;
    }
    *bytes = ws_bytes_for(n, m, algo);
    return PICO_OK;
}

}  // extern "C"

namespace {

// pico_coreness_ws and pico_coreness_update: warm == nullptr starts from the
// degrees.
int coreness_ws(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m, int algo,
                int32_t *out_core, void *workspace, size_t ws_bytes, pico_stats *stats, void *stream,
                const int32_t *warm, int warm_add, pico_step *sched = nullptr, int64_t sched_cap = 0,
                int64_t *sched_len = nullptr) {
    if (stats) memset(stats, 0, sizeof(*stats));
    int rc = check_args(csr_offsets, csr_cols, n, m, algo, out_core);
    if (rc) return rc;
    if (n == 0) return PICO_OK;
    rc = check_device();
    if (rc) return rc;
    size_t need = ws_bytes_for(n, m, algo);
    if (ws_bytes < need || !workspace) {
        set_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
        return PICO_ENOMEM;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return PICO_EINVAL;
    }
    auto t0 = std::chrono::steady_clock::now();
    rc = dispatch(csr_offsets, csr_cols, n, m, algo, out_core, workspace, ws_bytes, stats,
                  static_cast<hipStream_t>(stream), warm, warm_add, sched, sched_cap, sched_len);
    if (rc) {
        g_prof.pending.clear();
        g_prof.used = 0;
        return rc;
    }
    PICO_HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    rc = prof_resolve();
    if (rc) return rc;
    if (stats) {
        stats->elapsed_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return PICO_OK;
}

}  // namespace

extern "C" {

int pico_coreness_ws(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                     int algo, int32_t *out_core, void *workspace, size_t ws_bytes,
                     pico_stats *stats, void *stream) {
    clear_error();
    return coreness_ws(csr_offsets, csr_cols, n, m, algo, out_core, workspace, ws_bytes, stats, stream,
                       nullptr, 0);
}

int pico_coreness_schedule(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m, int algo,
                           int32_t *out_core, void *workspace, size_t ws_bytes, pico_stats *stats,
                           pico_step *steps, int64_t cap, int64_t *num_steps, void *stream) {
    clear_error();
    if (stats) memset(stats, 0, sizeof(*stats));
    if (num_steps) *num_steps = 0;
    const int a = algo & PICO_ALGO_MASK;
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO) ||
        (algo & ~(PICO_ALGO_MASK | PICO_OFFSETS_I64 | PICO_PATH_GRID)) != 0) {
        set_error("pico_coreness_schedule records PeelOne, HistoCore or AUTO on the grid path (algo 0x%x)",
                  algo);
        return PICO_EINVAL;
    }
    if (cap < 0 || (cap > 0 && !steps)) {
        set_error("bad schedule array (cap %lld)", (long long)cap);
        return PICO_EINVAL;
    }
    return coreness_ws(csr_offsets, csr_cols, n, m, algo | PICO_PATH_GRID, out_core, workspace, ws_bytes,
                       stats, stream, nullptr, 0, cap > 0 ? steps : nullptr, cap, num_steps);
}

int pico_select_algorithm(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m, int algo,
                          void *workspace, size_t ws_bytes, int *algo_out, int64_t *features, void *stream) {
    clear_error();
    if ((algo & PICO_ALGO_MASK) != PICO_ALGO_AUTO || (algo & ~(PICO_ALGO_MASK | PICO_OFFSETS_I64)) != 0) {
        set_error("pico_select_algorithm takes PICO_ALGO_AUTO (| PICO_OFFSETS_I64), got 0x%x", algo);
        return PICO_EINVAL;
    }
    if (!algo_out) {
        set_error("NULL algo_out");
        return PICO_EINVAL;
    }
    int32_t dummy_out = 0;
    int rc = check_args(csr_offsets, csr_cols, n, m, algo, &dummy_out);
    if (rc) return rc;
    int64_t feat[3] = {0, 0, 0};
    *algo_out = PICO_ALGO_PEELONE;
    if (n > 0) {
        rc = check_device();
        if (rc) return rc;
        const size_t need = ws_bytes_for(n, m, algo);
        if (ws_bytes < need || !workspace) {
            set_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
            return PICO_ENOMEM;
        }
        rc = pick_algo(csr_offsets, csr_cols, n, m, algo, workspace, ws_bytes, static_cast<hipStream_t>(stream),
                       algo_out, feat);
        if (rc) return rc;
    }
    if (features)
        for (int i = 0; i < 3; ++i) features[i] = feat[i];
    return PICO_OK;
}

int pico_coreness_update(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                         int algo, const int32_t *prev_core, int32_t bound_add, int32_t *out_core,
                         void *workspace, size_t ws_bytes, pico_stats *stats, void *stream) {
    clear_error();
    if (stats) memset(stats, 0, sizeof(*stats));
    if ((algo & PICO_ALGO_MASK) != PICO_ALGO_HISTOCORE) {
        set_error("pico_coreness_update runs HistoCore only (PeelOne cannot start from bounds)");
        return (algo & PICO_ALGO_MASK) == PICO_ALGO_PEELONE ? PICO_ENOTSUP : PICO_EINVAL;
    }
    if (bound_add < 0) {
        set_error("bound_add must be >= 0 (got %d)", bound_add);
        return PICO_EINVAL;
    }
    if (n > 0 && !prev_core) {
        set_error("NULL prev_core with n=%lld", (long long)n);
        return PICO_EINVAL;
    }
    return coreness_ws(csr_offsets, csr_cols, n, m, algo, out_core, workspace, ws_bytes, stats, stream,
                       prev_core, bound_add);
}

int pico_coreness(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m, int algo,
                  int32_t *out_core, void *stream) {
    clear_error();
    int rc = check_args(csr_offsets, csr_cols, n, m, algo, out_core);
    if (rc) return rc;
    if (n == 0) return PICO_OK;
    rc = check_device();
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t need = ws_bytes_for(n, m, algo);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, need, s);
    if (e != hipSuccess) {
        set_error("hipMallocAsync(%zu) failed: %s", need, hipGetErrorString(e));
        return PICO_ENOMEM;
    }
    rc = dispatch(csr_offsets, csr_cols, n, m, algo, out_core, ws, need, nullptr, s);
    hipError_t fe = hipFreeAsync(ws, s);
    if (rc) {
        g_prof.pending.clear();
        g_prof.used = 0;
        return rc;
    }
    if (fe != hipSuccess) {
        set_error("hipFreeAsync failed: %s", hipGetErrorString(fe));
        return PICO_EHIP;
    }
    PICO_HIP_TRY(hipStreamSynchronize(s));
    return prof_resolve();
}

int pico_coreness_noalloc(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m, int algo,
                          int32_t *out_core, void *stream) {
    clear_error();
    int rc = check_args(csr_offsets, csr_cols, n, m, algo, out_core);
    if (rc) return rc;
    if (n == 0) return PICO_OK;
    const size_t need = ws_bytes_for(n, m, algo);
    if (need > (size_t)PICO_NOALLOC_SCRATCH_BYTES) {
        set_error("graph needs %zu bytes of scratch; the static scratch holds %zu (n=%lld, m=%lld)", need,
                  (size_t)PICO_NOALLOC_SCRATCH_BYTES, (long long)n, (long long)m);
        return PICO_ENOMEM;
    }
    rc = check_device();
    if (rc) return rc;
    void *ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    NoAllocScope scope;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = dispatch(csr_offsets, csr_cols, n, m, algo, out_core, ws, need, nullptr, s);
    if (rc) return rc;
    PICO_HIP_TRY(hipStreamSynchronize(s));
    return PICO_OK;
}

int pico_batched_workspace_bytes(int64_t num_graphs, int64_t total_n, int64_t total_m, int algo,
                                 size_t *bytes) {
    clear_error();
    int a = algo & PICO_ALGO_MASK;
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO) || num_graphs < 0 || total_n < 0 ||
        total_m < 0 || !bytes) {
        set_error("bad arguments to pico_batched_workspace_bytes");
        return PICO_EINVAL;
    }
    *bytes = batched_ws_bytes(num_graphs, total_n, total_m, algo);
    return PICO_OK;
}

int pico_coreness_batched(const int64_t *graph_vptr, const int64_t *csr_offsets,
                          const int32_t *csr_cols, int64_t num_graphs, int64_t total_n,
                          int64_t total_m, int algo, const int32_t *order, int32_t *out_core,
                          const pico_batch_tune *tune, void *workspace, size_t ws_bytes,
                          pico_batch_stats *stats, void *stream) {
    clear_error();
    if (stats) memset(stats, 0, sizeof(*stats));
    int a = algo & PICO_ALGO_MASK;
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO) ||
        (algo & ~(PICO_ALGO_MASK | PICO_OFFSETS_I64)) != 0) {
        set_error("unknown algo %d", algo);
        return PICO_EINVAL;
    }
    if (num_graphs < 0 || total_n < 0 || total_m < 0) {
        set_error("negative size");
        return PICO_EINVAL;
    }
    if (!tune_ok(tune)) return PICO_EINVAL;
    if (num_graphs == 0) return PICO_OK;
    if (!graph_vptr || (total_n > 0 && (!csr_offsets || !out_core)) || (total_m > 0 && !csr_cols)) {
        set_error("NULL pointer with a non-empty batch");
        return PICO_EINVAL;
    }
    int rc = check_device();
    if (rc) return rc;
    size_t need = batched_ws_bytes(num_graphs, total_n, total_m, algo);
    if (!workspace || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
        return PICO_ENOMEM;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return PICO_EINVAL;
    }
    rc = run_batched(reinterpret_cast<const long long *>(graph_vptr),
                     reinterpret_cast<const long long *>(csr_offsets), csr_cols, num_graphs, total_n,
                     total_m, a, order, out_core, workspace, ws_bytes, tune, stats,
                     static_cast<hipStream_t>(stream));
    if (rc) {
        g_prof.pending.clear();
        g_prof.used = 0;
        return rc;
    }
    if (g_prof.on) {
        PICO_HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
        return prof_resolve();
    }
    return PICO_OK;
}


int pico_task_scratch_bytes(int64_t n, int64_t m, int algo, size_t *bytes) {
    clear_error();
    int a = algo & PICO_ALGO_MASK;
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO) || n < 0 || n > INT32_MAX ||
        m < 0 || !bytes) {
        set_error("bad arguments to pico_task_scratch_bytes");
        return PICO_EINVAL;
    }
    *bytes = task_scratch_bytes(n, m, a);
    return PICO_OK;
}

int pico_tasks_workspace_bytes(int64_t num_tasks, size_t *bytes) {
    clear_error();
    if (num_tasks < 0 || !bytes) {
        set_error("bad arguments to pico_tasks_workspace_bytes");
        return PICO_EINVAL;
    }
    *bytes = tasks_ws_bytes(num_tasks);
    return PICO_OK;
}

int pico_coreness_tasks(const pico_task *tasks, int64_t num_tasks, int algo,
                        const pico_batch_tune *tune, void *workspace, size_t ws_bytes,
                        pico_batch_stats *stats, void *stream) {
    clear_error();
    if (stats) memset(stats, 0, sizeof(*stats));
    int a = algo & PICO_ALGO_MASK;
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO) ||
        (algo & ~(PICO_ALGO_MASK | PICO_OFFSETS_I64)) != 0) {
        set_error("unknown algo %d", algo);
        return PICO_EINVAL;
    }
    if (num_tasks < 0 || (num_tasks > 0 && !tasks) || !tune_ok(tune)) {
        if (num_tasks < 0 || (num_tasks > 0 && !tasks)) set_error("bad task list");
        return PICO_EINVAL;
    }
    if (num_tasks == 0) return PICO_OK;
    for (int64_t i = 0; i < num_tasks; ++i) {
        const pico_task &t = tasks[i];
        if (t.n < 0 || t.n > INT32_MAX || t.m < 0 || (t.n > 0 && (!t.offsets || !t.out_core)) ||
            (t.m > 0 && !t.cols)) {
            set_error("task %lld: bad sizes or NULL pointer (n %lld, m %lld)", (long long)i,
                      (long long)t.n, (long long)t.m);
            return PICO_EINVAL;
        }
        if (t.n == 0) continue;
        const size_t need = task_scratch_bytes(t.n, t.m, a);
        if (!t.scratch || t.scratch_bytes < need) {
            set_error("task %lld: scratch of %zu bytes given, %zu needed", (long long)i,
                      t.scratch_bytes, need);
            return PICO_ENOMEM;
        }
        if (((uintptr_t)t.scratch & 255) != 0) {
            set_error("task %lld: scratch must be 256-byte aligned", (long long)i);
            return PICO_EINVAL;
        }
    }
    int rc = check_device();
    if (rc) return rc;
    const size_t need = tasks_ws_bytes(num_tasks);
    if (!workspace || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
        return PICO_ENOMEM;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return PICO_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    pico_task *dev = tasks_table(workspace, ws_bytes, num_tasks);
    PICO_HIP_TRY(hipMemcpyAsync(dev, tasks, sizeof(pico_task) * num_tasks, hipMemcpyHostToDevice, s));
    const int hm = help_min_large(tune, a);
    int64_t n_large = 0;
    for (int64_t i = 0; i < num_tasks; ++i) n_large += (hm > 0 && tasks[i].n >= hm) ? 1 : 0;
    rc = run_tasks_device(dev, num_tasks, a, workspace, ws_bytes, tune, stats, s, n_large);
    if (rc) {
        g_prof.pending.clear();
        g_prof.used = 0;
        return rc;
    }
    if (g_prof.on) {
        PICO_HIP_TRY(hipStreamSynchronize(s));
        return prof_resolve();
    }
    return PICO_OK;
}

int pico_batch_status(const void *workspace, size_t ws_bytes, int64_t count, int32_t *status, void *stream) {
    clear_error();
    if (count < 0 || (count > 0 && !workspace) || ws_bytes < (size_t)count * 4) {
        set_error("bad arguments to pico_batch_status (count %lld, %zu workspace bytes)", (long long)count,
                  ws_bytes);
        return PICO_EINVAL;
    }
    if (count == 0) return PICO_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> host;
    int32_t *dst = status;
    if (!dst) {
        host.resize((size_t)count);
        dst = host.data();
    }
    PICO_HIP_TRY(hipStreamSynchronize(s));
    PICO_HIP_TRY(hipMemcpy(dst, status_words(workspace), sizeof(int32_t) * (size_t)count, hipMemcpyDeviceToHost));
    int64_t unfinished = 0, invalid = 0, other = 0;
    int first = PICO_OK;
    for (int64_t i = 0; i < count; ++i) {
        const int v = dst[i];
        if (v == PICO_OK) continue;
        if (first == PICO_OK) first = v == PICO_EHIP || v == PICO_EINVAL ? v : PICO_EHIP;
        if (v == PICO_EHIP) ++unfinished;
        else if (v == PICO_EINVAL) ++invalid;
        else ++other;
    }
    if (first != PICO_OK)
        set_error("%lld graphs unfinished, %lld with an invalid vertex range, %lld with an unknown status word",
                  (long long)unfinished, (long long)invalid, (long long)other);
    return first;
}

int pico_validate_csr(const void *csr_offsets, const int32_t *csr_cols, int64_t n, int64_t m,
                      int algo, void *stream) {
    clear_error();
    int rc = check_args(csr_offsets, csr_cols, n, m, algo, (const int32_t *)1);
    if (rc) return rc;
    if (n == 0) return m == 0 ? PICO_OK : PICO_EBADCSR;
    rc = check_device();
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int *bad = nullptr;
    PICO_HIP_TRY(hipMallocAsync((void **)&bad, sizeof(int), s));
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
    if (e == hipSuccess) {
        int grid = (int)((n + 255) / 256 > 4096 ? 4096 : (n + 255) / 256);
        if (algo & PICO_OFFSETS_I64)
            hipLaunchKernelGGL(validate_kernel<int64_t>, dim3(grid), dim3(256), 0, s,
                               static_cast<const int64_t *>(csr_offsets), csr_cols, (long long)n,
                               (long long)m, bad);
        else
            hipLaunchKernelGGL(validate_kernel<int32_t>, dim3(grid), dim3(256), 0, s,
                               static_cast<const int32_t *>(csr_offsets), csr_cols, (long long)n,
                               (long long)m, bad);
        e = hipGetLastError();
    }
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    hipError_t fe = hipFreeAsync(bad, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || fe != hipSuccess) {
        set_error("validation failed to run: %s", hipGetErrorString(e != hipSuccess ? e : fe));
        return PICO_EHIP;
    }
    if (hbad) {
        set_error("malformed CSR (flags 0x%x: 1 off[0]!=0, 2 off[n]!=m, 4 bad offsets, "
                  "8 column out of range, 16 self-loop)", hbad);
        return PICO_EBADCSR;
    }
    return PICO_OK;
}

}  // extern "C"
