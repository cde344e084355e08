// Request server: continuous batching of decomposition requests.
//
// Requests name a device-resident CSR graph and a device output.  A request
// is admitted when its per-request scratch (the decomposition's working
// arrays) fits in the HBM arena the caller hands over.
//
// Small and medium requests (by vertex count) are launched together, largest
// first, as one batched-kernel call on a free launch slot (each slot its own
// stream; a workgroup per graph), and a slot is reused as soon as its launch
// has completed, so requests that arrive while others run are launched on a
// free slot right away and overlap on the device with the launches in
// flight.  A launch holds requests of one class only and completes with its
// slowest graph, so a small request never waits for a medium graph.
//
// Large requests would hold a workgroup -- and their launch -- for a long
// time; they run instead through the single-graph path (the persistent
// cooperative kernels, the whole GPU per graph) in an exclusive window: when
// large requests are waiting, no new batched launch starts, the slots drain,
// and then the waiting large requests (up to giant_window of them) are run
// back to back on the window's stream; batched launches resume when the
// window completes.  A cooperative kernel therefore never shares the device
// with a batched kernel, and windows alternate with batched launches so
// neither side starves.
//
// The server is driven by the caller: pico_server_submit queues a request,
// pico_server_progress reaps finished launches and windows (completion is an
// event per slot / window), launches what fits, and hands back completions.
// Nothing here blocks except pico_server_destroy.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "common.hpp"

namespace pico {
namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, bytes) of the arena, 256-byte granules, with
// coalescing of neighbouring free blocks.
class Arena {
  public:
    void reset(size_t bytes) {
        free_.clear();
        cap_ = bytes & ~(size_t)255;
        if (cap_) free_[0] = cap_;
        used_ = 0;
    }
    static size_t granule(size_t bytes) { return bytes ? (bytes + 255) & ~(size_t)255 : 256; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = granule(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = granule(bytes);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0;
};

constexpr int kClasses = 3;  // small, medium, large

struct Req {
    pico_request r;
    size_t bytes = 0, arena_off = 0;
    uint64_t t_submit = 0, t_launch = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    pico_task *staging = nullptr;  // pinned host copy of the task table
    void *ws = nullptr;            // device tasks workspace
    size_t ws_bytes = 0;
    std::vector<Req> reqs;
    int cls = 0;
    bool busy = false;
};

}  // namespace
}  // namespace pico

struct pico_server {
    pico_server_config cfg;
    int device = 0;
    int64_t bound[2] = {0, 0};  // vertex-count bounds of the small and medium classes
    int giant_window = 64;
    pico::Arena arena;
    std::deque<pico::Req> waiting[pico::kClasses];  // [2]: large requests for the window
    std::deque<pico_completion> ready;
    std::vector<pico::Slot> slots;
    // exclusive window of large requests
    hipStream_t gstream = nullptr;
    hipEvent_t gdone = nullptr;
    unsigned long long *gerr = nullptr;  // pinned: one error word per request of the window
    std::vector<pico::Req> gw;
    bool grunning = false;
    bool batched_turn = false;  // after a window, batched launches go first
    int64_t launches = 0, windows = 0, completed = 0;
};

namespace pico {
namespace {

int class_of(const pico_server *s, int64_t n) { return n < s->bound[0] ? 0 : n < s->bound[1] ? 1 : 2; }

void destroy_slots(pico_server *s) {
    if (s->gstream) (void)hipStreamSynchronize(s->gstream);
    if (s->gdone) (void)hipEventDestroy(s->gdone);
    if (s->gstream) (void)hipStreamDestroy(s->gstream);
    if (s->gerr) (void)hipHostFree(s->gerr);
    s->gstream = nullptr;
    s->gdone = nullptr;
    s->gerr = nullptr;
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.ws) (void)hipFree(sl.ws);
    }
    s->slots.clear();
}

int reap(pico_server *s) {
    for (Slot &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            set_error("launch slot failed: %s", hipGetErrorString(q));
            return PICO_EHIP;
        }
        const uint64_t t = now_ns();
        for (Req &r : sl.reqs) {
            s->arena.release(r.arena_off, r.bytes);
            pico_completion c;
            c.tag = r.r.tag;
            c.status = PICO_OK;
            c.reserved = 0;
            c.t_submit_ns = r.t_submit;
            c.t_launch_ns = r.t_launch;
            c.t_done_ns = t;
            s->ready.push_back(c);
            ++s->completed;
        }
        sl.reqs.clear();
        sl.busy = false;
    }
    return PICO_OK;
}

// Large requests take the exclusive window with PeelOne only: the
// single-graph HistoCore kernel indexes its histogram by CSR position and so
// needs offsets starting at 0, which a request's rows need not.  A HistoCore
// server launches its large requests in batched launches of their own class.
bool uses_window(const pico_server *s) { return (s->cfg.algo & PICO_ALGO_MASK) == PICO_ALGO_PEELONE; }

// The class a free slot serves next: the batched class whose oldest waiting
// request was submitted first, or -1.
int pick_class(const pico_server *s) {
    int best = -1;
    uint64_t t_best = 0;
    const int nc = uses_window(s) ? 2 : kClasses;
    for (int c = 0; c < nc; ++c) {
        if (s->waiting[c].empty()) continue;
        const uint64_t t = s->waiting[c].front().t_submit;
        if (best < 0 || t < t_best) {
            best = c;
            t_best = t;
        }
    }
    return best;
}

int reap_window(pico_server *s) {
    if (!s->grunning) return PICO_OK;
    const hipError_t q = hipEventQuery(s->gdone);
    if (q == hipErrorNotReady) return PICO_OK;
    if (q != hipSuccess) {
        set_error("large-request window failed: %s", hipGetErrorString(q));
        return PICO_EHIP;
    }
    const uint64_t t = now_ns();
    for (size_t i = 0; i < s->gw.size(); ++i) {
        Req &r = s->gw[i];
        s->arena.release(r.arena_off, r.bytes);
        pico_completion c;
        c.tag = r.r.tag;
        c.status = s->gerr[i] ? PICO_EHIP : PICO_OK;
        c.reserved = 0;
        c.t_submit_ns = r.t_submit;
        c.t_launch_ns = r.t_launch;
        c.t_done_ns = t;
        s->ready.push_back(c);
        ++s->completed;
    }
    s->gw.clear();
    s->grunning = false;
    s->batched_turn = true;
    return PICO_OK;
}

// Run the waiting large requests (up to giant_window, as the arena allows)
// back to back on the window stream.  Called only with every slot idle.
int launch_window(pico_server *s) {
    char *base = static_cast<char *>(s->cfg.arena);
    std::deque<Req> &q = s->waiting[2];
    const int algo = (s->cfg.algo & PICO_ALGO_MASK) | PICO_OFFSETS_I64;
    while (!q.empty() && (int)s->gw.size() < s->giant_window) {
        Req &r = q.front();
        const size_t need = ws_bytes_for(r.r.n, r.r.m, algo);
        size_t off = 0;
        if (!s->arena.alloc(need, &off)) break;
        r.bytes = need;
        r.arena_off = off;
        r.t_launch = now_ns();
        const size_t i = s->gw.size();
        s->gerr[i] = 0;
        int rc = r.r.n == 0 ? PICO_OK
                 : (algo & PICO_ALGO_MASK) == PICO_ALGO_PEELONE
                     ? run_peelone<int64_t>(r.r.offsets, r.r.cols, r.r.n, r.r.m, r.r.out_core, base + off,
                                            need, nullptr, s->gstream, &s->gerr[i])
                     : run_histocore<int64_t>(r.r.offsets, r.r.cols, r.r.n, r.r.m, r.r.out_core,
                                              base + off, need, nullptr, s->gstream, &s->gerr[i]);
        if (rc) {
            s->arena.release(off, need);
            return rc;
        }
        s->gw.push_back(r);
        q.pop_front();
    }
    if (s->gw.empty()) return PICO_OK;
    PICO_HIP_TRY(hipEventRecord(s->gdone, s->gstream));
    s->grunning = true;
    ++s->windows;
    return PICO_OK;
}

int launch(pico_server *s, Slot &sl, int cls) {
    const int64_t cap = s->cfg.max_tasks_per_launch;
    char *base = static_cast<char *>(s->cfg.arena);
    std::deque<Req> &q = s->waiting[cls];
    while (!q.empty() && (int64_t)sl.reqs.size() < cap) {
        Req &r = q.front();
        size_t off = 0;
        if (!s->arena.alloc(r.bytes, &off)) break;  // first come, first served
        r.arena_off = off;
        sl.reqs.push_back(r);
        q.pop_front();
    }
    if (sl.reqs.empty()) return PICO_OK;
    std::stable_sort(sl.reqs.begin(), sl.reqs.end(),
                     [](const Req &a, const Req &b) { return a.r.n > b.r.n; });
    const uint64_t t = now_ns();
    const int64_t T = (int64_t)sl.reqs.size();
    for (int64_t i = 0; i < T; ++i) {
        Req &r = sl.reqs[i];
        r.t_launch = t;
        pico_task &pt = sl.staging[i];
        pt.offsets = r.r.offsets;
        pt.cols = r.r.cols;
        pt.n = r.r.n;
        pt.m = r.r.m;
        pt.out_core = r.r.out_core;
        pt.scratch = base + r.arena_off;
        pt.scratch_bytes = r.bytes;
    }
    pico_task *dev = tasks_table(sl.ws, sl.ws_bytes, T);
    PICO_HIP_TRY(hipMemcpyAsync(dev, sl.staging, sizeof(pico_task) * T, hipMemcpyHostToDevice, sl.stream));
    const int algo = s->cfg.algo & PICO_ALGO_MASK;
    int rc = run_tasks_device(dev, T, algo, sl.ws, sl.ws_bytes, &s->cfg.tune, nullptr, sl.stream);
    if (rc) return rc;
    PICO_HIP_TRY(hipEventRecord(sl.done, sl.stream));
    sl.cls = cls;
    sl.busy = true;
    ++s->launches;
    return PICO_OK;
}

}  // namespace
}  // namespace pico

using namespace pico;

int pico_server_create(const pico_server_config *cfg, pico_server **out) {
    clear_error();
    if (!cfg || !out) {
        set_error("NULL argument to pico_server_create");
        return PICO_EINVAL;
    }
    *out = nullptr;
    const int a = cfg->algo & PICO_ALGO_MASK;
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE) || (cfg->algo & ~PICO_ALGO_MASK) != 0) {
        set_error("unknown algo %d", cfg->algo);
        return PICO_EINVAL;
    }
    if (cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->max_tasks_per_launch < 1 ||
        cfg->giant_window < 0 || cfg->giant_window > 4096 || (cfg->arena_bytes > 0 && !cfg->arena) ||
        ((uintptr_t)cfg->arena & 255) != 0 || cfg->tune.reserved != 0 || cfg->class_bounds[0] < 0 ||
        cfg->class_bounds[1] < 0 ||
        (cfg->class_bounds[0] > 0 && cfg->class_bounds[1] > 0 && cfg->class_bounds[1] < cfg->class_bounds[0])) {
        set_error("bad server configuration (max_inflight %d, max_tasks_per_launch %lld, arena %p)",
                  cfg->max_inflight, (long long)cfg->max_tasks_per_launch, cfg->arena);
        return PICO_EINVAL;
    }
    int rc = check_device();
    if (rc) return rc;
    pico_server *s = new (std::nothrow) pico_server();
    if (!s) {
        set_error("host allocation failed");
        return PICO_ENOMEM;
    }
    s->cfg = *cfg;
    s->bound[0] = cfg->class_bounds[0] > 0 ? cfg->class_bounds[0] : 16384;
    s->bound[1] = cfg->class_bounds[1] > 0 ? cfg->class_bounds[1] : 65536;
    if (s->bound[1] < s->bound[0]) s->bound[1] = s->bound[0];
    s->giant_window = cfg->giant_window > 0 ? cfg->giant_window : 64;
    (void)hipGetDevice(&s->device);
    s->arena.reset(cfg->arena_bytes);
    s->slots.resize((size_t)cfg->max_inflight);
    const int64_t T = cfg->max_tasks_per_launch;
    hipError_t e = hipSuccess;
    for (Slot &sl : s->slots) {
        sl.ws_bytes = tasks_ws_bytes(T);
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipHostMalloc((void **)&sl.staging, sizeof(pico_task) * T, hipHostMallocDefault)) !=
            hipSuccess)
            break;
        if ((e = hipMalloc(&sl.ws, sl.ws_bytes)) != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->gdone, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->gerr, sizeof(unsigned long long) * (size_t)s->giant_window,
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        set_error("server set-up failed: %s", hipGetErrorString(e));
        destroy_slots(s);
        delete s;
        return e == hipErrorOutOfMemory ? PICO_ENOMEM : PICO_EHIP;
    }
    *out = s;
    return PICO_OK;
}

int pico_server_submit(pico_server *s, const pico_request *req) {
    clear_error();
    if (!s || !req) {
        set_error("NULL argument to pico_server_submit");
        return PICO_EINVAL;
    }
    if (req->n < 0 || req->n > INT32_MAX || req->m < 0 ||
        (req->n > 0 && (!req->offsets || !req->out_core)) || (req->m > 0 && !req->cols)) {
        set_error("bad request (n %lld, m %lld)", (long long)req->n, (long long)req->m);
        return PICO_EINVAL;
    }
    Req r;
    r.r = *req;
    const int cls = class_of(s, req->n);
    r.bytes = cls == 2 && uses_window(s)
                  ? ws_bytes_for(req->n, req->m, (s->cfg.algo & PICO_ALGO_MASK) | PICO_OFFSETS_I64)
                  : task_scratch_bytes(req->n, req->m, s->cfg.algo);
    if (Arena::granule(r.bytes) > s->arena.capacity()) {
        set_error("request needs %zu bytes of scratch, the arena holds %zu", r.bytes, s->arena.capacity());
        return PICO_ENOMEM;
    }
    r.t_submit = now_ns();
    s->waiting[cls].push_back(r);
    return PICO_OK;
}

int pico_server_progress(pico_server *s, pico_completion *done, int max_done, int *num_done) {
    clear_error();
    if (!s || (max_done > 0 && !done) || max_done < 0) {
        set_error("bad arguments to pico_server_progress");
        return PICO_EINVAL;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != s->device) PICO_HIP_TRY(hipSetDevice(s->device));
    int rc = reap(s);
    if (!rc) rc = reap_window(s);
    bool any_busy = false;
    for (const Slot &sl : s->slots) any_busy = any_busy || sl.busy;
    const bool giants = uses_window(s) && !s->waiting[2].empty();
    if (!rc && !s->grunning && giants && !any_busy && !s->batched_turn) {
        rc = launch_window(s);  // the device is free of batched kernels
    } else if (!rc && !s->grunning && !(giants && !s->batched_turn)) {
        // batched launches (held while large requests wait for the device to drain)
        for (Slot &sl : s->slots) {
            if (rc) break;
            if (sl.busy) continue;
            const int c = pick_class(s);
            if (c < 0) break;
            rc = launch(s, sl, c);
            if (!rc && !sl.busy) break;  // nothing fitted in the arena: wait for completions
        }
        s->batched_turn = false;
    }
    if (cur != s->device) (void)hipSetDevice(cur);
    int k = 0;
    while (k < max_done && !s->ready.empty()) {
        done[k++] = s->ready.front();
        s->ready.pop_front();
    }
    if (num_done) *num_done = k;
    return rc;
}

int pico_server_query(const pico_server *s, pico_server_status *st) {
    clear_error();
    if (!s || !st) {
        set_error("NULL argument to pico_server_query");
        return PICO_EINVAL;
    }
    int64_t inflight = (int64_t)s->gw.size(), busy = s->grunning ? 1 : 0;
    for (const Slot &sl : s->slots) {
        inflight += (int64_t)sl.reqs.size();
        busy += sl.busy ? 1 : 0;
    }
    int64_t waiting = 0;
    for (int c = 0; c < kClasses; ++c) waiting += (int64_t)s->waiting[c].size();
    st->waiting = waiting;
    st->inflight = inflight;
    st->ready = (int64_t)s->ready.size();
    st->busy_slots = busy;
    st->launches = s->launches + s->windows;
    st->completed = s->completed;
    st->arena_used = (int64_t)s->arena.used();
    st->arena_bytes = (int64_t)s->arena.capacity();
    return PICO_OK;
}

int pico_server_destroy(pico_server *s) {
    clear_error();
    if (!s) return PICO_OK;
    destroy_slots(s);
    delete s;
    return PICO_OK;
}
