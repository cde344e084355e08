// Request server: continuous batching of decomposition requests.
//
// Requests name a device-resident CSR graph and a device output.  A request
// is admitted when its per-request scratch (the decomposition's working
// arrays) fits in the HBM arena the caller hands over.  Admitted requests are
// launched together, largest first, as one batched-kernel call on a free
// launch slot (each slot its own stream), and a slot is reused as soon as its
// launch has completed, so requests that arrive while others run are launched
// on a free slot right away and their work overlaps on the device with the
// launches already in flight.
//
// A launch completes only with its slowest graph, so requests are kept in
// three size classes (by vertex count) and a launch takes requests of one
// class only: a small request never waits for a large graph of the same
// launch.  Large requests may hold at most max_large_slots slots at a time,
// so the small and medium classes always find a slot.  Among the classes
// allowed on a free slot, the one whose oldest request has waited longest
// goes first.
//
// The server is driven by the caller: pico_server_submit queues a request,
// pico_server_progress reaps finished launches (completion is an event per
// slot), launches what fits, and hands back completions.  Nothing here blocks
// except pico_server_destroy.
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
    int32_t *status = nullptr;     // pinned host copy of the launch's status words
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
    int max_large = 1;
    pico::Arena arena;
    std::deque<pico::Req> waiting[pico::kClasses];
    std::deque<pico_completion> ready;
    std::vector<pico::Slot> slots;
    int64_t launches = 0, completed = 0;
};

namespace pico {
namespace {

int class_of(const pico_server *s, int64_t n) { return n < s->bound[0] ? 0 : n < s->bound[1] ? 1 : 2; }

void destroy_slots(pico_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.status) (void)hipHostFree(sl.status);
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
        for (size_t i = 0; i < sl.reqs.size(); ++i) {
            Req &r = sl.reqs[i];
            s->arena.release(r.arena_off, r.bytes);
            pico_completion c;
            c.tag = r.r.tag;
            // the launch's status word for this request (copied after the
            // kernels, before the slot's event): PICO_OK, or PICO_EHIP if a
            // wait bound left it unfinished
            c.status = sl.status[i];
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

// The class a free slot serves next: the allowed class whose oldest waiting
// request was submitted first, or -1.
int pick_class(const pico_server *s) {
    int large_busy = 0;
    for (const Slot &sl : s->slots) large_busy += (sl.busy && sl.cls == 2) ? 1 : 0;
    int best = -1;
    uint64_t t_best = 0;
    for (int c = 0; c < kClasses; ++c) {
        if (s->waiting[c].empty()) continue;
        if (c == 2 && large_busy >= s->max_large) continue;
        const uint64_t t = s->waiting[c].front().t_submit;
        if (best < 0 || t < t_best) {
            best = c;
            t_best = t;
        }
    }
    return best;
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
    const int hm = help_min_large(&s->cfg.tune, algo);
    int64_t n_large = 0;
    for (const Req &r : sl.reqs) n_large += (hm > 0 && r.r.n >= hm) ? 1 : 0;
    int rc = run_tasks_device(dev, T, algo, sl.ws, sl.ws_bytes, &s->cfg.tune, nullptr, sl.stream,
                              n_large);
    if (rc) return rc;
    PICO_HIP_TRY(hipMemcpyAsync(sl.status, status_words(sl.ws), sizeof(int32_t) * T, hipMemcpyDeviceToHost,
                                sl.stream));
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
    if ((a != PICO_ALGO_PEELONE && a != PICO_ALGO_HISTOCORE && a != PICO_ALGO_AUTO) ||
        (cfg->algo & ~PICO_ALGO_MASK) != 0) {
        set_error("unknown algo %d", cfg->algo);
        return PICO_EINVAL;
    }
    if (cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->max_tasks_per_launch < 1 ||
        cfg->max_large_slots < 0 || (cfg->arena_bytes > 0 && !cfg->arena) ||
        ((uintptr_t)cfg->arena & 255) != 0 || cfg->tune.help_min_vertices < -1 || cfg->class_bounds[0] < 0 ||
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
    s->bound[1] = cfg->class_bounds[1] > 0 ? cfg->class_bounds[1] : 131072;
    if (s->bound[1] < s->bound[0]) s->bound[1] = s->bound[0];
    s->max_large = cfg->max_large_slots > 0 ? cfg->max_large_slots : std::max(1, cfg->max_inflight / 2);
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
        if ((e = hipHostMalloc((void **)&sl.status, sizeof(int32_t) * T, hipHostMallocDefault)) != hipSuccess)
            break;
        if ((e = hipMalloc(&sl.ws, sl.ws_bytes)) != hipSuccess) break;
    }
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
    r.bytes = task_scratch_bytes(req->n, req->m, s->cfg.algo);
    if (Arena::granule(r.bytes) > s->arena.capacity()) {
        set_error("request needs %zu bytes of scratch, the arena holds %zu", r.bytes, s->arena.capacity());
        return PICO_ENOMEM;
    }
    r.t_submit = now_ns();
    s->waiting[class_of(s, req->n)].push_back(r);
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
    for (Slot &sl : s->slots) {
        if (rc) break;
        if (sl.busy) continue;
        const int c = pick_class(s);
        if (c < 0) break;
        rc = launch(s, sl, c);
        if (!rc && !sl.busy) break;  // nothing fitted in the arena: wait for completions
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
    int64_t inflight = 0, busy = 0;
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
    st->launches = s->launches;
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
