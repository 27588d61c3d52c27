// Runtime services of the library: thread-local error messages, the caching
// device memory pool, pinned staging buffers and event-based kernel timing.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>

#include "gw_internal.h"

namespace gw {

// ------------------------------------------------------------------ errors --
static thread_local std::string t_last_error;

void set_last_error(const std::string &msg) { t_last_error = msg; }

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

// -------------------------------------------------------------------- pool --
namespace {

struct BlockInfo {
    size_t cls;
    int device;
};

// Free lists are per (device, host thread, size class): a block freed while
// kernels of its thread's stream may still read it can only be reused by the
// same thread, hence on the same stream, in stream order.  Every blocking
// entry point synchronizes its stream before returning, so a thread never
// switches streams with such work pending.
struct Key {
    int device;
    int thread;
    size_t cls;
    bool operator<(const Key &o) const {
        if (device != o.device) return device < o.device;
        if (thread != o.thread) return thread < o.thread;
        return cls < o.cls;
    }
};

int thread_tag() {
    static std::atomic<int> next{0};
    static thread_local int tag = next.fetch_add(1);
    return tag;
}

struct Pool {
    std::mutex mu;
    std::map<Key, std::vector<void *>> free_lists;
    std::unordered_map<void *, BlockInfo> live;
    size_t cached = 0, in_use = 0;
};

Pool &pool() {
    static Pool *p = new Pool();  // never destroyed: blocks may be freed at exit
    return *p;
}

}  // namespace

size_t pool_class_bytes(size_t bytes) {
    if (bytes <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)bytes);
    size_t step = (size_t)1 << (e - 3);
    return (bytes + step - 1) / step * step;
}

void *pool_alloc(size_t bytes) {
    size_t cls = pool_class_bytes(bytes);
    int dev = 0;
    GW_HIP(hipGetDevice(&dev));
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto it = P.free_lists.find(Key{dev, thread_tag(), cls});
        if (it != P.free_lists.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            P.cached -= cls;
            P.in_use += cls;
            P.live[p] = {cls, dev};
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give cached blocks back and retry once
        GW_HIP(hipDeviceSynchronize());
        pool_trim();
        e = hipMalloc(&p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(GW_ENOMEM, "device allocation of " + std::to_string(cls) + " bytes failed");
        }
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.live[p] = {cls, dev};
    P.in_use += cls;
    return p;
}

namespace {
// Set while a SideJob enqueues its work: blocks freed then are held by it.
thread_local std::vector<void *> *t_defer = nullptr;
}  // namespace

void pool_free(void *p) {
    if (!p) return;
    if (t_defer) {
        t_defer->push_back(p);
        return;
    }
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    BlockInfo bi = it->second;
    P.live.erase(it);
    P.in_use -= bi.cls;
    P.cached += bi.cls;
    P.free_lists[Key{bi.device, thread_tag(), bi.cls}].push_back(p);
}

void pool_trim() {
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : P.free_lists) {
        if (kv.second.empty()) continue;
        (void)hipSetDevice(kv.first.device);
        for (void *p : kv.second) (void)hipFree(p);
        P.cached -= kv.first.cls * kv.second.size();
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

void pool_release_thread() {
    // blocks this thread freed and nobody took since: no stream of this
    // thread uses them any more once the thread's work is synchronized
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    const int me = thread_tag();
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : P.free_lists) {
        if (kv.first.thread != me || kv.second.empty()) continue;
        (void)hipSetDevice(kv.first.device);
        for (void *p : kv.second) (void)hipFree(p);
        P.cached -= kv.first.cls * kv.second.size();
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

// ------------------------------------------------------------------ pinned --
namespace {

void *&thread_stage() {
    static thread_local void *stage = nullptr;
    return stage;
}

std::map<int, hipStream_t> &thread_side_streams() {
    static thread_local std::map<int, hipStream_t> streams;
    return streams;
}

}  // namespace

void *host_stage() {
    // one per host thread, kept until the thread calls
    // release_thread_resources (threads that never do keep it for the life
    // of the process, which avoids freeing pinned memory during runtime
    // teardown)
    void *&stage = thread_stage();
    if (!stage) {
        GW_HIP(hipHostMalloc(&stage, kHostStageBytes, hipHostMallocDefault));
        std::memset(stage, 0, kHostStageBytes);
    }
    return stage;
}

hipStream_t side_stream() {
    // one per (host thread, device), created on first use; non-blocking, so
    // that it is ordered against the caller's stream by events only, and at
    // the default priority
    auto &streams = thread_side_streams();
    int dev = 0;
    GW_HIP(hipGetDevice(&dev));
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    GW_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams[dev] = st;
    return st;
}

void SideJob::begin(hipStream_t s) {
    GW_REQUIRE(!pending && !deferring_, "side job already running");
    q = side_stream();
    if (!start) GW_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    if (!done) GW_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    GW_HIP(hipEventRecord(start, s));
    GW_HIP(hipStreamWaitEvent(q, start, 0));
    prev_ = t_defer;
    t_defer = &held;
    deferring_ = true;
}

void SideJob::end_defer() {
    if (!deferring_) return;
    t_defer = prev_;
    deferring_ = false;
}

void SideJob::join(hipStream_t s) {
    if (!pending) return;
    GW_HIP(hipStreamWaitEvent(s, done, 0));
    pending = false;
    // every later kernel of s runs after the side work: its blocks may go back
    for (void *p : held) pool_free(p);
    held.clear();
}

SideJob::~SideJob() {
    end_defer();
    if (q && (pending || !held.empty())) (void)hipStreamSynchronize(q);
    for (void *p : held) pool_free(p);
    if (start) (void)hipEventDestroy(start);
    if (done) (void)hipEventDestroy(done);
}

void release_thread_resources() {
    auto &streams = thread_side_streams();
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : streams) {
        (void)hipSetDevice(kv.first);
        (void)hipStreamSynchronize(kv.second);
        (void)hipStreamDestroy(kv.second);
    }
    streams.clear();
    (void)hipSetDevice(cur);
    void *&stage = thread_stage();
    if (stage) {
        (void)hipHostFree(stage);
        stage = nullptr;
    }
    pool_release_thread();
}

Pinned::Pinned(size_t bytes) : n(bytes) {
    GW_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    std::memset(p, 0, bytes);
}
Pinned::~Pinned() {
    if (p) (void)hipHostFree(p);
}

// ------------------------------------------------------------------ timing --
namespace {

struct ProfState {
    std::mutex mu;
    bool on = false;
    int only = -1;  // record one kernel class only (-1: all)
    struct Pending {
        int id;
        double bytes, cbytes;
        hipEvent_t e0, e1;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    int64_t launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    double bytes[K_COUNT] = {};
    double cbytes[K_COUNT] = {};
};

ProfState &prof() {
    static ProfState *p = new ProfState();
    return *p;
}

const char *const kNames[K_COUNT] = {
    "fv_assemble", "darcy_flux", "tt_assemble",
    "setup_misc", "transpose", "strength", "mis2", "aggregate", "spgemm", "coarse_lu", "sell_build",
    "smooth_first_l0", "smooth_l0", "residual_l0", "restrict_l0", "prolong_l0",
    "smooth_first_l1", "smooth_l1", "residual_l1", "restrict_l1", "prolong_l1",
    "smooth_first_lc", "smooth_lc", "residual_lc", "restrict_lc", "prolong_lc", "coarse_solve",
    "krylov_spmv", "krylov_update", "krylov_dot", "true_residual",
    "sweep_lists", "sweep"};

hipEvent_t take_event(ProfState &P) {
    if (!P.spare.empty()) {
        hipEvent_t e = P.spare.back();
        P.spare.pop_back();
        return e;
    }
    hipEvent_t e;
    GW_HIP(hipEventCreate(&e));
    return e;
}

}  // namespace

const char *kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? kNames[id] : "?"; }

bool prof_on() { return prof().on; }

ProfScope::ProfScope(int id_, double bytes_, hipStream_t s_, bool ext_, double cbytes_)
    : id(id_), bytes(bytes_), cbytes(cbytes_ < 0.0 ? bytes_ : cbytes_), s(s_), ext(ext_) {
    ProfState &P = prof();
    if (!P.on || (P.only >= 0 && P.only != id)) return;
    // launches being captured into a graph are not timed one by one
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> g(P.mu);
    e0 = take_event(P);
    e1 = take_event(P);
    if (!ext) GW_HIP(hipEventRecord(e0, s));
}

ProfScope::~ProfScope() {
    if (!e0) return;
    ProfState &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (!ext && hipEventRecord(e1, s) != hipSuccess) return;
    P.pending.push_back({id, bytes, cbytes, e0, e1});
}

void prof_flush() {
    ProfState &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto &x : P.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(x.e1) == hipSuccess && hipEventElapsedTime(&ms, x.e0, x.e1) == hipSuccess) {
            P.launches[x.id] += 1;
            P.ms[x.id] += ms;
            P.bytes[x.id] += x.bytes;
            P.cbytes[x.id] += x.cbytes;
        }
        P.spare.push_back(x.e0);
        P.spare.push_back(x.e1);
    }
    P.pending.clear();
}

}  // namespace gw

// ------------------------------------------------------------- C entries --
extern "C" {

const char *gw_last_error(void) { return gw::t_last_error.c_str(); }

int gw_trim(void) {
    return gw::guarded([&] {
        GW_HIP(hipDeviceSynchronize());
        gw::pool_trim();
        return GW_OK;
    });
}

int gw_prof_enable(int32_t on) {
    return gw::guarded([&] {
        gw::prof_flush();
        auto &P = gw::prof();
        std::lock_guard<std::mutex> g(P.mu);
        if (on) {
            std::fill(P.launches, P.launches + gw::K_COUNT, 0);
            std::fill(P.ms, P.ms + gw::K_COUNT, 0.0);
            std::fill(P.bytes, P.bytes + gw::K_COUNT, 0.0);
            std::fill(P.cbytes, P.cbytes + gw::K_COUNT, 0.0);
        }
        P.on = on != 0;
        return GW_OK;
    });
}

int gw_prof_select(const char *name) {
    return gw::guarded([&] {
        auto &P = gw::prof();
        std::lock_guard<std::mutex> g(P.mu);
        if (!name || !*name) {
            P.only = -1;
            return GW_OK;
        }
        for (int i = 0; i < gw::K_COUNT; ++i)
            if (std::strcmp(name, gw::kNames[i]) == 0) {
                P.only = i;
                return GW_OK;
            }
        gw::fail(GW_EINVAL, std::string("gw_prof_select: unknown kernel ") + name);
    });
}

int gw_prof_read(gw_kernel_stat *out, int32_t max, int32_t *n) {
    return gw::guarded([&] {
        gw::prof_flush();
        auto &P = gw::prof();
        std::lock_guard<std::mutex> g(P.mu);
        int32_t k = 0;
        for (int i = 0; i < gw::K_COUNT; ++i) {
            if (k < max && out) {
                std::memset(&out[k], 0, sizeof(gw_kernel_stat));
                std::strncpy(out[k].name, gw::kNames[i], sizeof(out[k].name) - 1);
                out[k].launches = P.launches[i];
                out[k].ms = P.ms[i];
                out[k].bytes = P.bytes[i];
                out[k].bytes_csr = P.cbytes[i];
            }
            ++k;
        }
        if (n) *n = k;
        return GW_OK;
    });
}

}  // extern "C"
