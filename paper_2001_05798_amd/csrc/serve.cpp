// Serving loop: continuous batching of dual-delineation requests (a flow
// solve, then the travel-time pair on its Darcy velocities).
//
// A queue owns `max_slots` slot workers, each with its own HIP stream.  A
// free slot takes the oldest waiting request as soon as the request's device
// footprint fits in what the HBM budget has left (first come, first served:
// a request that does not fit holds back the ones behind it, so nothing
// starves).  Requests in different slots run concurrently and their kernels
// overlap on the device; a request that arrives while others run joins as
// soon as a slot and memory free up.  Hierarchies stay resident for the
// duration of a request: the travel-time hierarchy serves both right-hand
// sides.  With the setup cache on (queue_set_setup_cache), the flow
// hierarchy outlives its request: a later request with the same conductance
// field, grid, boundary heads and AMG parameters takes it instead of a new
// setup, since wells change only the right-hand side (the Discussion's
// setup caching, here across requests such as the runs of a sensitivity
// analysis on well rates).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "gw_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kMaxWaiting = 4096;

// Upper bound of the device bytes one request can hold at its peak (setup
// temporaries included), per cell, plus a fixed part; measured hierarchies
// stay well below it (see amg_hierarchy_info).
size_t footprint_bytes(const gw_request &r) {
    const double n = (double)r.grid.nx * r.grid.ny * r.grid.nz;
    // (the travel-time pair solve keeps 20 FP64 vectors and two-column level
    // vectors: about 200 B per cell of its own)
    const double per_cell = (r.flow_params.precision == GW_PRECISION_MIXED ? 1900.0 : 1700.0);
    return (size_t)(n * per_cell) + ((size_t)64 << 20);
}

// Two independent 64-bit hashes of the bytes (words mixed by multiply and
// xor-shift), with everything else that determines the flow matrix.
void mix(uint64_t &h, uint64_t w) {
    h ^= w + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
}

struct SetupKey {
    uint64_t h[2];
    bool operator==(const SetupKey &o) const { return h[0] == o.h[0] && h[1] == o.h[1]; }
};

SetupKey setup_key(const gw_request &r) {
    SetupKey k{{0x243F6A8885A308D3ull, 0x13198A2E03707344ull}};
    auto word = [&](uint64_t w) {
        mix(k.h[0], w);
        mix(k.h[1], w ^ 0xA4093822299F31D0ull);
    };
    auto dbl = [&](double d) {
        uint64_t w;
        std::memcpy(&w, &d, 8);
        word(w);
    };
    const gw_grid &g = r.grid;
    word((uint64_t)g.nx);
    word((uint64_t)g.ny);
    word((uint64_t)g.nz);
    dbl(g.dx);
    dbl(g.dy);
    dbl(g.dz);
    dbl(r.bc.h_west);
    dbl(r.bc.h_east);
    const amg_params &p = r.flow_params;
    dbl(p.eps_strong);
    word((uint64_t)p.smoother);
    dbl(p.omega);
    word((uint64_t)p.npre);
    word((uint64_t)p.npost);
    word((uint64_t)p.n_coarse);
    word((uint64_t)p.max_levels);
    word((uint64_t)p.precision);
    word((uint64_t)p.seed);
    word((uint64_t)p.coarsening);
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const uint64_t *K = reinterpret_cast<const uint64_t *>(r.K);
    for (int64_t i = 0; i < n; ++i) word(K[i]);
    return k;
}

struct CachedSetup {
    SetupKey key;
    amg_hierarchy *H = nullptr;
    size_t bytes = 0;
    bool in_use = false;
    uint64_t last_use = 0;
};

struct Job {
    uint64_t ticket;
    gw_request req;
    std::vector<gw_well> wells;
    size_t bytes;
    double t_arrival;
};

}  // namespace

struct gw_queue {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job> waiting;
    std::map<uint64_t, gw_result> finished;
    std::map<uint64_t, int> state;  // 0 waiting, 1 running
    size_t budget = 0, reserved = 0;
    int running = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    int device = 0;
    Clock::time_point t0;
    std::vector<std::thread> workers;
    // flow hierarchies kept after their request (bytes counted in `reserved`)
    std::vector<CachedSetup> cache;
    int cache_max = 0;
    uint64_t use_clock = 0;

    double clock() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void worker();
    int run(Job &job, hipStream_t s, gw_result &res);
    // With mu held: drop the least recently used idle entry; false if none.
    bool evict_one() {
        int best = -1;
        for (int i = 0; i < (int)cache.size(); ++i)
            if (!cache[i].in_use && (best < 0 || cache[i].last_use < cache[best].last_use)) best = i;
        if (best < 0) return false;
        amg_free(cache[best].H);
        reserved -= cache[best].bytes;
        cache.erase(cache.begin() + best);
        return true;
    }
    bool can_evict() const {
        for (const auto &c : cache)
            if (!c.in_use) return true;
        return false;
    }
};

namespace {

struct DevArrays {
    gw::DBuf<double> K, b, h, qx, qy, qz, tau, c, val;
    gw::DBuf<int32_t> rowptr, col;
};

}  // namespace

// One request on stream s: assemble, flow setup + solve, Darcy, travel time.
int gw_queue::run(Job &job, hipStream_t s, gw_result &res) {
    const gw_request &r = job.req;
    const gw_grid &g = r.grid;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    DevArrays d;
    d.K.alloc(n);
    d.b.alloc(n);
    d.h.alloc(n);
    d.rowptr.alloc((size_t)n + 1);
    const int64_t nnz = fv_nnz(&g);
    d.col.alloc((size_t)nnz);
    d.val.alloc((size_t)nnz);
    GW_HIP(hipMemcpyAsync(d.K.p, r.K, sizeof(double) * n, hipMemcpyHostToDevice, s));
    int st = fv_assemble(&g, d.K.p, &r.bc, job.wells.data(), (int32_t)job.wells.size(), d.rowptr.p, d.col.p,
                         d.val.p, d.b.p, s);
    if (st != GW_OK) return st;
    amg_hierarchy *H = nullptr;
    const double ts = std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
    SetupKey key{};
    bool caching = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        caching = cache_max > 0;
    }
    if (caching) {
        key = setup_key(r);
        std::lock_guard<std::mutex> lk(mu);
        for (auto &c : cache)
            if (!c.in_use && c.key == key) {
                c.in_use = true;
                H = c.H;
                res.setup_reused = 1;
                break;
            }
    }
    if (!H) {
        gw_csr A{(int32_t)n, nnz, d.rowptr.p, d.col.p, d.val.p};
        st = amg_setup(&A, &r.flow_params, &H, s);
        if (st != GW_OK) return st;
    }
    const double setup_ms =
        std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count() - ts;
    st = amg_solve_pcg(H, d.b.p, d.h.p, &r.solve, &res.flow, s);
    GW_HIP(hipStreamSynchronize(s));
    {
        // hand the hierarchy back to the cache, or keep a new one there
        std::lock_guard<std::mutex> lk(mu);
        bool kept = false;
        for (auto &c : cache)
            if (c.H == H) {
                c.in_use = false;
                c.last_use = ++use_clock;
                kept = true;
            }
        if (!kept && caching && cache_max > 0 && st >= 0) {
            while ((int)cache.size() >= cache_max && evict_one()) {
            }
            if ((int)cache.size() < cache_max) {
                CachedSetup c;
                c.key = key;
                c.H = H;
                int32_t nl = 0;
                (void)amg_hierarchy_info(H, nullptr, 0, &nl, &c.bytes);
                c.last_use = ++use_clock;
                reserved += c.bytes;
                cache.push_back(c);
                kept = true;
            }
        }
        if (!kept) amg_free(H);
    }
    res.flow.setup_ms = setup_ms;
    d.val.release();
    d.col.release();
    d.rowptr.release();
    d.b.release();
    if (st < 0) return st;
    int flow_status = st;
    d.qx.alloc((size_t)(g.nx + 1) * g.ny * g.nz);
    d.qy.alloc((size_t)g.nx * (g.ny + 1) * g.nz);
    d.qz.alloc((size_t)g.nx * g.ny * (g.nz + 1));
    st = darcy_flux(&g, d.K.p, &r.bc, d.h.p, d.qx.p, d.qy.p, d.qz.p, s);
    if (st != GW_OK) return st;
    if (r.h_out) GW_HIP(hipMemcpyAsync(r.h_out, d.h.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    d.tau.alloc(n);
    d.c.alloc(n);
    st = tt_solve(&g, d.qx.p, d.qy.p, d.qz.p, r.phi, &r.zone, &r.tt_params, &r.solve, d.tau.p, d.c.p, res.tt, s);
    if (st < 0) return st;
    if (r.tau_out) GW_HIP(hipMemcpyAsync(r.tau_out, d.tau.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    if (r.c_out) GW_HIP(hipMemcpyAsync(r.c_out, d.c.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    if (flow_status != GW_OK) return flow_status;
    return st;
}

void gw_queue::worker() {
    hipStream_t s = nullptr;
    bool have_stream = false;
    for (;;) {
        Job job;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop || (!waiting.empty() && (reserved + waiting.front().bytes <= budget || can_evict()));
            });
            if (stop) break;
            // cached setups give way to a request that does not fit beside them
            while (reserved + waiting.front().bytes > budget && evict_one()) {
            }
            if (reserved + waiting.front().bytes > budget) continue;
            job = std::move(waiting.front());
            waiting.pop_front();
            reserved += job.bytes;
            ++running;
            state[job.ticket] = 1;
        }
        gw_result res{};
        res.t_arrival = job.t_arrival;
        res.t_start = clock();
        res.bytes_reserved = job.bytes;
        int st = gw::guarded([&] {
            if (!have_stream) {
                GW_HIP(hipSetDevice(device));
                GW_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                have_stream = true;
            }
            return run(job, s, res);
        });
        res.status = st;
        res.t_done = clock();
        if (st < 0) std::strncpy(res.error, gw_last_error(), sizeof(res.error) - 1);
        {
            std::lock_guard<std::mutex> lk(mu);
            reserved -= job.bytes;
            --running;
            state.erase(job.ticket);
            finished[job.ticket] = res;
        }
        cv_work.notify_all();
        cv_done.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(s);
}

extern "C" {

int queue_create(size_t hbm_budget_bytes, int32_t max_slots, gw_queue **q) {
    return gw::guarded([&] {
        GW_REQUIRE(q, "queue_create: null output");
        *q = nullptr;
        GW_REQUIRE(max_slots >= 1 && max_slots <= 64, "queue_create: max_slots must be in [1, 64]");
        GW_REQUIRE(hbm_budget_bytes > 0, "queue_create: empty budget");
        std::unique_ptr<gw_queue> Q(new gw_queue());
        Q->budget = hbm_budget_bytes;
        Q->t0 = Clock::now();
        int dev = 0;
        (void)hipGetDevice(&dev);  // no device yet is fine: workers bind lazily
        (void)hipGetLastError();
        Q->device = dev;
        for (int i = 0; i < max_slots; ++i) Q->workers.emplace_back([p = Q.get()] { p->worker(); });
        *q = Q.release();
        return GW_OK;
    });
}

double queue_clock(const gw_queue *q) { return q ? q->clock() : 0.0; }

int queue_submit(gw_queue *q, const gw_request *req, uint64_t *ticket) {
    return gw::guarded([&] {
        GW_REQUIRE(q && req && ticket, "queue_submit: null pointer");
        const gw_grid &g = req->grid;
        GW_REQUIRE(g.nx > 0 && g.ny > 0 && g.nz > 0 && (int64_t)g.nx * g.ny * g.nz < ((int64_t)1 << 30),
                   "queue_submit: bad grid");
        GW_REQUIRE(g.dx > 0 && g.dy > 0 && g.dz > 0, "queue_submit: bad spacing");
        GW_REQUIRE(req->K, "queue_submit: null K");
        GW_REQUIRE(req->nwells >= 0 && req->nwells <= 64 && (req->nwells == 0 || req->wells),
                   "queue_submit: bad wells");
        GW_REQUIRE(req->phi > 0 && std::isfinite(req->phi), "queue_submit: porosity must be positive");
        Job job;
        job.req = *req;
        job.wells.assign(req->wells, req->wells + req->nwells);
        job.bytes = footprint_bytes(*req);
        std::lock_guard<std::mutex> lk(q->mu);
        if (job.bytes > q->budget) gw::fail(GW_ENOMEM, "queue_submit: request footprint exceeds the HBM budget");
        if (q->waiting.size() >= kMaxWaiting) gw::fail(GW_EAGAIN, "queue_submit: queue full");
        job.t_arrival = req->t_arrival >= 0 ? req->t_arrival : q->clock();
        job.ticket = q->next_ticket++;
        *ticket = job.ticket;
        q->state[job.ticket] = 0;
        q->waiting.push_back(std::move(job));
        q->cv_work.notify_one();
        return GW_OK;
    });
}

int queue_poll(gw_queue *q, uint64_t ticket, gw_result *res) {
    return gw::guarded([&] {
        GW_REQUIRE(q, "queue_poll: null queue");
        std::lock_guard<std::mutex> lk(q->mu);
        auto it = q->finished.find(ticket);
        if (it == q->finished.end()) {
            GW_REQUIRE(q->state.count(ticket), "queue_poll: unknown ticket");
            return GW_PENDING;
        }
        if (res) *res = it->second;
        int st = it->second.status;
        q->finished.erase(it);
        return st;
    });
}

int queue_drain(gw_queue *q) {
    return gw::guarded([&] {
        GW_REQUIRE(q, "queue_drain: null queue");
        std::unique_lock<std::mutex> lk(q->mu);
        q->cv_done.wait(lk, [&] { return q->waiting.empty() && q->running == 0; });
        return GW_OK;
    });
}

int queue_set_setup_cache(gw_queue *q, int32_t max_entries) {
    return gw::guarded([&] {
        GW_REQUIRE(q, "queue_set_setup_cache: null queue");
        GW_REQUIRE(max_entries >= 0 && max_entries <= 64, "queue_set_setup_cache: max_entries must be in [0, 64]");
        {
            std::lock_guard<std::mutex> lk(q->mu);
            q->cache_max = max_entries;
            while ((int)q->cache.size() > max_entries && q->evict_one()) {
            }
        }
        q->cv_work.notify_all();
        return GW_OK;
    });
}

void queue_destroy(gw_queue *q) {
    if (!q) return;
    {
        std::unique_lock<std::mutex> lk(q->mu);
        q->cv_done.wait(lk, [&] { return q->running == 0; });
        q->stop = true;
        q->waiting.clear();
    }
    q->cv_work.notify_all();
    for (auto &t : q->workers) t.join();
    for (auto &c : q->cache) amg_free(c.H);
    delete q;
}

}  // extern "C"
