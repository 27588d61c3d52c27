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
// sides.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
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

    double clock() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void worker();
    int run(Job &job, hipStream_t s, gw_result &res);
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
    gw_csr A{(int32_t)n, nnz, d.rowptr.p, d.col.p, d.val.p};
    const double ts = std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
    st = amg_setup(&A, &r.flow_params, &H, s);
    if (st != GW_OK) return st;
    const double setup_ms =
        std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count() - ts;
    st = amg_solve_pcg(H, d.b.p, d.h.p, &r.solve, &res.flow, s);
    amg_free(H);
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
                return stop || (!waiting.empty() && reserved + waiting.front().bytes <= budget);
            });
            if (stop) break;
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
    delete q;
}

}  // extern "C"
