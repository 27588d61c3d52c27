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
//
// Solves may share launches (queue_set_batch): a slot that reaches a solve
// (after its setup on its own stream) then hands it to the queue's solver
// thread, whose engines (flow CG; travel-time pairs) run the iterations of
// every solve they hold in shared launches, one launch per kernel step for
// all of them; a solve joins at the next block of iterations and leaves as
// soon as it is final.  By default each slot solves on its own stream: with
// four hardware queues the slots' small kernels already overlap on the
// device, and the shared launches measured 10-25 % fewer solves/s.  Either
// way each system's iterates are those of its solve alone, bit for bit, so a
// result does not depend on the mix it was served in.  With the setup cache on (queue_set_setup_cache), the flow
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

// The inputs that determine the flow matrix, kept with a cached hierarchy:
// a hash match is confirmed by comparing them in full.
struct SetupInputs {
    gw_grid grid;
    gw_bc bc;
    amg_params params;
    std::vector<double> K;
    bool same(const gw_request &r) const {
        const int64_t n = (int64_t)r.grid.nx * r.grid.ny * r.grid.nz;
        return std::memcmp(&grid, &r.grid, sizeof(gw_grid)) == 0 && std::memcmp(&bc, &r.bc, sizeof(gw_bc)) == 0 &&
               std::memcmp(&params, &r.flow_params, sizeof(amg_params)) == 0 && (int64_t)K.size() == n &&
               std::memcmp(K.data(), r.K, sizeof(double) * (size_t)n) == 0;
    }
};

struct CachedSetup {
    SetupKey key;
    std::shared_ptr<SetupInputs> inputs;
    amg_hierarchy *H = nullptr;
    size_t bytes = 0;
    bool in_use = false;
    uint64_t last_use = 0;
};

// A solve handed to the solver thread: kind 0 = flow (CG), 1 = travel-time
// pair (BiCGSTAB on two right-hand sides).
struct SolveTask {
    int kind = 0;
    amg_hierarchy *H = nullptr;
    const double *b0 = nullptr, *b1 = nullptr;
    double *x0 = nullptr, *x1 = nullptr;
    amg_solve_params sp{};
    amg_solve_info info[2] = {};
    int status = GW_OK;
    bool done = false;
    char error[160] = {};
};

// Solves that may share launches: same kind, hierarchy precision and sweep
// counts, and stopping parameters.
bool same_batch(const SolveTask &a, const SolveTask &b) {
    return a.kind == b.kind && a.H->prm.precision == b.H->prm.precision && a.H->prm.npre == b.H->prm.npre &&
           a.H->prm.npost == b.H->prm.npost && a.sp.rtol == b.sp.rtol && a.sp.maxiter == b.sp.maxiter &&
           a.sp.check_every == b.sp.check_every && a.sp.flexible == b.sp.flexible && a.sp.graph == b.sp.graph;
}

// A hierarchy the shared-launch solvers take (a diagonal smoother with at
// least one sweep each way).
bool batchable(const amg_hierarchy *H) {
    return H->nlev >= 1 && H->prm.smoother != GW_SMOOTHER_ILU0 && H->prm.npre >= 1 && H->prm.npost >= 1;
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
    // flow hierarchies kept after their request (bytes counted in `reserved`)
    std::vector<CachedSetup> cache;
    int cache_max = 0;
    uint64_t use_clock = 0;
    // solves waiting for the solver thread, and its batches
    std::deque<SolveTask *> solves;
    std::condition_variable cv_solve, cv_solved;
    int max_batch = 1;      // 1: every slot solves on its own stream (measured faster, see DESIGN)
    double window_s = 0.0;  // how long a batch waits for more solves to join
    bool stop_solver = false;
    std::vector<std::thread> solvers;  // solver threads, each with its own stream
    int n_solvers = 0, want_solvers = 1;
    uint64_t n_batches = 0, n_batched = 0;  // blocks run for two or more solves at once; solves taken

    double clock() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void worker();
    void solver_loop();
    int solve(SolveTask &t, hipStream_t s);
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
            if (!c.in_use && c.key == key && c.inputs->same(r)) {
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
    size_t flow_h_bytes = 0;
    {
        SolveTask t;
        t.kind = 0;
        t.H = H;
        t.b0 = d.b.p;
        t.x0 = d.h.p;
        t.sp = r.solve;
        try {
            st = solve(t, s);
        } catch (...) {
            st = GW_EDEVICE;
        }
        res.flow = t.info[0];
        if (st < 0) gw::set_last_error(t.error);
        int32_t nl = 0;
        (void)amg_hierarchy_info(H, nullptr, 0, &nl, &flow_h_bytes);
    }
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
                c.inputs = std::make_shared<SetupInputs>();
                c.inputs->grid = r.grid;
                c.inputs->bc = r.bc;
                c.inputs->params = r.flow_params;
                c.inputs->K.assign(r.K, r.K + n);
                c.H = H;
                c.bytes = flow_h_bytes;
                c.last_use = ++use_clock;
                reserved += c.bytes;
                cache.push_back(c);
                kept = true;
            }
        }
        if (!kept) amg_free(H);
    }
    res.flow.setup_ms = setup_ms;
    // device bytes held while the flow system was solved
    const size_t flow_phase = d.K.bytes() + d.b.bytes() + d.h.bytes() + d.rowptr.bytes() + d.col.bytes() +
                              d.val.bytes() + (res.setup_reused ? 0 : flow_h_bytes);
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
    // travel time (Eq. 1): the upwind matrix and its two right-hand sides, one
    // hierarchy, then the pair solve
    const double tt0 = std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
    gw::DBuf<int32_t> trp((size_t)n + 1), tcol((size_t)nnz);
    gw::DBuf<double> tval((size_t)nnz), bt(n), bc(n);
    int64_t tnnz = 0, nid = 0;
    st = tt_assemble(&g, d.qx.p, d.qy.p, d.qz.p, r.phi, &r.zone, trp.p, tcol.p, tval.p, bt.p, bc.p, &tnnz, &nid, s);
    if (st != GW_OK) return st;
    amg_hierarchy *Ht = nullptr;
    {
        gw_csr At{(int32_t)n, tnnz, trp.p, tcol.p, tval.p};
        st = amg_setup(&At, &r.tt_params, &Ht, s);
        if (st != GW_OK) return st;
    }
    std::unique_ptr<amg_hierarchy, void (*)(amg_hierarchy *)> Ht_owner(Ht, amg_free);
    const size_t tt_csr_bytes = trp.bytes() + tcol.bytes() + tval.bytes();
    trp.release();
    tcol.release();
    tval.release();
    const double tt_setup_ms =
        std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count() - tt0;
    SolveTask t;
    t.kind = 1;
    t.H = Ht;
    t.b0 = bt.p;
    t.b1 = bc.p;
    t.x0 = d.tau.p;
    t.x1 = d.c.p;
    t.sp = r.solve;
    try {
        st = solve(t, s);
    } catch (...) {
        st = GW_EDEVICE;
    }
    if (st < 0) gw::set_last_error(t.error);
    res.tt[0] = t.info[0];
    res.tt[1] = t.info[1];
    res.tt[0].setup_ms = res.tt[1].setup_ms = tt_setup_ms;
    size_t tt_h_bytes = 0;
    {
        int32_t nl = 0;
        (void)amg_hierarchy_info(Ht, nullptr, 0, &nl, &tt_h_bytes);
    }
    // device bytes held during the travel-time setup and solve (the CSR is
    // released after the setup, but counted: both live during it)
    const size_t tt_phase = d.K.bytes() + d.h.bytes() + d.qx.bytes() + d.qy.bytes() + d.qz.bytes() +
                            d.tau.bytes() + d.c.bytes() + bt.bytes() + bc.bytes() + tt_csr_bytes + tt_h_bytes;
    res.bytes_used = std::max(flow_phase, tt_phase);
    if (st < 0) return st;
    if (r.tau_out) GW_HIP(hipMemcpyAsync(r.tau_out, d.tau.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    if (r.c_out) GW_HIP(hipMemcpyAsync(r.c_out, d.c.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    if (flow_status != GW_OK) return flow_status;
    return st;
}

// A solve of a slot: handed to the solver thread (shared launches with the
// other slots' solves), or run on the slot's own stream when batching is off
// or the hierarchy is not one the shared-launch solvers take.  The inputs
// are complete on the device when it is called (every entry point before it
// synchronized the slot's stream), and so are the outputs when it returns.
int gw_queue::solve(SolveTask &t, hipStream_t s) {
    bool batch = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        batch = max_batch > 1 && batchable(t.H);
    }
    if (!batch) {
        const int st = t.kind == 0 ? amg_solve_pcg(t.H, t.b0, t.x0, &t.sp, &t.info[0], s)
                                   : amg_solve_bicgstab_pair(t.H, t.b0, t.b1, t.x0, t.x1, &t.sp, t.info, s);
        if (st < 0) std::strncpy(t.error, gw_last_error(), sizeof(t.error) - 1);
        return st;
    }
    std::unique_lock<std::mutex> lk(mu);
    solves.push_back(&t);
    cv_solve.notify_one();
    cv_solved.wait(lk, [&] { return t.done; });
    return t.status;
}

// A solver thread: one shared-launch engine per kind (flow CG, travel-time
// pair).  Each round it moves the waiting solves that fit an engine (same
// parameters as the solves already there, up to max_batch) into it, then
// runs one block of iterations of every engine that holds solves; a solve
// leaves as soon as it is final and its slot wakes up, and a solve that
// arrives meanwhile joins at the next block.  With window_us > 0, an idle
// solver waits that long for the solves of the other running requests
// before the first block.
void gw_queue::solver_loop() {
    hipStream_t s = nullptr;
    std::unique_ptr<gw::BatchEngine> eng[2];
    std::vector<SolveTask *> in[2];  // the solves each engine holds
    for (;;) {
        std::vector<SolveTask *> take[2];
        int cap = 1;
        {
            std::unique_lock<std::mutex> lk(mu);
            auto busy = [&] { return !in[0].empty() || !in[1].empty(); };
            cv_solve.wait(lk, [&] { return stop_solver || !solves.empty() || busy(); });
            if (!busy() && solves.empty()) break;  // stop_solver, nothing left
            cap = std::max(1, max_batch);
            if (!busy() && window_s > 0.0) {
                const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                                      std::chrono::duration<double>(window_s));
                cv_solve.wait_until(lk, until, [&] { return stop_solver || (int)solves.size() >= cap ||
                                                            (int)solves.size() >= running; });
            }
            for (auto it = solves.begin(); it != solves.end();) {
                SolveTask *t = *it;
                const int k = t->kind;
                const int have = (int)(in[k].size() + take[k].size());
                bool ok = have < cap;
                if (ok && have > 0) ok = same_batch(*t, !in[k].empty() ? *in[k][0] : *take[k][0]);
                if (ok) {
                    take[k].push_back(t);
                    it = solves.erase(it);
                } else {
                    ++it;
                }
            }
            n_batched += take[0].size() + take[1].size();
        }
        for (int k = 0; k < 2; ++k) {
            if (in[k].empty() && take[k].empty()) continue;
            std::vector<gw::BatchEngine::Result> res;
            int active = 0;
            const int st = gw::guarded([&] {
                if (!s) {
                    GW_HIP(hipSetDevice(device));
                    GW_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                }
                if (!take[k].empty()) {
                    if (!eng[k] || eng[k]->empty()) eng[k].reset(new gw::BatchEngine(k, take[k][0]->sp, cap, s));
                    for (SolveTask *t : take[k]) {
                        in[k].push_back(t);
                        eng[k]->join(t, t->H, t->b0, t->b1, t->x0, t->x1);
                    }
                }
                active = eng[k]->size();
                res = eng[k]->step();
                return GW_OK;
            });
            {
                std::lock_guard<std::mutex> lk(mu);
                if (st < 0) {
                    // the engine's solves all fail with the error
                    for (SolveTask *t : in[k]) {
                        t->status = st;
                        std::strncpy(t->error, gw_last_error(), sizeof(t->error) - 1);
                        t->done = true;
                    }
                    in[k].clear();
                    eng[k].reset();
                } else {
                    if (active >= 2) ++n_batches;
                    for (const auto &r : res) {
                        SolveTask *t = static_cast<SolveTask *>(r.tag);
                        t->status = r.status;
                        t->info[0] = r.info[0];
                        t->info[1] = r.info[1];
                        t->done = true;
                        in[k].erase(std::find(in[k].begin(), in[k].end(), t));
                    }
                }
            }
            if (st < 0 || !res.empty()) cv_solved.notify_all();
        }
    }
    eng[0].reset();
    eng[1].reset();
    if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    gw::release_thread_resources();
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
    if (have_stream) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    gw::release_thread_resources();
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
        {
            std::lock_guard<std::mutex> lk(Q->mu);
            for (; Q->n_solvers < Q->want_solvers; ++Q->n_solvers)
                Q->solvers.emplace_back([p = Q.get()] { p->solver_loop(); });
        }
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
    {
        // the slots are gone, so no solve waits any more
        std::lock_guard<std::mutex> lk(q->mu);
        q->stop_solver = true;
    }
    q->cv_solve.notify_all();
    for (auto &t : q->solvers) t.join();
    for (auto &c : q->cache) amg_free(c.H);
    delete q;
}

int queue_set_batch(gw_queue *q, int32_t max_batch, double window_us, int32_t streams) {
    return gw::guarded([&] {
        GW_REQUIRE(q, "queue_set_batch: null queue");
        GW_REQUIRE(max_batch >= 1 && max_batch <= 256, "queue_set_batch: max_batch must be in [1, 256]");
        GW_REQUIRE(window_us >= 0.0 && window_us <= 1e7, "queue_set_batch: window_us must be in [0, 1e7]");
        GW_REQUIRE(streams >= 1 && streams <= 16, "queue_set_batch: streams must be in [1, 16]");
        {
            std::lock_guard<std::mutex> lk(q->mu);
            q->max_batch = max_batch;
            q->window_s = window_us * 1e-6;
            q->want_solvers = std::max(q->want_solvers, (int)streams);
            // more solver threads start now; fewer than running never
            for (; q->n_solvers < q->want_solvers; ++q->n_solvers)
                q->solvers.emplace_back([q] { q->solver_loop(); });
        }
        q->cv_solve.notify_all();
        return GW_OK;
    });
}

int queue_stats(const gw_queue *q, uint64_t *shared_blocks, uint64_t *solves) {
    return gw::guarded([&] {
        GW_REQUIRE(q, "queue_stats: null queue");
        std::lock_guard<std::mutex> lk(const_cast<gw_queue *>(q)->mu);
        if (shared_blocks) *shared_blocks = q->n_batches;
        if (solves) *solves = q->n_batched;
        return GW_OK;
    });
}

}  // extern "C"
