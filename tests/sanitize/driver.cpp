// Host-side exercise of the library for the sanitizer builds (AddressSanitizer
// + UndefinedBehaviorSanitizer, ThreadSanitizer): argument validation of the
// entry points, and the serving queue driven from two submitting threads with
// batching and the setup cache on.  On a host without a GPU every request
// ends as a finished ticket with EDEVICE (its worker's first HIP call fails);
// with a GPU they solve.  Exit status 0 when every check holds.
#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "gwamg.h"

static int failures = 0;
#define CHECK(cond)                                                       \
    do {                                                                  \
        if (!(cond)) {                                                    \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

int main() {
    // validation before any device work
    gw_grid bad{0, 4, 4, 1.0, 1.0, 1.0};
    CHECK(fv_nnz(&bad) == -1);
    gw_grid g{6, 5, 4, 1.0, 1.0, 1.0};
    CHECK(fv_nnz(&g) == 7 * 120 - 2 * (30 + 20 + 24));
    CHECK(amg_setup(nullptr, nullptr, nullptr, nullptr) == GW_EINVAL);
    CHECK(std::strlen(gw_last_error()) > 0);
    CHECK(amg_solve_pcg_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == GW_EINVAL);
    CHECK(amg_solve_pcg_batch(nullptr, nullptr, nullptr, 1, nullptr, nullptr, nullptr) == GW_EINVAL);
    CHECK(tt_sweep(nullptr, 1, nullptr, nullptr, nullptr, nullptr) == GW_EINVAL);

    gw_queue *q = nullptr;
    CHECK(queue_create(0, 4, &q) == GW_EINVAL);
    CHECK(queue_create((size_t)8 << 30, 4, &q) == GW_OK && q);
    CHECK(queue_set_batch(q, 0, 0.0, 1) == GW_EINVAL);
    CHECK(queue_set_batch(q, 8, 200.0, 3) == GW_OK);
    CHECK(queue_set_setup_cache(q, 65) == GW_EINVAL);
    CHECK(queue_set_setup_cache(q, 2) == GW_OK);

    const int n = g.nx * g.ny * g.nz;
    std::vector<double> K(n, 1e-4);
    for (int i = 0; i < n; ++i) K[i] *= 1.0 + 0.01 * (i % 7);
    gw_well w{2, 2, 2, 1e-6};
    amg_params ap{0.08, GW_SMOOTHER_SPAI0, 2.0 / 3.0, 2, 2, 20, 20, GW_PRECISION_MIXED, 0x5EED, GW_COARSEN_SA};
    amg_params tp = ap;
    tp.eps_strong = 0.25;
    amg_solve_params sp{1e-8, 1000, 4, -1, -1};
    gw_request r{};
    r.grid = g;
    r.K = K.data();
    r.bc = gw_bc{10.0, 0.0};
    r.wells = &w;
    r.nwells = 1;
    r.phi = 0.25;
    r.zone = gw_zone{0, g.ny, 0, g.nz};
    r.flow_params = ap;
    r.tt_params = tp;
    r.solve = sp;
    r.t_arrival = -1.0;
    gw_request badr = r;
    badr.phi = 0.0;
    uint64_t t = 0;
    CHECK(queue_submit(q, &badr, &t) == GW_EINVAL);

    // two threads submit and poll concurrently
    std::atomic<int> finished{0};
    auto client = [&](int k) {
        std::vector<std::vector<double>> outs(6, std::vector<double>(n));
        std::vector<uint64_t> tick;
        for (int j = 0; j < 6; ++j) {
            gw_request rq = r;
            rq.h_out = outs[j].data();
            uint64_t tk = 0;
            if (queue_submit(q, &rq, &tk) == GW_OK) tick.push_back(tk);
        }
        for (uint64_t tk : tick) {
            gw_result res{};
            int st;
            while ((st = queue_poll(q, tk, &res)) == GW_PENDING) std::this_thread::yield();
            if (st == GW_OK || st == GW_EDEVICE) finished++;
            (void)k;
        }
    };
    std::thread a(client, 0), b(client, 1);
    a.join();
    b.join();
    CHECK(finished.load() == 12);
    CHECK(queue_drain(q) == GW_OK);
    uint64_t nb = 0, ns = 0;
    CHECK(queue_stats(q, &nb, &ns) == GW_OK);
    gw_result res{};
    CHECK(queue_poll(q, 999999, &res) == GW_EINVAL);
    queue_destroy(q);
    if (failures == 0) std::printf("sanitizer driver: all checks passed\n");
    return failures == 0 ? 0 : 1;
}
