// Workspace of the allocation-free PCG entry point (amg_solve_pcg_noalloc):
// one statically sized array of device memory in this file's code object,
// so that only a process that calls the entry point has it placed on the
// device (on the first call, with the rest of this code object); each
// device then holds its own copy until the process ends.  Every call on a
// device shares that device's copy.  Host code reaches it only through the
// address hipGetSymbolAddress gives for the current device: the array's
// name in host code is a host-side stand-in, not a device address.
#include <mutex>
#include <string>

#include "gw_internal.h"

namespace gw {

namespace {

// Six n-vectors for n <= GW_NOALLOC_MAX_ROWS, then the block partials
// (kKrylovMaxBlocks x 4), then one scalar record: 48 MiB + 64 KiB + 160 B.
constexpr size_t kVecDoubles = 6 * (size_t)GW_NOALLOC_MAX_ROWS;
constexpr size_t kPartDoubles = (size_t)kKrylovMaxBlocks * 4;
constexpr size_t kKsDoubles = (sizeof(KScalars) + 7) / 8;
constexpr size_t kScratchDoubles = kVecDoubles + kPartDoubles + kKsDoubles;
static_assert(sizeof(KScalars) % 8 == 0, "the scalar record follows the partials at 8-byte alignment");

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;

// Address of the current device's copy, looked up once per device (with
// that device current) and kept.
double *scratch_address() {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    GW_HIP(hipGetDevice(&dev));
    GW_REQUIRE(dev >= 0 && dev < kMaxDevices, "amg_solve_pcg_noalloc: device index out of range");
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        GW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        GW_REQUIRE(p, "amg_solve_pcg_noalloc: no device address for the workspace array");
        addr[dev] = static_cast<double *>(p);
    }
    return addr[dev];
}

}  // namespace

int pcg_noalloc(amg_hierarchy *H, const double *b, double *x, const amg_solve_params &sp, amg_solve_info *info,
                hipStream_t s) {
    const int64_t n = H->L[0].A.n;
    GW_REQUIRE(n <= GW_NOALLOC_MAX_ROWS, "amg_solve_pcg_noalloc: " + std::to_string(n) +
                                             " rows exceed the workspace limit of " +
                                             std::to_string(GW_NOALLOC_MAX_ROWS));
    double *base = scratch_address();
    // fixed offsets from the array's start whatever n is; the solve writes
    // every vector entry, partial and scalar before it reads it
    return krylov_pcg_in(H, base, base + kVecDoubles, reinterpret_cast<KScalars *>(base + kVecDoubles + kPartDoubles),
                         b, x, sp, info, s);
}

}  // namespace gw
