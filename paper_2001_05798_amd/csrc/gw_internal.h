// Internal declarations of the gfx950 groundwater AMG library: error
// plumbing, the device memory pool, device-resident matrix/level structures
// and the kernel launchers shared between the .hip translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <memory>
#include <vector>

#include "gwamg.h"

namespace gw {

// ---------------------------------------------------------------- errors --
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void set_last_error(const std::string &msg);

#define GW_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            ::gw::fail(GW_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GW_REQUIRE(cond, msg)                        \
    do {                                             \
        if (!(cond)) ::gw::fail(GW_EINVAL, (msg));   \
    } while (0)

// Run `f` and turn exceptions into a status code + thread-local message.
template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return GW_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return GW_EDEVICE;
    }
}

// ------------------------------------------------------------ memory pool --
// Device allocations are served from per-device free lists of size classes
// (1/8-octave steps above 4 KiB), so repeated setups and solves do not call
// hipMalloc.  Thread safe.  gw_trim() returns cached blocks to HIP.
void *pool_alloc(size_t bytes);
void pool_free(void *p);
void pool_trim();
size_t pool_class_bytes(size_t bytes);

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        p = count ? static_cast<T *>(pool_alloc(count * sizeof(T))) : nullptr;
    }
    void release() {
        if (p) pool_free(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    T *get() const { return p; }
};

// 4 KiB of pinned host memory owned by the calling host thread, for the
// small device<->host copies of sizes and Krylov scalars (allocated once per
// thread: pinned allocation is far too slow to do per call).
constexpr size_t kHostStageBytes = 4096;
void *host_stage();

// A second stream of the calling host thread on the current device, for work
// that overlaps the caller's stream (ordered against it by events).
hipStream_t side_stream();
// Work of the calling thread on its side stream, overlapping the work that
// follows on the caller's stream s.  run(s, f) makes the side stream wait for
// the work already on s and enqueues f(side) there; join(s) makes s wait for
// it.  Pool blocks freed while f runs (the side work's temporaries) are held
// back from the thread's free lists until join, so no kernel enqueued on s
// in between can receive a block the side stream may still use; the
// destructor (error paths) synchronizes the side stream before it releases
// them.  One job at a time per thread.
struct SideJob {
    hipStream_t q = nullptr;
    hipEvent_t start = nullptr, done = nullptr;
    std::vector<void *> held;
    bool pending = false;
    SideJob() = default;
    SideJob(const SideJob &) = delete;
    SideJob &operator=(const SideJob &) = delete;
    template <class F>
    void run(hipStream_t s, F &&f) {
        begin(s);
        struct Restore {
            SideJob *j;
            ~Restore() { j->end_defer(); }
        } r{this};
        f(q);
        end_defer();
        GW_HIP(hipEventRecord(done, q));
        pending = true;
    }
    void join(hipStream_t s);
    ~SideJob();

  private:
    void begin(hipStream_t s);
    void end_defer();
    std::vector<void *> *prev_ = nullptr;
    bool deferring_ = false;
};
// For a host thread that ends (a serving worker): synchronize and destroy
// its side streams, free its pinned stage and the pool blocks cached on its
// free lists.
void release_thread_resources();
void pool_release_thread();

// Pinned host buffer.
struct Pinned {
    void *p = nullptr;
    size_t n = 0;
    explicit Pinned(size_t bytes);
    ~Pinned();
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
};

// --------------------------------------------------------- kernel timing --
// When enabled, launches wrapped in a ProfScope are bracketed by HIP events
// on their stream; durations are summed at the next prof_flush().
enum KernelId : int {
    K_FV_ASSEMBLE, K_DARCY, K_TT_ASSEMBLE,
    K_SETUP_MISC, K_TRANSPOSE, K_STRENGTH, K_MIS2, K_AGGREGATE, K_SPGEMM, K_COARSE_LU, K_SELL_BUILD,
    // V-cycle kernels in three classes: level 0, level 1, levels >= 2
    K_SMOOTH_FIRST0, K_SMOOTH0, K_RESIDUAL0, K_RESTRICT0, K_PROLONG0,
    K_SMOOTH_FIRST1, K_SMOOTH1, K_RESIDUAL1, K_RESTRICT1, K_PROLONG1,
    K_SMOOTH_FIRSTC, K_SMOOTHC, K_RESIDUALC, K_RESTRICTC, K_PROLONGC, K_COARSE_SOLVE,
    K_KRYLOV_SPMV, K_KRYLOV_UPDATE, K_KRYLOV_DOT, K_TRUE_RESIDUAL,
    // direct upwind sweep: dependency lists, then the sweep itself
    K_SWEEP_LISTS, K_SWEEP,
    K_COUNT
};
const char *kernel_name(int id);
bool prof_on();
// Times the work enqueued on s during its lifetime with a pair of events
// (when profiling is on and the class is selected).  With ext = true the
// scope holds exactly one launch, made through GW_LAUNCH_TIMED, and the
// events are taken by that dispatch itself (kernel start and end), without
// the barrier packets of two hipEventRecord calls (about 3 us per launch).
// `bytes` counts the launch's operators in the format it reads (sliced copy
// or CSR); `cbytes` the same launch with every operator pass counted as a
// CSR pass (nnz (value + 4-byte column) + 4 (n + 1)), the accounting of the
// plain formula; negative: the same as `bytes`.
struct ProfScope {
    int id;
    double bytes, cbytes;
    hipStream_t s;
    bool ext;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfScope(int id_, double bytes_, hipStream_t s_, bool ext_ = false, double cbytes_ = -1.0);
    ~ProfScope();
};

#define GW_LAUNCH_TIMED(ps, kernel, grid, block, shm, stream, ...)                                          \
    do {                                                                                                    \
        if ((ps).e0 && (ps).ext)                                                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, (ps).e0, (ps).e1, 0u, __VA_ARGS__);     \
        else                                                                                                \
            hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                              \
    } while (0)
void prof_flush();

// ------------------------------------------------------- device matrices --
struct Csr {
    int32_t n = 0, ncols = 0;
    int64_t nnz = 0;
    int32_t grp = 1;    // lanes per row in the solve-phase products (a power of two <= 64)
    DBuf<int32_t> rowptr, col;
    DBuf<double> val;
    DBuf<float> val32;  // FP32 copy (mixed precision levels)
    void alloc(int32_t n_, int32_t ncols_, int64_t nnz_) {
        n = n_; ncols = ncols_; nnz = nnz_;
        rowptr.alloc((size_t)n + 1);
        col.alloc((size_t)nnz);
        val.alloc((size_t)nnz);
    }
    size_t bytes() const { return rowptr.bytes() + col.bytes() + val.bytes() + val32.bytes(); }
};

// Read-only view of a CSR on the device.
struct CsrView {
    int32_t n, ncols;
    int64_t nnz;
    const int32_t *rowptr, *col;
    const double *val;
};
inline CsrView view(const Csr &A) { return {A.n, A.ncols, A.nnz, A.rowptr.p, A.col.p, A.val.p}; }

// Sliced ELL copy of an operator for the solve phase: slices of C rows (C =
// 64, one wave, or 32, 16 or 8, chosen per operator), entries column-major
// inside a slice so the lanes of a slice read consecutive addresses; short
// rows are padded with zero values pointing at the row itself.  Each slice is
// as wide as its longest row, so operators whose row lengths vary from row to
// row (the upwind travel-time operator: 1 to 7 entries) take shorter slices,
// which pad less.  When the operator has at most 255 distinct offsets
// (col - row), as stencil matrices do, each column is stored as a one-byte
// index into a small dictionary of offsets; otherwise as an int32 column.
constexpr int kSellMaxC = 64, kSellMinC = 8;
constexpr int kSellMaxDict = 255;
struct Sell {
    int32_t n = 0, nslices = 0;
    int32_t cshift = 6;          // slice height C = 1 << cshift
    int64_t nnz_padded = 0;
    int32_t ndict = 0;           // 0: int32 columns, else dictionary size
    DBuf<int32_t> soff;          // nslices + 1, entry offset of each slice
    DBuf<uint8_t> idx;           // dictionary indices (ndict > 0)
    DBuf<int32_t> col;           // columns (ndict == 0)
    DBuf<int32_t> dict;          // offsets, ascending
    DBuf<double> val;
    DBuf<float> val32;
    bool built() const { return nslices > 0; }
    size_t bytes() const {
        return soff.bytes() + idx.bytes() + col.bytes() + dict.bytes() + val.bytes() + val32.bytes();
    }
};

struct SellView {
    int32_t n, ndict, cshift;
    const int32_t *soff;
    const uint8_t *idx;
    const int32_t *col;
    const int32_t *dict;
};
inline SellView view(const Sell &S) { return {S.n, S.ndict, S.cshift, S.soff.p, S.idx.p, S.col.p, S.dict.p}; }

// Symmetric stencil copy of the level-0 operator, taken before the sliced
// copy: when the column offsets (col - row) are a symmetric set {-d_K ..
// -d_1, 0, d_1 .. d_K} with K <= kStenMax (the 3-, 5- and 7-point
// operators) and every a_{i,i-d} equals a_{i-d,i} bit for bit, row i is
// read from the diagonal and c_k[i] = a_{i,i+d_k} (0 where absent), and its
// entries left of the diagonal from the mirror rows, c_k[i-d_k]: K+1 values
// a row, every load coalesced, no column indices.
// One-sided form, for upwind operators (every off-diagonal strictly
// negative, and a_{i,i+d} and a_{i+d,i} never both stored): c_k[i] holds the
// face between rows i and i+d_k, as a_{i,i+d_k} (negative) when row i holds
// it, as -a_{i+d_k,i} (positive) when row i+d_k does, 0 when neither; row i
// takes c_k[i] when negative and -c_k[i-d_k] when c_k[i-d_k] is positive.
constexpr int kStenMax = 3;
struct Stencil {
    int32_t n = 0, K = 0;
    int32_t d[kStenMax] = {};  // positive offsets, ascending
    int32_t onesided = 0;       // the one-sided (upwind) form
    DBuf<double> c;             // (K+1) n: the diagonal, then c_1 .. c_K
    DBuf<float> c32;
    bool built() const { return K > 0; }
    size_t bytes() const { return c.bytes() + c32.bytes(); }
};

// ------------------------------------------------------------ hierarchy --
// Level-synchronous schedule of a triangular (more generally acyclic) system
// M x = b: per row its count of off-diagonal dependencies, the rows that
// depend on it, and the rows with none; plus the work copies a run mutates.
struct TriPlan {
    Csr M;                       // the system, diagonal stored (unit for L)
    DBuf<int32_t> indeg0, drow, dcol, q0;
    DBuf<int64_t> first;         // size of the first frontier (device)
    DBuf<int32_t> indeg, qa, qb; // per-run copies
    DBuf<int64_t> out;
    size_t bytes() const {
        return M.bytes() + indeg0.bytes() + drow.bytes() + dcol.bytes() + q0.bytes() + indeg.bytes() + qa.bytes() +
               qb.bytes();
    }
};

// ILU(0) smoother of a level: the factors on A's pattern, the two triangles
// as systems for the substitutions, and the vectors of one smoothing step.
struct IluData {
    DBuf<double> lu;
    DBuf<int32_t> dpos;
    TriPlan lo, up;
    DBuf<double> r, y, z;
    size_t bytes() const { return lu.bytes() + dpos.bytes() + lo.bytes() + up.bytes() + r.bytes() * 3; }
};

struct Level {
    Csr A;           // operator A_l (level 0: copy of the caller's matrix)
    Sell As;         // sliced ELL copy of A_l used by the solve phase (level 0)
    Stencil St;      // symmetric stencil copy (level 0), preferred to As
    Csr P, R;        // prolongator n x nc and its transpose (empty on coarsest)
    DBuf<int32_t> agg;
    DBuf<double> M;  // smoother diagonal
    DBuf<float> M32;
    int32_t nc = 0;
    int64_t nnz_s = 0;
    int32_t mis_rounds = 0;
    double omega_p = 0.0;
    DBuf<double> omega_dev;  // omega_P on the device (read back after setup)
    // V-cycle vectors of this level, element size 8 (FP64) or 4 (mixed):
    // b (right-hand side), x (iterate) and t (ping-pong / residual)
    DBuf<char> vb, vx, vt;
    std::unique_ptr<IluData> ilu;  // ILU(0) smoother (else the diagonal M)
    size_t bytes() const {
        return A.bytes() + As.bytes() + St.bytes() + P.bytes() + R.bytes() + agg.bytes() + M.bytes() + M32.bytes() +
               vb.bytes() + vx.bytes() + vt.bytes() + (ilu ? ilu->bytes() : 0);
    }
};

// Device-resident Krylov scalars (one block of them per hierarchy).
struct KScalars {
    double bnorm, tol;               // ||b||, rtol ||b||
    double rz, pq, alpha, beta, rr;  // CG
    double zq;                       // flexible CG: z . q
    double rho, rho_prev, omega, rv, ts, tt, ss;  // BiCGSTAB
    double rel_true;
    int32_t iters, maxiter, done, status, flexible, pending_x;
    uint32_t counter;                // last-block ticket
    int32_t pad;
};

}  // namespace gw

struct amg_hierarchy {
    amg_params prm{};
    int device = 0;
    int nlev = 0;  // number of levels including the coarsest (0 = no preconditioner)
    std::vector<gw::Level> L;
    int32_t nd = 0;  // coarsest size
    int sym_pattern = -1;  // level-0 pattern symmetric: -1 not known yet, 0 no, 1 yes
    int sym_values = -1;   // level-0 values symmetric bit for bit (probed with the pattern)
    gw::DBuf<double> lu, inv;  // row-major LU, column-major inverse
    gw::DBuf<int32_t> piv;
    // Krylov workspace
    gw::DBuf<double> kvec;  // up to 9 vectors of n
    int kvec_count = 0;
    gw::DBuf<double> partials;
    gw::DBuf<gw::KScalars> ks;
    // Captured blocks of Krylov iterations (they hold the workspace
    // addresses: dropped whenever the workspace moves)
    struct Graph {
        int kind, check, parity;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t cap = nullptr;  // capture-only stream
    bool mixed() const { return prm.precision == GW_PRECISION_MIXED; }
    size_t bytes() const;
    void drop_graphs();
    amg_hierarchy() = default;
    amg_hierarchy(const amg_hierarchy &) = delete;
    amg_hierarchy &operator=(const amg_hierarchy &) = delete;
    ~amg_hierarchy();
};

namespace gw {

// ---------------------------------------------------------- launchers ----
// All launchers enqueue on `s` and return immediately.
constexpr int kBlock = 256;
inline unsigned blocks_for(int64_t n, int per_thread = 1, int block = kBlock) {
    int64_t b = (n + (int64_t)block * per_thread - 1) / ((int64_t)block * per_thread);
    return (unsigned)(b < 1 ? 1 : b);
}

// scan.hip / util
// In place inclusive scan of a[0..n) (int32), total returned in *total (device int64).
// When max_out is given, the largest element of a (before the scan) is
// written there too.
void scan_inclusive_i32(int32_t *a, int64_t n, int64_t *total, hipStream_t s, int32_t *max_out = nullptr);
void fill_i32(int32_t *a, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double *a, double v, int64_t n, hipStream_t s);
void copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t s);

// assemble.hip
void launch_fv_assemble(const gw_grid &g, const double *K, const gw_bc &bc, const gw_well *wells,
                        int nwells, int32_t *rowptr, int32_t *col, double *val, double *b,
                        int32_t *bad, hipStream_t s);
void launch_darcy(const gw_grid &g, const double *K, const gw_bc &bc, const double *h, double *qx,
                  double *qy, double *qz, hipStream_t s);
void launch_tt_count(const gw_grid &g, const double *qx, const double *qy, const double *qz,
                     int32_t *rowlen, hipStream_t s);
void launch_tt_fill(const gw_grid &g, const double *qx, const double *qy, const double *qz,
                    double phi, const gw_zone &z, const int32_t *rowptr, int32_t *col, double *val,
                    double *bt, double *bc, int32_t *n_ident, hipStream_t s);

// setup.hip
void launch_csr_check(const CsrView &A, double *diag, int32_t *bad, hipStream_t s);
void transpose(const CsrView &A, Csr &T, hipStream_t s, int64_t *scratch_total);
void build_level(amg_hierarchy *H, int l, hipStream_t s, bool *is_coarsest);
// The coarsest level's dense LU and its inverse.  start_coarsest enqueues
// them on the thread's side stream, after the work already on s, so that
// they overlap the rest of the setup; finish_coarsest makes s wait for them
// and reports a zero pivot.  The job's destructor waits for the side stream,
// so the hierarchy's buffers outlive its kernels on every path, errors
// included (declare the job after the hierarchy it fills).
struct CoarseJob {
    hipStream_t side = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    DBuf<int32_t> status;
    CoarseJob() = default;
    CoarseJob(const CoarseJob &) = delete;
    CoarseJob &operator=(const CoarseJob &) = delete;
    ~CoarseJob();
};
void start_coarsest(amg_hierarchy *H, int l, hipStream_t s, CoarseJob &job);
void finish_coarsest(CoarseJob &job, hipStream_t s);
void make_smoother(amg_hierarchy *H, int l, hipStream_t s);
void convert_level_fp32(amg_hierarchy *H, int l, hipStream_t s);
// Build the sliced ELL copy of level l's operator (values in FP64, plus FP32
// when `fp32`).
void build_sell(amg_hierarchy *H, int l, bool fp32, hipStream_t s);

// solve.hip
void vcycle(amg_hierarchy *H, const double *r, double *z, const int32_t *done, hipStream_t s);
// y = A_0 x in FP64 with the level's solve-phase operator.
void spmv_level0(amg_hierarchy *H, const double *x, double *y, hipStream_t s);
// Lanes per row for a matrix with this mean row length (setup kernels), and
// for the solve phase's products.
int lane_group_for(double mean_row_len);
int solve_group_for(double mean_row_len);
int krylov_pcg(amg_hierarchy *H, const double *b, double *x, const amg_solve_params &sp,
               amg_solve_info *info, hipStream_t s);
// Krylov workspace of a hierarchy: nvec n-vectors, block partials, scalars
// (grown on demand); V-cycle level vectors for nr interleaved right-hand
// sides.
void ensure_krylov_workspace(amg_hierarchy *H, int nvec);
void ensure_level_vectors(amg_hierarchy *H, int nr);
// batch.hip: the shared-launch solver.  An engine holds an active set of
// systems of one kind (0: CG, 1: the BiCGSTAB pair) with the same hierarchy
// precision, sweep counts and stopping parameters; step() admits the systems
// that joined, runs one block of iterations of all of them in shared
// launches, and returns those that finished (each with exactly the result of
// its own solve).  Vectors stay owned by the caller until their result is
// returned.
class BatchEngine {
   public:
    struct Result {
        void *tag;
        int status;
        amg_solve_info info[2];
    };
    struct Member;
    struct State;
    BatchEngine(int kind, const amg_solve_params &sp, int capacity, hipStream_t s);
    ~BatchEngine();
    BatchEngine(const BatchEngine &) = delete;
    BatchEngine &operator=(const BatchEngine &) = delete;
    bool accepts(const amg_hierarchy *H, const amg_solve_params &sp) const;
    void join(void *tag, amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1);
    std::vector<Result> step();
    bool empty() const;
    int size() const;
    int kind() const { return kind_; }

   private:
    int kind_;
    amg_solve_params sp_;
    int cap_;
    hipStream_t s_;
    int nrec_ = 1, check_ = 4, cnt_ = 4, parity_ = 0;
    bool dirty_ = true;
    DBuf<KScalars> ks_;
    std::unique_ptr<Pinned> stage_;
    std::vector<int> free_;
    std::vector<std::unique_ptr<Member>> members_, joining_;
    std::unique_ptr<State> st_;
    void read_ks();
    KScalars *hks(const Member &m);
    void write_ks(const Member &m);
    template <class Rec>
    void run_once(const std::vector<Member *> &ms, Rec &&rec);
    void admit(std::vector<Member *> &done_now);
    void first_z(const std::vector<Member *> &ms);
    void record_iterations();
    void complete(const std::vector<Member *> &ms, std::vector<Member *> &done_now);
};

// Several independent systems in shared launches, each with the iterates of
// its own solve (info: nsys entries; the pair: 2 nsys).
int krylov_pcg_batch(amg_hierarchy *const *H, const double *const *b, double *const *x, int32_t nsys,
                     const amg_solve_params &sp, amg_solve_info *info, hipStream_t s);
int krylov_bicgstab2_batch(amg_hierarchy *const *H, const double *const *b0, const double *const *b1,
                           double *const *x0, double *const *x1, int32_t nsys, const amg_solve_params &sp,
                           amg_solve_info *info, hipStream_t s);
// Blocks of a Krylov reduction (each leaves its partial sums).
constexpr int kKrylovMaxBlocks = 2048;
// krylov_pcg in a workspace the caller provides: `vec` six n-vectors, `part`
// kKrylovMaxBlocks x 4 doubles, `ks` one scalar record (all device memory);
// nothing is allocated, kernels are launched one by one.
int krylov_pcg_in(amg_hierarchy *H, double *vec, double *part, KScalars *ks, const double *b, double *x,
                  const amg_solve_params &sp, amg_solve_info *info, hipStream_t s);
// amg_solve_pcg_noalloc's solve in the library's static workspace array.
int pcg_noalloc(amg_hierarchy *H, const double *b, double *x, const amg_solve_params &sp, amg_solve_info *info,
                hipStream_t s);
// PCG on A + diag(shift), preconditioned by the hierarchy of A.
int krylov_pcg_shifted(amg_hierarchy *H, const double *shift, const double *b, double *x, const amg_solve_params &sp,
                       amg_solve_info *info, hipStream_t s);
int krylov_bicgstab(amg_hierarchy *H, const double *b, double *x, const amg_solve_params &sp,
                    amg_solve_info *info, hipStream_t s);
// Two systems with the hierarchy's matrix, solved in lockstep (each exactly
// as krylov_bicgstab solves it alone).  Returns the worse of the statuses.
int krylov_bicgstab2(amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1,
                     const amg_solve_params &sp, amg_solve_info info[2], hipStream_t s);

// transient.hip (Eq. 2)
// shift = S_i V_i / dt with vol = V_i.
void storage_shift(int64_t n, const double *Ss, double vol, double dt, double *shift, hipStream_t s);
// max_i shift_i / C_ii (blocks for the host read).
double shift_ratio(const CsrView &C, const double *shift, hipStream_t s);
// rhs = b + shift h.
void storage_rhs(int64_t n, const double *b, const double *shift, const double *h, double *rhs, hipStream_t s);
// val = values of C + diag(shift) (same pattern as C).
void add_diagonal(const CsrView &C, const double *shift, double *val, hipStream_t s);

// sweep.hip
// Exact solve of a system whose rows couple each cell to its inflow
// neighbours only, by levels of a topological order of the inflow graph.
// b, x: nrhs blocks of A.n values.  Returns the number of cells solved (below
// A.n when the inflow graph has a cycle) and the number of levels.
int64_t upwind_sweep(const CsrView &A, int32_t nrhs, const double *b, double *x, int32_t *levels,
                     hipStream_t s);
// Schedule of an acyclic system (built once), and one solve with it on one
// right-hand side; skipped when *done is set.  The run does not read back.
void sweep_plan(TriPlan &P, hipStream_t s);
void sweep_run(TriPlan &P, const double *b, double *x, const int32_t *done, hipStream_t s);
// ILU(0) smoother of level l (ilu.hip); EINVAL-style failure on a zero pivot.
void build_ilu0(amg_hierarchy *H, int l, hipStream_t s);
// z = (LU)^{-1} r with the level's factors.
void ilu_apply(IluData &I, const double *r, double *z, const int32_t *done, hipStream_t s);
// The same for an upwind matrix on the 7-point grid g (rows of at most the
// six face neighbours), through one 64-byte record per row.
int64_t grid_sweep(const gw_grid &g, const CsrView &A, int32_t nrhs, const double *b, double *x, int32_t *levels,
                   hipStream_t s);
// The forward and backward systems of the dual delineation, assembled into A
// (capacity: the 7-point bound) and swept into out: forward blocks (tau_f,
// one per zone, one per injection well), then backward blocks (tau_b, one per
// production well).  levels/solved per direction.
void delineate(const gw_grid &g, const double *qx, const double *qy, const double *qz, double phi,
               const gw_zone *zones, int32_t nzones, const gw_well *wells, int32_t nwells, Csr &A, double *out,
               int32_t levels[2], int64_t solved[2], hipStream_t s);

}  // namespace gw
