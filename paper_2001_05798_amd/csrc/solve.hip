// Solve phase: the V-cycle (Introduction: restrict the residual, smooth,
// recurse to a direct solve on the coarsest level, interpolate and correct,
// smooth -- only sparse matrix-vector products) and the Krylov methods it
// preconditions: CG for the symmetric flow system and BiCGSTAB for the
// upwind travel-time system (Benchmarking Examples).
//
// Every product kernel is written once against an operator type: OpSell (the
// sliced ELL copy of the level-0 operator, one lane per row, dictionary of
// column offsets in LDS) or OpCsr<G> (G lanes per CSR row, G picked per
// matrix from its mean row length, so the lanes of a wave read consecutive
// entries).  The Krylov scalars live on the device: a product kernel leaves
// per-block partial sums, a one-block finalize kernel adds them in a fixed
// order and forms alpha/beta/omega and the convergence flag; every later
// kernel reads the flag and returns at once, so the host only polls it every
// few iterations.  FP64 throughout the Krylov layer; the hierarchy is FP64 or
// FP32 (mixed mode).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

// ----------------------------------------------------------- operators ---
// NR right-hand sides travel together: vectors hold the NR values of a row
// next to each other (x[i*NR + r]), so one pass over a matrix serves all of
// them and the gather of x_j is one NR-wide load.  Each right-hand side sees
// exactly the arithmetic, in the same order, of a single-vector pass.
template <class V, int NR>
struct VecN {
    V v[NR];
};

template <class T, int NR>
__device__ __forceinline__ VecN<T, NR> load_n(const T *__restrict__ p, int64_t j) {
    VecN<T, NR> r;
    if constexpr (NR == 2) {
        using T2 = std::conditional_t<std::is_same<T, double>::value, double2, float2>;
        const T2 t = *reinterpret_cast<const T2 *>(p + 2 * j);
        r.v[0] = t.x;
        r.v[1] = t.y;
    } else {
        static_assert(NR == 1, "one or two right-hand sides");
        r.v[0] = p[j];
    }
    return r;
}

template <class T, int NR>
__device__ __forceinline__ void store_n(T *__restrict__ p, int64_t j, const VecN<T, NR> &x) {
    if constexpr (NR == 2) {
        using T2 = std::conditional_t<std::is_same<T, double>::value, double2, float2>;
        T2 t;
        t.x = x.v[0];
        t.y = x.v[1];
        *reinterpret_cast<T2 *>(p + 2 * j) = t;
    } else {
        p[j] = x.v[0];
    }
}

template <class To, class From, int NR>
__device__ __forceinline__ VecN<To, NR> cvt(const VecN<From, NR> &x) {
    VecN<To, NR> r;
#pragma unroll
    for (int k = 0; k < NR; ++k) r.v[k] = (To)x.v[k];
    return r;
}

// Lanes of a group own one row: strided partial sums, then a butterfly over
// the group (groups are aligned power-of-two lane ranges of one wave).  Each
// lane loads U of its entries before summing their products, so the gathers
// overlap (U*G slots cover a typical row of a matrix given G lanes: G is
// picked from the mean row length by solve_group_for); slots past the row end take value 0 at
// the row's first column (a finite x makes them exact zeros; a non-finite x
// there makes the row non-finite in any case).
template <int G, int NR, class V, class F>
__device__ __forceinline__ VecN<V, NR> group_row_sum(int32_t b, int32_t e, const int32_t *__restrict__ col,
                                                     const V *__restrict__ val, int lane, F &&xj) {
    // one-lane rows (prolongators, ~3.5 entries a row) take 4: with 8, the
    // clamped slots past the row end doubled the L1 requests (level-0
    // prolongation 3.0 -> 3.6 TB/s at 4)
    constexpr int U = (G == 1 || G == 64) ? 4 : 8;
    VecN<V, NR> s;
#pragma unroll
    for (int k = 0; k < NR; ++k) s.v[k] = 0;
    if (b < e) {
        const int32_t cb = col[b];
        for (int32_t q = b + lane; q < e; q += U * G) {
            V a[U];
            int32_t c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t p = q + u * G;
                const bool in = p < e;
                const int32_t pc = in ? p : b;
                const V av = val[pc];
                const int32_t cv = col[pc];
                a[u] = in ? av : V(0);
                c[u] = in ? cv : cb;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const VecN<V, NR> xv = xj(c[u]);
#pragma unroll
                for (int k = 0; k < NR; ++k) s.v[k] += a[u] * xv.v[k];
            }
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NR; ++k) s.v[k] += __shfl_xor(s.v[k], o, dev::kWave);
    return s;
}

// An operator's head(i) loads what locates row i (its CSR range, or its
// slice's range in the sliced copy); kernels issue it before the block
// prologue and their `done` test so that those latencies overlap.
template <int G_, class V>
struct OpCsr {
    static constexpr int G = G_;
    static constexpr bool kShared = false;  // no block prologue
    struct Head {
        int32_t b, e;
        // An empty asm that reads the head: where a kernel returns early,
        // it keeps the head's loads above the return (otherwise the
        // compiler sinks them below the `done` test).
        __device__ __forceinline__ void keep() const { asm volatile("" ::"v"(b), "v"(e)); }
    };
    const int32_t *rowptr, *col;
    const V *val;
    __device__ __forceinline__ void load(int32_t *) const {}
    __device__ __forceinline__ Head head(int64_t i) const { return Head{rowptr[i], rowptr[i + 1]}; }
    // xj(j) returns the NR values of column j
    template <int NR, class F>
    __device__ __forceinline__ VecN<V, NR> rows_at(const Head &h, int64_t, int lane, const int32_t *,
                                                   F &&xj) const {
        return group_row_sum<G, NR, V>(h.b, h.e, col, val, lane, xj);
    }
    template <int NR, class F>
    __device__ __forceinline__ VecN<V, NR> rows(int64_t i, int lane, const int32_t *sd, F &&xj) const {
        return rows_at<NR>(head(i), i, lane, sd, xj);
    }
    template <class F>
    __device__ __forceinline__ V row(int64_t i, int lane, const int32_t *sd, F &&xj) const {
        return rows<1>(i, lane, sd, [&](int32_t j) { return VecN<V, 1>{{(V)xj(j)}}; }).v[0];
    }
};

template <class V>
struct OpSell {
    static constexpr int G = 1;
    static constexpr bool kShared = true;  // the offset dictionary in LDS
    struct Head {
        int32_t off, w;
        __device__ __forceinline__ void keep() const { asm volatile("" ::"v"(off), "v"(w)); }
    };
    SellView S;
    const V *val;
    __device__ __forceinline__ void load(int32_t *sd) const {
        for (int t = threadIdx.x; t < S.ndict; t += blockDim.x) sd[t] = S.dict[t];
    }
    __device__ __forceinline__ Head head(int64_t i) const {
        const int64_t sl = i / kSellC;
        const int32_t off = S.soff[sl];
        return Head{off, (S.soff[sl + 1] - off) / kSellC};
    }
    // Entries k of row i sit at soff[slice] + k*64 + (i mod 64).  Eight
    // entries are loaded before their products are summed, so the gathers
    // of x overlap; the sum still runs in entry order.  Slots past the slice
    // width re-read the last entry and are replaced by the padding entry
    // (value 0 at the row's own column) in registers, without branches.
    template <bool DICT, int NR, class F>
    __device__ __forceinline__ VecN<V, NR> row_impl(const Head &h, int64_t i, const int32_t *sd, F &&xj) const {
        const int l = (int)(i % kSellC);
        const int32_t off = h.off, w = h.w;
        VecN<V, NR> acc;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc.v[k] = 0;
        for (int32_t k0 = 0; k0 < w; k0 += 8) {
            V a[8];
            int32_t c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t k = min(k0 + u, w - 1);
                const int64_t e = off + (int64_t)k * kSellC + l;
                const V av = val[e];
                const int32_t cv = DICT ? (int32_t)i + sd[S.idx[e]] : S.col[e];
                const bool in = k0 + u < w;
                a[u] = in ? av : V(0);
                c[u] = in ? cv : (int32_t)i;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const VecN<V, NR> xv = xj(c[u]);
#pragma unroll
                for (int k = 0; k < NR; ++k) acc.v[k] += a[u] * xv.v[k];
            }
        }
        return acc;
    }
    template <int NR, class F>
    __device__ __forceinline__ VecN<V, NR> rows_at(const Head &h, int64_t i, int, const int32_t *sd,
                                                   F &&xj) const {
        return S.ndict ? row_impl<true, NR>(h, i, sd, xj) : row_impl<false, NR>(h, i, sd, xj);
    }
    template <int NR, class F>
    __device__ __forceinline__ VecN<V, NR> rows(int64_t i, int lane, const int32_t *sd, F &&xj) const {
        return rows_at<NR>(head(i), i, lane, sd, xj);
    }
    template <class F>
    __device__ __forceinline__ V row(int64_t i, int lane, const int32_t *sd, F &&xj) const {
        return rows<1>(i, lane, sd, [&](int32_t j) { return VecN<V, 1>{{(V)xj(j)}}; }).v[0];
    }
};

// A + diag(d): the level-0 operator with a diagonal added, for the storage
// term S/dt of Eq. 2 when the hierarchy of the conductance matrix is kept.
template <class B>
struct OpShift {
    static constexpr int G = B::G;
    static constexpr bool kShared = B::kShared;
    using Head = typename B::Head;
    B base;
    const double *d;
    __device__ __forceinline__ void load(int32_t *sd) const { base.load(sd); }
    __device__ __forceinline__ Head head(int64_t i) const { return base.head(i); }
    template <int NR, class F>
    __device__ __forceinline__ VecN<double, NR> rows_at(const Head &h, int64_t i, int lane, const int32_t *sd,
                                                        F &&xj) const {
        VecN<double, NR> s = base.template rows_at<NR>(h, i, lane, sd, xj);
        const VecN<double, NR> xi = xj((int32_t)i);
        const double di = d[i];
#pragma unroll
        for (int k = 0; k < NR; ++k) s.v[k] += di * xi.v[k];
        return s;
    }
    template <int NR, class F>
    __device__ __forceinline__ VecN<double, NR> rows(int64_t i, int lane, const int32_t *sd, F &&xj) const {
        return rows_at<NR>(head(i), i, lane, sd, xj);
    }
    template <class F>
    __device__ __forceinline__ double row(int64_t i, int lane, const int32_t *sd, F &&xj) const {
        return rows<1>(i, lane, sd, [&](int32_t j) { return VecN<double, 1>{{(double)xj(j)}}; }).v[0];
    }
};

// Block prologue of every product kernel: the offset dictionary of a sliced
// operator into LDS (nothing for CSR operators).
#define OP_PROLOGUE(op)                                                   \
    __shared__ int32_t sd_[kSellMaxDict + 1];                             \
    if constexpr (std::decay_t<decltype(op)>::kShared) {                  \
        (op).load(sd_);                                                   \
        __syncthreads();                                                  \
    }

#define GROUP_ROW(G)                                                              \
    const int64_t gtid = dev::xcd_block() * (int64_t)blockDim.x + threadIdx.x;     \
    const int64_t i = gtid / (G);                                                 \
    const int lane = (int)(gtid % (G));                                           \
    if (i >= n) return;

// Read in place of a null `done` flag (a select, not a branch, so the flag's
// load joins the first batch of loads).
__device__ const int32_t kNotDone = 0;

// Prologue of a V-cycle kernel (blocks of kBlock threads, G lanes per row,
// n >= 1): the `done` flag, the row's head and the statements `...` (loads
// of the row's own vector entries, through `i`) are issued together, rows
// past the end reading row n-1; then the dictionary (sliced operators only);
// then the flag is tested.  A small level's kernel thus waits for one round
// of loads where a test first would wait for three in a row.
#define VROW_PROLOGUE(OP, op, ...)                                                \
    const int64_t gtid = dev::xcd_block() * (int64_t)kBlock + threadIdx.x;         \
    const int64_t row_ = gtid / OP::G;                                            \
    const int lane = (int)(gtid % OP::G);                                         \
    const bool live_ = row_ < n;                                                  \
    const int32_t stop_ = *(done ? done : &kNotDone);                             \
    const int64_t i = live_ ? row_ : n - 1;                                       \
    const typename OP::Head h_ = (op).head(i);                                    \
    __VA_ARGS__                                                                   \
    __shared__ int32_t sd_[OP::kShared ? kSellMaxDict + 1 : 1];                   \
    if constexpr (OP::kShared) {                                                  \
        (op).load(sd_);                                                           \
        __syncthreads();                                                          \
    }                                                                             \
    if (stop_ || !live_) {                                                        \
        h_.keep();                                                                \
        return;                                                                   \
    }

// ------------------------------------------------------------ V-cycle ----
// Sweep x <- x + M (b - A x); the first two sweeps from x = 0 are fused:
// x1 = M b, x2 = x1 + M (b - A x1) with x1_j recomputed on the fly.
template <class OP, class V, class Bt, class Yt, int NR>
__global__ void k_smooth_first(int64_t n, OP op, const V *__restrict__ M, const Bt *__restrict__ b,
                               Yt *__restrict__ y, int two, const int32_t *done) {
    VecN<V, NR> bi{};
    V mi = 0;
    VROW_PROLOGUE(OP, op, bi = cvt<V>(load_n<Bt, NR>(b, i)); mi = M[i];)
    VecN<V, NR> x1;
#pragma unroll
    for (int k = 0; k < NR; ++k) x1.v[k] = mi * bi.v[k];
    if (two) {
        const VecN<V, NR> ax = op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) {
            const VecN<V, NR> bj = cvt<V>(load_n<Bt, NR>(b, j));
            const V mj = M[j];
            VecN<V, NR> o;
#pragma unroll
            for (int k = 0; k < NR; ++k) o.v[k] = mj * bj.v[k];
            return o;
        });
#pragma unroll
        for (int k = 0; k < NR; ++k) x1.v[k] = x1.v[k] + mi * (bi.v[k] - ax.v[k]);
    }
    if (lane == 0) store_n<Yt, NR>(y, i, cvt<Yt>(x1));
}

template <class OP, class V, class Bt, class Xt, class Yt, int NR>
__global__ void k_smooth(int64_t n, OP op, const V *__restrict__ M, const Bt *__restrict__ b,
                         const Xt *__restrict__ x, Yt *__restrict__ y, const int32_t *done) {
    VecN<V, NR> xi{}, bi{};
    V mi = 0;
    VROW_PROLOGUE(OP, op, xi = cvt<V>(load_n<Xt, NR>(x, i)); bi = cvt<V>(load_n<Bt, NR>(b, i)); mi = M[i];)
    const VecN<V, NR> ax =
        op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) { return cvt<V>(load_n<Xt, NR>(x, j)); });
    if (lane == 0) {
        VecN<V, NR> o;
#pragma unroll
        for (int k = 0; k < NR; ++k) o.v[k] = xi.v[k] + mi * (bi.v[k] - ax.v[k]);
        store_n<Yt, NR>(y, i, cvt<Yt>(o));
    }
}

template <class OP, class V, class Bt, class Xt, class Rt, int NR>
__global__ void k_residual(int64_t n, OP op, const Bt *__restrict__ b, const Xt *__restrict__ x,
                           Rt *__restrict__ r, const int32_t *done) {
    VecN<V, NR> bi{};
    VROW_PROLOGUE(OP, op, bi = cvt<V>(load_n<Bt, NR>(b, i));)
    const VecN<V, NR> ax =
        op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) { return cvt<V>(load_n<Xt, NR>(x, j)); });
    if (lane == 0) {
        VecN<V, NR> o;
#pragma unroll
        for (int k = 0; k < NR; ++k) o.v[k] = bi.v[k] - ax.v[k];
        store_n<Rt, NR>(r, i, cvt<Rt>(o));
    }
}

template <class OP, class V, class Xt, class Yt, int NR>
__global__ void k_spmv(int64_t n, OP op, const Xt *__restrict__ x, Yt *__restrict__ y, const int32_t *done) {
    VROW_PROLOGUE(OP, op, )
    const VecN<V, NR> s =
        op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) { return cvt<V>(load_n<Xt, NR>(x, j)); });
    if (lane == 0) store_n<Yt, NR>(y, i, cvt<Yt>(s));
}

// x += P x_c
template <class OP, class V, class Xt, int NR>
__global__ void k_prolong(int64_t n, OP op, const Xt *__restrict__ xc, Xt *__restrict__ x, const int32_t *done) {
    VecN<V, NR> xi{};
    VROW_PROLOGUE(OP, op, xi = cvt<V>(load_n<Xt, NR>(x, i));)
    const VecN<V, NR> s =
        op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) { return cvt<V>(load_n<Xt, NR>(xc, j)); });
    if (lane == 0) {
        VecN<V, NR> o;
#pragma unroll
        for (int k = 0; k < NR; ++k) o.v[k] = xi.v[k] + s.v[k];
        store_n<Xt, NR>(x, i, cvt<Xt>(o));
    }
}

// Coarsest level: x = A_L^{-1} b with the row-major inverse, one wave per
// row, accumulated in FP64.
// The first kCoarseU columns of a lane are loaded with the done flag, before
// any is used (a coarsest level of up to kCoarseU*64 rows takes one round of
// loads); the products are added in column order all the same.
constexpr int kCoarseU = 8;

template <class Bt, class Yt, int NR>
__global__ void k_coarse_gemv(int32_t n, const double *__restrict__ inv, const Bt *__restrict__ b,
                              Yt *__restrict__ y, const int32_t *done) {
    const int32_t stop = *(done ? done : &kNotDone);
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / dev::kWave;
    const int lane = threadIdx.x & (dev::kWave - 1);
    const int64_t ir = i < n ? i : n - 1;
    double a[kCoarseU];
    VecN<double, NR> bc[kCoarseU];
#pragma unroll
    for (int u = 0; u < kCoarseU; ++u) {
        const int32_t c = min(lane + u * dev::kWave, n - 1);
        a[u] = inv[ir * n + c];
        bc[u] = cvt<double>(load_n<Bt, NR>(b, c));
    }
    if (stop || i >= n) return;
    VecN<double, NR> s;
#pragma unroll
    for (int k = 0; k < NR; ++k) s.v[k] = 0.0;
#pragma unroll
    for (int u = 0; u < kCoarseU; ++u)
        if (lane + u * dev::kWave < n)
#pragma unroll
            for (int k = 0; k < NR; ++k) s.v[k] += a[u] * bc[u].v[k];
    for (int32_t c = lane + kCoarseU * dev::kWave; c < n; c += dev::kWave) {
        const double av = inv[i * n + c];
        const VecN<double, NR> bv = cvt<double>(load_n<Bt, NR>(b, c));
#pragma unroll
        for (int k = 0; k < NR; ++k) s.v[k] += av * bv.v[k];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) s.v[k] = dev::wave_sum(s.v[k]);
    if (lane == 0) store_n<Yt, NR>(y, i, cvt<Yt>(s));
}

template <class X>
__global__ void k_zero(X *x, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = (X)0;
}

// y = x + z (ILU(0) smoothing step; y may be x)
__global__ void k_add(const double *x, const double *__restrict__ z, double *y, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + z[i];
}

template <class Xt, class Yt>
__global__ void k_convert(const Xt *__restrict__ x, Yt *__restrict__ y, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (Yt)x[i];
}

// Bytes one pass over an operator touches: values and column information
// (int32 columns + row pointers for CSR; one-byte offsets or int32 columns,
// padding included, + slice offsets for sliced ELL).
double csr_bytes(int64_t n, int64_t nnz, int vbytes) { return (double)nnz * (vbytes + 4) + 4.0 * (n + 1); }
double op_bytes(const Csr &A, const Sell &S, int vbytes) {
    if (S.built()) return (double)S.nnz_padded * (vbytes + (S.ndict ? 1 : 4)) + 4.0 * (S.nslices + 1);
    return csr_bytes(A.n, A.nnz, vbytes);
}

unsigned grid_rows(int64_t n, int G) { return blocks_for(n * G); }

// Timing class of a V-cycle kernel on level l (ids of level 0, 1 and >= 2
// are five apart).
int level_kid(int id0, int l) { return id0 + 5 * (l < 2 ? l : 2); }

template <class V>
struct LevelOps;
template <>
struct LevelOps<double> {
    static const double *aval(const Level &L) { return L.A.val.p; }
    static const double *asval(const Level &L) { return L.As.val.p; }
    static const double *pval(const Level &L) { return L.P.val.p; }
    static const double *rval(const Level &L) { return L.R.val.p; }
    static const double *mval(const Level &L) { return L.M.p; }
};
template <>
struct LevelOps<float> {
    static const float *aval(const Level &L) { return L.A.val32.p; }
    static const float *asval(const Level &L) { return L.As.val32.p; }
    static const float *pval(const Level &L) { return L.P.val32.p; }
    static const float *rval(const Level &L) { return L.R.val32.p; }
    static const float *mval(const Level &L) { return L.M32.p; }
};

// Call f(op) with the operator type of a CSR matrix (its lane group).
template <class V, class F>
void with_csr(const Csr &A, const V *val, F &&f) {
    switch (A.grp) {
        case 1: f(OpCsr<1, V>{A.rowptr.p, A.col.p, val}); break;
        case 2: f(OpCsr<2, V>{A.rowptr.p, A.col.p, val}); break;
        case 4: f(OpCsr<4, V>{A.rowptr.p, A.col.p, val}); break;
        case 8: f(OpCsr<8, V>{A.rowptr.p, A.col.p, val}); break;
        case 16: f(OpCsr<16, V>{A.rowptr.p, A.col.p, val}); break;
        case 32: f(OpCsr<32, V>{A.rowptr.p, A.col.p, val}); break;
        default: f(OpCsr<64, V>{A.rowptr.p, A.col.p, val}); break;
    }
}

// Call f(op) with the level's operator: the sliced ELL copy when built.
template <class V, class F>
void with_level_op(const Level &Lv, F &&f) {
    if (Lv.As.built() && LevelOps<V>::asval(Lv)) f(OpSell<V>{view(Lv.As), LevelOps<V>::asval(Lv)});
    else with_csr<V>(Lv.A, LevelOps<V>::aval(Lv), f);
}

// One V-cycle on level l for NR right-hand sides (interleaved).  `b` is the
// right-hand side (type Bt), the result goes to `out` (type Zt) when given,
// else into one of the level's own buffers, whose address is returned.  V =
// value type of the hierarchy (also the type of all internal vectors).
template <class V, class Bt, class Zt, int NR>
void *vcycle_level(amg_hierarchy *H, int l, const Bt *b, Zt *out, const int32_t *done, hipStream_t s);

// A level with the ILU(0) smoother (FP64, one right-hand side): each sweep is
// x <- x + (LU)^{-1} (b - A x), the first from x = 0 being x = (LU)^{-1} b.
template <class Zt>
void *vcycle_level_ilu(amg_hierarchy *H, int l, const double *b, Zt *out, const int32_t *done, hipStream_t s) {
    Level &Lv = H->L[l];
    IluData &I = *Lv.ilu;
    const int64_t n = Lv.A.n;
    double *x = reinterpret_cast<double *>(Lv.vx.p);
    double *t = reinterpret_cast<double *>(Lv.vt.p);
    const int npre = H->prm.npre, npost = H->prm.npost;
    const double abytes = op_bytes(Lv.A, Lv.As, 8);
    auto residual = [&](const double *xin, double *r) {
        ProfScope ps(level_kid(K_RESIDUAL0, l), abytes + n * 24.0, s, true);
        with_level_op<double>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_residual<OP, double, double, double, double, 1>), dim3(grid_rows(n, OP::G)),
                               dim3(kBlock), 0, s, n, op, b, xin, r, done);
        });
    };
    auto step = [&](double *xio, double *dst) {  // dst = x + (LU)^{-1}(b - A x)
        residual(xio, I.r.p);
        ilu_apply(I, I.r.p, I.z.p, done, s);
        hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(kBlock), 0, s, xio, I.z.p, dst, n, done);
    };
    if (npre == 0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n, done);
    } else {
        ilu_apply(I, b, x, done, s);
        for (int k = 1; k < npre; ++k) step(x, x);
    }
    residual(x, t);
    Level &Nx = H->L[l + 1];
    double *bc = reinterpret_cast<double *>(Nx.vb.p);
    const int64_t nc = Lv.nc;
    {
        ProfScope ps(level_kid(K_RESTRICT0, l), csr_bytes(nc, Lv.R.nnz, 8) + (double)(n + nc) * 8, s, true);
        with_csr<double>(Lv.R, Lv.R.val.p, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_spmv<OP, double, double, double, 1>), dim3(grid_rows(nc, OP::G)), dim3(kBlock), 0,
                               s, nc, op, t, bc, done);
        });
    }
    double *xc = static_cast<double *>(vcycle_level<double, double, double, 1>(H, l + 1, bc, (double *)nullptr,
                                                                               done, s));
    {
        ProfScope ps(level_kid(K_PROLONG0, l), csr_bytes(n, Lv.P.nnz, 8) + (double)(2 * n + nc) * 8, s, true);
        with_csr<double>(Lv.P, Lv.P.val.p, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_prolong<OP, double, double, 1>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n,
                               op, xc, x, done);
        });
    }
    for (int k = 0; k < npost; ++k) {
        if (k == npost - 1 && out && std::is_same_v<Zt, double>) {
            step(x, reinterpret_cast<double *>(out));
            return out;
        }
        step(x, x);
    }
    if (out) {
        hipLaunchKernelGGL((k_convert<double, Zt>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, out, n, done);
        return out;
    }
    return x;
}

template <class V, class Bt, class Zt, int NR>
void *vcycle_level(amg_hierarchy *H, int l, const Bt *b, Zt *out, const int32_t *done, hipStream_t s) {
    Level &Lv = H->L[l];
    const int64_t n = Lv.A.n;
    const int vb = (int)sizeof(V);
    const double nr = NR;
    if (l == H->nlev - 1) {
        Zt *y = out ? out : reinterpret_cast<Zt *>(Lv.vx.p);
        ProfScope ps(K_COARSE_SOLVE, (double)n * n * 8 + nr * n * (double)(sizeof(Bt) + sizeof(Zt)), s);
        hipLaunchKernelGGL((k_coarse_gemv<Bt, Zt, NR>), dim3(blocks_for(n * dev::kWave)), dim3(kBlock), 0, s,
                           (int32_t)n, H->inv.p, b, y, done);
        return y;
    }
    const V *M = LevelOps<V>::mval(Lv);
    const double abytes = op_bytes(Lv.A, Lv.As, vb);
    V *x = reinterpret_cast<V *>(Lv.vx.p);
    V *t = reinterpret_cast<V *>(Lv.vt.p);
    const int npre = H->prm.npre, npost = H->prm.npost;
    if constexpr (std::is_same_v<V, double> && std::is_same_v<Bt, double> && NR == 1) {
        if (Lv.ilu) return vcycle_level_ilu<Zt>(H, l, b, out, done, s);
    }

    // pre-smoothing
    if (npre == 0) {
        hipLaunchKernelGGL((k_zero<V>), dim3(blocks_for(n * NR)), dim3(kBlock), 0, s, x, n * NR, done);
    } else {
        ProfScope ps(level_kid(K_SMOOTH_FIRST0, l),
                     (npre >= 2 ? abytes : 0.0) + n * (double)vb + nr * n * (double)(sizeof(Bt) + vb), s, true);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_smooth_first<OP, V, Bt, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n,
                               op, M, b, x, npre >= 2 ? 1 : 0, done);
        });
    }
    auto sweep = [&](auto *xin, auto *yout) {
        using YT = std::remove_pointer_t<decltype(yout)>;
        ProfScope ps(level_kid(K_SMOOTH0, l),
                     abytes + n * (double)vb + nr * n * (double)(sizeof(Bt) + vb + sizeof(YT)), s, true);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_smooth<OP, V, Bt, V, YT, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, op,
                               M, b, xin, yout, done);
        });
    };
    for (int k = 2; k < npre; ++k) {
        sweep(x, t);
        std::swap(x, t);
    }
    // residual and restriction
    {
        ProfScope ps(level_kid(K_RESIDUAL0, l), abytes + nr * n * (double)(sizeof(Bt) + 2 * vb), s, true);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_residual<OP, V, Bt, V, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, op,
                               b, x, t, done);
        });
    }
    Level &Nx = H->L[l + 1];
    V *bc = reinterpret_cast<V *>(Nx.vb.p);
    const int64_t nc = Lv.nc;
    {
        ProfScope ps(level_kid(K_RESTRICT0, l), csr_bytes(nc, Lv.R.nnz, vb) + nr * (double)(n + nc) * vb, s, true);
        with_csr<V>(Lv.R, LevelOps<V>::rval(Lv), [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_spmv<OP, V, V, V, NR>), dim3(grid_rows(nc, OP::G)), dim3(kBlock), 0, s, nc, op, t,
                               bc, done);
        });
    }
    V *xc = static_cast<V *>(vcycle_level<V, V, V, NR>(H, l + 1, bc, (V *)nullptr, done, s));
    {
        ProfScope ps(level_kid(K_PROLONG0, l), csr_bytes(n, Lv.P.nnz, vb) + nr * (double)(2 * n + nc) * vb, s, true);
        with_csr<V>(Lv.P, LevelOps<V>::pval(Lv), [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_prolong<OP, V, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, op, xc, x,
                               done);
        });
    }
    // post-smoothing; the last sweep writes the requested output
    for (int k = 0; k < npost; ++k) {
        if (k == npost - 1 && out) {
            sweep(x, out);
            return out;
        }
        sweep(x, t);
        std::swap(x, t);
    }
    if (out) {
        hipLaunchKernelGGL((k_convert<V, Zt>), dim3(blocks_for(n * NR)), dim3(kBlock), 0, s, x, out, n * NR, done);
        return out;
    }
    return x;
}

// -------------------------------------------------------------- Krylov ---
constexpr int kKBlock = 256;
constexpr int kKMaxBlocks = 2048;

// Grid of a grouped row loop: rows are visited by (block, group) in a
// grid-stride loop over at most kKMaxBlocks blocks.
unsigned kgrid(int64_t n, int G) {
    int64_t b = (n * G + kKBlock - 1) / kKBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kKMaxBlocks));
}

#define GROUP_LOOP(G, i, lane, n)                                                         \
    const int lane = (int)(threadIdx.x % (G));                                            \
    for (int64_t i = (dev::xcd_block() * (int64_t)blockDim.x + threadIdx.x) / (G); i < (n); \
         i += (int64_t)gridDim.x * blockDim.x / (G))

#define GRID_LOOP(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// r = b - A x (and BiCGSTAB's r_hat = r, p = v = 0); partials b.b, r.r
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_kr_init(int64_t n, OP op, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ rh, double *__restrict__ p,
                                                     double *__restrict__ v, double *partials) {
    OP_PROLOGUE(op)
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        double ax = op.row(i, lane, sd_, [&](int32_t j) { return x[j]; });
        if (lane == 0) {
            double ri = b[i] - ax;
            r[i] = ri;
            if (rh) rh[i] = ri;
            if (p) p[i] = 0.0;
            if (v) v[i] = 0.0;
            acc[0] += b[i] * b[i];
            acc[1] += ri * ri;
        }
    }
    dev::block_partials<2>(acc, partials);
}

// CG: partials r.z and z.q
__global__ void __launch_bounds__(kKBlock) k_cg_dot(int64_t n, const double *__restrict__ r,
                                                    const double *__restrict__ z, const double *__restrict__ q,
                                                    double *partials, const KScalars *ks) {
    if (ks->done) return;
    double acc[2] = {0.0, 0.0};
    GRID_LOOP(i, n) {
        acc[0] += r[i] * z[i];
        acc[1] += z[i] * q[i];
    }
    dev::block_partials<2>(acc, partials);
}

// p_new = z + beta p_old;  q = A p_new;  partial p_new . q
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_cg_spmv(int64_t n, OP op, const double *__restrict__ z,
                                                     const double *__restrict__ p_old, double *__restrict__ p_new,
                                                     double *__restrict__ q, double *partials, const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks->done) return;
    const double beta = ks->beta;
    double acc[1] = {0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        double s = op.row(i, lane, sd_, [&](int32_t j) { return z[j] + beta * p_old[j]; });
        if (lane == 0) {
            double pi = z[i] + beta * p_old[i];
            p_new[i] = pi;
            q[i] = s;
            acc[0] += pi * s;
        }
    }
    dev::block_partials<1>(acc, partials);
}

// x += alpha p;  r -= alpha q;  partial r.r
__global__ void __launch_bounds__(kKBlock) k_cg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                       const double *__restrict__ p, const double *__restrict__ q,
                                                       double *partials, const KScalars *ks) {
    if (ks->done) return;
    const double alpha = ks->alpha;
    double acc[1] = {0.0};
    GRID_LOOP(i, n) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    dev::block_partials<1>(acc, partials);
}

// partial (b - A x).(b - A x)
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_true_res(int64_t n, OP op, const double *__restrict__ b,
                                                      const double *__restrict__ x, double *partials) {
    OP_PROLOGUE(op)
    double acc[1] = {0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        double ax = op.row(i, lane, sd_, [&](int32_t j) { return x[j]; });
        if (lane == 0) {
            double ri = b[i] - ax;
            acc[0] += ri * ri;
        }
    }
    dev::block_partials<1>(acc, partials);
}

// BiCGSTAB: p = r + beta (p - omega v)
__global__ void __launch_bounds__(kKBlock) k_bcg_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                                   const double *__restrict__ v, const KScalars *ks) {
    if (ks->done) return;
    const double beta = ks->beta, omega = ks->omega;
    GRID_LOOP(i, n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// v = A p_hat;  partial r_hat . v
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_v(int64_t n, OP op, const double *__restrict__ ph,
                                                   double *__restrict__ v, const double *__restrict__ rh,
                                                   double *partials, const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks->done) return;
    double acc[1] = {0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        double vi = op.row(i, lane, sd_, [&](int32_t j) { return ph[j]; });
        if (lane == 0) {
            v[i] = vi;
            acc[0] += rh[i] * vi;
        }
    }
    dev::block_partials<1>(acc, partials);
}

// s = r - alpha v;  partial s.s
__global__ void __launch_bounds__(kKBlock) k_bcg_s(int64_t n, const double *__restrict__ r,
                                                   const double *__restrict__ v, double *__restrict__ sv,
                                                   double *partials, const KScalars *ks) {
    if (ks->done) return;
    const double alpha = ks->alpha;
    double acc[1] = {0.0};
    GRID_LOOP(i, n) {
        double si = r[i] - alpha * v[i];
        sv[i] = si;
        acc[0] += si * si;
    }
    dev::block_partials<1>(acc, partials);
}

// t = A s_hat;  partials t.s, t.t
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_t(int64_t n, OP op, const double *__restrict__ sh,
                                                   double *__restrict__ t, const double *__restrict__ sv,
                                                   double *partials, const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks->done) return;
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        double ti = op.row(i, lane, sd_, [&](int32_t j) { return sh[j]; });
        if (lane == 0) {
            t[i] = ti;
            acc[0] += ti * sv[i];
            acc[1] += ti * ti;
        }
    }
    dev::block_partials<2>(acc, partials);
}

// x += alpha p_hat + omega s_hat;  r = s - omega t;  partials r.r, r_hat.r.
// After an early stop on ||s|| only x += alpha p_hat is applied.
__global__ void __launch_bounds__(kKBlock) k_bcg_xr(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ ph, const double *__restrict__ sh,
                                                    const double *__restrict__ sv, const double *__restrict__ t,
                                                    const double *__restrict__ rh, double *partials,
                                                    const KScalars *ks) {
    const int pending = ks->pending_x;
    if (ks->done && !pending) return;
    const double alpha = ks->alpha, omega = ks->omega;
    double acc[2] = {0.0, 0.0};
    if (pending) {
        GRID_LOOP(i, n) x[i] += alpha * ph[i];
    } else {
        GRID_LOOP(i, n) {
            x[i] += alpha * ph[i] + omega * sh[i];
            double ri = sv[i] - omega * t[i];
            r[i] = ri;
            acc[0] += ri * ri;
            acc[1] += rh[i] * ri;
        }
    }
    dev::block_partials<2>(acc, partials);
}

// The scalar step that follows each reduction.
enum FinOp : int {
    FIN_INIT_FIRST, FIN_INIT_RESTART, FIN_CG_BETA_FIRST, FIN_CG_BETA, FIN_CG_ALPHA, FIN_CG_CONV,
    FIN_TRUE_RES, FIN_BCG_ALPHA, FIN_BCG_S, FIN_BCG_OMEGA, FIN_BCG_XR
};

// The scalar step that follows reduction `op`, from the reduced values.
__device__ void fin_apply(int op, const double (&tot)[2], double rtol, KScalars *ks) {
    switch (op) {
        case FIN_INIT_FIRST:
        case FIN_INIT_RESTART:
            if (op == FIN_INIT_FIRST) {
                ks->bnorm = sqrt(tot[0]);
                ks->tol = rtol * ks->bnorm;
            }
            ks->rr = tot[1];
            ks->done = 0;
            // BiCGSTAB start: r_hat = r, rho = r_hat.r, rho_prev = alpha = omega = 1
            ks->rho_prev = 1.0;
            ks->alpha = 1.0;
            ks->omega = 1.0;
            ks->rho = tot[1];
            ks->beta = tot[1];
            ks->pending_x = 0;
            if (!dev::finite_nz(tot[1]) && ks->bnorm != 0.0) {
                ks->status = GW_BREAKDOWN;
                ks->done = 1;
            }
            break;
        case FIN_CG_BETA_FIRST:
            ks->beta = 0.0;
            ks->rz = tot[0];
            break;
        case FIN_CG_BETA:
            // Polak-Ribiere: z.(r - r_old) = -alpha z.q since r - r_old = -alpha q
            ks->beta = ks->flexible ? (-ks->alpha * tot[1]) / ks->rz : tot[0] / ks->rz;
            ks->rz = tot[0];
            break;
        case FIN_CG_ALPHA:
            ks->pq = tot[0];
            if (!dev::finite_nz(tot[0]) || !isfinite(ks->rz)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else ks->alpha = ks->rz / tot[0];
            break;
        case FIN_CG_CONV: {
            ks->rr = tot[0];
            ks->iters += 1;
            double rn = sqrt(tot[0]);
            if (!isfinite(rn)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else if (rn <= ks->tol) { ks->status = GW_OK; ks->done = 1; }
            else if (ks->iters >= ks->maxiter) { ks->status = GW_NOT_CONVERGED; ks->done = 1; }
            break;
        }
        case FIN_TRUE_RES:
            ks->rel_true = sqrt(tot[0]) / ks->bnorm;
            break;
        case FIN_BCG_ALPHA:
            ks->rv = tot[0];
            if (!dev::finite_nz(tot[0])) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else ks->alpha = ks->rho / tot[0];
            break;
        case FIN_BCG_S: {
            ks->ss = tot[0];
            ks->iters += 1;
            double sn = sqrt(tot[0]);
            if (!isfinite(sn)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else if (sn <= ks->tol) { ks->status = GW_OK; ks->rr = tot[0]; ks->done = 1; ks->pending_x = 1; }
            break;
        }
        case FIN_BCG_OMEGA:
            ks->ts = tot[0];
            ks->tt = tot[1];
            if (!dev::finite_nz(tot[1])) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else {
                double om = tot[0] / tot[1];
                if (!dev::finite_nz(om)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
                else ks->omega = om;
            }
            break;
        case FIN_BCG_XR: {
            if (ks->pending_x) { ks->pending_x = 0; break; }
            ks->rr = tot[0];
            double rn = sqrt(tot[0]);
            if (!isfinite(rn)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else if (rn <= ks->tol) { ks->status = GW_OK; ks->done = 1; }
            else if (ks->iters >= ks->maxiter) { ks->status = GW_NOT_CONVERGED; ks->done = 1; }
            else {
                ks->rho_prev = ks->rho;
                ks->rho = tot[1];
                if (!dev::finite_nz(tot[1])) { ks->status = GW_BREAKDOWN; ks->done = 1; }
                else ks->beta = (ks->rho / ks->rho_prev) * (ks->alpha / ks->omega);
            }
            break;
        }
        default: break;
    }
}

__device__ __forceinline__ bool fin_skip(int op, const KScalars *ks) {
    const bool always = op == FIN_INIT_FIRST || op == FIN_INIT_RESTART || op == FIN_TRUE_RES || op == FIN_BCG_XR;
    if (!always && ks->done) return true;
    return op == FIN_BCG_XR && ks->done && !ks->pending_x;
}

__host__ __device__ constexpr int fin_nv(int op) {
    return (op == FIN_INIT_FIRST || op == FIN_INIT_RESTART || op == FIN_CG_BETA_FIRST || op == FIN_CG_BETA ||
            op == FIN_BCG_OMEGA || op == FIN_BCG_XR) ? 2 : 1;
}

// The partials are loaded before the skip test reads the scalars, so both
// latencies overlap.
__global__ void __launch_bounds__(kKBlock) k_finalize(int op, unsigned nb, const double *partials, double rtol,
                                                      KScalars *ks) {
    double tot[2] = {0.0, 0.0};
    if (fin_nv(op) == 2) {
        const int off[2] = {0, 1};
        dev::sum_partials_batched<2>(partials, nb, 2, off, tot);
    } else {
        const int off[1] = {0};
        double t1[1];
        dev::sum_partials_batched<1>(partials, nb, 1, off, t1);
        tot[0] = t1[0];
    }
    if (threadIdx.x == 0 && !fin_skip(op, ks)) fin_apply(op, tot, rtol, ks);
}

// Two right-hand sides: block records hold NV values of each (first, then
// second); ks[0], ks[1] are their scalars, ks[2].done / ks[2].pending_x the
// joint flags read by the product kernels.  Only the right-hand sides in
// `mask` are touched.
__global__ void __launch_bounds__(kKBlock) k_finalize2(int op, unsigned nb, const double *partials, double rtol,
                                                       KScalars *ks, int mask) {
    // both systems' sums in one pass over the records (each added in the
    // order of a one-system finalize)
    double tot[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (fin_nv(op) == 2) {
        const int off[4] = {0, 1, 2, 3};
        double t[4];
        dev::sum_partials_batched<4>(partials, nb, 4, off, t);
        tot[0][0] = t[0], tot[0][1] = t[1], tot[1][0] = t[2], tot[1][1] = t[3];
    } else {
        const int off[2] = {0, 1};
        double t[2];
        dev::sum_partials_batched<2>(partials, nb, 2, off, t);
        tot[0][0] = t[0], tot[1][0] = t[1];
    }
    if (threadIdx.x == 0)
        for (int r = 0; r < 2; ++r)
            if ((mask >> r & 1) && !fin_skip(op, ks + r)) fin_apply(op, tot[r], rtol, ks + r);
    if (threadIdx.x == 0) {
        ks[2].done = ks[0].done && ks[1].done;
        ks[2].pending_x = ks[0].pending_x || ks[1].pending_x;
    }
}

// ------------------------------------------- two right-hand sides -------
// BiCGSTAB for two systems with one matrix, in lockstep: vectors hold the
// two values of a row next to each other, every product reads the matrix
// once for both, and each system keeps its own scalars (ks[0], ks[1]) and
// stops on its own flag; the kernels leave a stopped system untouched.  The
// grids and per-thread row sets equal those of the one-system kernels, so
// each system's partial sums, and therefore its iterates, are the ones a
// separate solve produces.

// r = b - A x, r_hat = r, p = v = 0 for the systems in `mask`; partials b.b,
// r.r per system
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_kr_init2(int64_t n, OP op, const double *__restrict__ b,
                                                      const double *__restrict__ x, double *__restrict__ r,
                                                      double *__restrict__ rh, double *__restrict__ p,
                                                      double *__restrict__ v, double *partials, int mask) {
    OP_PROLOGUE(op)
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        const VecN<double, 2> ax = op.template rows<2>(i, lane, sd_, [&](int32_t j) { return load_n<double, 2>(x, j); });
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (!(mask >> k & 1)) continue;
                const double bi = b[2 * i + k], ri = bi - ax.v[k];
                r[2 * i + k] = ri;
                rh[2 * i + k] = ri;
                p[2 * i + k] = 0.0;
                v[2 * i + k] = 0.0;
                acc[2 * k] += bi * bi;
                acc[2 * k + 1] += ri * ri;
            }
        }
    }
    dev::block_partials<4>(acc, partials);
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(kKBlock) k_bcg_p2(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                                    const double *__restrict__ v, const KScalars *ks) {
    if (ks[2].done) return;
    const bool on0 = !ks[0].done, on1 = !ks[1].done;
    const double b0 = ks[0].beta, w0 = ks[0].omega, b1 = ks[1].beta, w1 = ks[1].omega;
    GRID_LOOP(i, n) {
        if (on0) p[2 * i] = r[2 * i] + b0 * (p[2 * i] - w0 * v[2 * i]);
        if (on1) p[2 * i + 1] = r[2 * i + 1] + b1 * (p[2 * i + 1] - w1 * v[2 * i + 1]);
    }
}

// v = A p_hat; partials r_hat . v
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_v2(int64_t n, OP op, const double *__restrict__ ph,
                                                    double *__restrict__ v, const double *__restrict__ rh,
                                                    double *partials, const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks[2].done) return;
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        const VecN<double, 2> vi = op.template rows<2>(i, lane, sd_, [&](int32_t j) { return load_n<double, 2>(ph, j); });
        if (lane == 0) {
            store_n<double, 2>(v, i, vi);
            acc[0] += rh[2 * i] * vi.v[0];
            acc[1] += rh[2 * i + 1] * vi.v[1];
        }
    }
    dev::block_partials<2>(acc, partials);
}

// s = r - alpha v; partials s.s
__global__ void __launch_bounds__(kKBlock) k_bcg_s2(int64_t n, const double *__restrict__ r,
                                                    const double *__restrict__ v, double *__restrict__ sv,
                                                    double *partials, const KScalars *ks) {
    if (ks[2].done) return;
    const bool on0 = !ks[0].done, on1 = !ks[1].done;
    const double a0 = ks[0].alpha, a1 = ks[1].alpha;
    double acc[2] = {0.0, 0.0};
    GRID_LOOP(i, n) {
        if (on0) {
            const double si = r[2 * i] - a0 * v[2 * i];
            sv[2 * i] = si;
            acc[0] += si * si;
        }
        if (on1) {
            const double si = r[2 * i + 1] - a1 * v[2 * i + 1];
            sv[2 * i + 1] = si;
            acc[1] += si * si;
        }
    }
    dev::block_partials<2>(acc, partials);
}

// t = A s_hat; partials t.s, t.t
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_t2(int64_t n, OP op, const double *__restrict__ sh,
                                                    double *__restrict__ t, const double *__restrict__ sv,
                                                    double *partials, const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks[2].done) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        const VecN<double, 2> ti = op.template rows<2>(i, lane, sd_, [&](int32_t j) { return load_n<double, 2>(sh, j); });
        if (lane == 0) {
            store_n<double, 2>(t, i, ti);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                acc[2 * k] += ti.v[k] * sv[2 * i + k];
                acc[2 * k + 1] += ti.v[k] * ti.v[k];
            }
        }
    }
    dev::block_partials<4>(acc, partials);
}

// x += alpha p_hat + omega s_hat; r = s - omega t; partials r.r, r_hat.r.
// A system stopped early on ||s|| gets only x += alpha p_hat.
__global__ void __launch_bounds__(kKBlock) k_bcg_xr2(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ ph, const double *__restrict__ sh,
                                                     const double *__restrict__ sv, const double *__restrict__ t,
                                                     const double *__restrict__ rh, double *partials,
                                                     const KScalars *ks) {
    if (ks[2].done && !ks[2].pending_x) return;
    int mode[2];
    double al[2], om[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        mode[k] = ks[k].pending_x ? 1 : (ks[k].done ? 0 : 2);
        al[k] = ks[k].alpha;
        om[k] = ks[k].omega;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    GRID_LOOP(i, n) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t e = 2 * i + k;
            if (mode[k] == 1) {
                x[e] += al[k] * ph[e];
            } else if (mode[k] == 2) {
                x[e] += al[k] * ph[e] + om[k] * sh[e];
                const double ri = sv[e] - om[k] * t[e];
                r[e] = ri;
                acc[2 * k] += ri * ri;
                acc[2 * k + 1] += rh[e] * ri;
            }
        }
    }
    dev::block_partials<4>(acc, partials);
}

// partials (b - A x).(b - A x) per system
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_true_res2(int64_t n, OP op, const double *__restrict__ b,
                                                       const double *__restrict__ x, double *partials) {
    OP_PROLOGUE(op)
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(OP::G, i, lane, n) {
        const VecN<double, 2> ax = op.template rows<2>(i, lane, sd_, [&](int32_t j) { return load_n<double, 2>(x, j); });
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double ri = b[2 * i + k] - ax.v[k];
                acc[k] += ri * ri;
            }
        }
    }
    dev::block_partials<2>(acc, partials);
}

// Interleave two vectors / split them again.
__global__ void k_interleave(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                             double *__restrict__ ab) {
    GRID_LOOP(i, n) {
        ab[2 * i] = a[i];
        ab[2 * i + 1] = b[i];
    }
}

__global__ void k_split(int64_t n, const double *__restrict__ ab, double *__restrict__ a, double *__restrict__ b) {
    GRID_LOOP(i, n) {
        a[i] = ab[2 * i];
        b[i] = ab[2 * i + 1];
    }
}

template <class OP>
__global__ void k_spmv_f64(int64_t n, OP op, const double *__restrict__ x, double *__restrict__ y) {
    OP_PROLOGUE(op)
    GROUP_ROW(OP::G)
    double s = op.row(i, lane, sd_, [&](int32_t j) { return x[j]; });
    if (lane == 0) y[i] = s;
}

void ensure_krylov_workspace(amg_hierarchy *H, int nvec) {
    const size_t n = (size_t)H->L[0].A.n;
    if (H->kvec_count < nvec) {
        H->drop_graphs();
        H->kvec.alloc(n * nvec);
        H->kvec_count = nvec;
    }
    if (!H->partials.p) H->partials.alloc((size_t)kKMaxBlocks * 4);
    if (!H->ks.p) H->ks.alloc(3);
}

static_assert(sizeof(KScalars) <= kHostStageBytes, "Krylov scalars must fit the pinned stage");

static_assert(3 * sizeof(KScalars) <= kHostStageBytes, "two systems' scalars must fit the pinned stage");

void read_ks3(amg_hierarchy *H, KScalars (&k)[3], hipStream_t s) {
    void *stage = host_stage();
    GW_HIP(hipMemcpyAsync(stage, H->ks.p, 3 * sizeof(KScalars), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    std::memcpy(k, stage, 3 * sizeof(KScalars));
}

void write_ks3(amg_hierarchy *H, const KScalars (&k)[3], hipStream_t s) {
    void *stage = host_stage();
    std::memcpy(stage, k, 3 * sizeof(KScalars));
    GW_HIP(hipMemcpyAsync(H->ks.p, stage, 3 * sizeof(KScalars), hipMemcpyHostToDevice, s));
    GW_HIP(hipStreamSynchronize(s));
}

KScalars read_ks(amg_hierarchy *H, hipStream_t s) {
    void *stage = host_stage();
    GW_HIP(hipMemcpyAsync(stage, H->ks.p, sizeof(KScalars), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    KScalars k;
    std::memcpy(&k, stage, sizeof(KScalars));
    return k;
}

void write_ks(amg_hierarchy *H, const KScalars &k, hipStream_t s) {
    void *stage = host_stage();
    std::memcpy(stage, &k, sizeof(KScalars));
    GW_HIP(hipMemcpyAsync(H->ks.p, stage, sizeof(KScalars), hipMemcpyHostToDevice, s));
    GW_HIP(hipStreamSynchronize(s));
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum BlockKind : int { BLOCK_PCG = 1, BLOCK_BICGSTAB = 2, BLOCK_BICGSTAB2 = 3 };

// Enqueue one block of Krylov iterations on s: `emit(stream)` launches its
// kernels.  With `graph`, the block is captured once per (kind, length,
// parity) on the hierarchy's capture stream, which runs nothing, and the
// instantiated graph is launched on s.  Every kernel reads its scalars and
// the convergence flag from device memory, so a replay after convergence is
// a run of early exits, exactly as the one-by-one launches are.
// Iterations to enqueue before the next convergence poll: check_every, or
// fewer once the residual's rate of decrease over the last block predicts
// convergence sooner, so that few iterations run as early exits after it
// (each still launches its kernels).  Graph replays keep their captured
// check_every.  Only the launching changes: the iterates are the same.
struct PollPlan {
    int check;
    bool graph;
    double rn_prev = -1.0;
    int it_prev = 0;
    int predict(double rn, double goal, int iters) const {
        if (graph || rn_prev <= 0.0 || iters <= it_prev || !(rn < rn_prev) || !(rn > goal) || !(goal > 0.0))
            return check;
        const double rate = std::pow(rn / rn_prev, 1.0 / (iters - it_prev));
        const double need = std::log(goal / rn) / std::log(rate);
        if (!std::isfinite(need)) return check;
        return std::max(1, std::min(check, (int)std::ceil(need)));
    }
    int next(double rn, double goal, int iters) {
        const int c = predict(rn, goal, iters);
        rn_prev = rn;
        it_prev = iters;
        return c;
    }
};

template <class Emit>
void run_block(amg_hierarchy *H, bool graph, int kind, int check, int parity, hipStream_t s, Emit &&emit) {
    if (!graph) {
        emit(s);
        return;
    }
    hipGraphExec_t ex = nullptr;
    for (const auto &g : H->graphs)
        if (g.kind == kind && g.check == check && g.parity == parity) ex = g.exec;
    if (!ex) {
        if (!H->cap) GW_HIP(hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
        GW_HIP(hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal));
        hipGraph_t g = nullptr;
        try {
            emit(H->cap);
        } catch (...) {
            if (hipStreamEndCapture(H->cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            throw;
        }
        GW_HIP(hipStreamEndCapture(H->cap, &g));
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        GW_HIP(e);
        H->graphs.push_back({kind, check, parity, ex});
    }
    GW_HIP(hipGraphLaunch(ex, s));
}

bool use_graph(const amg_solve_params &sp) { return sp.graph > 0; }

// Host-side helper binding the level-0 operator and the scalar block.
struct Kry {
    amg_hierarchy *H;
    const Level &L0;
    int G;
    int64_t n;
    unsigned g1, gG;  // grids of element-wise and row-product kernels
    double *part;
    KScalars *ks;
    hipStream_t s;
    double rtol;
    double vec, abytes;
    const double *shift = nullptr;  // diagonal added to A (OpShift), or none

    Kry(amg_hierarchy *H_, hipStream_t s_, double rtol_) : H(H_), L0(H_->L[0]), s(s_), rtol(rtol_) {
        G = L0.As.built() ? 1 : L0.A.grp;
        n = L0.A.n;
        g1 = kgrid(n, 1);
        gG = kgrid(n, G);
        part = H->partials.p;
        ks = H->ks.p;
        vec = 8.0 * n;
        abytes = op_bytes(L0.A, L0.As, 8);
    }
    template <bool SHIFT = false, class F>
    void op(F &&f) const {
        if constexpr (SHIFT) {
            if (L0.As.built()) f(OpShift<OpSell<double>>{OpSell<double>{view(L0.As), L0.As.val.p}, shift});
            else with_csr<double>(L0.A, L0.A.val.p, [&](auto o) { f(OpShift<decltype(o)>{o, shift}); });
        } else {
            if (L0.As.built()) f(OpSell<double>{view(L0.As), L0.As.val.p});
            else with_csr<double>(L0.A, L0.A.val.p, f);
        }
    }
    void fin(int code, unsigned nb) {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kKBlock), 0, s, code, nb, part, rtol, ks);
    }
    template <bool SHIFT = false>
    void init(const double *b, const double *x, double *r, double *rh, double *p, double *v, bool first) {
        {
            ProfScope ps(K_KRYLOV_SPMV, abytes + 4 * vec + (rh ? 3 * vec : 0), s);
            op<SHIFT>([&](auto o) {
                hipLaunchKernelGGL((k_kr_init<decltype(o)>), dim3(gG), dim3(kKBlock), 0, s, n, o, b, x, r, rh, p, v,
                                   part);
            });
        }
        fin(first ? FIN_INIT_FIRST : FIN_INIT_RESTART, gG);
    }
    template <bool SHIFT = false>
    void true_res(const double *b, const double *x) {
        {
            ProfScope ps(K_TRUE_RESIDUAL, abytes + 2 * vec, s);
            op<SHIFT>([&](auto o) {
                hipLaunchKernelGGL((k_true_res<decltype(o)>), dim3(gG), dim3(kKBlock), 0, s, n, o, b, x, part);
            });
        }
        fin(FIN_TRUE_RES, gG);
    }
};

}  // namespace

int lane_group_for(double mean_row_len) {
    if (mean_row_len <= 3.0) return 1;
    if (mean_row_len <= 12.0) return 4;
    if (mean_row_len <= 48.0) return 16;
    return 64;
}

// Solve-phase products load 8 entries per lane (4 with 64 lanes) before
// summing: a row gets the fewest lanes G (a power of two) whose 8G slots
// hold 1.4 times the mean row length, so a typical row is one round and the
// wave covers as many rows as possible.  Measured against 1/4/16/64 lanes
// with 4/2/2/1 loads per lane: 8.4M-cell pass 215 -> 172 ms, 1M-cell pass
// 32.0 -> 30.5 ms (level-1 sweeps of ~33-entry rows 15 -> 11.6 us).
int solve_group_for(double mean_row_len) {
    int g = 1;
    while (g < 64 && 8.0 * g < 1.4 * mean_row_len) g *= 2;
    return g;
}

void vcycle(amg_hierarchy *H, const double *r, double *z, const int32_t *done, hipStream_t s) {
    if (H->nlev == 0) {
        // preconditioner off: z = r
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks_for(H->L[0].A.n)), dim3(kBlock), 0, s, r, z,
                           (int64_t)H->L[0].A.n, done);
        GW_HIP(hipGetLastError());
        return;
    }
    if (H->mixed()) vcycle_level<float, double, double, 1>(H, 0, r, z, done, s);
    else vcycle_level<double, double, double, 1>(H, 0, r, z, done, s);
    GW_HIP(hipGetLastError());
}

namespace {

// Level vectors sized for nr interleaved right-hand sides.
void ensure_level_vectors(amg_hierarchy *H, int nr) {
    const size_t es = H->mixed() ? 4 : 8;
    for (int l = 0; l < H->nlev; ++l) {
        Level &Lv = H->L[l];
        const size_t need = (size_t)Lv.A.n * es * nr;
        if (Lv.vx.n >= need) continue;
        H->drop_graphs();
        Lv.vx.alloc(need);
        Lv.vt.alloc(need);
        if (l > 0) Lv.vb.alloc(need);
    }
}

// One V-cycle on two interleaved right-hand sides.
void vcycle2(amg_hierarchy *H, const double *r, double *z, const int32_t *done, hipStream_t s) {
    if (H->nlev == 0) {
        const int64_t n2 = 2 * (int64_t)H->L[0].A.n;
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks_for(n2)), dim3(kBlock), 0, s, r, z, n2, done);
        GW_HIP(hipGetLastError());
        return;
    }
    if (H->mixed()) vcycle_level<float, double, double, 2>(H, 0, r, z, done, s);
    else vcycle_level<double, double, double, 2>(H, 0, r, z, done, s);
    GW_HIP(hipGetLastError());
}

}  // namespace

void spmv_level0(amg_hierarchy *H, const double *x, double *y, hipStream_t s) {
    const Level &L0 = H->L[0];
    const int64_t n = L0.A.n;
    ProfScope ps(K_KRYLOV_SPMV, op_bytes(L0.A, L0.As, 8) + 16.0 * n, s);
    auto launch = [&](auto o) {
        using OP = decltype(o);
        hipLaunchKernelGGL((k_spmv_f64<OP>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, o, x, y);
    };
    if (L0.As.built()) launch(OpSell<double>{view(L0.As), L0.As.val.p});
    else with_csr<double>(L0.A, L0.A.val.p, launch);
    GW_HIP(hipGetLastError());
}

namespace {

// PCG on A (SHIFT false) or on A + diag(shift) with the hierarchy of A as the
// preconditioner (SHIFT true; launched one by one: a captured graph would
// keep the shift pointer of its first call).
template <bool SHIFT>
int pcg_impl(amg_hierarchy *H, const double *shift, const double *b, double *x_out, const amg_solve_params &sp,
             amg_solve_info *info, hipStream_t s) {
    const double t0 = now_ms();
    ensure_krylov_workspace(H, 6);
    Kry K(H, s, sp.rtol);
    K.shift = shift;
    const int64_t n = K.n;
    // the iterate lives in the workspace (a captured block then serves any
    // output buffer) and is copied out at the end
    double *r = H->kvec.p, *z = r + n, *pa = z + n, *pb = pa + n, *q = pb + n, *x = q + n;
    KScalars k0{};
    k0.maxiter = std::max(0, sp.maxiter);
    k0.flexible = sp.flexible < 0 ? (H->mixed() ? 1 : 0) : (sp.flexible ? 1 : 0);
    k0.status = GW_NOT_CONVERGED;
    write_ks(H, k0, s);
    fill_f64(x, 0.0, n, s);
    K.template init<SHIFT>(b, x, r, nullptr, pa, nullptr, true);
    KScalars k = read_ks(H, s);
    int restarts = 0;
    if (k.bnorm == 0.0) {
        fill_f64(x_out, 0.0, n, s);
        if (info) *info = {0, GW_OK, 0, 0.0, 0.0, 0.0, now_ms() - t0};
        return GW_OK;
    }
    const int check = std::max(1, sp.check_every);
    const bool graph = !SHIFT && use_graph(sp);
    int32_t *done = &H->ks.p->done;
    int parity = 0;
    int cnt = check;  // iterations in the next block
    // check_every iterations: q = A p, alpha, x and r updates with the
    // convergence test, z = M r, beta
    auto block = [&](int parity0) {
        return [&, parity0](hipStream_t cs) {
            Kry Kc(H, cs, sp.rtol);
            Kc.shift = shift;
            int par = parity0;
            for (int c = 0; c < cnt; ++c) {
                double *po = par ? pb : pa, *pn = par ? pa : pb;
                {
                    ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 4 * Kc.vec, cs, true);
                    Kc.template op<SHIFT>([&](auto o) {
                        GW_LAUNCH_TIMED(ps, (k_cg_spmv<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, z, po,
                                           pn, q, Kc.part, Kc.ks);
                    });
                }
                Kc.fin(FIN_CG_ALPHA, Kc.gG);
                {
                    ProfScope ps(K_KRYLOV_UPDATE, 6 * Kc.vec, cs);
                    hipLaunchKernelGGL(k_cg_update, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, x, r, pn, q, Kc.part,
                                       Kc.ks);
                }
                Kc.fin(FIN_CG_CONV, Kc.g1);
                vcycle(H, r, z, done, cs);
                {
                    ProfScope ps(K_KRYLOV_DOT, 3 * Kc.vec, cs);
                    hipLaunchKernelGGL(k_cg_dot, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, z, q, Kc.part, Kc.ks);
                }
                Kc.fin(FIN_CG_BETA, Kc.g1);
                par ^= 1;
            }
            GW_HIP(hipGetLastError());
        };
    };
    for (;;) {
        if (!k.done) {
            vcycle(H, r, z, done, s);
            {
                ProfScope ps(K_KRYLOV_DOT, 3 * K.vec, s);
                hipLaunchKernelGGL(k_cg_dot, dim3(K.g1), dim3(kKBlock), 0, s, n, r, z, q, K.part, K.ks);
            }
            K.fin(FIN_CG_BETA_FIRST, K.g1);
            PollPlan plan{check, graph};
            cnt = check;
            for (;;) {
                run_block(H, graph, BLOCK_PCG, check, parity, s, block(parity));
                parity ^= cnt & 1;
                k = read_ks(H, s);
                if (k.done) break;
                cnt = plan.next(std::sqrt(k.rr), k.tol, k.iters);
            }
        }
        K.template true_res<SHIFT>(b, x);
        k = read_ks(H, s);
        if (k.status == GW_BREAKDOWN) break;
        if (k.rel_true <= sp.rtol) { k.status = GW_OK; break; }
        if (k.iters >= k.maxiter || restarts >= 8) { k.status = GW_NOT_CONVERGED; break; }
        ++restarts;
        parity = 0;
        K.template init<SHIFT>(b, x, r, nullptr, pa, nullptr, false);
        k = read_ks(H, s);
    }
    copy_bytes(x_out, x, sizeof(double) * (size_t)n, s);
    if (info) {
        info->iters = k.iters;
        info->status = k.status;
        info->restarts = restarts;
        info->rel_res = std::sqrt(k.rr) / k.bnorm;
        info->rel_res_true = k.rel_true;
        info->setup_ms = 0.0;
        info->solve_ms = now_ms() - t0;
    }
    return k.status;
}

}  // namespace

int krylov_pcg(amg_hierarchy *H, const double *b, double *x_out, const amg_solve_params &sp, amg_solve_info *info,
               hipStream_t s) {
    return pcg_impl<false>(H, nullptr, b, x_out, sp, info, s);
}

int krylov_pcg_shifted(amg_hierarchy *H, const double *shift, const double *b, double *x_out,
                       const amg_solve_params &sp, amg_solve_info *info, hipStream_t s) {
    return pcg_impl<true>(H, shift, b, x_out, sp, info, s);
}

int krylov_bicgstab(amg_hierarchy *H, const double *b, double *x_out, const amg_solve_params &sp,
                    amg_solve_info *info, hipStream_t s) {
    const double t0 = now_ms();
    ensure_krylov_workspace(H, 9);
    Kry K(H, s, sp.rtol);
    const int64_t n = K.n;
    double *r = H->kvec.p, *rh = r + n, *p = rh + n, *v = p + n, *sv = v + n, *t = sv + n, *ph = t + n,
           *sh = ph + n, *x = sh + n;
    KScalars k0{};
    k0.maxiter = std::max(0, sp.maxiter);
    k0.status = GW_NOT_CONVERGED;
    write_ks(H, k0, s);
    fill_f64(x, 0.0, n, s);
    K.init(b, x, r, rh, p, v, true);
    KScalars k = read_ks(H, s);
    int restarts = 0;
    if (k.bnorm == 0.0) {
        fill_f64(x_out, 0.0, n, s);
        if (info) *info = {0, GW_OK, 0, 0.0, 0.0, 0.0, now_ms() - t0};
        return GW_OK;
    }
    const int check = std::max(1, sp.check_every);
    const bool graph = use_graph(sp);
    int32_t *done = &H->ks.p->done;
    int cnt = check;  // iterations in the next block
    // cnt iterations of right-preconditioned BiCGSTAB
    auto block = [&](hipStream_t cs) {
        Kry Kc(H, cs, sp.rtol);
        for (int c = 0; c < cnt; ++c) {
            {
                ProfScope ps(K_KRYLOV_UPDATE, 4 * Kc.vec, cs);
                hipLaunchKernelGGL(k_bcg_p, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, p, v, Kc.ks);
            }
            vcycle(H, p, ph, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * Kc.vec, cs, true);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_v<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, ph, v, rh,
                                       Kc.part, Kc.ks);
                });
            }
            Kc.fin(FIN_BCG_ALPHA, Kc.gG);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 3 * Kc.vec, cs);
                hipLaunchKernelGGL(k_bcg_s, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, v, sv, Kc.part, Kc.ks);
            }
            Kc.fin(FIN_BCG_S, Kc.g1);
            vcycle(H, sv, sh, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * Kc.vec, cs, true);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_t<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, sh, t, sv,
                                       Kc.part, Kc.ks);
                });
            }
            Kc.fin(FIN_BCG_OMEGA, Kc.gG);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 8 * Kc.vec, cs);
                hipLaunchKernelGGL(k_bcg_xr, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, x, r, ph, sh, sv, t, rh, Kc.part,
                                   Kc.ks);
            }
            Kc.fin(FIN_BCG_XR, Kc.g1);
        }
        GW_HIP(hipGetLastError());
    };
    for (;;) {
        PollPlan plan{check, graph};
        cnt = check;
        while (!k.done) {
            run_block(H, graph, BLOCK_BICGSTAB, check, 0, s, block);
            k = read_ks(H, s);
            cnt = plan.next(std::sqrt(k.rr), k.tol, k.iters);
        }
        K.true_res(b, x);
        k = read_ks(H, s);
        if (k.status == GW_BREAKDOWN) break;
        if (k.rel_true <= sp.rtol) { k.status = GW_OK; break; }
        if (k.iters >= k.maxiter || restarts >= 8) { k.status = GW_NOT_CONVERGED; break; }
        ++restarts;
        K.init(b, x, r, rh, p, v, false);
        k = read_ks(H, s);
    }
    copy_bytes(x_out, x, sizeof(double) * (size_t)n, s);
    if (info) {
        info->iters = k.iters;
        info->status = k.status;
        info->restarts = restarts;
        info->rel_res = std::sqrt(k.rr) / k.bnorm;
        info->rel_res_true = k.rel_true;
        info->setup_ms = 0.0;
        info->solve_ms = now_ms() - t0;
    }
    return k.status;
}

int krylov_bicgstab2(amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1,
                     const amg_solve_params &sp, amg_solve_info info[2], hipStream_t s) {
    if (H->prm.smoother == GW_SMOOTHER_ILU0) {
        // the substitution sweeps take one right-hand side: one system at a time
        const int s0 = krylov_bicgstab(H, b0, x0, sp, &info[0], s);
        const int s1 = krylov_bicgstab(H, b1, x1, sp, &info[1], s);
        return std::max(s0, s1);
    }
    const double t0 = now_ms();
    ensure_krylov_workspace(H, 20);
    ensure_level_vectors(H, 2);
    Kry K(H, s, sp.rtol);
    const int64_t n = K.n, n2 = 2 * n;
    double *b = H->kvec.p, *r = b + n2, *rh = r + n2, *p = rh + n2, *v = p + n2, *sv = v + n2, *t = sv + n2,
           *ph = t + n2, *sh = ph + n2, *x = sh + n2;
    double *part = K.part;
    KScalars *ks = K.ks;
    const double vec2 = 2 * K.vec;
    auto fin2 = [&](hipStream_t cs, int code, unsigned nb, int mask) {
        hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(kKBlock), 0, cs, code, nb, part, sp.rtol, ks, mask);
    };
    auto init2 = [&](int mask, bool first) {
        {
            ProfScope ps(K_KRYLOV_SPMV, K.abytes + 7 * vec2, s);
            K.op([&](auto o) {
                hipLaunchKernelGGL((k_kr_init2<decltype(o)>), dim3(K.gG), dim3(kKBlock), 0, s, n, o, b, x, r, rh, p,
                                   v, part, mask);
            });
        }
        fin2(s, first ? FIN_INIT_FIRST : FIN_INIT_RESTART, K.gG, mask);
    };
    hipLaunchKernelGGL(k_interleave, dim3(K.g1), dim3(kKBlock), 0, s, n, b0, b1, b);
    KScalars kk[3] = {};
    kk[0].maxiter = kk[1].maxiter = std::max(0, sp.maxiter);
    kk[0].status = kk[1].status = GW_NOT_CONVERGED;
    write_ks3(H, kk, s);
    fill_f64(x, 0.0, n2, s);
    init2(3, true);
    read_ks3(H, kk, s);
    bool final[2] = {false, false};
    int restarts[2] = {0, 0}, status[2] = {GW_NOT_CONVERGED, GW_NOT_CONVERGED};
    bool zero_rhs = false;
    for (int k = 0; k < 2; ++k) {
        if (kk[k].bnorm != 0.0) continue;
        // b = 0: x = 0, nothing to iterate
        final[k] = true;
        status[k] = GW_OK;
        kk[k].done = 1;
        kk[k].iters = 0;
        kk[k].rr = 0.0;
        kk[k].rel_true = 0.0;
        zero_rhs = true;
    }
    if (zero_rhs) {
        kk[2].done = kk[0].done && kk[1].done;
        write_ks3(H, kk, s);
    }
    const int check = std::max(1, sp.check_every);
    const bool graph = use_graph(sp);
    const int32_t *done = &ks[2].done;
    int cnt = check;  // iterations in the next block
    auto block = [&](hipStream_t cs) {
        Kry Kc(H, cs, sp.rtol);
        for (int c = 0; c < cnt; ++c) {
            {
                ProfScope ps(K_KRYLOV_UPDATE, 4 * vec2, cs);
                hipLaunchKernelGGL(k_bcg_p2, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, p, v, ks);
            }
            vcycle2(H, p, ph, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * vec2, cs, true);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_v2<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, ph, v, rh,
                                       part, ks);
                });
            }
            fin2(cs, FIN_BCG_ALPHA, Kc.gG, 3);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 3 * vec2, cs);
                hipLaunchKernelGGL(k_bcg_s2, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, v, sv, part, ks);
            }
            fin2(cs, FIN_BCG_S, Kc.g1, 3);
            vcycle2(H, sv, sh, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * vec2, cs, true);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_t2<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, sh, t, sv,
                                       part, ks);
                });
            }
            fin2(cs, FIN_BCG_OMEGA, Kc.gG, 3);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 8 * vec2, cs);
                hipLaunchKernelGGL(k_bcg_xr2, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, x, r, ph, sh, sv, t, rh, part, ks);
            }
            fin2(cs, FIN_BCG_XR, Kc.g1, 3);
        }
        GW_HIP(hipGetLastError());
    };
    for (;;) {
        // the block ends when the slower of the running systems is predicted
        // to converge
        PollPlan plan[2] = {{check, graph}, {check, graph}};
        cnt = check;
        while (!kk[2].done) {
            run_block(H, graph, BLOCK_BICGSTAB2, check, 0, s, block);
            read_ks3(H, kk, s);
            int c2 = 1;
            for (int q = 0; q < 2; ++q) {
                const int cq = plan[q].next(std::sqrt(kk[q].rr), kk[q].tol, kk[q].iters);
                if (!kk[q].done) c2 = std::max(c2, cq);
            }
            cnt = c2;
        }
        {
            ProfScope ps(K_TRUE_RESIDUAL, K.abytes + 2 * vec2, s);
            K.op([&](auto o) {
                hipLaunchKernelGGL((k_true_res2<decltype(o)>), dim3(K.gG), dim3(kKBlock), 0, s, n, o, b, x, part);
            });
        }
        fin2(s, FIN_TRUE_RES, K.gG, 3);
        read_ks3(H, kk, s);
        int mask = 0;
        for (int k = 0; k < 2; ++k) {
            if (final[k]) continue;
            const KScalars &q = kk[k];
            if (q.status == GW_BREAKDOWN) { status[k] = GW_BREAKDOWN; final[k] = true; continue; }
            if (q.rel_true <= sp.rtol) { status[k] = GW_OK; final[k] = true; continue; }
            if (q.iters >= q.maxiter || restarts[k] >= 8) { status[k] = GW_NOT_CONVERGED; final[k] = true; continue; }
            ++restarts[k];
            mask |= 1 << k;
        }
        if (!mask) break;
        init2(mask, false);
        read_ks3(H, kk, s);
    }
    hipLaunchKernelGGL(k_split, dim3(K.g1), dim3(kKBlock), 0, s, n, x, x0, x1);
    GW_HIP(hipGetLastError());
    const double ms = now_ms() - t0;
    for (int k = 0; k < 2; ++k) {
        if (!info) break;
        const KScalars &q = kk[k];
        info[k].iters = q.iters;
        info[k].status = status[k];
        info[k].restarts = restarts[k];
        info[k].rel_res = q.bnorm != 0.0 ? std::sqrt(q.rr) / q.bnorm : 0.0;
        info[k].rel_res_true = q.bnorm != 0.0 ? q.rel_true : 0.0;
        info[k].setup_ms = 0.0;
        info[k].solve_ms = ms;
    }
    if (status[0] == GW_BREAKDOWN || status[1] == GW_BREAKDOWN) return GW_BREAKDOWN;
    if (status[0] != GW_OK || status[1] != GW_OK) return GW_NOT_CONVERGED;
    return GW_OK;
}

}  // namespace gw
