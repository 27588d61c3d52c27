// Kernels of the solve phase, shared by the one-system drivers (solve.hip)
// and the shared-launch drivers that run several independent systems per
// launch (batch.hip): the operators, the V-cycle and Krylov kernel bodies,
// the scalar steps that follow each reduction, and the shared-launch kernel.
//
// Every product kernel is written once against an operator type: OpSell (the
// sliced ELL copy of the level-0 operator, one lane per row, dictionary of
// column offsets in LDS) or OpCsr<G> (G lanes per CSR row, G picked per
// matrix from its mean row length, so the lanes of a wave read consecutive
// entries).  The Krylov scalars live on the device: a product kernel leaves
// per-block partial sums, a one-block finalize kernel adds them in a fixed
// order and forms alpha/beta/omega and the convergence flag; every later
// kernel reads the flag and returns at once.
#pragma once

#include <algorithm>
#include <cstdint>
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
    __device__ __host__ static constexpr int lanes() { return G; }
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

// group_row_sum with the lane group a runtime value G (1..64, a power of
// two): lane l adds entries b+l, b+l+G, ... in order and the group is
// combined by the same butterfly, with the same number of padding slots as
// the compile-time form (4 loads a batch for G = 1 or 64, else 8), so every
// row sum is the compile-time form's bit for bit.
template <int NR, class V, class F>
__device__ __forceinline__ VecN<V, NR> group_row_sum_dyn(int32_t b, int32_t e, const int32_t *__restrict__ col,
                                                         const V *__restrict__ val, int lane, int G, F &&xj) {
    VecN<V, NR> s;
#pragma unroll
    for (int k = 0; k < NR; ++k) s.v[k] = 0;
    if (b < e) {
        const int32_t cb = col[b];
        if (G == 1 || G == 64) {
            for (int32_t q = b + lane; q < e; q += 4 * G) {
                V a[4];
                int32_t c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t p = q + u * G;
                    const bool in = p < e;
                    const int32_t pc = in ? p : b;
                    const V av = val[pc];
                    const int32_t cv = col[pc];
                    a[u] = in ? av : V(0);
                    c[u] = in ? cv : cb;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const VecN<V, NR> xv = xj(c[u]);
#pragma unroll
                    for (int k = 0; k < NR; ++k) s.v[k] += a[u] * xv.v[k];
                }
            }
        } else {
            for (int32_t q = b + lane; q < e; q += 8 * G) {
                V a[8];
                int32_t c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t p = q + u * G;
                    const bool in = p < e;
                    const int32_t pc = in ? p : b;
                    const V av = val[pc];
                    const int32_t cv = col[pc];
                    a[u] = in ? av : V(0);
                    c[u] = in ? cv : cb;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const VecN<V, NR> xv = xj(c[u]);
#pragma unroll
                    for (int k = 0; k < NR; ++k) s.v[k] += a[u] * xv.v[k];
                }
            }
        }
    }
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NR; ++k) s.v[k] += __shfl_xor(s.v[k], o, dev::kWave);
    return s;
}

// A CSR operator whose lane group is chosen at run time: the systems of a
// shared launch, whose matrices pick different groups, then take one launch
// instead of one per group.  Row sums equal OpCsr<g>'s bit for bit.
template <class V>
struct OpCsrDyn {
    static constexpr int G = 0;  // see lanes()
    static constexpr bool kShared = false;
    using Head = typename OpCsr<1, V>::Head;
    const int32_t *rowptr, *col;
    const V *val;
    int g;
    __device__ __host__ int lanes() const { return g; }
    __device__ __forceinline__ void load(int32_t *) const {}
    __device__ __forceinline__ Head head(int64_t i) const { return Head{rowptr[i], rowptr[i + 1]}; }
    template <int NR, class F>
    __device__ __forceinline__ VecN<V, NR> rows_at(const Head &h, int64_t, int lane, const int32_t *,
                                                   F &&xj) const {
        return group_row_sum_dyn<NR, V>(h.b, h.e, col, val, lane, g, xj);
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
    __device__ __host__ static constexpr int lanes() { return 1; }
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
        const int64_t sl = i >> S.cshift;
        const int32_t off = S.soff[sl];
        return Head{off, (S.soff[sl + 1] - off) >> S.cshift};
    }
    // Entries k of row i sit at soff[slice] + k*C + (i mod C).  Eight
    // entries are loaded before their products are summed, so the gathers
    // of x overlap; the sum still runs in entry order.  Slots past the slice
    // width re-read the last entry and are replaced by the padding entry
    // (value 0 at the row's own column) in registers, without branches.
    template <bool DICT, int NR, class F>
    __device__ __forceinline__ VecN<V, NR> row_impl(const Head &h, int64_t i, const int32_t *sd, F &&xj) const {
        const int l = (int)(i & ((1 << S.cshift) - 1));
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
                const int64_t e = off + ((int64_t)k << S.cshift) + l;
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

// The stencil copy (Stencil): one lane a row, its 2K+1 terms in column order
// -- left neighbours i - d_k from the arrays c_k[i - d_k], the diagonal,
// right neighbours from c_k[i] -- summed as the sliced copy sums the same
// entries.  Symmetric form: the values as stored; one-sided form: c_k[i]
// where negative, -c_k[i - d_k] where c_k[i - d_k] is positive (an exact
// negation back to the stored a_{i,i-d_k}).  Terms of a neighbour outside
// the matrix, absent from the row, or of k >= K carry 0 and read x at a
// clamped index (a finite x adds an exact zero).  No head to load and no
// dictionary.
template <class V>
struct OpSten {
    static constexpr int G = 1;
    static constexpr bool kShared = false;
    __device__ __host__ static constexpr int lanes() { return 1; }
    struct Head {
        __device__ __forceinline__ void keep() const {}
    };
    int32_t n, K;
    int32_t d[kStenMax];
    int32_t onesided;
    const V *c;
    __device__ __forceinline__ void load(int32_t *) const {}
    __device__ __forceinline__ Head head(int64_t) const { return {}; }
    template <int NR, class F>
    __device__ __forceinline__ VecN<V, NR> rows_at(const Head &, int64_t i, int, const int32_t *, F &&xj) const {
        constexpr int T = 2 * kStenMax + 1;
        V a[T];
        int32_t cj[T];
        const int32_t ii = (int32_t)i;
        // slot kStenMax-1-k: left term of d_k; kStenMax: the diagonal;
        // kStenMax+1+k: right term of d_k
#pragma unroll
        for (int k = 0; k < kStenMax; ++k) {
            const int32_t dk = k < K ? d[k] : 0;
            const bool lin = k < K && ii >= dk;
            const bool rin = k < K && ii + dk < n;
            const int64_t base = (int64_t)(k < K ? 1 + k : 0) * n;
            const V gl = c[base + (lin ? ii - dk : ii)];
            const V gr = c[base + ii];
            const V al = onesided ? (gl > V(0) ? -gl : V(0)) : gl;
            const V ar = onesided ? (gr < V(0) ? gr : V(0)) : gr;
            a[kStenMax - 1 - k] = lin ? al : V(0);
            cj[kStenMax - 1 - k] = lin ? ii - dk : ii;
            a[kStenMax + 1 + k] = rin ? ar : V(0);
            cj[kStenMax + 1 + k] = rin ? ii + dk : ii;
        }
        a[kStenMax] = c[ii];
        cj[kStenMax] = ii;
        VecN<V, NR> acc;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc.v[k] = 0;
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const VecN<V, NR> xv = xj(cj[u]);
#pragma unroll
            for (int k = 0; k < NR; ++k) acc.v[k] += a[u] * xv.v[k];
        }
        return acc;
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
    __device__ __host__ static constexpr int lanes() { return B::lanes(); }
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

// ---------------------------------------------------------- launch grid ---
// The block a workgroup plays and the block count of its grid: the launch's
// own (VG::here()), or, inside a shared launch of several systems, the
// system's own grid, so that each system sees exactly the rows, block
// partials and summation order of a launch of its own.
struct VG {
    int64_t b, nb;
    __device__ static VG here() { return VG{(int64_t)blockIdx.x, (int64_t)gridDim.x}; }
    // dev::xcd_block's renumbering within this grid: each XCD walks one
    // contiguous range of rows (a launch of its own keeps the gathers of its
    // rows in that XCD's L2)
    __device__ int64_t xcd() const {
        const int64_t full = nb / dev::kXcds * dev::kXcds;
        if (b >= full) return b;
        return (b % dev::kXcds) * (full / dev::kXcds) + b / dev::kXcds;
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

// Prologue of a V-cycle kernel body (blocks of kBlock threads, G lanes per
// row, n >= 1, grid vg_): the `done` flag, the row's head and the
// statements `...` (loads of the row's own vector entries, through `i`) are
// issued together, rows past the end reading row n-1; then the dictionary
// (sliced operators only); then the flag is tested.  A small level's kernel
// thus waits for one round of loads where a test first would wait for three
// in a row.
#define VROW_PROLOGUE(OP, op, ...)                                                \
    const int64_t gtid = vg_.xcd() * (int64_t)kBlock + threadIdx.x;               \
    const int64_t row_ = gtid / (op).lanes();                                     \
    const int lane = (int)(gtid % (op).lanes());                                  \
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

// Each kernel below is a body (a device function of its grid vg_ and of its
// arguments, which keep their __restrict__ promises) and an argument record
// K whose run(vg) calls the body: a kernel of its own launches the body on
// VG::here(), a shared launch (k_seg) runs the records of several systems.

// ------------------------------------------------------------ V-cycle ----
// Sweep x <- x + M (b - A x); the first two sweeps from x = 0 are fused:
// x1 = M b, x2 = x1 + M (b - A x1) with x1_j recomputed on the fly.
template <class OP, class V, class Bt, class Yt, int NR>
__device__ __forceinline__ void smooth_first_body(VG vg_, int64_t n, OP op, const V *__restrict__ M,
                                                  const Bt *__restrict__ b, Yt *__restrict__ y, int two,
                                                  const int32_t *done) {
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
template <class OP, class V, class Bt, class Yt, int NR>
struct SmoothFirstK {
    int64_t n;
    OP op;
    const V *M;
    const Bt *b;
    Yt *y;
    int two;
    const int32_t *done;
    __device__ void run(VG vg) const { smooth_first_body<OP, V, Bt, Yt, NR>(vg, n, op, M, b, y, two, done); }
};

// One pre-smoothing sweep from x = 0 and the residual after it in one pass
// (one pre-sweep): x1 = M b and r = b - A x1, with x1_j recomputed on the
// fly as the fused first sweeps do, so that the residual does not wait for
// the sweep's launch and x1 is not read back.  x1 and r take exactly the
// values of the sweep kernel followed by the residual kernel.
template <class OP, class V, class Bt, class Rt, int NR>
__device__ __forceinline__ void smooth_res_body(VG vg_, int64_t n, OP op, const V *__restrict__ M,
                                                const Bt *__restrict__ b, V *__restrict__ y, Rt *__restrict__ r,
                                                const int32_t *done) {
    VecN<V, NR> bi{};
    V mi = 0;
    VROW_PROLOGUE(OP, op, bi = cvt<V>(load_n<Bt, NR>(b, i)); mi = M[i];)
    const VecN<V, NR> ax = op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) {
        const VecN<V, NR> bj = cvt<V>(load_n<Bt, NR>(b, j));
        const V mj = M[j];
        VecN<V, NR> o;
#pragma unroll
        for (int k = 0; k < NR; ++k) o.v[k] = mj * bj.v[k];
        return o;
    });
    if (lane == 0) {
        VecN<V, NR> x1, o;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            x1.v[k] = mi * bi.v[k];
            o.v[k] = bi.v[k] - ax.v[k];
        }
        store_n<V, NR>(y, i, x1);
        store_n<Rt, NR>(r, i, cvt<Rt>(o));
    }
}

template <class OP, class V, class Bt, class Xt, class Yt, int NR>
__device__ __forceinline__ void smooth_body(VG vg_, int64_t n, OP op, const V *__restrict__ M,
                                            const Bt *__restrict__ b, const Xt *__restrict__ x, Yt *__restrict__ y,
                                            const int32_t *done) {
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
template <class OP, class V, class Bt, class Xt, class Yt, int NR>
struct SmoothK {
    int64_t n;
    OP op;
    const V *M;
    const Bt *b;
    const Xt *x;
    Yt *y;
    const int32_t *done;
    __device__ void run(VG vg) const { smooth_body<OP, V, Bt, Xt, Yt, NR>(vg, n, op, M, b, x, y, done); }
};

template <class OP, class V, class Bt, class Xt, class Rt, int NR>
__device__ __forceinline__ void residual_body(VG vg_, int64_t n, OP op, const Bt *__restrict__ b,
                                              const Xt *__restrict__ x, Rt *__restrict__ r, const int32_t *done) {
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
template <class OP, class V, class Bt, class Xt, class Rt, int NR>
struct ResidualK {
    int64_t n;
    OP op;
    const Bt *b;
    const Xt *x;
    Rt *r;
    const int32_t *done;
    __device__ void run(VG vg) const { residual_body<OP, V, Bt, Xt, Rt, NR>(vg, n, op, b, x, r, done); }
};

template <class OP, class V, class Xt, class Yt, int NR>
__device__ __forceinline__ void spmv_body(VG vg_, int64_t n, OP op, const Xt *__restrict__ x, Yt *__restrict__ y,
                                          const int32_t *done) {
    VROW_PROLOGUE(OP, op, )
    const VecN<V, NR> s =
        op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) { return cvt<V>(load_n<Xt, NR>(x, j)); });
    if (lane == 0) store_n<Yt, NR>(y, i, cvt<Yt>(s));
}
template <class OP, class V, class Xt, class Yt, int NR>
struct SpmvK {
    int64_t n;
    OP op;
    const Xt *x;
    Yt *y;
    const int32_t *done;
    __device__ void run(VG vg) const { spmv_body<OP, V, Xt, Yt, NR>(vg, n, op, x, y, done); }
};

// Restriction b_c = R t; with x1 given, also the first sweep of the next
// level from x = 0, x1 = M_c b_c (the value that level's fused first sweep
// would form), so that level starts from a plain sweep or residual.
template <class OP, class V, int NR>
__device__ __forceinline__ void restrict_body(VG vg_, int64_t n, OP op, const V *__restrict__ t, V *__restrict__ bc,
                                              const V *__restrict__ Mc, V *__restrict__ x1, const int32_t *done) {
    V mi = 0;
    VROW_PROLOGUE(OP, op, mi = x1 ? Mc[i] : (V)0;)
    const VecN<V, NR> s =
        op.template rows_at<NR>(h_, i, lane, sd_, [&](int32_t j) { return load_n<V, NR>(t, j); });
    if (lane == 0) {
        store_n<V, NR>(bc, i, s);
        if (x1) {
            VecN<V, NR> o;
#pragma unroll
            for (int k = 0; k < NR; ++k) o.v[k] = mi * s.v[k];
            store_n<V, NR>(x1, i, o);
        }
    }
}
template <class OP, class V, int NR>
struct RestrictK {
    int64_t n;
    OP op;
    const V *t;
    V *bc;
    const V *Mc;
    V *x1;
    const int32_t *done;
    __device__ void run(VG vg) const { restrict_body<OP, V, NR>(vg, n, op, t, bc, Mc, x1, done); }
};

// x += P x_c
template <class OP, class V, class Xt, int NR>
__device__ __forceinline__ void prolong_body(VG vg_, int64_t n, OP op, const Xt *__restrict__ xc,
                                             Xt *__restrict__ x, const int32_t *done) {
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
template <class OP, class V, class Xt, int NR>
struct ProlongK {
    int64_t n;
    OP op;
    const Xt *xc;
    Xt *x;
    const int32_t *done;
    __device__ void run(VG vg) const { prolong_body<OP, V, Xt, NR>(vg, n, op, xc, x, done); }
};

// Coarsest level: x = A_L^{-1} b with the row-major inverse, one wave per
// row, accumulated in FP64.
// The first kCoarseU columns of a lane are loaded with the done flag, before
// any is used (a coarsest level of up to kCoarseU*64 rows takes one round of
// loads); the products are added in column order all the same.
constexpr int kCoarseU = 8;

template <class Bt, class Yt, int NR>
__device__ __forceinline__ void coarse_gemv_body(VG vg_, int32_t n, const double *__restrict__ inv,
                                                 const Bt *__restrict__ b, Yt *__restrict__ y, const int32_t *done) {
    const int32_t stop = *(done ? done : &kNotDone);
    const int64_t i = (vg_.b * (int64_t)blockDim.x + threadIdx.x) / dev::kWave;
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
template <class Bt, class Yt, int NR>
struct CoarseGemvK {
    int32_t n;
    const double *inv;
    const Bt *b;
    Yt *y;
    const int32_t *done;
    __device__ void run(VG vg) const { coarse_gemv_body<Bt, Yt, NR>(vg, n, inv, b, y, done); }
};

// -------------------------------------------------------------- Krylov ---
constexpr int kKBlock = 256;
constexpr int kKMaxBlocks = 2048;
static_assert(kKBlock == kBlock, "V-cycle and Krylov kernels share one block size (shared launches)");

// Grid of a grouped row loop: rows are visited by (block, group) in a
// grid-stride loop over at most kKMaxBlocks blocks.
inline unsigned kgrid(int64_t n, int G) {
    int64_t b = (n * G + kKBlock - 1) / kKBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kKMaxBlocks));
}

#define GROUP_LOOP(G, i, lane, n)                                                    \
    const int lane = (int)(threadIdx.x % (G));                                       \
    for (int64_t i = (vg_.xcd() * (int64_t)blockDim.x + threadIdx.x) / (G); i < (n); \
         i += vg_.nb * (int64_t)blockDim.x / (G))

#define GRID_LOOP(i, n) \
    for (int64_t i = vg_.b * (int64_t)blockDim.x + threadIdx.x; i < (n); i += vg_.nb * (int64_t)blockDim.x)

// r = b - A x (and BiCGSTAB's r_hat = r, p = v = 0); partials b.b, r.r
template <class OP>
__device__ __forceinline__ void kr_init_body(VG vg_, int64_t n, OP op, const double *__restrict__ b,
                                             const double *__restrict__ x, double *__restrict__ r,
                                             double *__restrict__ rh, double *__restrict__ p,
                                             double *__restrict__ v, double *partials) {
    OP_PROLOGUE(op)
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
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
    dev::block_partials<2>(acc, partials, vg_.b);
}
template <class OP>
struct KrInitK {
    int64_t n;
    OP op;
    const double *b, *x;
    double *r, *rh, *p, *v, *partials;
    __device__ void run(VG vg) const { kr_init_body<OP>(vg, n, op, b, x, r, rh, p, v, partials); }
};

// CG: partials r.z and z.q
__device__ __forceinline__ void cg_dot_body(VG vg_, int64_t n, const double *__restrict__ r,
                                            const double *__restrict__ z, const double *__restrict__ q,
                                            double *partials, const KScalars *ks) {
    if (ks->done) return;
    double acc[2] = {0.0, 0.0};
    GRID_LOOP(i, n) {
        acc[0] += r[i] * z[i];
        acc[1] += z[i] * q[i];
    }
    dev::block_partials<2>(acc, partials, vg_.b);
}
struct CgDotK {
    int64_t n;
    const double *r, *z, *q;
    double *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { cg_dot_body(vg, n, r, z, q, partials, ks); }
};

// p_new = z + beta p_old;  q = A p_new;  partial p_new . q
template <class OP>
__device__ __forceinline__ void cg_spmv_body(VG vg_, int64_t n, OP op, const double *__restrict__ z,
                                             const double *__restrict__ p_old, double *__restrict__ p_new,
                                             double *__restrict__ q, double *partials, const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks->done) return;
    const double beta = ks->beta;
    double acc[1] = {0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
        double s = op.row(i, lane, sd_, [&](int32_t j) { return z[j] + beta * p_old[j]; });
        if (lane == 0) {
            double pi = z[i] + beta * p_old[i];
            p_new[i] = pi;
            q[i] = s;
            acc[0] += pi * s;
        }
    }
    dev::block_partials<1>(acc, partials, vg_.b);
}
template <class OP>
struct CgSpmvK {
    int64_t n;
    OP op;
    const double *z, *p_old;
    double *p_new, *q, *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { cg_spmv_body<OP>(vg, n, op, z, p_old, p_new, q, partials, ks); }
};

// x += alpha p;  r -= alpha q;  partial r.r
__device__ __forceinline__ void cg_update_body(VG vg_, int64_t n, double *__restrict__ x, double *__restrict__ r,
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
    dev::block_partials<1>(acc, partials, vg_.b);
}
struct CgUpdateK {
    int64_t n;
    double *x, *r;
    const double *p, *q;
    double *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { cg_update_body(vg, n, x, r, p, q, partials, ks); }
};

// partial (b - A x).(b - A x)
template <class OP>
__device__ __forceinline__ void true_res_body(VG vg_, int64_t n, OP op, const double *__restrict__ b,
                                              const double *__restrict__ x, double *partials) {
    OP_PROLOGUE(op)
    double acc[1] = {0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
        double ax = op.row(i, lane, sd_, [&](int32_t j) { return x[j]; });
        if (lane == 0) {
            double ri = b[i] - ax;
            acc[0] += ri * ri;
        }
    }
    dev::block_partials<1>(acc, partials, vg_.b);
}
template <class OP>
struct TrueResK {
    int64_t n;
    OP op;
    const double *b, *x;
    double *partials;
    __device__ void run(VG vg) const { true_res_body<OP>(vg, n, op, b, x, partials); }
};

// BiCGSTAB: p = r + beta (p - omega v)
__device__ __forceinline__ void bcg_p_body(VG vg_, int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                           const double *__restrict__ v, const KScalars *ks) {
    if (ks->done) return;
    const double beta = ks->beta, omega = ks->omega;
    GRID_LOOP(i, n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// v = A p_hat;  partial r_hat . v
template <class OP>
__device__ __forceinline__ void bcg_v_body(VG vg_, int64_t n, OP op, const double *__restrict__ ph,
                                           double *__restrict__ v, const double *__restrict__ rh, double *partials,
                                           const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks->done) return;
    double acc[1] = {0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
        double vi = op.row(i, lane, sd_, [&](int32_t j) { return ph[j]; });
        if (lane == 0) {
            v[i] = vi;
            acc[0] += rh[i] * vi;
        }
    }
    dev::block_partials<1>(acc, partials, vg_.b);
}

// s = r - alpha v;  partial s.s
__device__ __forceinline__ void bcg_s_body(VG vg_, int64_t n, const double *__restrict__ r,
                                           const double *__restrict__ v, double *__restrict__ sv, double *partials,
                                           const KScalars *ks) {
    if (ks->done) return;
    const double alpha = ks->alpha;
    double acc[1] = {0.0};
    GRID_LOOP(i, n) {
        double si = r[i] - alpha * v[i];
        sv[i] = si;
        acc[0] += si * si;
    }
    dev::block_partials<1>(acc, partials, vg_.b);
}

// t = A s_hat;  partials t.s, t.t
template <class OP>
__device__ __forceinline__ void bcg_t_body(VG vg_, int64_t n, OP op, const double *__restrict__ sh,
                                           double *__restrict__ t, const double *__restrict__ sv, double *partials,
                                           const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks->done) return;
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
        double ti = op.row(i, lane, sd_, [&](int32_t j) { return sh[j]; });
        if (lane == 0) {
            t[i] = ti;
            acc[0] += ti * sv[i];
            acc[1] += ti * ti;
        }
    }
    dev::block_partials<2>(acc, partials, vg_.b);
}

// x += alpha p_hat + omega s_hat;  r = s - omega t;  partials r.r, r_hat.r.
// After an early stop on ||s|| only x += alpha p_hat is applied.
__device__ __forceinline__ void bcg_xr_body(VG vg_, int64_t n, double *__restrict__ x, double *__restrict__ r,
                                            const double *__restrict__ ph, const double *__restrict__ sh,
                                            const double *__restrict__ sv, const double *__restrict__ t,
                                            const double *__restrict__ rh, double *partials, const KScalars *ks) {
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
    dev::block_partials<2>(acc, partials, vg_.b);
}

enum FinOp : int {
    FIN_INIT_FIRST, FIN_INIT_RESTART, FIN_CG_BETA_FIRST, FIN_CG_BETA, FIN_CG_ALPHA, FIN_CG_CONV,
    FIN_TRUE_RES, FIN_BCG_ALPHA, FIN_BCG_S, FIN_BCG_OMEGA, FIN_BCG_XR
};

// The scalar step that follows reduction `op`, from the reduced values.
__device__ __forceinline__ void fin_apply(int op, const double (&tot)[2], double rtol, KScalars *ks) {
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

// The scalars are read into registers before the records are summed, so
// their load overlaps the records' instead of following the block's two
// barriers; thread 0 writes them back when the step changes them.  One block.
__device__ __forceinline__ void finalize_body(int op, unsigned nb, const double *partials, double rtol,
                                              KScalars *ks) {
    KScalars k = *ks;
    double tot[2] = {0.0, 0.0};
    if (fin_nv(op) == 2) {
        const int off[2] = {0, 1};
        dev::sum_partials_batched<2, kKBlock>(partials, nb, 2, off, tot);
    } else {
        const int off[1] = {0};
        double t1[1];
        dev::sum_partials_batched<1, kKBlock>(partials, nb, 1, off, t1);
        tot[0] = t1[0];
    }
    if (threadIdx.x == 0 && !fin_skip(op, &k)) {
        fin_apply(op, tot, rtol, &k);
        *ks = k;
    }
}
struct FinK {
    int op;
    unsigned nb;
    const double *partials;
    double rtol;
    KScalars *ks;
    __device__ void run(VG) const { finalize_body(op, nb, partials, rtol, ks); }
};

// Two right-hand sides: block records hold NV values of each (first, then
// second); ks[0], ks[1] are their scalars, ks[2].done / ks[2].pending_x the
// joint flags read by the product kernels.  Only the right-hand sides in
// `mask` are touched.  One block.
__device__ __forceinline__ void finalize2_body(int op, unsigned nb, const double *partials, double rtol,
                                               KScalars *ks, int mask) {
    // both systems' sums in one pass over the records (each added in the
    // order of a one-system finalize)
    KScalars k[2] = {ks[0], ks[1]};  // read before the sums, as in finalize_body
    double tot[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (fin_nv(op) == 2) {
        const int off[4] = {0, 1, 2, 3};
        double t[4];
        dev::sum_partials_batched<4, kKBlock>(partials, nb, 4, off, t);
        tot[0][0] = t[0], tot[0][1] = t[1], tot[1][0] = t[2], tot[1][1] = t[3];
    } else {
        const int off[2] = {0, 1};
        double t[2];
        dev::sum_partials_batched<2, kKBlock>(partials, nb, 2, off, t);
        tot[0][0] = t[0], tot[1][0] = t[1];
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if ((mask >> r & 1) && !fin_skip(op, &k[r])) {
                fin_apply(op, tot[r], rtol, &k[r]);
                ks[r] = k[r];
            }
        ks[2].done = k[0].done && k[1].done;
        ks[2].pending_x = k[0].pending_x || k[1].pending_x;
    }
}
struct Fin2K {
    int op;
    unsigned nb;
    const double *partials;
    double rtol;
    KScalars *ks;
    int mask;
    __device__ void run(VG) const { finalize2_body(op, nb, partials, rtol, ks, mask); }
};

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
__device__ __forceinline__ void kr_init2_body(VG vg_, int64_t n, OP op, const double *__restrict__ b,
                                              const double *__restrict__ x, double *__restrict__ r,
                                              double *__restrict__ rh, double *__restrict__ p,
                                              double *__restrict__ v, double *partials, int mask) {
    OP_PROLOGUE(op)
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
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
    dev::block_partials<4>(acc, partials, vg_.b);
}
template <class OP>
struct KrInit2K {
    int64_t n;
    OP op;
    const double *b, *x;
    double *r, *rh, *p, *v, *partials;
    int mask;
    __device__ void run(VG vg) const { kr_init2_body<OP>(vg, n, op, b, x, r, rh, p, v, partials, mask); }
};

// p = r + beta (p - omega v)
__device__ __forceinline__ void bcg_p2_body(VG vg_, int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                            const double *__restrict__ v, const KScalars *ks) {
    if (ks[2].done) return;
    const bool on0 = !ks[0].done, on1 = !ks[1].done;
    const double b0 = ks[0].beta, w0 = ks[0].omega, b1 = ks[1].beta, w1 = ks[1].omega;
    GRID_LOOP(i, n) {
        if (on0) p[2 * i] = r[2 * i] + b0 * (p[2 * i] - w0 * v[2 * i]);
        if (on1) p[2 * i + 1] = r[2 * i + 1] + b1 * (p[2 * i + 1] - w1 * v[2 * i + 1]);
    }
}
struct BcgP2K {
    int64_t n;
    const double *r;
    double *p;
    const double *v;
    const KScalars *ks;
    __device__ void run(VG vg) const { bcg_p2_body(vg, n, r, p, v, ks); }
};

// v = A p_hat; partials r_hat . v
template <class OP>
__device__ __forceinline__ void bcg_v2_body(VG vg_, int64_t n, OP op, const double *__restrict__ ph,
                                            double *__restrict__ v, const double *__restrict__ rh, double *partials,
                                            const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks[2].done) return;
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
        const VecN<double, 2> vi = op.template rows<2>(i, lane, sd_, [&](int32_t j) { return load_n<double, 2>(ph, j); });
        if (lane == 0) {
            store_n<double, 2>(v, i, vi);
            acc[0] += rh[2 * i] * vi.v[0];
            acc[1] += rh[2 * i + 1] * vi.v[1];
        }
    }
    dev::block_partials<2>(acc, partials, vg_.b);
}
template <class OP>
struct BcgV2K {
    int64_t n;
    OP op;
    const double *ph;
    double *v;
    const double *rh;
    double *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { bcg_v2_body<OP>(vg, n, op, ph, v, rh, partials, ks); }
};

// s = r - alpha v; partials s.s
__device__ __forceinline__ void bcg_s2_body(VG vg_, int64_t n, const double *__restrict__ r,
                                            const double *__restrict__ v, double *__restrict__ sv, double *partials,
                                            const KScalars *ks) {
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
    dev::block_partials<2>(acc, partials, vg_.b);
}
struct BcgS2K {
    int64_t n;
    const double *r, *v;
    double *sv, *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { bcg_s2_body(vg, n, r, v, sv, partials, ks); }
};

// t = A s_hat; partials t.s, t.t
template <class OP>
__device__ __forceinline__ void bcg_t2_body(VG vg_, int64_t n, OP op, const double *__restrict__ sh,
                                            double *__restrict__ t, const double *__restrict__ sv, double *partials,
                                            const KScalars *ks) {
    OP_PROLOGUE(op)
    if (ks[2].done) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
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
    dev::block_partials<4>(acc, partials, vg_.b);
}
template <class OP>
struct BcgT2K {
    int64_t n;
    OP op;
    const double *sh;
    double *t;
    const double *sv;
    double *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { bcg_t2_body<OP>(vg, n, op, sh, t, sv, partials, ks); }
};

// x += alpha p_hat + omega s_hat; r = s - omega t; partials r.r, r_hat.r.
// A system stopped early on ||s|| gets only x += alpha p_hat.
__device__ __forceinline__ void bcg_xr2_body(VG vg_, int64_t n, double *__restrict__ x, double *__restrict__ r,
                                             const double *__restrict__ ph, const double *__restrict__ sh,
                                             const double *__restrict__ sv, const double *__restrict__ t,
                                             const double *__restrict__ rh, double *partials, const KScalars *ks) {
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
    dev::block_partials<4>(acc, partials, vg_.b);
}
struct BcgXr2K {
    int64_t n;
    double *x, *r;
    const double *ph, *sh, *sv, *t, *rh;
    double *partials;
    const KScalars *ks;
    __device__ void run(VG vg) const { bcg_xr2_body(vg, n, x, r, ph, sh, sv, t, rh, partials, ks); }
};

// partials (b - A x).(b - A x) per system
template <class OP>
__device__ __forceinline__ void true_res2_body(VG vg_, int64_t n, OP op, const double *__restrict__ b,
                                               const double *__restrict__ x, double *partials) {
    OP_PROLOGUE(op)
    double acc[2] = {0.0, 0.0};
    GROUP_LOOP(op.lanes(), i, lane, n) {
        const VecN<double, 2> ax = op.template rows<2>(i, lane, sd_, [&](int32_t j) { return load_n<double, 2>(x, j); });
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double ri = b[2 * i + k] - ax.v[k];
                acc[k] += ri * ri;
            }
        }
    }
    dev::block_partials<2>(acc, partials, vg_.b);
}
template <class OP>
struct TrueRes2K {
    int64_t n;
    OP op;
    const double *b, *x;
    double *partials;
    __device__ void run(VG vg) const { true_res2_body<OP>(vg, n, op, b, x, partials); }
};

// Interleave two vectors / split them again.
__device__ __forceinline__ void interleave_body(VG vg_, int64_t n, const double *__restrict__ a,
                                                const double *__restrict__ b, double *__restrict__ ab) {
    GRID_LOOP(i, n) {
        ab[2 * i] = a[i];
        ab[2 * i + 1] = b[i];
    }
}
struct InterleaveK {
    int64_t n;
    const double *a, *b;
    double *ab;
    __device__ void run(VG vg) const { interleave_body(vg, n, a, b, ab); }
};

__device__ __forceinline__ void split_body(VG vg_, int64_t n, const double *__restrict__ ab, double *__restrict__ a,
                                           double *__restrict__ b) {
    GRID_LOOP(i, n) {
        a[i] = ab[2 * i];
        b[i] = ab[2 * i + 1];
    }
}
struct SplitK {
    int64_t n;
    const double *ab;
    double *a, *b;
    __device__ void run(VG vg) const { split_body(vg, n, ab, a, b); }
};

// ------------------------------------------------------- shared launch ---
// One launch for several independent systems: record j holds system j's
// arguments, the first block it takes in the launch (blk0, ascending) and
// its own grid size nb; each block runs its system's body on the grid that
// system would have had alone (so its rows, block partials and sums are the
// same bit for bit), and a system whose flag says done returns at once, as
// it would alone.
template <class A>
struct Seg {
    A a;
    uint32_t blk0, nb;
};

// `sid` maps each block of the launch to its record (one load, then the
// record's fields).
template <class A>
__global__ void __launch_bounds__(kBlock) k_seg(const Seg<A> *__restrict__ t, const uint16_t *__restrict__ sid) {
    const Seg<A> &sg = t[sid[blockIdx.x]];
    sg.a.run(VG{(int64_t)blockIdx.x - (int64_t)sg.blk0, (int64_t)sg.nb});
}

// -------------------------------------------------------- host helpers ---
// Bytes one pass over an operator touches: values and column information
// (int32 columns + row pointers for CSR; one-byte offsets or int32 columns,
// padding included, + slice offsets for sliced ELL).
inline double csr_bytes(int64_t n, int64_t nnz, int vbytes) { return (double)nnz * (vbytes + 4) + 4.0 * (n + 1); }
// Bytes of one pass over a level's operator in the format the solve
// kernels read: the stencil copy's K+1 arrays (the mirror rows' reads hit
// the same arrays), the sliced copy, or the CSR arrays.
inline double op_bytes(const Level &L, int vbytes) {
    if (L.St.built()) return (double)(L.St.K + 1) * L.St.n * vbytes;
    const Sell &S = L.As;
    if (S.built()) return (double)S.nnz_padded * (vbytes + (S.ndict ? 1 : 4)) + 4.0 * (S.nslices + 1);
    return csr_bytes(L.A.n, L.A.nnz, vbytes);
}

inline unsigned grid_rows(int64_t n, int G) { return blocks_for(n * G); }

// Timing class of a V-cycle kernel on level l (ids of level 0, 1 and >= 2
// are five apart).
inline int level_kid(int id0, int l) { return id0 + 5 * (l < 2 ? l : 2); }

// Whether the restriction into level l+1 also writes that level's first
// sweep: it is smoothed (not the coarsest level, not ILU(0)) from x = 0 with
// at least one pre-sweep.
inline bool restrict_writes_x1(const amg_hierarchy *H, int l) {
    return H->prm.npre >= 1 && l + 1 < H->nlev - 1 && !H->L[l + 1].ilu;
}

template <class V>
struct LevelOps;
template <>
struct LevelOps<double> {
    static const double *stval(const Level &L) { return L.St.c.p; }
    static const double *aval(const Level &L) { return L.A.val.p; }
    static const double *asval(const Level &L) { return L.As.val.p; }
    static const double *pval(const Level &L) { return L.P.val.p; }
    static const double *rval(const Level &L) { return L.R.val.p; }
    static const double *mval(const Level &L) { return L.M.p; }
};
template <>
struct LevelOps<float> {
    static const float *stval(const Level &L) { return L.St.c32.p; }
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

template <class V>
OpSten<V> sten_op(const Stencil &S, const V *c) {
    OpSten<V> o{S.n, S.K, {}, S.onesided, c};
    for (int k = 0; k < kStenMax; ++k) o.d[k] = S.d[k];
    return o;
}

// Call f(op) with the level's operator: the stencil copy, else the sliced
// ELL copy, when built.
template <class V, class F>
void with_level_op(const Level &Lv, F &&f) {
    if (Lv.St.built() && LevelOps<V>::stval(Lv)) f(sten_op<V>(Lv.St, LevelOps<V>::stval(Lv)));
    else if (Lv.As.built() && LevelOps<V>::asval(Lv)) f(OpSell<V>{view(Lv.As), LevelOps<V>::asval(Lv)});
    else with_csr<V>(Lv.A, LevelOps<V>::aval(Lv), f);
}


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


}  // namespace
}  // namespace gw
