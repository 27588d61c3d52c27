// Sliced ELL layout of the level-0 operator for the solve phase.
//
// One slice = C consecutive rows (C = 64, one wave, or 32, 16, 8); inside a
// slice the k-th entries of all C rows are stored next to each other, so the
// lanes of a slice load values or column indices from one contiguous run.  A
// row keeps its CSR entry order; rows shorter than the slice width are padded
// with a zero value at the row's own column.  C is the largest height whose
// padded entry count is within 2 % of the count at C = 8: stencil operators
// (rows of equal length) keep whole-wave slices, the upwind travel-time
// operator (rows of 1 to 7 entries) takes short ones.  Stencil operators
// have a handful of distinct offsets col - row: those columns are stored as
// one-byte indices into a sorted offset dictionary (9 B per entry in FP64, 5
// B in FP32, instead of 12 / 8 with int32 columns).
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

constexpr int kOffsetTable = 4096;  // open-addressing set of offsets (device)
constexpr int kBlockTable = 512;    // per-block set in LDS
constexpr int32_t kEmpty = INT32_MIN;

// Padded entry totals at slice heights 8, 16, 32 and 64 (totals[0..3]): a
// slice is as wide as its longest row.  Grid-stride over whole waves, so the
// group maxima below always see full waves; the grid is capped, and each
// block adds its four sums with one integer atomic each.
__global__ void __launch_bounds__(kBlock) k_sell_pad(const int32_t *__restrict__ rowptr, int32_t n,
                                                      unsigned long long *__restrict__ totals) {
    __shared__ unsigned long long sm[kBlock / dev::kWave];
    const int lane = threadIdx.x & (dev::kWave - 1);
    unsigned long long t[4] = {0, 0, 0, 0};
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row - lane < n;
         row += (int64_t)gridDim.x * blockDim.x) {
        int32_t m = row < n ? rowptr[row + 1] - rowptr[row] : 0;
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) m = max(m, __shfl_xor(m, o, dev::kWave));
        if ((lane & 7) == 0) t[0] += (unsigned long long)m * 8;
#pragma unroll
        for (int c = 1; c < 4; ++c) {
            m = max(m, __shfl_xor(m, 4 << c, dev::kWave));
            if ((lane & ((8 << c) - 1)) == 0) t[c] += (unsigned long long)m * (8u << c);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const unsigned long long b = dev::block_sum(t[c], sm);
        if (threadIdx.x == 0 && b) atomicAdd(&totals[c], b);
    }
}

// Slice widths (entries per slice, at slice s + 1) at slice height 1 << cshift.
__global__ void k_sell_width(const int32_t *__restrict__ rowptr, int32_t n, int cshift, int32_t *__restrict__ width) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int C = 1 << cshift;
    int32_t len = row < n ? rowptr[row + 1] - rowptr[row] : 0;
    for (int o = 1; o < C; o <<= 1) len = max(len, __shfl_xor(len, o, dev::kWave));
    if ((threadIdx.x & (C - 1)) == 0 && row < n) width[(row >> cshift) + 1] = len << cshift;
}

__device__ __forceinline__ uint32_t offset_hash(int32_t d) { return ((uint32_t)d * 2654435761u) >> 16; }

// Insert d into an open-addressing set of `size` slots (power of two); the
// slot is read before any atomic so repeated offsets cost no contention.
template <int SCOPE>
__device__ __forceinline__ bool set_insert(int32_t *table, int size, int32_t d) {
    uint32_t h = offset_hash(d) & (size - 1);
    for (int probe = 0; probe < 64; ++probe) {
        int32_t cur = __hip_atomic_load(&table[h], __ATOMIC_RELAXED, SCOPE);
        if (cur == d) return true;
        if (cur == kEmpty) {
            int32_t old = atomicCAS(&table[h], kEmpty, d);
            if (old == kEmpty || old == d) return true;
        }
        h = (h + 1) & (size - 1);
    }
    return false;
}

// Distinct offsets col - row: each block collects its own in LDS, then adds
// that short list to the device-wide set.
__global__ void __launch_bounds__(kBlock) k_offset_set(const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col, int32_t n, int32_t *table,
                                                       int32_t *overflow) {
    __shared__ int32_t lt[kBlockTable];
    __shared__ int32_t lovf;
    for (int t = threadIdx.x; t < kBlockTable; t += blockDim.x) lt[t] = kEmpty;
    if (threadIdx.x == 0) lovf = 0;
    __syncthreads();
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row < n) {
        int32_t last = kEmpty;
        const int32_t e = rowptr[row + 1];
        for (int32_t p = rowptr[row]; p < e; ++p) {
            const int32_t d = col[p] - (int32_t)row;
            if (d == last) continue;
            last = d;
            if (!set_insert<__HIP_MEMORY_SCOPE_WORKGROUP>(lt, kBlockTable, d)) lovf = 1;
        }
    }
    __syncthreads();
    if (lovf) {
        if (threadIdx.x == 0) atomicOr(overflow, 1);
        return;
    }
    for (int t = threadIdx.x; t < kBlockTable; t += blockDim.x) {
        const int32_t d = lt[t];
        if (d != kEmpty && !set_insert<__HIP_MEMORY_SCOPE_AGENT>(table, kOffsetTable, d)) atomicOr(overflow, 1);
    }
}

// One block: the set's entries in ascending order into meta[kMetaDict + k]
// and their count into meta[1] (meta[0] is the overflow flag; a count above
// kSellMaxDict is reported as such and nothing is written).  The four padded
// entry totals are copied next to them so one small read returns everything.
constexpr int kMetaDict = 10;
__global__ void __launch_bounds__(1024) k_offset_compact(const int32_t *__restrict__ table, int32_t *meta,
                                                         const unsigned long long *__restrict__ totals) {
    __shared__ int32_t keys[kOffsetTable];
    __shared__ int32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < kOffsetTable; t += blockDim.x) {
        const int32_t d = table[t];
        if (d != kEmpty) keys[atomicAdd(&cnt, 1)] = d;
    }
    __syncthreads();
    const int m = cnt;
    if (threadIdx.x == 0) meta[1] = m;
    if (threadIdx.x < 4) reinterpret_cast<unsigned long long *>(meta)[1 + threadIdx.x] = totals[threadIdx.x];
    if (m > kSellMaxDict) return;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int32_t d = keys[t];
        int rank = 0;
        for (int u = 0; u < m; ++u) rank += keys[u] < d;
        meta[kMetaDict + rank] = d;
    }
}

__device__ __forceinline__ int32_t dict_index(const int32_t *dict, int32_t ndict, int32_t d) {
    int32_t lo = 0, hi = ndict - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (dict[mid] < d) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Thread per row: write the row's entries column-major into its slice.
__global__ void k_sell_fill(CsrView A, int cshift, const int32_t *__restrict__ soff, const int32_t *__restrict__ dict,
                            int32_t ndict, uint8_t *__restrict__ idx, int32_t *__restrict__ cols,
                            double *__restrict__ val, float *__restrict__ val32) {
    __shared__ int32_t sdict[kSellMaxDict + 1];
    for (int t = threadIdx.x; t < ndict; t += blockDim.x) sdict[t] = dict[t];
    __syncthreads();
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= A.n) return;
    const int64_t s = row >> cshift;
    const int l = (int)(row & ((1 << cshift) - 1));
    const int32_t off = soff[s], w = (soff[s + 1] - off) >> cshift;
    const int32_t b = A.rowptr[row], len = A.rowptr[row + 1] - b;
    const int32_t self = ndict ? dict_index(sdict, ndict, 0) : 0;
    for (int32_t k = 0; k < w; ++k) {
        const int64_t e = off + ((int64_t)k << cshift) + l;
        double v = 0.0;
        int32_t c = (int32_t)row;
        if (k < len) {
            v = A.val[b + k];
            c = A.col[b + k];
        }
        if (ndict) idx[e] = (uint8_t)(k < len ? dict_index(sdict, ndict, c - (int32_t)row) : self);
        else cols[e] = c;
        val[e] = v;
        if (val32) val32[e] = (float)v;
    }
}

// ---------------------------------------------------- stencil copy ------
struct StenArgs {
    int32_t K;
    int32_t d[kStenMax];  // positive offsets, ascending
};

// Thread per row: the diagonal and the entries right of it, by offset, into
// the stencil arrays (0 where the row has no such entry).
__global__ void k_sten_fill(CsrView A, StenArgs sa, double *__restrict__ c, float *__restrict__ c32) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= A.n) return;
    const int32_t i = (int32_t)row;
    double v[kStenMax + 1];
#pragma unroll
    for (int k = 0; k <= kStenMax; ++k) v[k] = 0.0;
    const int32_t e = A.rowptr[i + 1];
    for (int32_t p = A.rowptr[i]; p < e; ++p) {
        const int32_t dd = A.col[p] - i;
        const double a = A.val[p];
        if (dd == 0) v[0] = a;
#pragma unroll
        for (int k = 0; k < kStenMax; ++k)
            if (k < sa.K && dd == sa.d[k]) v[1 + k] = a;
    }
    const int64_t n = A.n;
#pragma unroll
    for (int k = 0; k <= kStenMax; ++k) {
        if (k > sa.K) break;
        c[k * n + i] = v[k];
        if (c32) c32[k * n + i] = (float)v[k];
    }
}

// Thread per row j: each entry left of the diagonal, a_{j,j-d_k} (0 where
// absent), against the mirror row's stored c_k[j-d_k], bit for bit; any
// difference sets *bad (one atomic per block).
__global__ void __launch_bounds__(kBlock) k_sten_check(CsrView A, StenArgs sa, const double *__restrict__ c,
                                                       int32_t *bad) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool mis = false;
    if (row < A.n) {
        const int32_t j = (int32_t)row;
        unsigned long long neg[kStenMax];
#pragma unroll
        for (int k = 0; k < kStenMax; ++k) neg[k] = 0ull;
        const int32_t e = A.rowptr[j + 1];
        for (int32_t p = A.rowptr[j]; p < e; ++p) {
            const int32_t dd = A.col[p] - j;
            if (dd >= 0) continue;
            const unsigned long long bits = (unsigned long long)__double_as_longlong(A.val[p]);
#pragma unroll
            for (int k = 0; k < kStenMax; ++k)
                if (k < sa.K && -dd == sa.d[k]) neg[k] = bits;
        }
        const int64_t n = A.n;
#pragma unroll
        for (int k = 0; k < kStenMax; ++k) {
            if (k >= sa.K) break;
            const int32_t m = j - sa.d[k];
            const unsigned long long got =
                m >= 0 ? (unsigned long long)__double_as_longlong(c[(1 + k) * n + m]) : 0ull;
            mis = mis || got != neg[k];
        }
    }
    if (__syncthreads_or(mis) && threadIdx.x == 0) atomicOr(bad, 1);
}

// One-sided (upwind) form, thread per row i: the diagonal, and for each d_k
// the face between rows i and i+d_k from row i's entry at +d_k (stored as
// is) or row i+d_k's entry at -d_k (stored negated).  Sets *bad when an
// off-diagonal entry of row i is not strictly negative or a face is stored
// by both rows.
__global__ void k_sten_onesided(CsrView A, StenArgs sa, double *__restrict__ c, float *__restrict__ c32,
                                int32_t *bad) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool mis = false;
    if (row < A.n) {
        const int32_t i = (int32_t)row;
        const int64_t n = A.n;
        double v0 = 0.0, right[kStenMax];
        bool has[kStenMax];
#pragma unroll
        for (int k = 0; k < kStenMax; ++k) {
            right[k] = 0.0;
            has[k] = false;
        }
        const int32_t e = A.rowptr[i + 1];
        for (int32_t p = A.rowptr[i]; p < e; ++p) {
            const int32_t dd = A.col[p] - i;
            const double a = A.val[p];
            if (dd == 0) {
                v0 = a;
                continue;
            }
            mis = mis || !(a < 0.0);
#pragma unroll
            for (int k = 0; k < kStenMax; ++k)
                if (k < sa.K && dd == sa.d[k]) {
                    right[k] = a;
                    has[k] = true;
                }
        }
        c[i] = v0;
        if (c32) c32[i] = (float)v0;
#pragma unroll
        for (int k = 0; k < kStenMax; ++k) {
            if (k >= sa.K) break;
            double f = has[k] ? right[k] : 0.0;
            const int32_t j = i + sa.d[k];
            if (j < A.n) {
                const int32_t ej = A.rowptr[j + 1];
                for (int32_t p = A.rowptr[j]; p < ej; ++p) {
                    if (A.col[p] != i) continue;
                    mis = mis || has[k];
                    f = -A.val[p];
                }
            }
            c[(1 + k) * n + i] = f;
            if (c32) c32[(1 + k) * n + i] = (float)f;
        }
    }
    if (__syncthreads_or(mis) && threadIdx.x == 0) atomicOr(bad, 1);
}

// Whether the offsets (ascending, `count` of them) are a symmetric set
// around 0 with at most kStenMax positive ones; their positive half into sa.
bool stencil_shape(const int32_t *offsets, int32_t count, StenArgs &sa) {
    if (count < 3 || count > 2 * kStenMax + 1 || (count & 1) == 0) return false;
    const int K = count / 2;
    if (offsets[K] != 0) return false;
    sa = StenArgs{};
    sa.K = K;
    for (int k = 0; k < K; ++k) {
        sa.d[k] = offsets[K + 1 + k];
        if (sa.d[k] <= 0 || offsets[K - 1 - k] != -sa.d[k]) return false;
    }
    return true;
}

// The stencil copy of A with the offsets sa when its values are symmetric
// bit for bit; false (nothing kept) otherwise.  check = false: the values
// are known to be symmetric (the setup's pattern probe compared every
// mirror pair), so the copy is filled without the check and its read.
bool build_stencil(Level &Lv, const StenArgs &sa, bool onesided, bool fp32, bool check, hipStream_t s,
                   double *bytes) {
    const int K = sa.K;
    const CsrView A = view(Lv.A);
    Stencil St;
    St.n = A.n;
    St.c.alloc((size_t)(K + 1) * A.n);
    if (fp32) St.c32.alloc((size_t)(K + 1) * A.n);
    if (onesided) {
        // the fill checks as it goes: the CSR read for row i and its K
        // neighbours' rows, the copy written
        DBuf<int32_t> bad(1);
        fill_i32(bad.p, 0, 1, s);
        hipLaunchKernelGGL(k_sten_onesided, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, sa, St.c.p, St.c32.p,
                           bad.p);
        GW_HIP(hipGetLastError());
        int32_t *stage = static_cast<int32_t *>(host_stage());
        GW_HIP(hipMemcpyAsync(stage, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        *bytes += 4.0 * (A.n + 1) + 12.0 * (double)A.nnz + (double)(K + 1) * A.n * (8 + (fp32 ? 4 : 0));
        if (stage[0] != 0) return false;
        St.K = K;
        St.onesided = 1;
        for (int k = 0; k < kStenMax; ++k) St.d[k] = sa.d[k];
        Lv.St = std::move(St);
        return true;
    }
    hipLaunchKernelGGL(k_sten_fill, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, sa, St.c.p, St.c32.p);
    // the fill reads the CSR arrays and writes the copy
    *bytes += 4.0 * (A.n + 1) + 12.0 * (double)A.nnz + (double)(K + 1) * A.n * (8 + (fp32 ? 4 : 0));
    if (check) {
        DBuf<int32_t> bad(1);
        fill_i32(bad.p, 0, 1, s);
        hipLaunchKernelGGL(k_sten_check, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, sa, St.c.p, bad.p);
        GW_HIP(hipGetLastError());
        int32_t *stage = static_cast<int32_t *>(host_stage());
        GW_HIP(hipMemcpyAsync(stage, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        // the check reads the CSR arrays again and K of the copy's arrays
        *bytes += 4.0 * (A.n + 1) + 12.0 * (double)A.nnz + 8.0 * K * A.n;
        if (stage[0] != 0) return false;
    }
    GW_HIP(hipGetLastError());
    St.K = K;
    for (int k = 0; k < kStenMax; ++k) St.d[k] = sa.d[k];
    Lv.St = std::move(St);
    return true;
}

}  // namespace

void build_sell(amg_hierarchy *H, int l, bool fp32, hipStream_t s) {
    Level &Lv = H->L[l];
    const CsrView A = view(Lv.A);
    Sell &S = Lv.As;
    S = Sell();
    // meta: [0] overflow, [1] count, [2..9] padded totals at C = 8..64
    // (int64), [kMetaDict..] offsets
    constexpr int kMeta = kMetaDict + kSellMaxDict;
    static_assert(kMeta * sizeof(int32_t) <= kHostStageBytes, "offset dictionary must fit the pinned stage");
    ProfScope ps(K_SELL_BUILD, 0.0, s);
    DBuf<unsigned long long> totals(4);
    DBuf<int32_t> table(kOffsetTable);
    DBuf<int32_t> meta(kMeta);
    // a stencil copy first (level 0; GWAMG_STENCIL=0 keeps the sliced copy):
    // the offsets are read first, and the sliced copy's slice-height totals
    // are formed only when the stencil is not taken.
    Lv.St = Stencil();
    const char *sten_env = std::getenv("GWAMG_STENCIL");
    const bool sten_on = l == 0 && !(sten_env && std::atoi(sten_env) == 0);
    // symmetric form unless the pattern or the values are known not to be
    // symmetric; the one-sided form for a pattern known not to be
    const bool onesided = H->sym_pattern == 0;
    const bool sten_try = sten_on && (onesided || H->sym_values != 0);
    const bool sten_known = sten_try && !onesided && H->sym_values == 1;
    fill_i32(reinterpret_cast<int32_t *>(totals.p), 0, 8, s);
    fill_i32(table.p, kEmpty, kOffsetTable, s);
    fill_i32(meta.p, 0, kMeta, s);
    auto launch_pad = [&] {
        hipLaunchKernelGGL(k_sell_pad, dim3(std::min<unsigned>(blocks_for(A.n), 1024)), dim3(kBlock), 0, s,
                           A.rowptr, A.n, totals.p);
    };
    int32_t *stage = static_cast<int32_t *>(host_stage());
    auto read_meta = [&] {
        hipLaunchKernelGGL(k_offset_compact, dim3(1), dim3(1024), 0, s, table.p, meta.p, totals.p);
        GW_HIP(hipGetLastError());
        GW_HIP(hipMemcpyAsync(stage, meta.p, sizeof(int32_t) * kMeta, hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
    };
    // with a stencil to try, the slice-height totals wait until it is refused
    if (!sten_try) launch_pad();
    hipLaunchKernelGGL(k_offset_set, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A.rowptr, A.col, A.n, table.p,
                       meta.p);
    read_meta();
    double sb = 4.0 * (A.n + 1) * (sten_try ? 1 : 2) + 4.0 * (double)A.nnz;  // offset set (and padded totals)
    if (sten_try && stage[0] == 0 && stage[1] <= kSellMaxDict) {
        StenArgs sa;
        if (stencil_shape(stage + kMetaDict, stage[1], sa)) {
            if (build_stencil(Lv, sa, onesided, fp32, !sten_known, s, &sb)) {
                ps.bytes = sb;
                ps.cbytes = sb;
                return;
            }
        }
    }
    // the sliced copy: its slice-height totals (when not launched yet) and
    // the words read again with them (a check may have reused the stage)
    if (sten_try) {
        launch_pad();
        sb += 4.0 * (A.n + 1);
        read_meta();
    }
    const bool overflow = stage[0] != 0;
    const int32_t count = stage[1];
    int64_t pad[4];
    std::memcpy(pad, stage + 2, sizeof(pad));
    // the tallest slices whose padding stays within 2 % of the shortest's
    int cshift = 3;
    for (int c = 3; c >= 1; --c)
        if ((double)pad[c] <= 1.02 * (double)pad[0]) {
            cshift = 3 + c;
            break;
        }
    const int64_t padded = pad[cshift - 3];
    // Rows of very uneven length would pad the copy far beyond the CSR
    // operator: keep the CSR kernels then (also past int32 entry offsets).
    if (padded >= INT32_MAX || (double)padded > 1.5 * (double)A.nnz + kSellMaxC) return;
    bool use_dict = !overflow && count <= kSellMaxDict && count > 0;
    if (use_dict) use_dict = std::binary_search(stage + kMetaDict, stage + kMetaDict + count, 0);
    const int32_t nslices = (int32_t)(((int64_t)A.n + (1 << cshift) - 1) >> cshift);
    DBuf<int32_t> soff((size_t)nslices + 1);
    DBuf<int64_t> total(1);
    fill_i32(soff.p, 0, 1, s);
    hipLaunchKernelGGL(k_sell_width, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A.rowptr, A.n, cshift, soff.p);
    scan_inclusive_i32(soff.p + 1, nslices, total.p, s);
    S.n = A.n;
    S.nslices = nslices;
    S.cshift = cshift;
    S.nnz_padded = padded;
    S.soff = std::move(soff);
    const size_t np = (size_t)std::max<int64_t>(padded, 1);
    if (use_dict) {
        S.ndict = count;
        S.dict.alloc((size_t)count);
        copy_bytes(S.dict.p, meta.p + kMetaDict, sizeof(int32_t) * (size_t)count, s);
        S.idx.alloc(np);
    } else {
        S.ndict = 0;
        S.col.alloc(np);
    }
    S.val.alloc(np);
    if (fp32) S.val32.alloc(np);
    hipLaunchKernelGGL(k_sell_fill, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, cshift, S.soff.p, S.dict.p,
                       S.ndict, S.idx.p, S.col.p, S.val.p, S.val32.p);
    GW_HIP(hipGetLastError());
    // the padded totals and the widths (row pointers, twice), the offset set
    // (row pointers and columns), the fill (the CSR read, the copy written)
    ps.bytes = sb + 4.0 * (A.n + 1) * 2 + 12.0 * (double)A.nnz +
               (double)padded * (8 + (S.ndict ? 1 : 4) + (fp32 ? 4 : 0)) + 4.0 * (nslices + 1);
    ps.cbytes = ps.bytes;
}

}  // namespace gw
