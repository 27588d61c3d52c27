// Smoothed-aggregation AMG setup on the device (Introduction: the setup
// phase builds the grid hierarchy and the transfer operators by nodal
// aggregation; Results: smoothed aggregation is the coarsening used).
//
// Every level is built from deterministic steps, so the hierarchy is
// bit-reproducible:
//   strength graph  {i,j} strong <=> a_ij^2 > eps2 a_ii a_jj or a_ji^2 > eps2 a_ii a_jj
//   MIS-2           synchronous rounds on hash priorities (integer only)
//   aggregates      roots numbered by index, pass 1 (root neighbours), pass 2
//   prolongator     P = (I - w D_F^-1 A_F) P_tent, w = (4/3)/Gershgorin bound
//   Galerkin        A_c = R (A P) with R = P^T, every entry summed in a fixed
//                   order (AP: ascending k; R(AP): ascending fine row)
//   coarsest        dense LU with partial pivoting, then its inverse
// Built with -ffp-contract=off so that a*b+c is never fused.
#include <algorithm>
#include <type_traits>
#include <cmath>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

constexpr uint32_t ST_OUT = 0, ST_UND = 1, ST_ROOT = 2;

// MurmurHash3 32-bit finalizer (Appleby), host and device.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

uint32_t level_salt(uint64_t seed, int32_t level) {
    return fmix32((uint32_t)seed ^ fmix32((uint32_t)(seed >> 32) + 0x9E3779B9u * (uint32_t)(level + 1)));
}

// Priority key (state rank, hash, index), compared as one uint64; OUT nodes
// carry 0 (lowest), ROOT outranks UNDECIDED.  Needs i < 2^30.
__device__ __forceinline__ uint64_t mis_key(uint32_t st, uint32_t salt, int32_t i) {
    if (st == ST_OUT) return 0ull;
    return ((uint64_t)st << 62) | ((uint64_t)fmix32((uint32_t)i ^ salt) << 30) | (uint64_t)(uint32_t)i;
}

// ------------------------------------------------------------ validation --
// bad bit 1: structure (rowptr, column range/order); bit 2: missing or
// non-positive diagonal; bit 4: non-finite value.
__global__ void k_csr_check(CsrView A, double *__restrict__ diag, int32_t *bad, int strict) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0 && (A.rowptr[0] != 0 || (int64_t)A.rowptr[A.n] != A.nnz)) atomicOr(bad, 1);
    if (i >= A.n) return;
    int64_t b = A.rowptr[i], e = A.rowptr[i + 1];
    if (b < 0 || e < b || e > A.nnz) { atomicOr(bad, 1); diag[i] = 0.0; return; }
    double d = 0.0;
    bool found = false;
    int32_t prev = -1;
    for (int64_t p = b; p < e; ++p) {
        int32_t c = A.col[p];
        double v = A.val[p];
        if (strict) {
            if (c < 0 || c >= A.ncols || c <= prev) atomicOr(bad, 1);
            if (!isfinite(v)) atomicOr(bad, 4);
        }
        prev = c;
        if (c == (int32_t)i) { d = v; found = true; }
    }
    if (strict && (!found || !(d > 0.0))) atomicOr(bad, 2);
    diag[i] = d;
}

// -------------------------------------------------------------- transpose --
__global__ void k_tr_count(const int32_t *__restrict__ col, int64_t nnz, int32_t *__restrict__ cnt) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[p] + 1], 1);
}

// G lanes per row of A (long coarse-level rows would serialize one lane).
template <int G>
__global__ void k_tr_fill(CsrView A, const int32_t *__restrict__ trow, int32_t *__restrict__ fill,
                          int32_t *__restrict__ tcol, double *__restrict__ tval, int32_t *__restrict__ rowid) {
    const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = gtid / G;
    const int lane = (int)(gtid % G);
    if (i >= A.n) return;
    const int32_t e = A.rowptr[i + 1];
    for (int32_t p = A.rowptr[i] + lane; p < e; p += G) {
        int32_t j = A.col[p];
        int32_t pos = trow[j] + atomicAdd(&fill[j], 1);
        tcol[pos] = (int32_t)i;
        tval[pos] = A.val[p];
        rowid[pos] = j;
    }
}

// Entries of a transposed row arrive in arbitrary order; each entry's final
// slot is its rank among the (unique) columns of its row.
__global__ void k_tr_sort(const int32_t *__restrict__ trow, const int32_t *__restrict__ rowid,
                          const int32_t *__restrict__ tcol, const double *__restrict__ tval, int64_t nnz,
                          int32_t *__restrict__ ocol, double *__restrict__ oval) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int32_t j = rowid[e];
    int32_t key = tcol[e];
    int32_t b = trow[j], en = trow[j + 1];
    int32_t rank = 0;
    for (int32_t u = b; u < en; ++u) rank += tcol[u] < key;
    ocol[b + rank] = key;
    oval[b + rank] = tval[e];
}

// Transpose by a stable least-significant-digit radix sort of the entries on
// their column.  The entries enter in row order (row i ascending, columns
// ascending within a row), so after a stable sort on the column every row
// of A^T holds its entries in ascending row index: the one CSR of A^T, the
// same as the count / fill / rank path above, without same-address atomics.
// A pass handles tiles of kRxTile entries: a histogram of the pass's digit
// per tile, an exclusive scan of the counts in digit-major order (so the
// offset of (digit, tile) is where that tile's entries of that digit start),
// then a scatter in which each entry's place among the tile's entries of its
// digit is its rank in entry order (ballots over the lanes of the wave
// holding the same digit, then the counts of the earlier waves).
constexpr int kRxItems = 16;
constexpr int kRxTile = kBlock * kRxItems;
constexpr int kRxWaves = kBlock / dev::kWave;
// Digits of at most 9 bits: with more buckets a 4096-entry tile leaves runs
// of about 4 entries per bucket, whose partial-line writes cost more than a
// third pass (1M-column operator: 88 us a pass at 10 bits).
constexpr int kRxMaxBits = 9;

// Row of every entry of A (the row order that the sort keeps).
template <int G>
__global__ void k_rx_rowid(CsrView A, int32_t *__restrict__ rowid) {
    const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = gtid / G;
    const int lane = (int)(gtid % G);
    if (i >= A.n) return;
    const int32_t e = A.rowptr[i + 1];
    for (int32_t p = A.rowptr[i] + lane; p < e; p += G) rowid[p] = (int32_t)i;
}

// cnt[1 + d * ntiles + t] = entries of tile t whose digit is d.
__global__ void __launch_bounds__(kBlock) k_rx_hist(const int32_t *__restrict__ key, int64_t nnz, int shift,
                                                    int bits, int32_t *__restrict__ cnt, int64_t ntiles) {
    __shared__ int32_t h[1 << kRxMaxBits];
    const int nd = 1 << bits;
    for (int d = threadIdx.x; d < nd; d += kBlock) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRxTile;
    const uint32_t mask = (uint32_t)nd - 1u;
#pragma unroll
    for (int u = 0; u < kRxItems; ++u) {
        const int64_t e = base + (int64_t)u * kBlock + threadIdx.x;
        if (e < nnz) atomicAdd(&h[((uint32_t)key[e] >> shift) & mask], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += kBlock) cnt[1 + (int64_t)d * ntiles + blockIdx.x] = h[d];
}

// One stable pass.  Wave w of the tile takes entries [w*64*kRxItems, ...)
// of it, 64 consecutive ones at a time, so the entry order is (wave, step,
// lane).  off[d * ntiles + t] holds the scanned offsets (exclusive).  The
// tile is first laid out in LDS in its sorted order (slot = the tile's
// entries of smaller digits, then of the same digit earlier in entry order),
// and written from there by consecutive threads, so that the stores of a
// wave cover runs of consecutive addresses.
__global__ void __launch_bounds__(kBlock) k_rx_scatter(const int32_t *__restrict__ kin,
                                                       const int32_t *__restrict__ rin,
                                                       const double *__restrict__ vin, int64_t nnz, int shift,
                                                       int bits, const int32_t *__restrict__ off, int64_t ntiles,
                                                       int32_t *__restrict__ kout, int32_t *__restrict__ rout,
                                                       double *__restrict__ vout) {
    __shared__ int32_t c[kRxWaves][1 << kRxMaxBits];
    __shared__ int32_t gofs[1 << kRxMaxBits];
    __shared__ int32_t wsum[kRxWaves];
    __shared__ int64_t stage[kRxTile];  // (key, row) pairs, then values
    const int nd = 1 << bits;
    const uint32_t mask = (uint32_t)nd - 1u;
    for (int d = threadIdx.x; d < nd; d += kBlock)
#pragma unroll
        for (int w = 0; w < kRxWaves; ++w) c[w][d] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (dev::kWave - 1), w = threadIdx.x / dev::kWave;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t tile0 = (int64_t)blockIdx.x * kRxTile;
    const int64_t base = tile0 + (int64_t)w * dev::kWave * kRxItems;
    const int32_t tcount = (int32_t)min<int64_t>(kRxTile, nnz - tile0);
    int32_t kk[kRxItems], rr[kRxItems], pos[kRxItems];
    double vv[kRxItems];
#pragma unroll
    for (int u = 0; u < kRxItems; ++u) {
        const int64_t e = base + (int64_t)u * dev::kWave + lane;
        const bool in = e < nnz;
        const int64_t es = in ? e : 0;
        kk[u] = kin[es];
        rr[u] = rin[es];
        vv[u] = vin[es];
        if (!in) kk[u] = -1;
    }
#pragma unroll
    for (int u = 0; u < kRxItems; ++u) {
        const bool in = kk[u] >= 0;
        const uint32_t d = ((uint32_t)kk[u] >> shift) & mask;
        uint64_t peers = __ballot(in);
        for (int b = 0; b < bits; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        int32_t before = 0;
        if (in) before = c[w][d];
        const int rank = __popcll(peers & lt);
        // the lowest lane of each digit's peers advances that digit's count
        // (one writer per digit; every lane has read it above)
        if (in && rank == 0) c[w][d] = before + __popcll(peers);
        pos[u] = before + rank;
    }
    __syncthreads();
    // Digit starts within the tile: thread t owns digits [t*dpt, (t+1)*dpt)
    // (dpt = nd / kBlock, at least 1), sums them, and an exclusive scan over
    // the threads gives each digit's first slot; c[w][d] becomes that slot
    // plus the digit's entries in the earlier waves.
    const int dpt = nd >= kBlock ? nd / kBlock : 1;
    const int d0 = threadIdx.x * dpt;
    int32_t mine = 0;
    if (d0 < nd)
        for (int d = d0; d < d0 + dpt; ++d)
#pragma unroll
            for (int ww = 0; ww < kRxWaves; ++ww) mine += c[ww][d];
    const int32_t incl = dev::wave_scan_incl(mine);
    if (lane == dev::kWave - 1) wsum[w] = incl;
    __syncthreads();
    int32_t start = incl - mine;
    for (int ww = 0; ww < w; ++ww) start += wsum[ww];
    if (d0 < nd)
        for (int d = d0; d < d0 + dpt; ++d) {
            gofs[d] = off[(int64_t)d * ntiles + blockIdx.x] - start;
#pragma unroll
            for (int ww = 0; ww < kRxWaves; ++ww) {
                const int32_t t = c[ww][d];
                c[ww][d] = start;
                start += t;
            }
        }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRxItems; ++u) {
        if (kk[u] < 0) continue;
        const uint32_t d = ((uint32_t)kk[u] >> shift) & mask;
        pos[u] += c[w][d];
        stage[pos[u]] = (int64_t)(((uint64_t)(uint32_t)rr[u] << 32) | (uint32_t)kk[u]);
    }
    __syncthreads();
    int32_t dst[kRxItems];
#pragma unroll
    for (int u = 0; u < kRxItems; ++u) {
        const int32_t sl = u * kBlock + threadIdx.x;
        dst[u] = -1;
        if (sl < tcount) {
            const uint64_t kr = (uint64_t)stage[sl];
            const int32_t key = (int32_t)(uint32_t)kr;
            dst[u] = gofs[((uint32_t)key >> shift) & mask] + sl;
            kout[dst[u]] = key;
            rout[dst[u]] = (int32_t)(uint32_t)(kr >> 32);
        }
    }
    __syncthreads();
    double *sv = reinterpret_cast<double *>(stage);
#pragma unroll
    for (int u = 0; u < kRxItems; ++u)
        if (kk[u] >= 0) sv[pos[u]] = vv[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRxItems; ++u)
        if (dst[u] >= 0) vout[dst[u]] = sv[u * kBlock + threadIdx.x];
}

// Row pointers of A^T from the sorted columns: rowptr[J] = first position
// whose column is >= J (the columns of entries e-1 and e bound the J that
// entry e starts); the entry past the end closes the trailing rows.
__global__ void k_rx_rowptr(const int32_t *__restrict__ key, int64_t nnz, int32_t ncols, int32_t *__restrict__ rp) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e > nnz) return;
    const int32_t prev = e > 0 ? key[e - 1] : -1;
    const int32_t cur = e < nnz ? key[e] : ncols;
    for (int32_t J = prev + 1; J <= cur; ++J) rp[J] = (int32_t)e;
}

// A^T on the pattern of A, when that pattern is symmetric: entry (i, j) of
// A^T is a_ji, found by binary search in row j of A; no counting, atomic
// fill or sort.  `miss` is set when some (j, i) is absent (the pattern is not
// symmetric and the result is discarded); one atomic per block at most, on a
// capped grid.
// a_ji into tval at the position of a_ij; *miss bit 0: an entry without its
// mirror (pattern not symmetric), bit 1: a mirror whose value differs bit for
// bit (values not symmetric).
template <int G>
__global__ void __launch_bounds__(kBlock) k_sym_transpose(CsrView A, double *__restrict__ tval, int32_t *miss) {
    int32_t bad = 0, vbad = 0;
    const int lane = (int)(threadIdx.x % G);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G; row < A.n;
         row += (int64_t)gridDim.x * blockDim.x / G) {
        const int32_t i = (int32_t)row, e = A.rowptr[i + 1];
        for (int32_t p = A.rowptr[i] + lane; p < e; p += G) {
            const int32_t j = A.col[p];
            const int32_t b = A.rowptr[j], len = A.rowptr[j + 1] - b;
            int32_t lo = 0, hi = len;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (A.col[b + mid] < i) lo = mid + 1;
                else hi = mid;
            }
            if (lo < len && A.col[b + lo] == i) {
                const double aji = A.val[b + lo];
                tval[p] = aji;
                vbad |= __double_as_longlong(aji) != __double_as_longlong(A.val[p]);
            } else {
                bad = 1;
            }
        }
    }
    const int32_t w = (__syncthreads_or(bad) ? 1 : 0) | (__syncthreads_or(vbad) ? 2 : 0);
    if (w && threadIdx.x == 0) atomicOr(miss, w);
}

// --------------------------------------------------------------- strength --
// Walk the union of row i of A and row i of A^T (both sorted).
template <class F>
__device__ __forceinline__ void union_row(const CsrView &A, const CsrView &T, int32_t i, F &&f) {
    int32_t pa = A.rowptr[i], ea = A.rowptr[i + 1];
    int32_t pt = T.rowptr[i], et = T.rowptr[i + 1];
    while (pa < ea || pt < et) {
        int32_t ja = pa < ea ? A.col[pa] : INT32_MAX;
        int32_t jt = pt < et ? T.col[pt] : INT32_MAX;
        int32_t j = ja < jt ? ja : jt;
        double aij = 0.0, aji = 0.0;
        int32_t posa = -1;
        if (ja == j) { aij = A.val[pa]; posa = pa; ++pa; }
        if (jt == j) { aji = T.val[pt]; ++pt; }
        f(j, aij, aji, posa);
    }
}

__device__ __forceinline__ bool strong_pair(double aij, double aji, double di, double dj, double eps2) {
    double dd = di * dj;
    return (aij * aij > eps2 * dd) || (aji * aji > eps2 * dd);
}

__device__ __forceinline__ int32_t strength_count_row(const CsrView &A, const CsrView &T,
                                                      const double *__restrict__ diag, double eps2, int32_t i) {
    const double di = diag[i];
    int32_t c = 0;
    union_row(A, T, i, [&](int32_t j, double aij, double aji, int32_t) {
        if (j != i && strong_pair(aij, aji, di, diag[j], eps2)) ++c;
    });
    return c;
}

__device__ __forceinline__ void strength_fill_row(const CsrView &A, const CsrView &T, const double *__restrict__ diag,
                                                  double eps2, int32_t i, const int32_t *__restrict__ srow,
                                                  int32_t *__restrict__ scol, double *__restrict__ sw,
                                                  uint8_t *__restrict__ strongA, double *__restrict__ dF) {
    const double di = diag[i];
    int32_t q = srow[i];
    double lump = di;  // a_ii + weak off-diagonals in ascending column order
    union_row(A, T, i, [&](int32_t j, double aij, double aji, int32_t posa) {
        if (j == i) {
            if (posa >= 0) strongA[posa] = 0;
            return;
        }
        bool s = strong_pair(aij, aji, di, diag[j], eps2);
        if (posa >= 0) {
            strongA[posa] = s ? 1 : 0;
            if (!s) lump = lump + aij;
        }
        if (s) {
            scol[q] = j;
            double x = fabs(aij), y = fabs(aji);
            sw[q] = x > y ? x : y;
            ++q;
        }
    });
    dF[i] = lump;
}

__global__ void k_strength_count(CsrView A, CsrView T, const double *__restrict__ diag, double eps2,
                                 int32_t *__restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    cnt[i + 1] = strength_count_row(A, T, diag, eps2, (int32_t)i);
}

__global__ void k_strength_fill(CsrView A, CsrView T, const double *__restrict__ diag, double eps2,
                                const int32_t *__restrict__ srow, int32_t *__restrict__ scol,
                                double *__restrict__ sw, uint8_t *__restrict__ strongA,
                                double *__restrict__ dF) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    strength_fill_row(A, T, diag, eps2, (int32_t)i, srow, scol, sw, strongA, dF);
}

// Number of entries of the sorted a[0..n) below key.
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t *__restrict__ a, int32_t n, int32_t key) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int G>
__device__ __forceinline__ int32_t grp_scan_incl(int32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int32_t w = __shfl_up(v, o, G);
        if (lane >= o) v += w;
    }
    return v;
}

// The same strength graph with G lanes per row, for rows of a few dozen
// entries (coarse levels), where walking the union one entry at a time is a
// long chain of dependent loads.  The union of row i of A and of A^T is not
// formed: the lanes take A's entries (a_ji found by binary search in row i
// of A^T), then the entries of A^T's row whose column A's row lacks (a_ij =
// 0).  A strong entry's place in the column-ordered union is its count of
// strong predecessors in its own list plus the strong entries of the other
// list with a smaller column (exclusive prefix counts kept in LDS).  The
// counting pass stores each entry's outcome in code[] (A's entries at their
// positions in A, then A^T's at nnz(A) + theirs): the lower-bound index in
// the other row when the entry is strong, -1 when not; the filling pass
// places entries from these codes without searching or gathering again.
// The lumped diagonal is summed in column order, one lane's value after the
// other.  Rows longer than the LDS lists take the one-lane walk in both
// passes.
template <int G, bool FILL>
__global__ void __launch_bounds__(kBlock) k_strength_grp(CsrView A, CsrView T, const double *__restrict__ diag,
                                                         double eps2, int32_t *__restrict__ cnt,
                                                         const int32_t *__restrict__ srow, int32_t *__restrict__ scol,
                                                         double *__restrict__ sw, uint8_t *__restrict__ strongA,
                                                         double *__restrict__ dF, int32_t *__restrict__ code) {
    constexpr int CAP = 16 * G;
    __shared__ int32_t pref[FILL ? (kBlock / G) * 2 * (CAP + 1) : 1];
    const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t row = gtid / G;
    const int lane = (int)(threadIdx.x % G);
    if (row >= A.n) return;
    const int32_t i = (int32_t)row;
    const int32_t pa = A.rowptr[i], la = A.rowptr[i + 1] - pa;
    const int32_t pt = T.rowptr[i], lt = T.rowptr[i + 1] - pt;
    if (la > CAP || lt > CAP) {
        if (lane == 0) {
            if (FILL) strength_fill_row(A, T, diag, eps2, i, srow, scol, sw, strongA, dF);
            else cnt[i + 1] = strength_count_row(A, T, diag, eps2, i);
        }
        return;
    }
    int32_t *codeA = code + pa, *codeT = code + A.nnz + pt;
    if (!FILL) {
        const double di = diag[i];
        int32_t run = 0;
        for (int32_t c0 = 0; c0 < la; c0 += G) {
            const int32_t a = c0 + lane;
            bool st = false;
            if (a < la) {
                const int32_t j = A.col[pa + a];
                const double aij = A.val[pa + a];
                const int32_t idx = lower_bound_i32(T.col + pt, lt, j);
                const double aji = (idx < lt && T.col[pt + idx] == j) ? T.val[pt + idx] : 0.0;
                st = j != i && strong_pair(aij, aji, di, diag[j], eps2);
                codeA[a] = st ? idx : -1;
            }
            run += __shfl(grp_scan_incl<G>(st ? 1 : 0, lane), G - 1, G);
        }
        for (int32_t c0 = 0; c0 < lt; c0 += G) {
            const int32_t u = c0 + lane;
            bool st = false;
            if (u < lt) {
                const int32_t j = T.col[pt + u];
                const double aji = T.val[pt + u];
                const int32_t idx = lower_bound_i32(A.col + pa, la, j);
                const bool only = !(idx < la && A.col[pa + idx] == j);
                st = only && j != i && strong_pair(0.0, aji, di, diag[j], eps2);
                codeT[u] = st ? idx : -1;
            }
            run += __shfl(grp_scan_incl<G>(st ? 1 : 0, lane), G - 1, G);
        }
        if (lane == 0) cnt[i + 1] = run;
        return;
    }
    int32_t *PA = pref + (threadIdx.x / G) * 2 * (CAP + 1);
    int32_t *PT = PA + (CAP + 1);
    int32_t runA = 0, runT = 0;
    double lump = diag[i];
    for (int32_t c0 = 0; c0 < la; c0 += G) {
        const int32_t a = c0 + lane;
        const bool in = a < la;
        const int32_t j = in ? A.col[pa + a] : i;
        const double aij = in ? A.val[pa + a] : 0.0;
        const bool st = in && codeA[a] >= 0;
        const int32_t sc = st ? 1 : 0;
        const int32_t incl = grp_scan_incl<G>(sc, lane);
        if (in) {
            strongA[pa + a] = st ? 1 : 0;
            PA[a] = runA + incl - sc;
        }
        const double weak = (in && j != i && !st) ? aij : 0.0;
        for (int t = 0; t < G; ++t) {
            const double w = __shfl(weak, t, G);
            if (c0 + t < la && w != 0.0) lump = lump + w;
        }
        runA += __shfl(incl, G - 1, G);
    }
    for (int32_t c0 = 0; c0 < lt; c0 += G) {
        const int32_t u = c0 + lane;
        const bool in = u < lt;
        const int32_t sc = (in && codeT[u] >= 0) ? 1 : 0;
        const int32_t incl = grp_scan_incl<G>(sc, lane);
        if (in) PT[u] = runT + incl - sc;
        runT += __shfl(incl, G - 1, G);
    }
    if (lane == 0) {
        PA[la] = runA;
        PT[lt] = runT;
    }
    __builtin_amdgcn_wave_barrier();
    const int32_t q0 = srow[i];
    for (int32_t a = lane; a < la; a += G) {
        const int32_t idx = codeA[a];
        if (idx < 0) continue;
        const int32_t j = A.col[pa + a];
        const double aji = (idx < lt && T.col[pt + idx] == j) ? T.val[pt + idx] : 0.0;
        const int32_t pos = PA[a] + PT[idx];
        scol[q0 + pos] = j;
        const double x = fabs(A.val[pa + a]), y = fabs(aji);
        sw[q0 + pos] = x > y ? x : y;
    }
    for (int32_t u = lane; u < lt; u += G) {
        const int32_t idx = codeT[u];
        if (idx < 0) continue;
        const int32_t pos = PT[u] + PA[idx];
        scol[q0 + pos] = T.col[pt + u];
        const double y = fabs(T.val[pt + u]);
        sw[q0 + pos] = 0.0 > y ? 0.0 : y;
    }
    if (lane == 0) dF[i] = lump;
}

// The strength graph when A's pattern is symmetric and tval holds A^T on it
// (a_ji at the position of a_ij): the union of the two rows is A's row, so
// each entry is classified where it stands.  Same results as the walk over
// the union.
template <int G, bool FILL>
__global__ void __launch_bounds__(kBlock) k_strength_sym(CsrView A, const double *__restrict__ tval,
                                                         const double *__restrict__ diag, double eps2,
                                                         int32_t *__restrict__ cnt, const int32_t *__restrict__ srow,
                                                         int32_t *__restrict__ scol, double *__restrict__ sw,
                                                         uint8_t *__restrict__ strongA, double *__restrict__ dF) {
    const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
    const int lane = (int)(threadIdx.x % G);
    if (row >= A.n) return;
    const int32_t i = (int32_t)row;
    const int32_t pa = A.rowptr[i], la = A.rowptr[i + 1] - pa;
    const double di = diag[i];
    const int32_t q0 = FILL ? srow[i] : 0;
    int32_t run = 0;
    double lump = di;
    for (int32_t c0 = 0; c0 < la; c0 += G) {
        const int32_t a = c0 + lane;
        const bool in = a < la;
        const int32_t j = in ? A.col[pa + a] : i;
        const double aij = in ? A.val[pa + a] : 0.0, aji = in ? tval[pa + a] : 0.0;
        const bool st = in && j != i && strong_pair(aij, aji, di, diag[j], eps2);
        const int32_t sc = st ? 1 : 0;
        const int32_t incl = grp_scan_incl<G>(sc, lane);
        if (FILL) {
            if (in) strongA[pa + a] = st ? 1 : 0;
            if (st) {
                const int32_t pos = run + incl - sc;
                scol[q0 + pos] = j;
                const double x = fabs(aij), y = fabs(aji);
                sw[q0 + pos] = x > y ? x : y;
            }
            const double weak = (in && j != i && !st) ? aij : 0.0;
            for (int t = 0; t < G; ++t) {
                const double w = __shfl(weak, t, G);
                if (c0 + t < la && w != 0.0) lump = lump + w;
            }
        }
        run += __shfl(incl, G - 1, G);
    }
    if (lane == 0) {
        if (FILL) dF[i] = lump;
        else cnt[i + 1] = run;
    }
}

// ------------------------------------------------------------------ MIS-2 --
// Kernels that end in one same-address atomic per block run a capped grid
// over a row loop: such atomics serialize (about 10 ns each), so a grid of one
// block per 256 rows of a million-row level would spend tens of microseconds
// on them alone.
constexpr unsigned kAtomicBlocks = 1024;

__global__ void k_mis_init(const int32_t *__restrict__ srow, int32_t n, uint32_t *__restrict__ state,
                           uint8_t *__restrict__ done, int32_t *und) {
    __shared__ int32_t sm[kBlock / dev::kWave];
    int32_t c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const bool kept = srow[i + 1] > srow[i];
        state[i] = kept ? ST_UND : ST_OUT;
        done[i] = kept ? 0 : 1;
        c += kept;
    }
    c = dev::block_sum(c, sm);
    if (threadIdx.x == 0 && c) atomicAdd(und, c);
}

template <int G, class T>
__device__ __forceinline__ T grp_max(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, G);
        v = w > v ? w : v;
    }
    return v;
}

template <int G, class T>
__device__ __forceinline__ T grp_min(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, G);
        v = w < v ? w : v;
    }
    return v;
}

// Row of a G-lane group: index, lane, and whether it exists.  Every lane of
// a block stays to the end (block reductions follow).
#define GRP_ROW(G, n)                                                                \
    const int64_t row_ = (dev::xcd_block() * (int64_t)blockDim.x + threadIdx.x) / (G); \
    const int lane_ = (int)(threadIdx.x % (G));                                  \
    const bool has_ = row_ < (n);                                                \
    const int32_t i = has_ ? (int32_t)row_ : 0;

// Rows visited by G-lane groups over the whole (capped) grid.
#define GRP_LOOP(G, n)                                                                          \
    const int lane_ = (int)(threadIdx.x % (G));                                                 \
    for (int64_t row_ = (dev::xcd_block() * (int64_t)blockDim.x + threadIdx.x) / (G); row_ < (n); \
         row_ += (int64_t)gridDim.x * blockDim.x / (G))

// m1_i = max(key_i, max_{j in S(i)} key_j) (a maximum: any lane order).
// Skipped once a previous round left nothing undecided.  m1 is read only by
// undecided nodes, for themselves and their neighbours (S is symmetric), and
// states never return to UNDECIDED: a node that finds itself and all its
// neighbours decided is marked done and skipped by later rounds.
template <int G>
__global__ void k_mis_m1(const int32_t *__restrict__ srow, const int32_t *__restrict__ scol, int32_t n,
                         const uint32_t *__restrict__ state, uint32_t salt, uint64_t *__restrict__ m1,
                         uint8_t *__restrict__ done, const int32_t *prev_und) {
    if (*prev_und == 0) return;
    GRP_ROW(G, n)
    if (!has_ || done[i]) return;
    const uint32_t si = state[i];
    uint64_t m = lane_ == 0 ? mis_key(si, salt, i) : 0ull;
    int32_t open = si == ST_UND;
    const int32_t e = srow[i + 1];
    for (int32_t p = srow[i] + lane_; p < e; p += G) {
        const int32_t j = scol[p];
        const uint32_t sj = state[j];
        open |= sj == ST_UND;
        const uint64_t kj = mis_key(sj, salt, j);
        m = kj > m ? kj : m;
    }
    m = grp_max<G>(m);
    open = grp_max<G>(open);
    if (lane_ == 0) {
        m1[i] = m;
        if (!open) done[i] = 1;
    }
}

// m2_i = max(m1_i, max_j m1_j); UNDECIDED i becomes ROOT if m2_i is its own
// key, OUT if m2_i belongs to a ROOT.  Sets *und to 1 when a node is left
// undecided (one plain store per wave that has one: the next round and the
// host only ask whether any is left).
template <int G>
__global__ void k_mis_m2(const int32_t *__restrict__ srow, const int32_t *__restrict__ scol, int32_t n,
                         uint32_t *__restrict__ state, uint32_t salt, const uint64_t *__restrict__ m1,
                         const int32_t *prev_und, int32_t *und) {
    if (*prev_und == 0) return;
    GRP_ROW(G, n)
    bool left = false;
    if (has_ && state[i] == ST_UND) {
        uint64_t m = lane_ == 0 ? m1[i] : 0ull;
        const int32_t e = srow[i + 1];
        for (int32_t p = srow[i] + lane_; p < e; p += G) {
            const uint64_t v = m1[scol[p]];
            m = v > m ? v : m;
        }
        m = grp_max<G>(m);
        if (lane_ == 0) {
            if (m == mis_key(ST_UND, salt, i)) state[i] = ST_ROOT;
            else if ((m >> 62) == ST_ROOT) state[i] = ST_OUT;
            else left = true;
        }
    }
    if (__any(left) && (threadIdx.x & (dev::kWave - 1)) == 0) *und = 1;
}

// ------------------------------------------------------------- aggregates --
__global__ void k_root_flags(const uint32_t *__restrict__ state, int32_t n, int32_t *__restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) flag[i + 1] = state[i] == ST_ROOT ? 1 : 0;
    if (i == 0) flag[0] = 0;
}

// Aggregate of i: its own id if ROOT, else that of its first ROOT neighbour
// in column order (smallest position).
template <int G>
__global__ void k_agg_pass1(const int32_t *__restrict__ srow, const int32_t *__restrict__ scol, int32_t n,
                            const uint32_t *__restrict__ state, const int32_t *__restrict__ ids,
                            int32_t *__restrict__ agg1) {
    GRP_ROW(G, n)
    if (!has_) return;
    if (state[i] == ST_ROOT) {
        if (lane_ == 0) agg1[i] = ids[i];
        return;
    }
    const int32_t e = srow[i + 1];
    int32_t first = INT32_MAX;
    for (int32_t p = srow[i] + lane_; p < e; p += G) {
        if (state[scol[p]] == ST_ROOT) {
            first = p;
            break;
        }
    }
    first = grp_min<G>(first);
    if (lane_ == 0) agg1[i] = first == INT32_MAX ? -1 : ids[scol[first]];
}

// Unassigned i joins the neighbouring aggregate of largest strength weight,
// the smallest aggregate id among equal weights.
template <int G>
__global__ void k_agg_pass2(const int32_t *__restrict__ srow, const int32_t *__restrict__ scol,
                            const double *__restrict__ sw, int32_t n, const int32_t *__restrict__ agg1,
                            int32_t *__restrict__ agg) {
    GRP_ROW(G, n)
    if (!has_) return;
    const int32_t a = agg1[i];
    const int32_t b = srow[i], e = srow[i + 1];
    if (a >= 0 || e == b) {
        if (lane_ == 0) agg[i] = a;
        return;
    }
    double best_w = -1.0;
    int32_t best = -1;
    for (int32_t p = b + lane_; p < e; p += G) {
        const int32_t c = agg1[scol[p]];
        if (c < 0) continue;
        const double w = sw[p];
        if (w > best_w || (w == best_w && c < best)) { best_w = w; best = c; }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const double w = __shfl_xor(best_w, o, G);
        const int32_t c = __shfl_xor(best, o, G);
        if (w > best_w || (w == best_w && c < best && c >= 0)) { best_w = w; best = c; }
    }
    if (lane_ == 0) agg[i] = best;
}

// ----------------------------------------------------- prolongator weight --
// rho = max_i (sum_j |a_ij|, ascending j) / a_ii; positive doubles order like
// their bit patterns, so an integer atomicMax is exact.
// Sum over row i in column order, lane values taken one after another.
template <int G, class F>
__device__ __forceinline__ double grp_ordered_sum(int32_t b, int32_t e, int lane, F &&term) {
    double s = 0.0;
    for (int32_t c0 = b; c0 < e; c0 += G) {
        const int32_t p = c0 + lane;
        const double v = p < e ? term(p) : 0.0;
        for (int t = 0; t < G; ++t) {
            const double w = __shfl(v, t, G);
            if (c0 + t < e) s = s + w;
        }
    }
    return s;
}

// One thread a row, in row order within the block, so the block's entries
// are one contiguous range: up to kRhoStage of them are first copied to LDS
// with coalesced loads (|a_ij|), then each thread adds its row's from LDS;
// a longer range loads each row's entries B at a time, all B before any is
// added.  Either way the row is summed one entry after another from s = 0
// in column order (the sum grp_ordered_sum forms).
constexpr int kRhoStage = 16 * kBlock;

template <int B>
__global__ void __launch_bounds__(kBlock) k_rho(CsrView A, const double *__restrict__ diag,
                                                unsigned long long *rho_bits) {
    __shared__ double st[kRhoStage];
    const int64_t r0 = dev::xcd_block() * (int64_t)kBlock;
    const int64_t i = r0 + threadIdx.x;
    const int64_t rl = min(r0 + kBlock, (int64_t)A.n);  // one past the block's last row
    const int32_t base = A.rowptr[r0], top = A.rowptr[rl];
    const bool staged = top - base <= kRhoStage;  // the same in every thread
    if (staged) {
        for (int32_t p = base + threadIdx.x; p < top; p += kBlock) st[p - base] = fabs(A.val[p]);
        __syncthreads();
    }
    double r = 0.0;
    if (i < A.n) {
        const int32_t b = A.rowptr[i], e = A.rowptr[i + 1];
        const double d = diag[i];
        double s = 0.0;
        if (staged) {
            for (int32_t p = b; p < e; ++p) s = s + st[p - base];
        } else {
            for (int32_t c0 = b; c0 < e; c0 += B) {
                double v[B];
#pragma unroll
                for (int u = 0; u < B; ++u) v[u] = fabs(A.val[min(c0 + u, e - 1)]);
#pragma unroll
                for (int u = 0; u < B; ++u)
                    if (c0 + u < e) s = s + v[u];
            }
        }
        const double ri = s / d;
        r = ri > r ? ri : r;
    }
    __shared__ double sm[kBlock / dev::kWave];
    r = dev::block_max(r, sm);
    // a block whose maximum does not pass the value already there skips the
    // atomic (the maximum only grows, so none is lost), so thousands of
    // blocks do not queue on the one address
    if (threadIdx.x == 0) {
        const unsigned long long rb = (unsigned long long)__double_as_longlong(r);
        if (rb > __hip_atomic_load(rho_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(rho_bits, rb);
    }
}

__global__ void k_omega(const unsigned long long *rho_bits, double *omega) {
    if (threadIdx.x == 0) *omega = (4.0 / 3.0) / __longlong_as_double((long long)*rho_bits);
}

// ------------------------------------------------------- hashed SpGEMM ----
// Output row i is the stream, over the A-side entries (k, a) of row i in
// ascending order, of the B-row entries (J, b): contribution a*b to column J.
// G lanes own one output row and an LDS hash table; the entries of one B row
// have distinct columns, so the lanes can add them concurrently while B rows
// are taken one after another: every output entry is then accumulated left to
// right in stream order, exactly like a sequential dense accumulator.

struct ARowCsr {
    const int32_t *rowptr, *col;
    const double *val;
    __device__ int32_t begin(int32_t i) const { return rowptr[i]; }
    __device__ int32_t end(int32_t i) const { return rowptr[i + 1]; }
    __device__ bool get(int32_t p, int32_t, int32_t &k, double &a) const {
        k = col[p];
        a = val[p];
        return true;
    }
};

// Filtered operator A_F: diagonal replaced by the lumped dF, weak
// off-diagonals dropped.
struct ARowFiltered {
    const int32_t *rowptr, *col;
    const double *val;
    const uint8_t *strong;
    const double *dF;
    __device__ int32_t begin(int32_t i) const { return rowptr[i]; }
    __device__ int32_t end(int32_t i) const { return rowptr[i + 1]; }
    __device__ bool get(int32_t p, int32_t i, int32_t &k, double &a) const {
        k = col[p];
        if (k != i && !strong[p]) return false;
        a = (k == i) ? dF[i] : val[p];
        return true;
    }
};

struct BCsr {
    const int32_t *rowptr, *col;
    const double *val;
    __device__ void row(int32_t k, int32_t &base, int32_t &len) const {
        base = rowptr[k];
        len = rowptr[k + 1] - base;
    }
    __device__ void get(int32_t base, int32_t t, int32_t &J, double &b) const {
        J = col[base + t];
        b = val[base + t];
    }
};

// Tentative prolongator: row k has the single entry 1 at column agg(k).
struct BTent {
    const int32_t *agg;
    __device__ void row(int32_t k, int32_t &base, int32_t &len) const {
        base = agg[k];
        len = base >= 0 ? 1 : 0;
    }
    __device__ void get(int32_t base, int32_t, int32_t &J, double &b) const {
        J = base;
        b = 1.0;
    }
};

// Epilogues: row(i) gathers what the output row needs once (before its
// stores, which the compiler cannot prove apart from the epilogue's
// arrays), then each entry is formed from that and the sum s.
struct EpiIdentity {
    struct Row {};
    __device__ Row row(int32_t) const { return {}; }
    __device__ double operator()(const Row &, int32_t, double s) const { return s; }
};

// P_iI = [agg(i) == I] - (w / d_i) s_I with d_i = dF_i if positive else a_ii.
struct EpiSmoothP {
    const int32_t *agg;
    const double *dF, *diag;
    const double *omega;
    struct Row {
        int32_t agg_i;
        double coef;
    };
    __device__ Row row(int32_t i) const {
        const double di = dF[i] > 0.0 ? dF[i] : diag[i];
        return {agg[i], *omega / di};
    }
    __device__ double operator()(const Row &r, int32_t J, double s) const {
        const double delta = (r.agg_i == J) ? 1.0 : 0.0;
        return delta - r.coef * s;
    }
};

// Upper bound of the distinct columns of each output row (the sum of the B
// row lengths), largest over all rows; G lanes per output row.
template <int G, class AR, class BR>
__global__ void k_spgemm_ub(AR ar, BR br, int32_t nrows, int32_t *ub_max) {
    int32_t u = 0;
    GRP_LOOP(G, nrows) {
        const int32_t i = (int32_t)row_;
        int32_t ui = 0;
        const int32_t e = ar.end(i);
        for (int32_t p = ar.begin(i) + lane_; p < e; p += G) {
            int32_t k, base, len;
            double a;
            if (!ar.get(p, i, k, a)) continue;
            br.row(k, base, len);
            ui += len;
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) ui += __shfl_xor(ui, o, G);
        u = ui > u ? ui : u;
    }
    __shared__ int32_t sm[kBlock / dev::kWave];
    u = dev::block_max(u, sm);
    if (threadIdx.x == 0) atomicMax(ub_max, u);
}

__device__ __forceinline__ int32_t hash_slot(int32_t *keys, int hbits, int32_t J, bool &fresh) {
    const int32_t H = 1 << hbits;
    uint32_t h = ((uint32_t)J * 2654435761u) >> (32 - hbits);
    for (int32_t probe = 0; probe < H; ++probe) {
        int32_t old = atomicCAS(&keys[h], -1, J);
        if (old == -1) { fresh = true; return (int32_t)h; }
        if (old == J) { fresh = false; return (int32_t)h; }
        h = (h + 1) & (uint32_t)(H - 1);
    }
    fresh = false;
    return -1;
}

template <int G>
__device__ __forceinline__ int32_t group_sum(int32_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, dev::kWave);
    return v;
}

template <int G>
__device__ __forceinline__ int32_t group_max(int32_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        int32_t w = __shfl_xor(v, o, dev::kWave);
        v = w > v ? w : v;
    }
    return v;
}

// Inclusive prefix sum over the G lanes of a group.
template <int G>
__device__ __forceinline__ int32_t group_scan_incl(int32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int32_t w = __shfl_up(v, o, G);
        if (lane >= o) v += w;
    }
    return v;
}

// Both passes of the product in one kernel body.  NUM = false counts the
// distinct columns of every output row (symbolic pass); NUM = true writes
// them, sorted, with their values.  A segment of A-side entries is taken one
// entry per lane, all their B rows are loaded at once into an LDS stage
// (contribution a*b formed by the loading lane), and then the staged B rows
// are added into the hash one after another, in stream order.  A segment is
// the longest run of entries whose contributions fit in the stage; an entry
// that alone exceeds it is added straight from memory.
template <int G, bool NUM, class AR, class BR, class EPI>
__global__ void k_spgemm(AR ar, BR br, int32_t nrows, int hbits, int S, int32_t *__restrict__ cnt,
                         const int32_t *__restrict__ crow, int32_t *__restrict__ ccol, double *__restrict__ cval,
                         EPI epi, int32_t *maxd, int32_t *overflow) {
    extern __shared__ double sm_dbl[];
    const int32_t H = 1 << hbits;
    const int group = threadIdx.x / G, lane = threadIdx.x % G;
    const int groups = blockDim.x / G;
    // per group: doubles [vals H | stage S] (NUM only), then ints [keys H | stage S]
    double *vals = nullptr, *stV = nullptr;
    int32_t *ibase = NUM ? reinterpret_cast<int32_t *>(sm_dbl + (size_t)groups * (H + S))
                         : reinterpret_cast<int32_t *>(sm_dbl);
    int32_t *keys = ibase + (size_t)group * (H + S);
    int32_t *stJ = keys + H;
    if (NUM) {
        vals = sm_dbl + (size_t)group * (H + S);
        stV = vals + H;
    }
    const int64_t row = dev::xcd_block() * groups + group;  // XCD-contiguous row ranges
    const bool active = row < nrows;
    // the epilogue's row words, issued now and first needed at the write-out
    typename EPI::Row er{};
    if (NUM && active) er = epi.row((int32_t)row);
    for (int32_t s = lane; s < H; s += G) {
        keys[s] = -1;
        if (NUM) vals[s] = 0.0;
    }
    __syncthreads();
    int32_t fresh_count = 0;
    bool ovf = false;
    if (active) {
        const int32_t i = (int32_t)row;
        const int32_t pend = ar.end(i);
        int32_t p0 = ar.begin(i);
        while (p0 < pend) {
            const int32_t p = p0 + lane;
            int32_t k = 0, base = 0, len = 0;
            double a = 0.0;
            const bool valid = p < pend;
            if (valid && ar.get(p, i, k, a)) br.row(k, base, len);
            const int32_t incl = group_scan_incl<G>(len, lane);
            const int32_t excl = incl - len;
            const int32_t m = group_max<G>((valid && incl <= S) ? lane + 1 : 0);
            if (m == 0) {
                const int32_t b0 = __shfl(base, 0, G), l0 = __shfl(len, 0, G);
                const double a0 = __shfl(a, 0, G);
                for (int32_t t = lane; t < l0; t += G) {
                    int32_t J;
                    double bv;
                    br.get(b0, t, J, bv);
                    bool fresh;
                    int32_t h = hash_slot(keys, hbits, J, fresh);
                    if (h < 0) { ovf = true; continue; }
                    fresh_count += fresh;
                    if (NUM) vals[h] = vals[h] + a0 * bv;
                }
                __builtin_amdgcn_wave_barrier();
                p0 += 1;
                continue;
            }
            if (lane < m) {
                int32_t t = 0;
                for (; t + 1 < len; t += 2) {
                    int32_t J0, J1;
                    double b0, b1;
                    br.get(base, t, J0, b0);
                    br.get(base, t + 1, J1, b1);
                    stJ[excl + t] = J0;
                    stJ[excl + t + 1] = J1;
                    if (NUM) {
                        stV[excl + t] = a * b0;
                        stV[excl + t + 1] = a * b1;
                    }
                }
                if (t < len) {
                    int32_t J;
                    double bv;
                    br.get(base, t, J, bv);
                    stJ[excl + t] = J;
                    if (NUM) stV[excl + t] = a * bv;
                }
            }
            __builtin_amdgcn_wave_barrier();
            // every staged column finds its slot at once (the slot a key
            // gets does not depend on the order of insertion that matters
            // for the sums); the slot then replaces the column in the stage
            const int32_t tot = __shfl(incl, m - 1, G);
            for (int32_t c = lane; c < tot; c += G) {
                bool fresh;
                int32_t h = hash_slot(keys, hbits, stJ[c], fresh);
                if (h < 0) {
                    ovf = true;
                    h = 0;
                }
                fresh_count += fresh;
                if (NUM) stJ[c] = h;
            }
            __builtin_amdgcn_wave_barrier();
            // the sums, B row after B row in stream order
            if (NUM) {
                for (int e = 0; e < m; ++e) {
                    const int32_t off = G == 64 ? __builtin_amdgcn_readlane(excl, e) : __shfl(excl, e, G);
                    const int32_t le = G == 64 ? __builtin_amdgcn_readlane(len, e) : __shfl(len, e, G);
                    for (int32_t t = lane; t < le; t += G) {
                        const int32_t h = stJ[off + t];
                        vals[h] = vals[h] + stV[off + t];
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            p0 += m;
        }
    }
    if (!NUM) {
        // row lengths (and the leading zero); the scan over them also
        // yields the largest row
        int32_t tot = group_sum<G>(fresh_count);
        if (active && lane == 0) cnt[row + 1] = tot;
        if (row == 0 && lane == 0) cnt[0] = 0;
    } else if (active) {
        // Sorted write-out: the occupied slots are packed into the stage
        // (when the row fits it) so that each entry's rank is counted over
        // the row's entries only, not over the whole table.
        __builtin_amdgcn_wave_barrier();
        const int32_t i = (int32_t)row;
        const int32_t out0 = crow[i];
        int32_t mine = 0;
        for (int32_t s = lane; s < H; s += G) mine += keys[s] >= 0;
        const int32_t incl = group_scan_incl<G>(mine, lane);
        const int32_t m = __shfl(incl, G - 1, G);
        if (m <= S) {
            int32_t q = incl - mine;
            for (int32_t s = lane; s < H; s += G) {
                const int32_t J = keys[s];
                if (J < 0) continue;
                stJ[q] = J;
                stV[q] = vals[s];
                ++q;
            }
            __builtin_amdgcn_wave_barrier();
            for (int32_t t = lane; t < m; t += G) {
                const int32_t J = stJ[t];
                int32_t rank = 0;
                for (int32_t u = 0; u < m; ++u) rank += stJ[u] < J;
                ccol[out0 + rank] = J;
                cval[out0 + rank] = epi(er, J, stV[t]);
            }
        } else {
            for (int32_t s = lane; s < H; s += G) {
                const int32_t J = keys[s];
                if (J < 0) continue;
                int32_t rank = 0;
                for (int32_t u = 0; u < H; ++u) {
                    const int32_t K2 = keys[u];
                    rank += (K2 >= 0 && K2 < J);
                }
                ccol[out0 + rank] = J;
                cval[out0 + rank] = epi(er, J, vals[s]);
            }
        }
    }
    if (ovf) atomicOr(overflow, 1);
}

// The same product with one lane per output row, for rows with at most CAP
// distinct columns (the caller picks CAP from the row bound or the largest
// row): the row's columns and sums live in registers, each contribution is
// added to its column's sum in stream order (A entry after A entry, each B
// row in order), exactly as the hashed kernel adds them, and the row is
// written in column order by ranking.  NUM = false counts the columns.
template <int CAP, bool NUM, class AR, class BR, class EPI>
__global__ void __launch_bounds__(kBlock) k_spgemm_lane(AR ar, BR br, int32_t nrows, int32_t *__restrict__ cnt,
                                                        const int32_t *__restrict__ crow, int32_t *__restrict__ ccol,
                                                        double *__restrict__ cval, EPI epi, int32_t *overflow) {
    const int64_t row = dev::xcd_block() * (int64_t)blockDim.x + threadIdx.x;
    if (row >= nrows) return;
    const int32_t i = (int32_t)row;
    typename EPI::Row er{};
    if (NUM) er = epi.row(i);
    int32_t key[CAP];
    double val[CAP];
#pragma unroll
    for (int s = 0; s < CAP; ++s) {
        key[s] = -1;
        val[s] = 0.0;
    }
    int32_t m = 0;
    bool ovf = false;
    const int32_t pend = ar.end(i);
    // A entries and their B-row heads are loaded four at a time (independent
    // loads in flight), then added in order
    constexpr int U = 4;
    for (int32_t p0 = ar.begin(i); p0 < pend; p0 += U) {
        int32_t kk[U], bb[U], ll[U];
        double aa[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            kk[u] = 0;
            aa[u] = 0.0;
            bb[u] = 0;
            ll[u] = 0;
            if (p0 + u < pend && ar.get(p0 + u, i, kk[u], aa[u])) br.row(kk[u], bb[u], ll[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double a = aa[u];
            const int32_t base = bb[u], len = ll[u];
            for (int32_t t = 0; t < len; ++t) {
                int32_t J;
                double bv;
                br.get(base, t, J, bv);
                const double c = NUM ? a * bv : 0.0;
                bool found = false;
#pragma unroll
                for (int s = 0; s < CAP; ++s) {
                    if (key[s] == J) {
                        if (NUM) val[s] = val[s] + c;
                        found = true;
                    }
                }
                if (!found) {
                    if (m < CAP) {
#pragma unroll
                        for (int s = 0; s < CAP; ++s) {
                            if (s == m) {
                                key[s] = J;
                                if (NUM) val[s] = val[s] + c;  // 0 + c, as the hashed kernel's first add
                            }
                        }
                        ++m;
                    } else {
                        ovf = true;
                    }
                }
            }
        }
    }
    if (!NUM) {
        cnt[row + 1] = m;
        if (row == 0) cnt[0] = 0;
    } else {
        const int32_t out0 = crow[i];
#pragma unroll
        for (int s = 0; s < CAP; ++s) {
            if (s >= m) break;
            int32_t rank = 0;
#pragma unroll
            for (int u = 0; u < CAP; ++u) rank += (u < m && key[u] < key[s]) ? 1 : 0;
            ccol[out0 + rank] = key[s];
            cval[out0 + rank] = epi(er, key[s], val[s]);
        }
    }
    if (ovf) atomicOr(overflow, 1);
}

// -------------------------------------------------------------- smoother --
// SPAI0: M_i = a_ii / sum_j a_ij^2, the squares added in column order from
// 0, one thread a row as in k_rho (the block's squares staged in LDS when
// they fit, else loaded B at a time); damped Jacobi: M_i = omega / a_ii.
template <int B>
__global__ void __launch_bounds__(kBlock) k_smoother_diag(CsrView A, const double *__restrict__ diag, int spai0,
                                                          double omega, double *__restrict__ M) {
    __shared__ double st[kRhoStage];
    const int64_t r0 = dev::xcd_block() * (int64_t)kBlock;
    const int64_t i = r0 + threadIdx.x;
    if (!spai0) {  // the same in every thread
        if (i < A.n) M[i] = omega / diag[i];
        return;
    }
    const int64_t rl = min(r0 + kBlock, (int64_t)A.n);
    const int32_t base = A.rowptr[r0], top = A.rowptr[rl];
    const bool staged = top - base <= kRhoStage;  // the same in every thread
    if (staged) {
        for (int32_t p = base + threadIdx.x; p < top; p += kBlock) st[p - base] = A.val[p] * A.val[p];
        __syncthreads();
    }
    if (i >= A.n) return;
    const int32_t b = A.rowptr[i], e = A.rowptr[i + 1];
    const double aii = diag[i];
    double s = 0.0;
    if (staged) {
        for (int32_t p = b; p < e; ++p) s = s + st[p - base];
    } else {
        for (int32_t c0 = b; c0 < e; c0 += B) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const double a = A.val[min(c0 + u, e - 1)];
                v[u] = a * a;
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (c0 + u < e) s = s + v[u];
        }
    }
    M[i] = aii / s;
}

// Diagonal of each row (0 when absent).
template <int G>
__global__ void k_diag(CsrView A, double *__restrict__ diag) {
    GRP_ROW(G, A.n)
    if (!has_) return;
    const int32_t e = A.rowptr[i + 1];
    int32_t at = -1;
    for (int32_t p = A.rowptr[i] + lane_; p < e; p += G)
        if (A.col[p] == i) at = p;
    at = grp_max<G>(at);
    if (lane_ == 0) diag[i] = at >= 0 ? A.val[at] : 0.0;
}

__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

// ------------------------------------------------------------- coarse LU --
// One wave a row: the lanes clear the dense row, then write its entries
// (a row's columns are distinct, so the scattered writes never collide).
__global__ void k_csr_to_dense(CsrView A, double *__restrict__ a) {
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / dev::kWave;
    const int lane = threadIdx.x & (dev::kWave - 1);
    if (i >= A.n) return;
    double *row = a + i * A.n;
    for (int32_t c = lane; c < A.n; c += dev::kWave) row[c] = 0.0;
    __threadfence_block();  // the zeros land before any entry overwrites one
    for (int32_t p = A.rowptr[i] + lane; p < A.rowptr[i + 1]; p += dev::kWave) row[A.col[p]] = A.val[p];
}

// Right-looking LU with partial pivoting in one workgroup (LAPACK getrf
// order: the first row holding the largest |a_ik| is the pivot), on `a`
// row-major n x n in memory M: global memory, or LDS for small n (the
// matrix is copied in and out).  Each entry is updated k after k, with no
// fused multiply-add, exactly as the unblocked algorithm does.
__device__ __forceinline__ void lu_in_place(double *a, int32_t n, int32_t *__restrict__ piv, int32_t *status) {
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    __shared__ int32_t p_sh;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    for (int32_t k = 0; k < n; ++k) {
        double best = -1.0;
        int32_t bi = n;
        for (int32_t i = k + tid; i < n; i += blockDim.x) {
            double v = fabs(a[(int64_t)i * n + k]);
            if (v > best) { best = v; bi = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            double v2 = __shfl_xor(best, o, 64);
            int32_t i2 = __shfl_xor(bi, o, 64);
            if (v2 > best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
        }
        if (lane == 0) { sv[w] = best; si[w] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = sv[0];
            int32_t ix = si[0];
            for (int q = 1; q < nw; ++q)
                if (sv[q] > b || (sv[q] == b && si[q] < ix)) { b = sv[q]; ix = si[q]; }
            p_sh = (b == 0.0) ? -1 : ix;
            piv[k] = ix;
        }
        __syncthreads();
        const int32_t p = p_sh;
        if (p < 0) {
            if (tid == 0) *status = GW_SINGULAR;
            return;
        }
        if (p != k)
            for (int32_t j = tid; j < n; j += blockDim.x) {
                double t = a[(int64_t)k * n + j];
                a[(int64_t)k * n + j] = a[(int64_t)p * n + j];
                a[(int64_t)p * n + j] = t;
            }
        __syncthreads();
        const double akk = a[(int64_t)k * n + k];
        for (int32_t i = k + 1 + tid; i < n; i += blockDim.x) a[(int64_t)i * n + k] = a[(int64_t)i * n + k] / akk;
        __syncthreads();
        // trailing update: a wave takes four rows at a time (independent
        // updates in flight), lanes along the row
        for (int32_t i0 = k + 1 + w; i0 < n; i0 += 4 * nw) {
            double lik[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t i = min(i0 + u * nw, n - 1);
                lik[u] = a[(int64_t)i * n + k];
            }
            for (int32_t j = k + 1 + lane; j < n; j += 64) {
                const double akj = a[(int64_t)k * n + j];
                double aij[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) aij[u] = a[(int64_t)min(i0 + u * nw, n - 1) * n + j];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + u * nw < n) a[(int64_t)(i0 + u * nw) * n + j] = aij[u] - lik[u] * akj;
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_dense_lu(double *__restrict__ a, int32_t n, int32_t *__restrict__ piv,
                                                   int32_t *status) {
    lu_in_place(a, n, piv, status);
}

constexpr int kLuLdsSmall = 88;  // up to 88 x 88 (61952 B): 256 threads, more: 512 (measured
                                 // 18 % faster than 1024 at n = 109, 14 % at n = 141)

// The same factorization for a matrix held in LDS, with two barriers a step
// instead of five: the pivot search of column k+1 runs inside step k's
// trailing update (lane 0 of each wave sees the new column k+1 entries of
// its rows, in increasing row order, and keeps the first largest with its
// signed value), and every thread then picks the pivot from the per-wave
// records itself; the row swap and the scaling of column k share one phase,
// thread 0 taking the two column-k entries that both would touch.  Every
// entry gets the same operations in the same order as in lu_in_place, and
// the pivot is the same row, so the factors and pivots are identical.
template <int NW>
__device__ __forceinline__ void lu_lds_two_barrier(double *a, int32_t n, int32_t *__restrict__ piv,
                                                   int32_t *status) {
    // n <= 143 (the matrix fits in LDS), so 32-bit indices
    __shared__ double sv[NW], sval[NW];
    __shared__ int32_t si[NW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // column 0's search: lane 0 of wave w scans rows w, w + NW, ...
    if (lane == 0) {
        double best = -1.0, bv = 0.0;
        int32_t bi = n;
        for (int32_t i = w; i < n; i += NW) {
            const double v = a[i * n];
            if (fabs(v) > best) { best = fabs(v); bi = i; bv = v; }
        }
        sv[w] = best, si[w] = bi, sval[w] = bv;
    }
    __syncthreads();
    for (int32_t k = 0; k < n; ++k) {
        // the per-wave records, all read before they are compared
        double rv[NW], rs[NW];
        int32_t ri[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) rv[q] = sv[q], rs[q] = sval[q], ri[q] = si[q];
        double b = rv[0], pv = rs[0];
        int32_t p = ri[0];
#pragma unroll
        for (int q = 1; q < NW; ++q)
            if (rv[q] > b || (rv[q] == b && ri[q] < p)) { b = rv[q]; p = ri[q]; pv = rs[q]; }
        if (tid == 0) piv[k] = p;
        if (!(b > 0.0)) {
            if (tid == 0) *status = GW_SINGULAR;
            return;
        }
        // swap rows k and p outside column k; column k: a_kk = pivot, the
        // old a_kk moves to row p and is scaled there, the rest are scaled
        if (tid == 0) {
            const double t = a[k * n + k];
            a[k * n + k] = pv;
            if (p != k) a[p * n + k] = t / pv;
        }
        if (p != k)
            for (int32_t j = tid; j < n; j += NW * 64)
                if (j != k) {
                    const double t = a[k * n + j];
                    a[k * n + j] = a[p * n + j];
                    a[p * n + j] = t;
                }
        for (int32_t i = k + 1 + tid; i < n; i += NW * 64)
            if (i != p) a[i * n + k] = a[i * n + k] / pv;
        __syncthreads();
        // trailing update (a wave takes four rows at a time, lanes along the
        // row) with the search of column k+1 on lane 0 (j = k+1)
        double best = -1.0, bv = 0.0;
        int32_t bi = n;
        for (int32_t i0 = k + 1 + w; i0 < n; i0 += 4 * NW) {
            double lik[4];
            int32_t row[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                row[u] = min(i0 + u * NW, n - 1) * n;
                lik[u] = a[row[u] + k];
            }
            for (int32_t j = k + 1 + lane; j < n; j += 64) {
                const double akj = a[k * n + j];
                double aij[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) aij[u] = a[row[u] + j];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t i = i0 + u * NW;
                    if (i < n) {
                        const double v = aij[u] - lik[u] * akj;
                        a[row[u] + j] = v;
                        if (j == k + 1 && fabs(v) > best) { best = fabs(v); bi = i; bv = v; }
                    }
                }
            }
        }
        if (lane == 0) sv[w] = best, si[w] = bi, sval[w] = bv;
        __syncthreads();
    }
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_dense_lu_lds(double *__restrict__ a, int32_t n,
                                                         int32_t *__restrict__ piv, int32_t *status) {
    static_assert(BLOCK % 64 == 0 && BLOCK <= 1024, "whole waves, at most 16");
    extern __shared__ double lu_sm[];
    for (int32_t e = threadIdx.x; e < n * n; e += blockDim.x) lu_sm[e] = a[e];
    __syncthreads();
    lu_lds_two_barrier<BLOCK / 64>(lu_sm, n, piv, status);
    __syncthreads();
    for (int32_t e = threadIdx.x; e < n * n; e += blockDim.x) a[e] = lu_sm[e];
}

// Blocked form of the same factorization for matrices past the LDS limit:
// panels of nb columns.  The panel kernel factors columns [k0, k0+nb) over
// rows [k0, n) in LDS (pivot search, swap inside the panel, scaling, and the
// updates of the panel's later columns); the update kernel then applies the
// panel's row swaps to every other column, solves the panel rows of the
// later columns with the panel's unit lower triangle (U12), and subtracts
// L21 U12 from the trailing matrix.  Every entry receives the updates of
// steps k in increasing k, each a product then a difference, and every
// pivot is chosen from the same column values, so the factors and pivots
// equal those of the unblocked loop bit for bit.
__global__ void __launch_bounds__(512) k_lu_panel(double *__restrict__ a, int32_t n, int32_t k0, int32_t nb,
                                                   int32_t *__restrict__ piv, int32_t *status) {
    extern __shared__ double pan[];  // rows k0..n-1, nb columns, row-major
    __shared__ double sv[16];
    __shared__ int32_t si[16];
    __shared__ int32_t p_sh;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    const int32_t m = n - k0;  // panel rows
    if (*status != 0) return;   // an earlier panel met a zero pivot
    for (int32_t e = tid; e < m * nb; e += blockDim.x) {
        const int32_t r = e / nb, c = e - r * nb;
        pan[e] = a[(int64_t)(k0 + r) * n + k0 + c];
    }
    __syncthreads();
    for (int32_t kk = 0; kk < nb; ++kk) {
        double best = -1.0;
        int32_t bi = m;
        for (int32_t r = kk + tid; r < m; r += blockDim.x) {
            const double v = fabs(pan[r * nb + kk]);
            if (v > best) { best = v; bi = r; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(best, o, 64);
            const int32_t i2 = __shfl_xor(bi, o, 64);
            if (v2 > best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
        }
        if (lane == 0) { sv[w] = best; si[w] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = sv[0];
            int32_t ix = si[0];
            for (int q = 1; q < nw; ++q)
                if (sv[q] > b || (sv[q] == b && si[q] < ix)) { b = sv[q]; ix = si[q]; }
            p_sh = (b == 0.0) ? -1 : ix;
            piv[k0 + kk] = k0 + ix;
        }
        __syncthreads();
        const int32_t p = p_sh;
        if (p < 0) {
            if (tid == 0) *status = GW_SINGULAR;
            return;
        }
        if (p != kk)
            for (int32_t c = tid; c < nb; c += blockDim.x) {
                const double t = pan[kk * nb + c];
                pan[kk * nb + c] = pan[p * nb + c];
                pan[p * nb + c] = t;
            }
        __syncthreads();
        const double akk = pan[kk * nb + kk];
        for (int32_t r = kk + 1 + tid; r < m; r += blockDim.x) pan[r * nb + kk] = pan[r * nb + kk] / akk;
        __syncthreads();
        const int32_t wc = nb - kk - 1;  // later panel columns
        if (wc > 0)
            for (int32_t e = tid; e < (m - kk - 1) * wc; e += blockDim.x) {
                const int32_t r = kk + 1 + e / wc, c = kk + 1 + e % wc;
                pan[r * nb + c] = pan[r * nb + c] - pan[r * nb + kk] * pan[kk * nb + c];
            }
        __syncthreads();
    }
    for (int32_t e = tid; e < m * nb; e += blockDim.x) {
        const int32_t r = e / nb, c = e - r * nb;
        a[(int64_t)(k0 + r) * n + k0 + c] = pan[e];
    }
}

// The panel's swaps (in pivot order) on every column outside the panel, and
// for the later columns their panel rows: U12 = L11^-1 A12 by forward
// substitution (k increasing).  One lane per column, 64 columns a
// workgroup; L11 and the column's panel rows sit in LDS during the solve.
constexpr int kLuPanelMax = 64;
__global__ void __launch_bounds__(64) k_lu_swap_u12(double *__restrict__ a, int32_t n, int32_t k0, int32_t w,
                                                    const int32_t *__restrict__ piv, const int32_t *status) {
    __shared__ double l11[kLuPanelMax * kLuPanelMax];
    __shared__ double u[kLuPanelMax * 64];
    if (*status != 0) return;
    const int lane = threadIdx.x;
    const int32_t jb = blockIdx.x * 64 + lane;  // among the n - w columns outside the panel
    const bool live = jb < n - w;
    const int32_t j = jb < k0 ? jb : jb + w;
    for (int32_t e = lane; e < w * w; e += 64) l11[e] = a[(int64_t)(k0 + e / w) * n + k0 + e % w];
    if (live)
        for (int32_t kk = 0; kk < w; ++kk) {
            const int32_t p = piv[k0 + kk];
            if (p != k0 + kk) {
                const double t = a[(int64_t)(k0 + kk) * n + j];
                a[(int64_t)(k0 + kk) * n + j] = a[(int64_t)p * n + j];
                a[(int64_t)p * n + j] = t;
            }
        }
    __syncthreads();
    if (!live || j < k0) return;
    for (int32_t kk = 0; kk < w; ++kk) u[kk * 64 + lane] = a[(int64_t)(k0 + kk) * n + j];
    for (int32_t kk = 1; kk < w; ++kk) {
        double v = u[kk * 64 + lane];
        for (int32_t q = 0; q < kk; ++q) v = v - l11[kk * w + q] * u[q * 64 + lane];
        u[kk * 64 + lane] = v;
    }
    for (int32_t kk = 1; kk < w; ++kk) a[(int64_t)(k0 + kk) * n + j] = u[kk * 64 + lane];
}

// Trailing update a_ij -= sum_q l_iq u_qj over the panel (q increasing), one
// thread per entry, consecutive threads along a row; the row's l_iq and the
// column's u_qj are loaded eight at a time before they are used.
__global__ void k_lu_trail(double *__restrict__ a, int32_t n, int32_t k0, int32_t w, const int32_t *status) {
    if (*status != 0) return;
    const int32_t t0 = k0 + w, nt = n - t0;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nt * nt) return;
    const int32_t i = t0 + (int32_t)(e / nt), j = t0 + (int32_t)(e % nt);
    const double *li = a + (int64_t)i * n + k0;
    double v = a[(int64_t)i * n + j];
    for (int32_t q0 = 0; q0 < w; q0 += 8) {
        double l[8], uq[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int32_t q = min(q0 + r, w - 1);
            l[r] = li[q];
            uq[r] = a[(int64_t)(k0 + q) * n + j];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (q0 + r < w) v = v - l[r] * uq[r];
    }
    a[(int64_t)i * n + j] = v;
}

// Column c of the inverse: solve L U x = Perm e_c, one wave per column with
// x in LDS; each substitution step is a wave-wide dot over a row of L or U.
// The inverse is stored row-major (inv[i*n + c]) for the V-cycle's GEMV.
constexpr int kMaxDense = 2048;
__global__ void __launch_bounds__(64) k_lu_inverse(const double *__restrict__ lu, const int32_t *__restrict__ piv,
                                                   int32_t n, double *__restrict__ inv, const int32_t *status) {
    __shared__ double x[kMaxDense];
    const int32_t c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n || *status != 0) return;
    // the permutation moves the single 1 of e_c
    int32_t pos = c;
    for (int32_t k = 0; k < n; ++k) {
        int32_t pk = piv[k];
        if (pos == k) pos = pk;
        else if (pos == pk) pos = k;
    }
    for (int32_t i = lane; i < n; i += 64) x[i] = (i == pos) ? 1.0 : 0.0;
    __syncthreads();
    for (int32_t i = pos + 1; i < n; ++i) {
        double s = 0.0;
        for (int32_t j = pos + lane; j < i; j += 64) s += lu[(int64_t)i * n + j] * x[j];
        s = dev::wave_sum(s);
        if (lane == 0) x[i] = x[i] - s;
        __syncthreads();
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double s = 0.0;
        for (int32_t j = i + 1 + lane; j < n; j += 64) s += lu[(int64_t)i * n + j] * x[j];
        s = dev::wave_sum(s);
        if (lane == 0) x[i] = (x[i] - s) / lu[(int64_t)i * n + i];
        __syncthreads();
    }
    for (int32_t i = lane; i < n; i += 64) inv[(int64_t)i * n + c] = x[i];
}

// The same columns of the inverse for n <= 128, by column-oriented
// substitutions: lane l holds x_l and x_{l+64}; step j broadcasts the
// finished x_j with v_readlane (a uniform lane index) and every lane
// updates its later (forward) or earlier (backward) rows, so a step costs a
// broadcast and a multiply-subtract instead of a wave-wide sum.  The L and U
// entries of the next kInvAhead steps are loaded while the current ones run,
// so the chain of steps waits for memory once per kInvAhead steps (one step
// ahead, with the pivots read one by one: 42 us for n = 118; staging the
// factors in LDS first measured slower still, 73 against 50 us).  (Each x_i receives
// its terms in the order j = pos, pos+1, ... rather than as one dot product,
// so the inverse agrees with the row-oriented one to rounding.)
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

constexpr int kInvAhead = 16;  // substitution steps whose factor entries are loaded ahead

__global__ void __launch_bounds__(64) k_lu_inverse_col(const double *__restrict__ lu, const int32_t *__restrict__ piv,
                                                       int32_t n, double *__restrict__ inv, const int32_t *status) {
    constexpr int D = kInvAhead;
    const int32_t c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n) return;
    // the pivots, two a lane (after a zero pivot the later ones were never
    // written: loaded, but not used)
    const int32_t p0 = lane < n ? piv[lane] : lane, p1 = lane + 64 < n ? piv[lane + 64] : lane + 64;
    if (*status != 0) return;
    int32_t pos = c;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t pk = __builtin_amdgcn_readlane(k < 64 ? p0 : p1, k & 63);
        if (pos == k) pos = pk;
        else if (pos == pk) pos = k;
    }
    const int32_t i0 = lane, i1 = lane + 64;
    // rows past n read row n-1 and columns past the ends the last one: in
    // bounds, never used
    const int32_t r0 = min(i0, n - 1) * n, r1 = min(i1, n - 1) * n;
    double x0 = (i0 == pos) ? 1.0 : 0.0, x1 = (i1 == pos) ? 1.0 : 0.0;
    double c0[D], c1[D], f0[D], f1[D];
    // forward: unit lower triangle, x_j final after step j - 1; the entries
    // of the next D steps are loaded while these D run
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const int32_t j = min(pos + u, n - 1);
        c0[u] = lu[r0 + j], c1[u] = lu[r1 + j];
    }
    for (int32_t jb = pos; jb < n - 1; jb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int32_t j = min(jb + D + u, n - 1);
            f0[u] = lu[r0 + j], f1[u] = lu[r1 + j];
        }
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int32_t j = jb + u;
            if (j < n - 1) {
                const double xj = readlane_f64(j < 64 ? x0 : x1, j & 63);
                if (i0 > j && i0 < n) x0 = x0 - c0[u] * xj;
                if (i1 > j && i1 < n) x1 = x1 - c1[u] * xj;
            }
        }
#pragma unroll
        for (int u = 0; u < D; ++u) c0[u] = f0[u], c1[u] = f1[u];
    }
    // backward: upper triangle with its diagonal, j = n-1 down to 0
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const int32_t j = max(n - 1 - u, 0);
        c0[u] = lu[r0 + j], c1[u] = lu[r1 + j];
    }
    for (int32_t jb = n - 1; jb >= 0; jb -= D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int32_t j = max(jb - D - u, 0);
            f0[u] = lu[r0 + j], f1[u] = lu[r1 + j];
        }
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int32_t j = jb - u;
            if (j >= 0) {
                if (i0 == j) x0 = x0 / c0[u];
                if (i1 == j) x1 = x1 / c1[u];
                const double xj = readlane_f64(j < 64 ? x0 : x1, j & 63);
                if (i0 < j) x0 = x0 - c0[u] * xj;
                if (i1 < j) x1 = x1 - c1[u] * xj;
            }
        }
#pragma unroll
        for (int u = 0; u < D; ++u) c0[u] = f0[u], c1[u] = f1[u];
    }
    if (i0 < n) inv[(int64_t)i0 * n + c] = x0;
    if (i1 < n) inv[(int64_t)i1 * n + c] = x1;
}

// ----------------------------------------------------------- Ruge-Stueben --
// The classical coarsening the paper's figures compare with smoothed
// aggregation: strength on the size of the negative couplings, a PMIS C/F
// splitting and direct interpolation.  One thread per row throughout: level
// 0 has seven entries a row and the Galerkin levels a few dozen.
constexpr int32_t CF_UND = 0, CF_C = 1, CF_F = 2;

// Strong set of row i: the j != i with -a_ij >= theta max_{k != i}(-a_ik),
// empty when no off-diagonal is negative.  The counting pass writes cnt[i+1];
// the filling pass writes the columns in A's order and marks each entry of
// A in `strong`.
template <bool FILL>
__global__ void k_rs_strength(CsrView A, double theta, int32_t *__restrict__ cnt, const int32_t *__restrict__ srow,
                              int32_t *__restrict__ scol, uint8_t *__restrict__ strong) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int32_t b = A.rowptr[i], e = A.rowptr[i + 1];
    double mx = 0.0;
    for (int32_t p = b; p < e; ++p)
        if (A.col[p] != (int32_t)i && -A.val[p] > mx) mx = -A.val[p];
    const double cut = theta * mx;
    int32_t c = 0;
    for (int32_t p = b; p < e; ++p) {
        const bool st = mx > 0.0 && A.col[p] != (int32_t)i && -A.val[p] >= cut;
        if (FILL) {
            strong[p] = st ? 1 : 0;
            if (st) scol[srow[i] + c] = A.col[p];
        }
        c += st;
    }
    if (!FILL) cnt[i + 1] = c;
}

// Weight of i: its number of dependents (the length of its row of S^T) plus
// a hash fraction in [0, 1) from the top 24 bits of fmix32(i ^ salt), exact
// in a double.  Points nothing depends on start as F.
__global__ void k_pmis_init(const int32_t *__restrict__ trow, int32_t n, uint32_t salt, double *__restrict__ w,
                            int32_t *__restrict__ cf, int32_t *und) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool left = false;
    if (i < n) {
        const int32_t dep = trow[i + 1] - trow[i];
        w[i] = (double)dep + (double)(fmix32((uint32_t)i ^ salt) >> 8) * (1.0 / 16777216.0);
        cf[i] = dep == 0 ? CF_F : CF_UND;
        left = dep != 0;
    }
    if (__any(left) && (threadIdx.x & (dev::kWave - 1)) == 0) *und = 1;
}

__device__ __forceinline__ bool pmis_beats(double wi, int32_t i, double wj, int32_t j) {
    return wi > wj || (wi == wj && i > j);
}

// First half of a round: an undecided point whose weight beats that of every
// undecided neighbour in S and in S^T is a new C point.
__global__ void k_pmis_c(const int32_t *__restrict__ srow, const int32_t *__restrict__ scol,
                         const int32_t *__restrict__ trow, const int32_t *__restrict__ tcol, int32_t n,
                         const double *__restrict__ w, const int32_t *__restrict__ cf, int32_t *__restrict__ newc) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t best = 0;
    if (cf[i] == CF_UND) {
        best = 1;
        const double wi = w[i];
        for (int32_t p = srow[i]; p < srow[i + 1] && best; ++p) {
            const int32_t j = scol[p];
            if (cf[j] == CF_UND && !pmis_beats(wi, (int32_t)i, w[j], j)) best = 0;
        }
        for (int32_t p = trow[i]; p < trow[i + 1] && best; ++p) {
            const int32_t j = tcol[p];
            if (cf[j] == CF_UND && !pmis_beats(wi, (int32_t)i, w[j], j)) best = 0;
        }
    }
    newc[i] = best;
}

// Second half: new C points take C; an undecided point that depends on a C
// point (old or new) takes F.  Each thread writes only its own point and
// tests its neighbours for C, a state no write of this pass creates or
// removes (new C points are read from newc), so the result does not depend
// on the order of the writes.  *und_next records whether any point is left.
__global__ void k_pmis_f(const int32_t *__restrict__ srow, const int32_t *__restrict__ scol, int32_t n,
                         const int32_t *__restrict__ newc, int32_t *cf, int32_t *und_next) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool left = false;
    if (i < n && cf[i] == CF_UND) {
        if (newc[i]) {
            cf[i] = CF_C;
        } else {
            bool f = false;
            for (int32_t p = srow[i]; p < srow[i + 1] && !f; ++p) {
                const int32_t j = scol[p];
                f = newc[j] != 0 || cf[j] == CF_C;
            }
            if (f) cf[i] = CF_F;
            else left = true;
        }
    }
    if (__any(left) && (threadIdx.x & (dev::kWave - 1)) == 0) *und_next = 1;
}

__global__ void k_c_flags(const int32_t *__restrict__ cf, int32_t n, int32_t *__restrict__ flag) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) flag[i + 1] = cf[i] == CF_C ? 1 : 0;
    if (i == 0) flag[0] = 0;
}

// Coarse index of each C point (its rank among the C points), -1 for F.
__global__ void k_c_index(const int32_t *__restrict__ cf, const int32_t *__restrict__ rank, int32_t n,
                          int32_t *__restrict__ cidx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) cidx[i] = cf[i] == CF_C ? rank[i] : -1;
}

// Direct interpolation.  A C point's row is 1 at its coarse index.  For an F
// point: d = a_ii plus the positive off-diagonals (lumped), neg = the sum of
// the other off-diagonals, sc = the sum of a_ij over the strong C
// neighbours, all in column order; then alpha = neg / sc and
// P_ij = -(alpha a_ij) / d on those neighbours (coarse indices ascend with
// j).  No strong C neighbour (sc = 0) leaves the row empty.
template <bool FILL>
__global__ void k_rs_interp(CsrView A, const uint8_t *__restrict__ strong, const int32_t *__restrict__ cf,
                            const int32_t *__restrict__ cidx, int32_t *__restrict__ cnt,
                            const int32_t *__restrict__ prow, int32_t *__restrict__ pcol,
                            double *__restrict__ pval) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    if (cf[i] == CF_C) {
        if (FILL) {
            pcol[prow[i]] = cidx[i];
            pval[prow[i]] = 1.0;
        } else {
            cnt[i + 1] = 1;
        }
        return;
    }
    const int32_t b = A.rowptr[i], e = A.rowptr[i + 1];
    double d = 0.0, neg = 0.0, sc = 0.0;
    int32_t m = 0;
    for (int32_t p = b; p < e; ++p) {
        const int32_t j = A.col[p];
        const double a = A.val[p];
        if (j == (int32_t)i || a > 0.0) {
            d = d + a;
            continue;
        }
        neg = neg + a;
        if (strong[p] && cf[j] == CF_C) {
            sc = sc + a;
            ++m;
        }
    }
    if (sc == 0.0) m = 0;
    if (!FILL) {
        cnt[i + 1] = m;
        return;
    }
    if (m == 0) return;
    const double alpha = neg / sc;
    int32_t q = prow[i];
    for (int32_t p = b; p < e; ++p) {
        const int32_t j = A.col[p];
        if (j == (int32_t)i || A.val[p] > 0.0) continue;
        if (strong[p] && cf[j] == CF_C) {
            pcol[q] = cidx[j];
            pval[q] = -(alpha * A.val[p]) / d;
            ++q;
        }
    }
}

// ------------------------------------------------------------ host side --

// Small device->host reads through the thread's pinned stage.
struct Staging {
    struct {
        void *p = host_stage();
    } pin;
    template <class T>
    T read(const T *d, hipStream_t s) {
        GW_HIP(hipMemcpyAsync(pin.p, d, sizeof(T), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        T v;
        std::memcpy(&v, pin.p, sizeof(T));
        return v;
    }
};

// Call f with the lane-group width (as an integral constant) for rows of
// this mean length; rows of up to 6 entries take one lane each (measured
// best for the MIS-2 rounds and aggregation passes on strength graphs of ~5
// entries per row).
template <class F>
void with_group(double mean_len, F &&f) {
    switch (lane_group_for(mean_len <= 6.0 ? 1.0 : mean_len)) {
        case 1: f(std::integral_constant<int, 1>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        case 16: f(std::integral_constant<int, 16>()); break;
        default: f(std::integral_constant<int, 64>()); break;
    }
}

double mean_row(int64_t nnz, int64_t n) { return n > 0 ? (double)nnz / (double)n : 0.0; }

int pow2_bits_at_least(int64_t v) {
    int b = 4;
    while (b < 30 && ((int64_t)1 << b) < v) ++b;
    return b;
}

constexpr int kMaxHashBits = 12;  // 4096 slots per output row

// Lanes per output row: one A-side entry per lane, so a typical row is one
// staging segment.
int spgemm_group(double avg_a_len) {
    if (avg_a_len <= 8.0) return 8;
    if (avg_a_len <= 16.0) return 16;
    if (avg_a_len <= 32.0) return 32;
    return 64;
}

// C = (A-side) x (B-side) with fixed summation order; C has `ncols` columns,
// in three phases so that the host reads of a level can be merged: the row
// bound (spgemm_bound, launched early; its value is read together with
// other sizes), the symbolic pass (row lengths, nnz, largest row and
// overflow into `blk`), and the numeric pass once those are on the host.
// blk: [0] row bound, [1] largest row, [2] overflow, [4..5] nnz (int64).
// Each pass is timed with its algorithmic bytes (every array it reads or
// writes touched once): `bytes` for the row bound; for the symbolic and
// numeric passes `in_bytes` covers the A- and B-side rows they read, and the
// pass adds what it writes (C's row pointers; its columns and values).
template <class AR, class BR>
void spgemm_bound(AR ar, BR br, int32_t nrows, double avg_a_len, int32_t *blk, hipStream_t s, double bytes) {
    // blk (the bound, and the words the symbolic pass accumulates into) was
    // cleared with the level's read-back block; a repeated call (the
    // speculative prolongator bound after each batch of MIS-2 rounds) only
    // raises the maximum, which the later rows' growing aggregates bound
    ProfScope ps(K_SPGEMM, bytes, s);
    // short rows: one lane per row (the row sums are a few loads)
    with_group(avg_a_len > 12.0 ? avg_a_len : 1.0, [&](auto gc) {
        constexpr int GU = decltype(gc)::value;
        hipLaunchKernelGGL((k_spgemm_ub<GU, AR, BR>), dim3(std::min(blocks_for((int64_t)nrows * GU), kAtomicBlocks)),
                           dim3(kBlock), 0, s, ar, br, nrows, blk);
    });
    GW_HIP(hipGetLastError());
}

struct SpgShape {
    int G, S;
};

// Lanes per output row and the staging length.
inline SpgShape spg_shape(double avg_a_len, double avg_b_len) {
    const int G = spgemm_group(avg_a_len);
    // stage: about one and a half average segments, 32..512 contributions,
    // rounded to 16 (LDS per row bounds the resident waves: no larger stage
    // than needed)
    const int S = std::max(32, std::min(512, ((int)(1.5 * G * avg_b_len) + 15) / 16 * 16));
    return {G, S};
}

// Launch shape: groups per block, grid, LDS bytes, stage length.
template <class K>
void spg_launch(const SpgShape &sh, int32_t nrows, bool num, int hbits, K &&kern) {
    constexpr size_t kMaxLds = 64 * 1024;
    const int G = sh.G;
    const size_t H = (size_t)1 << hbits;
    const size_t per = num ? 12 : 4;
    int Sx = sh.S;
    while (Sx > 32 && (H + Sx) * per > kMaxLds) Sx /= 2;
    const size_t bytes_group = (H + Sx) * per;
    int groups = (int)std::min<size_t>(kBlock / G, std::max<size_t>(1, kMaxLds / bytes_group));
    if (groups >= dev::kWave / G) groups -= groups % (dev::kWave / G);  // whole waves
    unsigned grid = (unsigned)((nrows + groups - 1) / groups);
    if (grid == 0) grid = 1;
    kern(dim3(grid), dim3(groups * G), groups * bytes_group, Sx);
}

// Rows of at most this many distinct columns, from A-side rows of at most
// kLaneMaxALen entries on average, take one lane each (k_spgemm_lane): the
// level-0 products (the prolongator smoothing, at most 7 columns a row, and
// A P).  The numeric pass keeps the sums in registers too and stops at 16
// (32 columns and their sums spill); on the Galerkin levels, whose A rows
// hold ~30 entries, one lane walking them measured slower than the lane
// groups (prolongator smoothing 68 -> 91 us).
constexpr int kLaneCapSym = 32, kLaneCapNum = 16;
constexpr double kLaneMaxALen = 8.0;

template <bool NUM, class AR, class BR, class EPI>
void launch_spgemm_lane(int32_t cap, AR ar, BR br, EPI epi, int32_t nrows, int32_t *cnt, const int32_t *crow,
                        int32_t *ccol, double *cval, int32_t *overflow, hipStream_t s) {
    const dim3 g(blocks_for(std::max<int32_t>(nrows, 1))), b(kBlock);
    if (cap <= 8)
        hipLaunchKernelGGL((k_spgemm_lane<8, NUM, AR, BR, EPI>), g, b, 0, s, ar, br, nrows, cnt, crow, ccol, cval,
                           epi, overflow);
    else if (cap <= 16)
        hipLaunchKernelGGL((k_spgemm_lane<16, NUM, AR, BR, EPI>), g, b, 0, s, ar, br, nrows, cnt, crow, ccol, cval,
                           epi, overflow);
    else if constexpr (!NUM)
        hipLaunchKernelGGL((k_spgemm_lane<32, NUM, AR, BR, EPI>), g, b, 0, s, ar, br, nrows, cnt, crow, ccol, cval,
                           epi, overflow);
    GW_HIP(hipGetLastError());
}

template <class AR, class BR, class EPI>
void spgemm_symbolic(AR ar, BR br, EPI epi, int32_t nrows, int32_t ncols, double avg_a_len, double avg_b_len,
                     int32_t ub, Csr &C, int32_t *blk, hipStream_t s, double in_bytes) {
    const int64_t cap = std::min<int64_t>(ub, ncols);
    const int hb = std::min(pow2_bits_at_least(2 * std::max<int64_t>(cap, 1)), kMaxHashBits);
    C.alloc(nrows, ncols, 0);  // blk[1..5] were cleared by the product's spgemm_bound
    if (cap <= kLaneCapSym && avg_a_len <= kLaneMaxALen) {
        ProfScope ps(K_SPGEMM, in_bytes + 4.0 * (nrows + 1), s);
        launch_spgemm_lane<false>((int32_t)cap, ar, br, epi, nrows, C.rowptr.p, nullptr, nullptr, nullptr, blk + 2, s);
        scan_inclusive_i32(C.rowptr.p + 1, nrows, reinterpret_cast<int64_t *>(blk + 4), s, blk + 1);
        return;
    }
    const SpgShape sh = spg_shape(avg_a_len, avg_b_len);
#define SPG_SYM(GG)                                                                                           \
    hipLaunchKernelGGL((k_spgemm<GG, false, AR, BR, EPI>), g, b, shm, s, ar, br, nrows, hb, Sx, C.rowptr.p, \
                       (const int32_t *)nullptr, (int32_t *)nullptr, (double *)nullptr, epi, blk + 1, blk + 2)
    {
        ProfScope ps(K_SPGEMM, in_bytes + 4.0 * (nrows + 1), s);
        spg_launch(sh, nrows, false, hb, [&](dim3 g, dim3 b, size_t shm, int Sx) {
            switch (sh.G) {
                case 8: SPG_SYM(8); break;
                case 16: SPG_SYM(16); break;
                case 32: SPG_SYM(32); break;
                default: SPG_SYM(64); break;
            }
        });
        GW_HIP(hipGetLastError());
    }
#undef SPG_SYM
    scan_inclusive_i32(C.rowptr.p + 1, nrows, reinterpret_cast<int64_t *>(blk + 4), s, blk + 1);
}

// hblk: the host copy of blk after the symbolic pass.
template <class AR, class BR, class EPI>
void spgemm_numeric(AR ar, BR br, EPI epi, int32_t nrows, double avg_a_len, double avg_b_len, const int32_t *hblk,
                    Csr &C, int32_t *blk, hipStream_t s, double in_bytes) {
    int64_t nnz;
    std::memcpy(&nnz, &hblk[4], sizeof(nnz));
    const int32_t maxd = hblk[1];
    if (hblk[2]) fail(GW_EINVAL, "amg_setup: a Galerkin row has more than 4096 distinct columns");
    GW_REQUIRE(nnz < INT32_MAX, "amg_setup: operator exceeds 2^31 nonzeros");
    C.nnz = nnz;
    C.col.alloc((size_t)nnz);
    C.val.alloc((size_t)nnz);
    if (maxd <= kLaneCapNum && avg_a_len <= kLaneMaxALen) {
        ProfScope ps(K_SPGEMM, in_bytes + 4.0 * (nrows + 1) + 12.0 * (double)nnz, s);
        launch_spgemm_lane<true>(maxd, ar, br, epi, nrows, nullptr, C.rowptr.p, C.col.p, C.val.p, blk + 2, s);
        return;
    }
    // numeric table: at least 1.5 slots per column of the longest row
    const int hbn = std::min(pow2_bits_at_least((int64_t)(1.5 * std::max<int32_t>(maxd, 1))), kMaxHashBits);
    const SpgShape sh = spg_shape(avg_a_len, avg_b_len);
#define SPG_NUM(GG)                                                                                        \
    hipLaunchKernelGGL((k_spgemm<GG, true, AR, BR, EPI>), g, b, shm, s, ar, br, nrows, hbn, Sx,          \
                       (int32_t *)nullptr, C.rowptr.p, C.col.p, C.val.p, epi, blk + 1, blk + 2)
    {
        ProfScope ps(K_SPGEMM, in_bytes + 4.0 * (nrows + 1) + 12.0 * (double)nnz, s);
        spg_launch(sh, nrows, true, hbn, [&](dim3 g, dim3 b, size_t shm, int Sx) {
            switch (sh.G) {
                case 8: SPG_NUM(8); break;
                case 16: SPG_NUM(16); break;
                case 32: SPG_NUM(32); break;
                default: SPG_NUM(64); break;
            }
        });
        GW_HIP(hipGetLastError());
    }
#undef SPG_NUM
}

// Device words of one level read back together at a few host reads.
//   [0..1] strength-graph nnz, [2] pattern-symmetry misses (SA) or [2..3]
//   P nnz (RS), [4..5] aggregates / coarse points, [6..7] the spectral
//   bound's bits (SA), [8..15] P, [16..23] AP, [24..31] A_c (each an spgemm
//   blk).
constexpr int kLevelWords = 32;
constexpr int kMaxMisRounds = 4096;
struct LevelReads {
    DBuf<int32_t> d;
    int32_t h[kLevelWords] = {};
    // the read words, then the per-round "undecided left" flags of the
    // MIS-2 / PMIS rounds, cleared by one launch
    explicit LevelReads(hipStream_t s) : d(kLevelWords + kMaxMisRounds + 1) {
        fill_i32(d.p, 0, kLevelWords + kMaxMisRounds + 1, s);
    }
    int32_t *und() { return d.p + kLevelWords; }
    int32_t *miss() { return d.p + 2; }  // pattern-symmetry misses (smoothed aggregation)
    unsigned long long *rho() { return reinterpret_cast<unsigned long long *>(d.p + 6); }  // words 6..7
    int32_t *blk(int k) { return d.p + 8 + 8 * k; }  // 0: P, 1: AP, 2: A_c
    const int32_t *hblk(int k) const { return h + 8 + 8 * k; }
    int64_t *total(int word) { return reinterpret_cast<int64_t *>(d.p + word); }
    int64_t h64(int word) const {
        int64_t v;
        std::memcpy(&v, h + word, sizeof(v));
        return v;
    }
    // Copy the words (and `extra_bytes` from `extra` behind them) to the host
    // in one synchronisation.
    void sync(hipStream_t s, const void *extra = nullptr, size_t extra_bytes = 0, void *extra_out = nullptr) {
        char *stage = static_cast<char *>(host_stage());
        static_assert(kLevelWords * sizeof(int32_t) + 64 <= kHostStageBytes, "level words fit the pinned stage");
        GW_HIP(hipMemcpyAsync(stage, d.p, sizeof(h), hipMemcpyDeviceToHost, s));
        if (extra_bytes) GW_HIP(hipMemcpyAsync(stage + sizeof(h), extra, extra_bytes, hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        std::memcpy(h, stage, sizeof(h));
        if (extra_bytes) std::memcpy(extra_out, stage + sizeof(h), extra_bytes);
    }
};

void csr_diag(const CsrView &A, double *diag, hipStream_t s) {
    with_group(mean_row(A.nnz, A.n), [&](auto gc) {
        constexpr int G = decltype(gc)::value;
        hipLaunchKernelGGL((k_diag<G>), dim3(blocks_for((int64_t)A.n * G)), dim3(kBlock), 0, s, A, diag);
    });
    GW_HIP(hipGetLastError());
}

}  // namespace

void launch_csr_check(const CsrView &A, double *diag, int32_t *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_csr_check, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, diag, bad, 1);
    GW_HIP(hipGetLastError());
}

// Transposes of at least this many entries, with at least kRxMinPerCol of
// them per column, take the radix sort; the others the count / fill / rank
// path (fewer launches, and its atomics are cheap when few entries share a
// column: 133 us against 236 us for the 1M-row upwind operator, about 4
// entries a column; the prolongator of the 1M-cell flow hierarchy, 38 a
// column, 350 us against 144 us).
constexpr int64_t kRxMinEntries = 1 << 17;
constexpr int64_t kRxMinPerCol = 6;

static void transpose_radix(const CsrView &A, Csr &T, hipStream_t s, int64_t *scratch_total) {
    const int64_t nnz = A.nnz;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)A.ncols) ++bits;
    const int npass = (bits + kRxMaxBits - 1) / kRxMaxBits;
    const int64_t ntiles = (nnz + kRxTile - 1) / kRxTile;
    const int nd_max = 1 << ((bits + npass - 1) / npass);
    DBuf<int32_t> rowid((size_t)nnz), k0((size_t)nnz), r0(npass > 1 ? (size_t)nnz : 0), k1((size_t)nnz),
        r1(npass > 2 ? (size_t)nnz : 0), cnt((size_t)nd_max * ntiles + 1);
    DBuf<double> v0(npass > 1 ? (size_t)nnz : 0), v1(npass > 2 ? (size_t)nnz : 0);
    const int G = lane_group_for(A.n ? (double)nnz / (double)A.n : 0.0);
    auto rowids = [&](auto gc) {
        constexpr int GG = decltype(gc)::value;
        hipLaunchKernelGGL((k_rx_rowid<GG>), dim3(blocks_for((int64_t)A.n * GG)), dim3(kBlock), 0, s, A, rowid.p);
    };
    switch (G) {
        case 1: rowids(std::integral_constant<int, 1>()); break;
        case 4: rowids(std::integral_constant<int, 4>()); break;
        case 16: rowids(std::integral_constant<int, 16>()); break;
        default: rowids(std::integral_constant<int, 64>()); break;
    }
    fill_i32(cnt.p, 0, 1, s);
    const int32_t *kin = A.col, *rin = rowid.p;
    const double *vin = A.val;
    int shift = 0;
    const int32_t *sorted_keys = nullptr;
    for (int p = 0; p < npass; ++p) {
        const int b = bits / npass + (p < bits % npass ? 1 : 0);
        const bool last = p == npass - 1;
        // outputs: the sets alternate (k0/r0/v0, k1/r1/v1); the last pass
        // writes rows and values straight into T
        int32_t *ko = (p % 2 == 0) ? k0.p : k1.p;
        int32_t *ro = last ? T.col.p : (p % 2 == 0 ? r0.p : r1.p);
        double *vo = last ? T.val.p : (p % 2 == 0 ? v0.p : v1.p);
        const int64_t nc = ((int64_t)1 << b) * ntiles;
        hipLaunchKernelGGL(k_rx_hist, dim3((unsigned)ntiles), dim3(kBlock), 0, s, kin, nnz, shift, b, cnt.p, ntiles);
        scan_inclusive_i32(cnt.p + 1, nc, scratch_total, s);
        hipLaunchKernelGGL(k_rx_scatter, dim3((unsigned)ntiles), dim3(kBlock), 0, s, kin, rin, vin, nnz, shift, b,
                           cnt.p, ntiles, ko, ro, vo);
        kin = ko;
        rin = ro;
        vin = vo;
        sorted_keys = ko;
        shift += b;
    }
    hipLaunchKernelGGL(k_rx_rowptr, dim3(blocks_for(nnz + 1)), dim3(kBlock), 0, s, sorted_keys, nnz, A.ncols,
                       T.rowptr.p);
    GW_HIP(hipGetLastError());
}

void transpose(const CsrView &A, Csr &T, hipStream_t s, int64_t *scratch_total) {
    ProfScope ps(K_TRANSPOSE, 24.0 * A.nnz + 4.0 * ((double)A.n + A.ncols + 2), s);
    T.alloc(A.ncols, A.n, A.nnz);
    if (A.nnz >= kRxMinEntries && A.nnz >= kRxMinPerCol * (int64_t)A.ncols) {
        transpose_radix(A, T, s, scratch_total);
        return;
    }
    fill_i32(T.rowptr.p, 0, (int64_t)A.ncols + 1, s);
    if (A.nnz > 0) {
        unsigned g = std::min<unsigned>(blocks_for(A.nnz, 4), 65536);
        hipLaunchKernelGGL(k_tr_count, dim3(g), dim3(kBlock), 0, s, A.col, A.nnz, T.rowptr.p);
    }
    scan_inclusive_i32(T.rowptr.p + 1, A.ncols, scratch_total, s);
    DBuf<int32_t> fill((size_t)A.ncols + 1), rowid((size_t)std::max<int64_t>(A.nnz, 1)),
        tcol((size_t)std::max<int64_t>(A.nnz, 1));
    DBuf<double> tval((size_t)std::max<int64_t>(A.nnz, 1));
    fill_i32(fill.p, 0, A.ncols, s);
    const int G = lane_group_for(A.n ? (double)A.nnz / (double)A.n : 0.0);
    auto fill_rows = [&](auto gc) {
        constexpr int GG = decltype(gc)::value;
        hipLaunchKernelGGL((k_tr_fill<GG>), dim3(blocks_for((int64_t)A.n * GG)), dim3(kBlock), 0, s, A, T.rowptr.p,
                           fill.p, tcol.p, tval.p, rowid.p);
    };
    switch (G) {
        case 1: fill_rows(std::integral_constant<int, 1>()); break;
        case 4: fill_rows(std::integral_constant<int, 4>()); break;
        case 16: fill_rows(std::integral_constant<int, 16>()); break;
        default: fill_rows(std::integral_constant<int, 64>()); break;
    }
    if (A.nnz > 0)
        hipLaunchKernelGGL(k_tr_sort, dim3(blocks_for(A.nnz)), dim3(kBlock), 0, s, T.rowptr.p, rowid.p, tcol.p,
                           tval.p, A.nnz, T.col.p, T.val.p);
    GW_HIP(hipGetLastError());
}

namespace {

// R = P^T and A_{l+1} = R (A P) for a level whose P is built; the row bound
// of A P must already be in rd (blk 1).  The symbolic pass of A P and the row
// bound of R (A P) share one read.
void galerkin(amg_hierarchy *H, int l, int64_t nc, LevelReads &rd, hipStream_t s) {
    Level &Lv = H->L[l];
    const CsrView A = view(Lv.A);
    const int32_t n = A.n;
    // R = P^T on the side stream, overlapping the symbolic pass of A P
    SideJob tr;
    tr.run(s, [&](hipStream_t q) {
        DBuf<int64_t> total(1);
        transpose(view(Lv.P), Lv.R, q, total.p);
    });
    Csr AP;
    const double arow = (double)A.nnz / std::max<int32_t>(n, 1);
    const double pavg = (double)Lv.P.nnz / std::max<int32_t>(n, 1);
    const double ravg = (double)Lv.R.nnz / std::max<int64_t>(nc, 1);
    const ARowCsr a_side{A.rowptr, A.col, A.val};
    const BCsr p_side{Lv.P.rowptr.p, Lv.P.col.p, Lv.P.val.p};
    // rows read by a pass: row pointers, then columns (symbolic) or columns
    // and values (numeric)
    auto rows = [](int64_t nr, int64_t nz, double per) { return 4.0 * (nr + 1) + per * (double)nz; };
    const int64_t np = Lv.P.nnz, nr_ = Lv.R.nnz;
    spgemm_symbolic(a_side, p_side, EpiIdentity{}, n, (int32_t)nc, arow, pavg, rd.hblk(1)[0], AP, rd.blk(1), s,
                    rows(n, A.nnz, 4) + rows(n, np, 4));
    tr.join(s);
    const ARowCsr r_side{Lv.R.rowptr.p, Lv.R.col.p, Lv.R.val.p};
    spgemm_bound(r_side, BCsr{AP.rowptr.p, nullptr, nullptr}, (int32_t)nc, ravg, rd.blk(2), s,
                 rows(nc, nr_, 4) + 4.0 * (n + 1));
    rd.sync(s);
    spgemm_numeric(a_side, p_side, EpiIdentity{}, n, arow, pavg, rd.hblk(1), AP, rd.blk(1), s,
                   rows(n, A.nnz, 12) + rows(n, np, 12));
    Level &Nx = H->L[l + 1];
    const double apavg = (double)AP.nnz / std::max<int32_t>(n, 1);
    const BCsr ap_side{AP.rowptr.p, AP.col.p, AP.val.p};
    spgemm_symbolic(r_side, ap_side, EpiIdentity{}, (int32_t)nc, (int32_t)nc, ravg, apavg, rd.hblk(2)[0], Nx.A,
                    rd.blk(2), s, rows(nc, nr_, 4) + rows(n, AP.nnz, 4));
    rd.sync(s);
    spgemm_numeric(r_side, ap_side, EpiIdentity{}, (int32_t)nc, ravg, apavg, rd.hblk(2), Nx.A, rd.blk(2), s,
                   rows(nc, nr_, 12) + rows(n, AP.nnz, 12));
}

// Ruge-Stueben level: strength with the threshold kept on every level, PMIS
// rounds batched between host reads (as the MIS-2 rounds), coarse indices,
// direct interpolation, then the Galerkin product.
void build_level_rs(amg_hierarchy *H, int l, hipStream_t s, bool *is_coarsest) {
    Level &Lv = H->L[l];
    const CsrView A = view(Lv.A);
    const int32_t n = A.n;
    const amg_params &prm = H->prm;
    const unsigned nb = blocks_for(n);
    LevelReads rd(s);

    Csr S, St;
    S.n = S.ncols = n;
    S.rowptr.alloc((size_t)n + 1);
    fill_i32(S.rowptr.p, 0, 1, s);
    S.col.alloc((size_t)std::max<int64_t>(A.nnz, 1));  // a subset of A's off-diagonal entries
    DBuf<uint8_t> strong((size_t)std::max<int64_t>(A.nnz, 1));
    {
        ProfScope ps(K_STRENGTH, (double)A.nnz * 25 + n * 8.0, s);
        hipLaunchKernelGGL((k_rs_strength<false>), dim3(nb), dim3(kBlock), 0, s, A, prm.eps_strong, S.rowptr.p,
                           (const int32_t *)nullptr, (int32_t *)nullptr, (uint8_t *)nullptr);
        scan_inclusive_i32(S.rowptr.p + 1, n, rd.total(0), s);
        hipLaunchKernelGGL((k_rs_strength<true>), dim3(nb), dim3(kBlock), 0, s, A, prm.eps_strong,
                           (int32_t *)nullptr, S.rowptr.p, S.col.p, strong.p);
        GW_HIP(hipGetLastError());
    }
    rd.sync(s);
    S.nnz = rd.h64(0);
    Lv.nnz_s = S.nnz;
    S.val.alloc((size_t)std::max<int64_t>(S.nnz, 1));
    fill_f64(S.val.p, 1.0, S.nnz, s);
    DBuf<int64_t> total(1);
    transpose(view(S), St, s, total.p);

    // PMIS rounds; und[r] = some point was undecided before round r
    DBuf<double> w(n);
    DBuf<int32_t> cf(n), newc(n);
    constexpr int kMaxRounds = kMaxMisRounds, kBatch = 12, kLate = 4;
    int32_t *und = rd.und();
    {
        ProfScope ps(K_MIS2, n * 20.0, s);
        hipLaunchKernelGGL(k_pmis_init, dim3(nb), dim3(kBlock), 0, s, St.rowptr.p, n, level_salt(prm.seed, l), w.p,
                           cf.p, und);
        GW_HIP(hipGetLastError());
    }
    int rounds = 0;
    for (;;) {
        // a first batch of kBatch rounds covers most levels; later ones
        // take kLate, so a level needing a few more rounds launches few
        // no-op rounds
        const int batch = rounds == 0 ? kBatch : kLate;
        GW_REQUIRE(rounds + batch <= kMaxRounds, "amg_setup: PMIS did not terminate");
        for (int b = 0; b < batch; ++b) {
            const int r = rounds + b;
            ProfScope ps(K_MIS2, (double)S.nnz * 16 + n * 24.0, s);
            hipLaunchKernelGGL(k_pmis_c, dim3(nb), dim3(kBlock), 0, s, S.rowptr.p, S.col.p, St.rowptr.p, St.col.p, n,
                               w.p, cf.p, newc.p);
            hipLaunchKernelGGL(k_pmis_f, dim3(nb), dim3(kBlock), 0, s, S.rowptr.p, S.col.p, n, newc.p, cf.p,
                               und + r + 1);
        }
        GW_HIP(hipGetLastError());
        int32_t flags[kBatch + 1];
        rd.sync(s, und + rounds, sizeof(int32_t) * (batch + 1), flags);
        if (flags[0] == 0) break;  // nothing was undecided before this batch
        int b = 0;
        while (b < batch && flags[1 + b] > 0) ++b;
        if (b < batch) {
            rounds += b + 1;
            break;
        }
        rounds += batch;
    }
    Lv.mis_rounds = rounds;
    St = Csr();
    w.release();

    // coarse indices, the rows of P, and the row bound of A P, one read
    DBuf<int32_t> rank((size_t)n + 1);
    Lv.agg.alloc(n);
    Csr &P = Lv.P;
    P.n = n;
    P.rowptr.alloc((size_t)n + 1);
    fill_i32(P.rowptr.p, 0, 1, s);
    {
        ProfScope ps(K_AGGREGATE, (double)A.nnz * 13 + n * 20.0, s);
        hipLaunchKernelGGL(k_c_flags, dim3(nb), dim3(kBlock), 0, s, cf.p, n, rank.p);
        scan_inclusive_i32(rank.p + 1, n, rd.total(4), s);
        hipLaunchKernelGGL(k_c_index, dim3(nb), dim3(kBlock), 0, s, cf.p, rank.p, n, Lv.agg.p);
        hipLaunchKernelGGL((k_rs_interp<false>), dim3(nb), dim3(kBlock), 0, s, A, strong.p, cf.p, Lv.agg.p,
                           P.rowptr.p, (const int32_t *)nullptr, (int32_t *)nullptr, (double *)nullptr);
        scan_inclusive_i32(P.rowptr.p + 1, n, rd.total(2), s);
        GW_HIP(hipGetLastError());
    }
    const double arow = (double)A.nnz / std::max<int32_t>(n, 1);
    spgemm_bound(ARowCsr{A.rowptr, A.col, A.val}, BCsr{P.rowptr.p, nullptr, nullptr}, n, arow, rd.blk(1), s,
                 4.0 * (n + 1) + 4.0 * (double)A.nnz + 4.0 * (n + 1));
    rd.sync(s);
    const int64_t nc = rd.h64(4);
    Lv.nc = (int32_t)nc;
    if (nc == 0 || (double)nc > 0.9 * (double)n) {
        *is_coarsest = true;
        Lv.agg.release();
        Lv.P = Csr();
        Lv.nc = 0;
        return;
    }
    P.ncols = (int32_t)nc;
    P.nnz = rd.h64(2);
    P.col.alloc((size_t)std::max<int64_t>(P.nnz, 1));
    P.val.alloc((size_t)std::max<int64_t>(P.nnz, 1));
    {
        ProfScope ps(K_SETUP_MISC, (double)A.nnz * 13 + P.nnz * 12.0 + n * 12.0, s);
        hipLaunchKernelGGL((k_rs_interp<true>), dim3(nb), dim3(kBlock), 0, s, A, strong.p, cf.p, Lv.agg.p,
                           (int32_t *)nullptr, P.rowptr.p, P.col.p, P.val.p);
        GW_HIP(hipGetLastError());
    }
    // no prolongator smoothing: omega_P is 0
    Lv.omega_dev.alloc(1);
    fill_f64(Lv.omega_dev.p, 0.0, 1, s);
    galerkin(H, l, nc, rd, s);
}

}  // namespace

// Build level l+1 from level l, or mark l as the coarsest.  Returns through
// *is_coarsest whether level l ended the hierarchy.
void build_level(amg_hierarchy *H, int l, hipStream_t s, bool *is_coarsest) {
    Staging st;
    Level &Lv = H->L[l];
    const int32_t n = Lv.A.n;
    const amg_params &prm = H->prm;
    const int maxl = std::max(1, std::min(prm.max_levels, 32));
    *is_coarsest = false;
    if (n <= prm.n_coarse || l == maxl - 1) {
        *is_coarsest = true;
        return;
    }
    GW_REQUIRE(n < (1 << 30), "amg_setup: at most 2^30 rows per level");
    if (prm.coarsening == GW_COARSEN_RS) {
        build_level_rs(H, l, s, is_coarsest);
        return;
    }
    const CsrView A = view(Lv.A);
    double eps2 = prm.eps_strong * prm.eps_strong;
    for (int k = 0; k < l; ++k) eps2 = eps2 * 0.25;

    DBuf<double> diag(n), dF(n), sw;
    DBuf<int64_t> total(1);
    csr_diag(A, diag.p, s);
    LevelReads rd(s);

    // strength graph on A and A^T (A^T from A's own pattern when that is
    // symmetric, as for the flow operator and all its Galerkin products)
    Csr T;
    DBuf<double> tval_sym;
    CsrView Tv{};
    bool sym = false;
    if (H->sym_pattern != 0) {
        tval_sym.alloc((size_t)std::max<int64_t>(A.nnz, 1));
        int32_t *miss = rd.miss();
        {
            ProfScope ps(K_TRANSPOSE, (double)A.nnz * 24, s);
            with_group(mean_row(A.nnz, n), [&](auto gc) {
                constexpr int G = decltype(gc)::value;
                hipLaunchKernelGGL((k_sym_transpose<G>), dim3(std::min(blocks_for((int64_t)n * G), kAtomicBlocks)),
                                   dim3(kBlock), 0, s, A, tval_sym.p, miss);
            });
            GW_HIP(hipGetLastError());
        }
        if (H->sym_pattern == 1) {
            // a Galerkin product R A P with R = P^T (cancelled entries kept)
            // has a symmetric pattern when A's is: no read here, the miss
            // word is checked with the level's next read
            sym = true;
        } else {
            const int32_t w = st.read(miss, s);
            sym = (w & 1) == 0;
            H->sym_pattern = sym ? 1 : 0;
            if (l == 0) H->sym_values = w == 0 ? 1 : 0;
        }
    }
    const bool check_sym = sym && l > 0;
    if (sym) {
        Tv = CsrView{n, n, A.nnz, A.rowptr, A.col, tval_sym.p};
    } else {
        tval_sym.release();
        transpose(A, T, s, total.p);
        Tv = view(T);
    }
    Csr S;  // pattern only: col + weights in sw
    S.n = S.ncols = n;
    S.rowptr.alloc((size_t)n + 1);
    fill_i32(S.rowptr.p, 0, 1, s);
    DBuf<uint8_t> strongA((size_t)std::max<int64_t>(A.nnz, 1));
    DBuf<int32_t> code;  // per-entry outcomes of the grouped counting pass
    const int Gs = lane_group_for(n ? (double)A.nnz / (double)n : 0.0);
    auto launch_strength = [&](bool fill) {
        auto grp = [&](auto gc) {
            constexpr int GG = decltype(gc)::value;
            const dim3 grid(blocks_for((int64_t)n * GG));
            if (!fill) code.alloc((size_t)std::max<int64_t>(A.nnz + Tv.nnz, 1));
            if (fill)
                hipLaunchKernelGGL((k_strength_grp<GG, true>), grid, dim3(kBlock), 0, s, A, Tv, diag.p, eps2,
                                   (int32_t *)nullptr, S.rowptr.p, S.col.p, sw.p, strongA.p, dF.p, code.p);
            else
                hipLaunchKernelGGL((k_strength_grp<GG, false>), grid, dim3(kBlock), 0, s, A, Tv, diag.p, eps2,
                                   S.rowptr.p, (const int32_t *)nullptr, (int32_t *)nullptr, (double *)nullptr,
                                   (uint8_t *)nullptr, (double *)nullptr, code.p);
        };
        if (sym) {
            // A^T lives on A's own pattern: classify in place
            auto symk = [&](auto gc) {
                constexpr int GG = decltype(gc)::value;
                const dim3 grid(blocks_for((int64_t)n * GG));
                if (fill)
                    hipLaunchKernelGGL((k_strength_sym<GG, true>), grid, dim3(kBlock), 0, s, A, tval_sym.p, diag.p,
                                       eps2, (int32_t *)nullptr, S.rowptr.p, S.col.p, sw.p, strongA.p, dF.p);
                else
                    hipLaunchKernelGGL((k_strength_sym<GG, false>), grid, dim3(kBlock), 0, s, A, tval_sym.p, diag.p,
                                       eps2, S.rowptr.p, (const int32_t *)nullptr, (int32_t *)nullptr,
                                       (double *)nullptr, (uint8_t *)nullptr, (double *)nullptr);
            };
            with_group(mean_row(A.nnz, n), symk);
            return;
        }
        switch (Gs) {
            case 1:
                if (fill)
                    hipLaunchKernelGGL(k_strength_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, Tv, diag.p, eps2,
                                       S.rowptr.p, S.col.p, sw.p, strongA.p, dF.p);
                else
                    hipLaunchKernelGGL(k_strength_count, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, Tv, diag.p,
                                       eps2, S.rowptr.p);
                break;
            case 4: grp(std::integral_constant<int, 4>()); break;
            case 16: grp(std::integral_constant<int, 16>()); break;
            default: grp(std::integral_constant<int, 64>()); break;
        }
    };
    {
        ProfScope ps(K_STRENGTH, (double)A.nnz * 24 + n * 16.0, s);
        launch_strength(false);
        GW_HIP(hipGetLastError());
    }
    // the graph's size is read later, with the MIS-2 flags: its arrays take
    // the bound (A's off-diagonal pattern, and that of A^T when not symmetric).
    // Its longest row goes to the prolongator product's row bound: a row of
    // the filtered A (the diagonal and A's strong entries, a subset of the
    // graph's row) adds at most that many + 1 contributions, one per
    // aggregate met.
    scan_inclusive_i32(S.rowptr.p + 1, n, rd.total(0), s, rd.blk(0));
    const int64_t s_cap = std::max<int64_t>(sym ? A.nnz : A.nnz + T.nnz, 1);
    S.col.alloc((size_t)s_cap);
    sw.alloc((size_t)s_cap);
    {
        ProfScope ps(K_STRENGTH, (double)A.nnz * 25 + n * 24.0, s);
        launch_strength(true);
        GW_HIP(hipGetLastError());
    }
    code.release();

    // MIS-2 rounds, batched between host reads; a round after the last
    // decision is a no-op.  After each batch the aggregates are formed from
    // the states reached, and read back with the round flags: they are final
    // when the rounds have ended.
    DBuf<uint32_t> state(n);
    DBuf<uint64_t> m1(n);
    DBuf<uint8_t> done(n);
    constexpr int kMaxRounds = kMaxMisRounds, kBatch = 12, kLate = 4;
    int32_t *und = rd.und();
    const uint32_t salt = level_salt(prm.seed, l);
    {
        ProfScope ps(K_MIS2, n * 8.0, s);
        hipLaunchKernelGGL(k_mis_init, dim3(std::min(blocks_for(n), kAtomicBlocks)), dim3(kBlock), 0, s, S.rowptr.p, n,
                           state.p, done.p, und);
        GW_HIP(hipGetLastError());
    }
    // lanes per row from A's off-diagonal row length (the graph's own size is
    // not on the host yet; it is a subset of those entries)
    const double srow_mean = mean_row(A.nnz - n, n);
    DBuf<int32_t> ids((size_t)n + 1), agg1(n);
    Lv.agg.alloc(n);
    ARowFiltered af{A.rowptr, A.col, A.val, strongA.p, dF.p};
    BTent bt{Lv.agg.p};
    const double arow = (double)A.nnz / std::max<int32_t>(n, 1);
    int rounds = 0;
    for (;;) {
        // a first batch of kBatch rounds covers most levels; later ones
        // take kLate, so a level needing a few more rounds launches few
        // no-op rounds
        const int batch = rounds == 0 ? kBatch : kLate;
        GW_REQUIRE(rounds + batch <= kMaxRounds, "amg_setup: MIS-2 did not terminate");
        for (int b = 0; b < batch; ++b) {
            int r = rounds + b;
            ProfScope ps(K_MIS2, (double)A.nnz * 8 + n * 20.0, s);
            with_group(srow_mean, [&](auto gc) {
                constexpr int G = decltype(gc)::value;
                const dim3 grid(blocks_for((int64_t)n * G));
                hipLaunchKernelGGL((k_mis_m1<G>), grid, dim3(kBlock), 0, s, S.rowptr.p, S.col.p, n, state.p, salt,
                                   m1.p, done.p, und + r);
                hipLaunchKernelGGL((k_mis_m2<G>), grid, dim3(kBlock), 0, s, S.rowptr.p, S.col.p, n, state.p, salt,
                                   m1.p, und + r, und + r + 1);
            });
        }
        GW_HIP(hipGetLastError());
        {
            ProfScope ps(K_AGGREGATE, (double)A.nnz * 16 + n * 24.0, s);
            hipLaunchKernelGGL(k_root_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, state.p, n, ids.p);
            scan_inclusive_i32(ids.p + 1, n, rd.total(4), s);
            with_group(srow_mean, [&](auto gc) {
                constexpr int G = decltype(gc)::value;
                const dim3 grid(blocks_for((int64_t)n * G));
                hipLaunchKernelGGL((k_agg_pass1<G>), grid, dim3(kBlock), 0, s, S.rowptr.p, S.col.p, n, state.p, ids.p,
                                   agg1.p);
                hipLaunchKernelGGL((k_agg_pass2<G>), grid, dim3(kBlock), 0, s, S.rowptr.p, S.col.p, sw.p, n, agg1.p,
                                   Lv.agg.p);
            });
            GW_HIP(hipGetLastError());
        }
        int32_t flags[kBatch + 1];
        rd.sync(s, und + rounds, sizeof(int32_t) * (batch + 1), flags);
        if (flags[0] == 0) break;  // nothing was undecided before this batch
        int b = 0;
        while (b < batch && flags[1 + b] > 0) ++b;
        if (b < batch) {
            rounds += b + 1;
            break;
        }
        rounds += batch;
    }
    Lv.mis_rounds = rounds;
    if (check_sym && (rd.h[2] & 1) != 0) fail(GW_EDEVICE, "amg_setup: a Galerkin level lost its symmetric pattern");
    m1.release();
    done.release();
    S.nnz = rd.h64(0);
    Lv.nnz_s = S.nnz;
    T = Csr();
    tval_sym.release();
    const int64_t nc = rd.h64(4);
    Lv.nc = (int32_t)nc;
    if (nc == 0 || (double)nc > 0.9 * (double)n) {
        *is_coarsest = true;
        Lv.agg.release();
        Lv.nc = 0;
        return;
    }

    // smoothed prolongator
    unsigned long long *rho_bits = rd.rho();
    DBuf<double> &omega = Lv.omega_dev;  // read back once the hierarchy is built
    omega.alloc(1);
    {
        ProfScope ps(K_SETUP_MISC, (double)A.nnz * 8 + n * 8.0, s);
        if (mean_row(A.nnz, n) <= 8.0)
            hipLaunchKernelGGL((k_rho<8>), dim3(blocks_for(n)), dim3(kBlock), 0, s, A, diag.p, rho_bits);
        else
            hipLaunchKernelGGL((k_rho<16>), dim3(blocks_for(n)), dim3(kBlock), 0, s, A, diag.p, rho_bits);
        hipLaunchKernelGGL(k_omega, dim3(1), dim3(64), 0, s, rho_bits, omega.p);
        GW_HIP(hipGetLastError());
    }
    EpiSmoothP ep{Lv.agg.p, dF.p, diag.p, omega.p};
    // P: symbolic pass, then the row bound of A P (it needs only P's row
    // pointers), one read for both
    spgemm_symbolic(af, bt, ep, n, (int32_t)nc, arow, 1.0, rd.hblk(0)[0] + 1, Lv.P, rd.blk(0), s,
                    4.0 * (n + 1) + 5.0 * (double)A.nnz + 4.0 * n);
    spgemm_bound(ARowCsr{A.rowptr, A.col, A.val}, BCsr{Lv.P.rowptr.p, nullptr, nullptr}, n, arow, rd.blk(1), s,
                 4.0 * (n + 1) + 4.0 * (double)A.nnz + 4.0 * (n + 1));
    rd.sync(s);
    // numeric: values too, the aggregate map, the lumped and the smoothing diagonals
    spgemm_numeric(af, bt, ep, n, arow, 1.0, rd.hblk(0), Lv.P, rd.blk(0), s,
                   4.0 * (n + 1) + 13.0 * (double)A.nnz + 4.0 * n + 16.0 * n);

    galerkin(H, l, nc, rd, s);
}

void make_smoother(amg_hierarchy *H, int l, hipStream_t s) {
    Level &Lv = H->L[l];
    const CsrView A = view(Lv.A);
    DBuf<double> diag(A.n);
    csr_diag(A, diag.p, s);
    Lv.M.alloc(A.n);
    ProfScope ps(K_SETUP_MISC, (double)A.nnz * 12 + A.n * 16.0, s);
    const int spai0 = H->prm.smoother == GW_SMOOTHER_SPAI0 ? 1 : 0;
    if (mean_row(A.nnz, A.n) <= 8.0)
        hipLaunchKernelGGL((k_smoother_diag<8>), dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, diag.p, spai0,
                           H->prm.omega, Lv.M.p);
    else
        hipLaunchKernelGGL((k_smoother_diag<16>), dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, diag.p, spai0,
                           H->prm.omega, Lv.M.p);
    GW_HIP(hipGetLastError());
}

void convert_level_fp32(amg_hierarchy *H, int l, hipStream_t s) {
    Level &Lv = H->L[l];
    auto conv = [&](const DBuf<double> &x, DBuf<float> &y) {
        y.alloc(x.n);
        if (!x.n) return;
        unsigned g = std::min<unsigned>(blocks_for((int64_t)x.n, 4), 65536);
        hipLaunchKernelGGL(k_to_f32, dim3(g), dim3(kBlock), 0, s, x.p, y.p, (int64_t)x.n);
    };
    conv(Lv.A.val, Lv.A.val32);
    if (Lv.P.n) conv(Lv.P.val, Lv.P.val32);
    if (Lv.R.n) conv(Lv.R.val, Lv.R.val32);
    if (Lv.M.n) conv(Lv.M, Lv.M32);
    GW_HIP(hipGetLastError());
}

// Dynamic LDS a workgroup of the LU may use for the matrix: the device's
// per-block limit (160 KB on gfx950, i.e. n <= 142) less the LU's own
// shared words.
static size_t lu_lds_bytes() {
    int dev = 0, v = 0;
    GW_HIP(hipGetDevice(&dev));
    GW_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return v > 1024 ? (size_t)(v - 1024) : 0;
}

CoarseJob::~CoarseJob() {
    if (side) (void)hipStreamSynchronize(side);
    if (ready) (void)hipEventDestroy(ready);
    if (done) (void)hipEventDestroy(done);
}

void start_coarsest(amg_hierarchy *H, int l, hipStream_t s, CoarseJob &job) {
    Level &Lv = H->L[l];
    const int32_t n = Lv.A.n;
    GW_REQUIRE(n <= 2048, "amg_setup: coarsening stalled at " + std::to_string(n) + " rows (> 2048)");
    H->nd = n;
    H->lu.alloc((size_t)n * n);
    H->inv.alloc((size_t)n * n);
    H->piv.alloc(n);
    job.status.alloc(1);
    GW_HIP(hipEventCreateWithFlags(&job.ready, hipEventDisableTiming));
    GW_HIP(hipEventCreateWithFlags(&job.done, hipEventDisableTiming));
    fill_i32(job.status.p, 0, 1, s);
    GW_HIP(hipEventRecord(job.ready, s));
    const hipStream_t q = side_stream();
    GW_HIP(hipStreamWaitEvent(q, job.ready, 0));
    job.side = q;
    int32_t *status = job.status.p;
    {
        ProfScope ps(K_COARSE_LU, (double)n * n * 24, q);
        hipLaunchKernelGGL(k_csr_to_dense, dim3(blocks_for((int64_t)n * dev::kWave)), dim3(kBlock), 0, q, view(Lv.A),
                           H->lu.p);
        const size_t lds = (size_t)n * n * sizeof(double);
        if (n <= kLuLdsSmall) {
            hipLaunchKernelGGL(k_dense_lu_lds<256>, dim3(1), dim3(256), lds, q, H->lu.p, n, H->piv.p, status);
        } else if (lds <= lu_lds_bytes()) {
            // past 64 KB of dynamic LDS the kernel has to ask for it
            GW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dense_lu_lds<512>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(k_dense_lu_lds<512>, dim3(1), dim3(512), lds, q, H->lu.p, n, H->piv.p, status);
        } else {
            // panels as wide as the LDS holds (n x nb doubles), at most 64
            int32_t nb = kLuPanelMax;
            while (nb > 1 && (size_t)n * nb * sizeof(double) > lu_lds_bytes()) nb /= 2;
            const size_t plds = (size_t)n * nb * sizeof(double);
            if (plds > 65536)
                GW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lu_panel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds));
            for (int32_t k0 = 0; k0 < n; k0 += nb) {
                const int32_t w = std::min(nb, n - k0), nt = n - k0 - w;
                hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(512), (size_t)(n - k0) * w * sizeof(double), q,
                                   H->lu.p, n, k0, w, H->piv.p, status);
                if (n - w > 0)
                    hipLaunchKernelGGL(k_lu_swap_u12, dim3((n - w + 63) / 64), dim3(64), 0, q, H->lu.p, n, k0, w,
                                       H->piv.p, status);
                if (nt > 0)
                    hipLaunchKernelGGL(k_lu_trail, dim3(blocks_for((int64_t)nt * nt)), dim3(kBlock), 0, q, H->lu.p,
                                       n, k0, w, status);
            }
        }
        GW_HIP(hipGetLastError());
    }
    {
        // skipped after a zero pivot (the pivots past it were never written)
        ProfScope ps(K_COARSE_LU, (double)n * n * 16, q);
        if (n <= 128)
            hipLaunchKernelGGL(k_lu_inverse_col, dim3(n), dim3(64), 0, q, H->lu.p, H->piv.p, n, H->inv.p, status);
        else
            hipLaunchKernelGGL(k_lu_inverse, dim3(n), dim3(64), 0, q, H->lu.p, H->piv.p, n, H->inv.p, status);
        GW_HIP(hipGetLastError());
    }
    GW_HIP(hipEventRecord(job.done, q));
}

void finish_coarsest(CoarseJob &job, hipStream_t s) {
    GW_HIP(hipStreamWaitEvent(s, job.done, 0));
    Staging st;
    if (st.read(job.status.p, s) != 0) fail(GW_SINGULAR, "amg_setup: zero pivot in the coarsest-level LU");
}

}  // namespace gw
