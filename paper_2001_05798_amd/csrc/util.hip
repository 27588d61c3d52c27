// Device-wide inclusive scan of int32 counts (used to turn row lengths into
// CSR row pointers and flags into ids) and small fill/copy helpers.
#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
// Up to this many tiles every block of the apply pass adds the sums of the
// tiles before its own (at most 8 KB, read from L2); past it a one-block
// pass forms the tiles' offsets first.
constexpr int64_t kScanDirectTiles = 1024;

// A wave scans a segment of contiguous elements in rounds of kSegRound: each
// round is loaded with one coalesced dword load per item (element k*64 + lane
// of the round), staged in LDS and read back in lane order (lane l takes
// elements 16l .. 16l+15), so a lane adds its own run sequentially and one
// wave scan joins the runs; the results go back through the stage and out
// with coalesced stores.  Stage index e sits at e + e/32 (no bank conflicts
// either way).
constexpr int kSegItems = 16;
constexpr int kSegRound = dev::kWave * kSegItems;
constexpr int kSegStage = kSegRound + kSegRound / 32;

__device__ __forceinline__ int stage_at(int e) { return e + (e >> 5); }

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Elements of the lane's column at and past `seg + lane` that lie before n,
// capped at `cap` (32-bit limits for the checked loads and stores).
__device__ __forceinline__ int seg_limit(int64_t n, int64_t seg, int lane, int cap) {
    const int64_t m = n - seg - lane;
    return m <= 0 ? 0 : (m >= cap ? cap : (int)m);
}

// x[j] = a[seg + j*64 + lane] for the R rounds of the segment at seg; entries
// at or past n read as 0.  FAST adds an unchecked path for whole segments
// (more code: kept out of the one-block kernel, whose code is fetched cold).
template <int R, bool FAST>
__device__ __forceinline__ void seg_load(const int32_t *__restrict__ a, int64_t n, int64_t seg, int lane,
                                         int32_t (&x)[R * kSegItems]) {
    const int32_t *p = a + seg + lane;
    if (FAST && seg + (int64_t)R * kSegRound <= n) {
#pragma unroll
        for (int j = 0; j < R * kSegItems; ++j) x[j] = p[j * dev::kWave];
    } else {
        const int lim = seg_limit(n, seg, lane, R * kSegRound);
#pragma unroll
        for (int j = 0; j < R * kSegItems; ++j) x[j] = j * dev::kWave < lim ? p[j * dev::kWave] : 0;
    }
}

// Stores the inclusive scan of the segment that seg_load read, plus carry
// (the sum of everything before the segment), into a[seg ...].  st is the
// wave's own stage of kSegStage entries.
template <int R, bool FAST>
__device__ __forceinline__ void seg_scan_store(int32_t *__restrict__ a, int64_t n, int64_t seg, int lane,
                                               const int32_t (&x)[R * kSegItems], int64_t carry,
                                               int32_t *__restrict__ st) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int k = 0; k < kSegItems; ++k) st[stage_at(k * dev::kWave + lane)] = x[r * kSegItems + k];
        __builtin_amdgcn_wave_barrier();
        int64_t run = 0;
#pragma unroll
        for (int k = 0; k < kSegItems; ++k) run += st[stage_at(lane * kSegItems + k)];
        const int64_t incl = dev::wave_scan_incl(run);
        int64_t acc = carry + incl - run;
#pragma unroll
        for (int k = 0; k < kSegItems; ++k) {
            const int e = stage_at(lane * kSegItems + k);
            acc += st[e];
            st[e] = (int32_t)acc;
        }
        __builtin_amdgcn_wave_barrier();
        const int64_t s0 = seg + (int64_t)r * kSegRound;
        int32_t *q = a + s0 + lane;
        if (FAST && s0 + kSegRound <= n) {
#pragma unroll
            for (int k = 0; k < kSegItems; ++k) q[k * dev::kWave] = st[stage_at(k * dev::kWave + lane)];
        } else {
            const int lim = seg_limit(n, s0, lane, kSegRound);
#pragma unroll
            for (int k = 0; k < kSegItems; ++k)
                if (k * dev::kWave < lim) q[k * dev::kWave] = st[stage_at(k * dev::kWave + lane)];
        }
        __builtin_amdgcn_wave_barrier();
        carry += readlane_i64(incl, dev::kWave - 1);
    }
}

// Per tile: the sum and the largest value (the latter only when bm != null).
// A wave reads one round of the tile (independent coalesced loads).
__global__ void __launch_bounds__(kScanThreads) k_scan_tile_sums(const int32_t *a, int64_t n, int64_t *bs,
                                                                 int32_t *bm) {
    constexpr int nw = kScanThreads / dev::kWave;
    static_assert(kScanTile == nw * kSegRound, "one round per wave");
    __shared__ int64_t sm[nw];
    __shared__ int32_t smx[nw];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t seg = (int64_t)blockIdx.x * kScanTile + (int64_t)w * kSegRound;
    int32_t x[kSegItems];
    seg_load<1, true>(a, n, seg, lane, x);
    const int lim = seg_limit(n, seg, lane, kSegRound);
    int64_t s = 0;
    int32_t mx = INT32_MIN;
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        s += x[j];
        if (j * dev::kWave < lim) mx = x[j] > mx ? x[j] : mx;
    }
    s = dev::block_sum(s, sm);
    if (bm) mx = dev::block_max(mx, smx);
    if (threadIdx.x == 0) {
        bs[blockIdx.x] = s;
        if (bm) bm[blockIdx.x] = mx;
    }
}

// Exclusive scan of the tile sums in one block; the grand total goes to
// *total and, when asked, the largest element to *max_out.
__global__ void __launch_bounds__(1024) k_scan_tile_offsets(int64_t *bs, int64_t nb, int64_t *total,
                                                            const int32_t *bm, int32_t *max_out) {
    __shared__ int64_t wsum[1024 / dev::kWave];
    __shared__ int32_t smx[1024 / dev::kWave];
    __shared__ int64_t carry;
    if (max_out) {
        int32_t mx = INT32_MIN;
        for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) mx = bm[i] > mx ? bm[i] : mx;
        mx = dev::block_max(mx, smx);
        if (threadIdx.x == 0) *max_out = mx;
    }
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nb ? bs[i] : 0;
        int64_t inc = dev::wave_scan_incl(v);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int64_t off = carry;
        for (int k = 0; k < w; ++k) off += wsum[k];
        if (i < nb) bs[i] = off + inc - v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry = off + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Scans tile blockIdx.x in place, one round per wave.  DIRECT: bs holds the
// tile sums, the block adds those before its own, and the last block writes
// the total and the largest element; otherwise bs holds the tiles' exclusive
// offsets.
template <bool DIRECT>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(int32_t *a, int64_t n, const int64_t *bs, int64_t nb,
                                                             int64_t *total, const int32_t *bm, int32_t *max_out) {
    constexpr int nw = kScanThreads / dev::kWave;
    static_assert(kScanTile == nw * kSegRound, "one round per wave");
    __shared__ int32_t stage[nw][kSegStage];
    __shared__ int64_t wsum[nw];
    __shared__ int64_t psum[nw];
    __shared__ int32_t smx[nw];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t b = blockIdx.x;
    const int64_t seg = b * kScanTile + (int64_t)w * kSegRound;
    int32_t x[kSegItems];
    seg_load<1, true>(a, n, seg, lane, x);
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) s += x[j];
    s = dev::wave_sum(s);
    if (lane == 0) wsum[w] = s;
    int64_t off;
    if (DIRECT) {
        int64_t p = 0;
        for (int64_t k = threadIdx.x; k < b; k += kScanThreads) p += bs[k];
        off = dev::block_sum(p, psum);  // its barriers also publish wsum
    } else {
        __syncthreads();
        off = bs[b];
    }
    int64_t before = off;
    for (int k = 0; k < w; ++k) before += wsum[k];
    seg_scan_store<1, true>(a, n, seg, lane, x, before, stage[w]);
    if (DIRECT && b == nb - 1) {
        if (threadIdx.x == 0) {
            int64_t t = off;
            for (int k = 0; k < nw; ++k) t += wsum[k];
            *total = t;
        }
        if (max_out) {
            int32_t mx = INT32_MIN;
            for (int64_t k = threadIdx.x; k < nb; k += kScanThreads) mx = bm[k] > mx ? bm[k] : mx;
            mx = dev::block_max(mx, smx);
            if (threadIdx.x == 0) *max_out = mx;
        }
    }
}

// Whole scan in one block for short arrays (up to kScanOneBlock elements):
// one launch instead of two.  A pass over the block takes one round per wave;
// waves past the end skip theirs.  Same result as the tiled scan (integer
// sums).
constexpr int kScanOneThreads = 1024;
constexpr int64_t kScanOneTile = (int64_t)(kScanOneThreads / dev::kWave) * kSegRound;
constexpr int64_t kScanOneBlock = kScanOneTile;

__global__ void __launch_bounds__(kScanOneThreads) k_scan_one_block(int32_t *a, int64_t n, int64_t *total,
                                                                    int32_t *max_out) {
    constexpr int nw = kScanOneThreads / dev::kWave;
    __shared__ int32_t stage[nw][kSegStage];
    __shared__ int64_t wsum[nw];
    __shared__ int32_t wmax[nw];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t carry = 0;  // same in every thread
    int32_t mx = INT32_MIN;
    for (int64_t base = 0; base < n; base += kScanOneTile) {
        const int64_t seg = base + (int64_t)w * kSegRound;
        const bool live = seg < n;  // uniform over the wave
        int32_t x[kSegItems];
        int64_t s = 0;
        if (live) {
            seg_load<1, false>(a, n, seg, lane, x);
            const int lim = seg_limit(n, seg, lane, kSegRound);
#pragma unroll
            for (int j = 0; j < kSegItems; ++j) {
                s += x[j];
                if (j * dev::kWave < lim) mx = x[j] > mx ? x[j] : mx;
            }
            s = dev::wave_sum(s);
        }
        if (lane == 0) wsum[w] = s;
        __syncthreads();
        int64_t before = carry, tile = 0;
        for (int k = 0; k < nw; ++k) {
            if (k == w) before += tile;
            tile += wsum[k];
        }
        if (live) seg_scan_store<1, false>(a, n, seg, lane, x, before, stage[w]);
        carry += tile;
        __syncthreads();  // wsum is rewritten by the next pass
    }
    if (max_out) {
        mx = dev::wave_max(mx);
        if (lane == 0) wmax[w] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t m = wmax[0];
            for (int k = 1; k < nw; ++k) m = wmax[k] > m ? wmax[k] : m;
            *max_out = m;
        }
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_fill_i32(int32_t *a, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_fill_f64(double *a, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

}  // namespace

void scan_inclusive_i32(int32_t *a, int64_t n, int64_t *total, hipStream_t s, int32_t *max_out) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill_f64, 1, 1, 0, s, reinterpret_cast<double *>(total), 0.0, 1);
        if (max_out) hipLaunchKernelGGL(k_fill_i32, 1, 1, 0, s, max_out, 0, 1);
        GW_HIP(hipGetLastError());
        return;
    }
    if (n <= kScanOneBlock) {
        hipLaunchKernelGGL(k_scan_one_block, dim3(1), dim3(kScanOneThreads), 0, s, a, n, total, max_out);
        GW_HIP(hipGetLastError());
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    DBuf<int64_t> bs((size_t)nb);
    DBuf<int32_t> bm(max_out ? (size_t)nb : 0);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, n, bs.p, bm.p);
    if (nb <= kScanDirectTiles) {
        hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, n, bs.p, nb, total,
                           bm.p, max_out);
    } else {
        hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(1024), 0, s, bs.p, nb, total, bm.p, max_out);
        hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, n, bs.p, nb, total,
                           bm.p, max_out);
    }
    GW_HIP(hipGetLastError());
}

void fill_i32(int32_t *a, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = blocks_for(n, 4);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(kBlock), 0, s, a, v, n);
    GW_HIP(hipGetLastError());
}

void fill_f64(double *a, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = blocks_for(n, 4);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_f64, dim3(g), dim3(kBlock), 0, s, a, v, n);
    GW_HIP(hipGetLastError());
}

void copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes) GW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
}

}  // namespace gw
