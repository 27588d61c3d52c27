// Device-wide inclusive scan of int32 counts (used to turn row lengths into
// CSR row pointers and flags into ids) and small fill/copy helpers.
#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Per tile: the sum and the largest value (the latter only when bm != null).
__global__ void __launch_bounds__(kScanThreads) k_scan_tile_sums(const int32_t *a, int64_t n, int64_t *bs,
                                                                 int32_t *bm) {
    __shared__ int64_t sm[kScanThreads / dev::kWave];
    __shared__ int32_t smx[kScanThreads / dev::kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    int32_t mx = INT32_MIN;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) {
            s += a[i];
            mx = a[i] > mx ? a[i] : mx;
        }
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

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(int32_t *a, int64_t n, const int64_t *bs) {
    __shared__ int64_t wsum[kScanThreads / dev::kWave];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        s += (i < n) ? a[i] : 0;
        v[k] = s;
    }
    int64_t inc = dev::wave_scan_incl(s);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t off = bs[blockIdx.x];
    for (int k = 0; k < w; ++k) off += wsum[k];
    off += inc - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) a[i] = (int32_t)(off + v[k]);
    }
}

// Whole scan in one block for short arrays (up to kScanOneBlock elements):
// one launch instead of three.  Same result as the three-kernel scan
// (integer sums).
constexpr int kScanOneThreads = 1024;
constexpr int kScanOneItems = 16;
constexpr int64_t kScanOneBlock = (int64_t)kScanOneThreads * kScanOneItems * 4;

__global__ void __launch_bounds__(kScanOneThreads) k_scan_one_block(int32_t *a, int64_t n, int64_t *total,
                                                                    int32_t *max_out) {
    __shared__ int64_t wsum[kScanOneThreads / dev::kWave];
    __shared__ int32_t wmax[kScanOneThreads / dev::kWave];
    __shared__ int64_t carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    int32_t mx = INT32_MIN;
    __syncthreads();
    constexpr int64_t tile = (int64_t)kScanOneThreads * kScanOneItems;
    for (int64_t base0 = 0; base0 < n; base0 += tile) {
        const int64_t base = base0 + (int64_t)threadIdx.x * kScanOneItems;
        int64_t v[kScanOneItems];
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanOneItems; ++k) {
            const int64_t i = base + k;
            const int32_t x = i < n ? a[i] : 0;
            if (i < n) mx = x > mx ? x : mx;
            s += x;
            v[k] = s;
        }
        const int64_t inc = dev::wave_scan_incl(s);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int64_t off = carry;
        for (int k = 0; k < w; ++k) off += wsum[k];
        off += inc - s;
#pragma unroll
        for (int k = 0; k < kScanOneItems; ++k) {
            const int64_t i = base + k;
            if (i < n) a[i] = (int32_t)(off + v[k]);
        }
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry = off + s;
        __syncthreads();
    }
    if (max_out) {
        mx = dev::wave_max(mx);
        if (lane == 0) wmax[w] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t m = wmax[0];
            for (int k = 1; k < kScanOneThreads / dev::kWave; ++k) m = wmax[k] > m ? wmax[k] : m;
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
    hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(1024), 0, s, bs.p, nb, total, bm.p, max_out);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, n, bs.p);
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
