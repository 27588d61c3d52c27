// Device-side helpers shared by the kernels: wave64 reductions and scans in
// a fixed order (results do not depend on scheduling), and the last-block
// pattern that finishes a grid-wide reduction without a second launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gw {
namespace dev {

constexpr int kWave = 64;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

// Inclusive scan across the wave (Hillis-Steele).
template <class T>
__device__ __forceinline__ T wave_scan_incl(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T w = __shfl_up(v, o, kWave);
        if (lane >= o) v += w;
    }
    return v;
}

// Block sum with a fixed combination order; result valid in every thread.
// `sm` needs blockDim.x / 64 entries.
template <class T>
__device__ __forceinline__ T block_sum(T v, T *sm) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    T t = sm[0];
    for (int i = 1; i < nw; ++i) t += sm[i];
    __syncthreads();
    return t;
}

// Block maximum (valid in every thread).  `sm` needs blockDim.x / 64 entries.
template <class T>
__device__ __forceinline__ T block_max(T v, T *sm) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    T t = sm[0];
    for (int i = 1; i < nw; ++i) t = sm[i] > t ? sm[i] : t;
    __syncthreads();
    return t;
}

// First stage of a grid-wide sum: every block stores its NV block sums in
// partials[b*NV + k], b = `block` (the block's index in its grid).  A one-block finalize kernel adds them in block order
// (fixed), so totals do not depend on scheduling.  Two kernels instead of a
// "last block" ticket: on a multi-XCD part a device-scope fence in every
// block would write back that XCD's L2 each time, while the kernel boundary
// makes the partials visible once.
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *partials, int64_t block) {
    __shared__ double sm[NV][16];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = block_sum(v[k], sm[k]);
        if (threadIdx.x == 0) partials[(size_t)block * NV + k] = s;
    }
}

// Second stage, one block: tot[k] = sum over nb blocks of the k-th value at
// `off` in each block's record of `stride` values, same order always.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *partials, unsigned nb, double (&tot)[NV],
                                             int stride = NV, int off = 0) {
    __shared__ double sm[NV][16];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (unsigned b = threadIdx.x; b < nb; b += blockDim.x) s += partials[(size_t)b * stride + off + k];
        tot[k] = block_sum(s, sm[k]);
    }
}

// sum_partials for several values at once (nb >= 1), in blocks of BS threads,
// with every block record this thread reads loaded before any is added
// (records b = threadIdx.x + u*BS, u < MAXU, then the rest in a loop), so
// the loads take one round of latency instead of one per record: tot[k] =
// the sum of value off[k] of the nb records, added in exactly the order of
// sum_partials.  BS is a constant so that no load of the launch's block size
// has to finish before the records' loads are issued.
template <int NV, int BS, int MAXU = 8>
__device__ __forceinline__ void sum_partials_batched(const double *partials, unsigned nb, int stride,
                                                     const int (&off)[NV], double (&tot)[NV]) {
    static_assert(BS % kWave == 0 && BS / kWave <= 16, "block of at most 16 waves");
    __shared__ double sm[NV][16];
    double s[NV], t[MAXU][NV];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
        const unsigned b = threadIdx.x + u * BS;
        const unsigned bb = b < nb ? b : 0;  // nb >= 1; unused, but no branch
#pragma unroll
        for (int k = 0; k < NV; ++k) t[u][k] = partials[(size_t)bb * stride + off[k]];
    }
    // Every load above is issued before the first addition waits for one:
    // memory operations cannot cross these empty statements, and each
    // addition needs its value out of one.
#pragma unroll
    for (int u = 0; u < MAXU; ++u)
#pragma unroll
        for (int k = 0; k < NV; ++k) asm volatile("" : "+v"(t[u][k])::"memory");
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
#pragma unroll
    for (int u = 0; u < MAXU; ++u)
        if (threadIdx.x + u * BS < nb)
#pragma unroll
            for (int k = 0; k < NV; ++k) s[k] += t[u][k];
    for (unsigned b = threadIdx.x + MAXU * BS; b < nb; b += BS)
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += partials[(size_t)b * stride + off[k]];
    // block sums in block_sum's order, one pair of barriers for all values
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    constexpr int nw = BS / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = wave_sum(s[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sm[k][w] = s[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = sm[k][0];
        for (int i = 1; i < nw; ++i) a += sm[k][i];
        tot[k] = a;
    }
    __syncthreads();
}

__device__ __forceinline__ bool finite_nz(double v) { return isfinite(v) && v != 0.0; }

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  Renumbered this way, each XCD walks one
// contiguous range of rows, so the x_j its rows gather (neighbours a row, a
// line or a plane away) stay in its own L2 instead of being fetched by all
// eight.  A bijection of [0, gridDim.x); the last gridDim.x mod 8 keep their
// number.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t full = nb / kXcds * kXcds;
    if (b >= full) return b;
    return (b % kXcds) * (full / kXcds) + b / kXcds;
}

}  // namespace dev
}  // namespace gw
