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

// Uncached (device-coherent) load of a value written by another workgroup.
__device__ __forceinline__ double load_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide sum of NV per-thread values with the "last block finishes"
// pattern.  Every block stores its NV block sums in partials[b*NV + k] and
// takes a ticket; the block that draws the last ticket adds all partials in
// block order (thread t takes blocks t, t+blockDim, ..., then a fixed tree),
// so the total is identical whichever block arrives last.  Returns true in
// the last block, where tot[] holds the totals (in every thread).
template <int NV>
__device__ bool grid_sum_last(double (&v)[NV], double *partials, uint32_t *counter, double (&tot)[NV]) {
    __shared__ double sm[NV][16];
    __shared__ bool last;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = block_sum(v[k], sm[k]);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * NV + k] = s;
    }
    if (threadIdx.x == 0) {
        __threadfence();
        uint32_t t = atomicAdd(counter, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
            s += load_coherent(&partials[(size_t)b * NV + k]);
        tot[k] = block_sum(s, sm[k]);
    }
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

__device__ __forceinline__ bool finite_nz(double v) { return isfinite(v) && v != 0.0; }

}  // namespace dev
}  // namespace gw
