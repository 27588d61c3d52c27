// Device pieces of transient flow, Eq. 2: (C + S/dt) h^{n+1} = b + (S/dt) h^n
// with S the diagonal of S_i V_i (specific storage times cell volume): the
// storage term, the right-hand side, C + S/dt, and the ratio
// max_i S_i V_i / (dt C_ii) that decides whether the setup of C may be kept
// (the criterion of the Discussion).
//
// Built with -ffp-contract=off: the storage term and the right-hand side are
// formed with the same operations as their definition, so the reuse ratio is
// exact and reproducible.
#include <cstring>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

// shift_i = S_i V_i / dt
__global__ void k_storage_shift(int64_t n, const double *__restrict__ Ss, double vol, double dt,
                                double *__restrict__ shift) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) shift[i] = (Ss[i] * vol) / dt;
}

// rhs = b + shift h
__global__ void k_storage_rhs(int64_t n, const double *__restrict__ b, const double *__restrict__ shift,
                              const double *__restrict__ h, double *__restrict__ rhs) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) rhs[i] = b[i] + shift[i] * h[i];
}

// Per-block maximum of shift_i / C_ii (non-negative values: the bits of a
// double order like the double, so the maximum is an integer maximum).
__global__ void k_shift_ratio(CsrView C, const double *__restrict__ shift, unsigned long long *out) {
    __shared__ unsigned long long wmax[kBlock / 64];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long m = 0;
    if (i < C.n) {
        double d = 0.0;
        for (int32_t p = C.rowptr[i]; p < C.rowptr[i + 1]; ++p)
            if (C.col[p] == (int32_t)i) d = C.val[p];
        const double r = shift[i] / d;
        m = __double_as_longlong(r > 0.0 ? r : 0.0);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long v = __shfl_xor(m, o, 64);
        m = v > m ? v : m;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = wmax[w] > b ? wmax[w] : b;
        out[blockIdx.x] = b;
    }
}

__global__ void k_max_u64(const unsigned long long *__restrict__ in, int64_t m, unsigned long long *out) {
    __shared__ unsigned long long part[1024];
    unsigned long long v = 0;
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x) v = in[t] > v ? in[t] : v;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = part[threadIdx.x + w] > part[threadIdx.x] ?
                                                          part[threadIdx.x + w] : part[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// A copy of C with shift added to the diagonal: C + S/dt.
__global__ void k_add_diagonal(CsrView C, const double *__restrict__ shift, double *__restrict__ val) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= C.n) return;
    for (int32_t p = C.rowptr[i]; p < C.rowptr[i + 1]; ++p)
        val[p] = C.col[p] == (int32_t)i ? C.val[p] + shift[i] : C.val[p];
}

}  // namespace

void storage_shift(int64_t n, const double *Ss, double vol, double dt, double *shift, hipStream_t s) {
    hipLaunchKernelGGL(k_storage_shift, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, Ss, vol, dt, shift);
    GW_HIP(hipGetLastError());
}

double shift_ratio(const CsrView &C, const double *shift, hipStream_t s) {
    const unsigned nb = blocks_for(C.n);
    DBuf<unsigned long long> part(nb), out(1);
    hipLaunchKernelGGL(k_shift_ratio, dim3(nb), dim3(kBlock), 0, s, C, shift, part.p);
    hipLaunchKernelGGL(k_max_u64, dim3(1), dim3(1024), 0, s, part.p, (int64_t)nb, out.p);
    GW_HIP(hipGetLastError());
    unsigned long long *stage = static_cast<unsigned long long *>(host_stage());
    GW_HIP(hipMemcpyAsync(stage, out.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    double r;
    std::memcpy(&r, stage, sizeof(double));
    return r;
}

void storage_rhs(int64_t n, const double *b, const double *shift, const double *h, double *rhs, hipStream_t s) {
    hipLaunchKernelGGL(k_storage_rhs, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, b, shift, h, rhs);
    GW_HIP(hipGetLastError());
}

void add_diagonal(const CsrView &C, const double *shift, double *val, hipStream_t s) {
    hipLaunchKernelGGL(k_add_diagonal, dim3(blocks_for(C.n)), dim3(kBlock), 0, s, C, shift, val);
    GW_HIP(hipGetLastError());
}

}  // namespace gw
