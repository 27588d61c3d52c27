// ILU(0) smoother: the relaxation the paper's AMG used on every level
// (Results).  The factorization keeps A's pattern: row by row, over the row's
// lower entries k in ascending column order, l_ik = a_ik / u_kk and then
// a_ij -= l_ik u_kj for every later entry j of row i that row k also holds.
// A row needs only the rows of its lower entries, so rows are factored level
// by level of that dependency graph (the schedule of the forward
// substitution), in one workgroup as the upwind sweep solves its levels; every
// entry receives its updates in the order of the sequential algorithm, so the
// factors are bit-identical to it.  A smoothing step x += (LU)^{-1}(b - A x)
// then runs two such sweeps: forward with the unit lower triangle, backward
// with the upper one.
//
// Built with -ffp-contract=off (each update is a product then a difference).
#include <algorithm>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

constexpr int kFactorThreads = 1024;
constexpr int kFactorQueue = 6144;

__global__ void k_ilu_dpos(CsrView A, int32_t *__restrict__ dpos, int32_t *__restrict__ lo_len,
                           int32_t *__restrict__ up_len) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t d = A.rowptr[i];
    for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
        if (A.col[p] == (int32_t)i) d = p;
    dpos[i] = d;
    lo_len[i] = d - A.rowptr[i] + 1;      // lower entries and the unit diagonal
    up_len[i] = A.rowptr[i + 1] - d;      // the diagonal and the upper entries
}

// The two triangles as systems for the substitutions: L = strict lower part
// of the factors plus a unit diagonal, U = diagonal and upper part.  With
// `values` off only the columns are written (the schedule of L is needed
// before the factors exist).
__global__ void k_ilu_split(CsrView A, const int32_t *__restrict__ dpos, const double *__restrict__ lu,
                            const int32_t *__restrict__ lrow, int32_t *__restrict__ lcol, double *__restrict__ lval,
                            const int32_t *__restrict__ urow, int32_t *__restrict__ ucol, double *__restrict__ uval,
                            int values) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int32_t b = A.rowptr[i], d = dpos[i], e = A.rowptr[i + 1];
    int32_t q = lrow[i];
    for (int32_t p = b; p < d; ++p, ++q) {
        lcol[q] = A.col[p];
        if (values) lval[q] = lu[p];
    }
    lcol[q] = (int32_t)i;
    if (values) lval[q] = 1.0;
    q = urow[i];
    for (int32_t p = d; p < e; ++p, ++q) {
        ucol[q] = A.col[p];
        if (values) uval[q] = lu[p];
    }
}

__global__ void k_ilu_prep(int64_t n, const int32_t *__restrict__ indeg0, const int32_t *__restrict__ q0,
                           const int64_t *__restrict__ first, int32_t *__restrict__ indeg, int32_t *__restrict__ qa,
                           int64_t *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) indeg[i] = indeg0[i];
    if (i < *first) qa[i] = q0[i];
    if (i == 0) out[0] = *first;
}

// Factor rows level by level (out[0]: size of the first level on entry).
// A zero pivot sets *bad.
__global__ void __launch_bounds__(kFactorThreads) k_ilu_factor(CsrView A, const int32_t *__restrict__ dpos, double *lu,
                                                               int32_t *__restrict__ indeg,
                                                               const int32_t *__restrict__ drow,
                                                               const int32_t *__restrict__ dcol, int32_t *qg0,
                                                               int32_t *qg1, int64_t *out, int32_t *bad) {
    __shared__ int32_t lq[2][kFactorQueue];
    __shared__ int32_t cnt[3];
    const int32_t first = (int32_t)out[0];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    for (int32_t t = threadIdx.x; t < first && t < kFactorQueue; t += blockDim.x) lq[0][t] = qg0[t];
    __syncthreads();
    int32_t size = first, lev = 0;
    int64_t total = 0;
    int32_t zero = 0;
    while (size > 0) {
        const int cb = lev & 1, nb = cb ^ 1;
        const int32_t *gcur = cb ? qg1 : qg0;
        int32_t *gnxt = cb ? qg0 : qg1;
        int32_t *app = &cnt[lev % 3];
        if (threadIdx.x == 0) cnt[(lev + 1) % 3] = 0;
        for (int32_t t = threadIdx.x; t < size; t += blockDim.x) {
            const int32_t i = t < kFactorQueue ? lq[cb][t] : gcur[t];
            const int32_t e = A.rowptr[i + 1], di = dpos[i];
            for (int32_t p = A.rowptr[i]; p < di; ++p) {
                const int32_t k = A.col[p];
                const double ukk = lu[dpos[k]];
                zero |= ukk == 0.0;
                const double lik = lu[p] / ukk;
                lu[p] = lik;
                int32_t r = dpos[k] + 1;
                const int32_t ek = A.rowptr[k + 1];
                for (int32_t q = p + 1; q < e; ++q) {
                    const int32_t j = A.col[q];
                    while (r < ek && A.col[r] < j) ++r;
                    if (r < ek && A.col[r] == j) lu[q] = lu[q] - lik * lu[r];
                }
            }
            zero |= lu[di] == 0.0;
            for (int32_t q = drow[i]; q < drow[i + 1]; ++q) {
                const int32_t k2 = dcol[q];
                if (atomicSub(&indeg[k2], 1) == 1) {
                    const int32_t pos = atomicAdd(app, 1);
                    if (pos < kFactorQueue) lq[nb][pos] = k2;
                    else gnxt[pos] = k2;
                }
            }
        }
        __syncthreads();
        total += size;
        size = *app;
        ++lev;
    }
    if (zero) atomicOr(bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = total;
        out[1] = lev;
    }
}

}  // namespace

void build_ilu0(amg_hierarchy *H, int l, hipStream_t s) {
    Level &Lv = H->L[l];
    const CsrView A = view(Lv.A);
    const int64_t n = A.n;
    auto I = std::make_unique<IluData>();
    I->dpos.alloc(n);
    I->lu.alloc((size_t)A.nnz);
    copy_bytes(I->lu.p, A.val, sizeof(double) * (size_t)A.nnz, s);
    Csr &Lm = I->lo.M, &Um = I->up.M;
    Lm.n = Lm.ncols = Um.n = Um.ncols = (int32_t)n;
    Lm.rowptr.alloc((size_t)n + 1);
    Um.rowptr.alloc((size_t)n + 1);
    fill_i32(Lm.rowptr.p, 0, 1, s);
    fill_i32(Um.rowptr.p, 0, 1, s);
    DBuf<int64_t> tot(2);
    DBuf<int32_t> bad(1);
    fill_i32(bad.p, 0, 1, s);
    hipLaunchKernelGGL(k_ilu_dpos, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, I->dpos.p, Lm.rowptr.p + 1,
                       Um.rowptr.p + 1);
    scan_inclusive_i32(Lm.rowptr.p + 1, n, tot.p, s);
    scan_inclusive_i32(Um.rowptr.p + 1, n, tot.p + 1, s);
    int64_t *stage = static_cast<int64_t *>(host_stage());
    GW_HIP(hipMemcpyAsync(stage, tot.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    Lm.nnz = stage[0];
    Um.nnz = stage[1];
    Lm.col.alloc((size_t)Lm.nnz);
    Lm.val.alloc((size_t)Lm.nnz);
    Um.col.alloc((size_t)Um.nnz);
    Um.val.alloc((size_t)Um.nnz);
    // the schedule of L (its pattern only), the factorization, then the values
    hipLaunchKernelGGL(k_ilu_split, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, I->dpos.p, I->lu.p, Lm.rowptr.p,
                       Lm.col.p, Lm.val.p, Um.rowptr.p, Um.col.p, Um.val.p, 0);
    sweep_plan(I->lo, s);
    {
        ProfScope ps(K_SETUP_MISC, (double)A.nnz * 28, s);
        hipLaunchKernelGGL(k_ilu_prep, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, I->lo.indeg0.p, I->lo.q0.p,
                           I->lo.first.p, I->lo.indeg.p, I->lo.qa.p, I->lo.out.p);
        hipLaunchKernelGGL(k_ilu_factor, dim3(1), dim3(kFactorThreads), 0, s, A, I->dpos.p, I->lu.p, I->lo.indeg.p,
                           I->lo.drow.p, I->lo.dcol.p, I->lo.qa.p, I->lo.qb.p, I->lo.out.p, bad.p);
        GW_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ilu_split, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, I->dpos.p, I->lu.p, Lm.rowptr.p,
                       Lm.col.p, Lm.val.p, Um.rowptr.p, Um.col.p, Um.val.p, 1);
    sweep_plan(I->up, s);
    I->r.alloc(n);
    I->y.alloc(n);
    I->z.alloc(n);
    int32_t *flag = static_cast<int32_t *>(host_stage());
    GW_HIP(hipMemcpyAsync(flag, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    if (flag[0]) fail(GW_SINGULAR, "amg_setup: zero pivot in the ILU(0) factorization of level " + std::to_string(l));
    Lv.ilu = std::move(I);
}

void ilu_apply(IluData &I, const double *r, double *z, const int32_t *done, hipStream_t s) {
    sweep_run(I.lo, r, I.y.p, done, s);
    sweep_run(I.up, I.y.p, z, done, s);
}

}  // namespace gw
