// Solve phase: the V-cycle (Introduction: restrict the residual, smooth,
// recurse to a direct solve on the coarsest level, interpolate and correct,
// smooth -- only sparse matrix-vector products) and the Krylov methods it
// preconditions: CG for the symmetric flow system and BiCGSTAB for the
// upwind travel-time system (Benchmarking Examples).
//
// The Krylov scalars live on the device: every dot product is finished by
// the last workgroup of its kernel, which also forms alpha/beta/omega and
// raises the convergence flag; all later kernels read the flag and return at
// once, so the host only polls it every few iterations.  FP64 throughout the
// Krylov layer; the hierarchy is FP64 or FP32 (mixed mode).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

template <class T>
__device__ __forceinline__ bool is_done(const int32_t *done) {
    return done && *done;
}

// ------------------------------------------------------------ V-cycle ----
// Sweep x <- x + M (b - A x); the first two sweeps from x = 0 are fused:
// x1 = M b, x2 = x1 + M (b - A x1) with x1_j recomputed on the fly.
template <class V, class Bt, class Yt>
__global__ void k_smooth_first(int32_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                               const V *__restrict__ val, const V *__restrict__ M, const Bt *__restrict__ b,
                               Yt *__restrict__ y, int two, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const V bi = (V)b[i], mi = M[i];
    V x1 = mi * bi;
    if (two) {
        V ax = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = col[p];
            ax += val[p] * (M[j] * (V)b[j]);
        }
        x1 = x1 + mi * (bi - ax);
    }
    y[i] = (Yt)x1;
}

template <class V, class Bt, class Xt, class Yt>
__global__ void k_smooth(int32_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                         const V *__restrict__ val, const V *__restrict__ M, const Bt *__restrict__ b,
                         const Xt *__restrict__ x, Yt *__restrict__ y, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    V ax = 0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) ax += val[p] * (V)x[col[p]];
    y[i] = (Yt)((V)x[i] + M[i] * ((V)b[i] - ax));
}

template <class V, class Bt, class Xt, class Rt>
__global__ void k_residual(int32_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const V *__restrict__ val, const Bt *__restrict__ b, const Xt *__restrict__ x,
                           Rt *__restrict__ r, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    V ax = 0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) ax += val[p] * (V)x[col[p]];
    r[i] = (Rt)((V)b[i] - ax);
}

template <class V, class Xt, class Yt>
__global__ void k_spmv(int32_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                       const V *__restrict__ val, const Xt *__restrict__ x, Yt *__restrict__ y,
                       const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    V s = 0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += val[p] * (V)x[col[p]];
    y[i] = (Yt)s;
}

// x += P x_c
template <class V, class Xt>
__global__ void k_prolong(int32_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                          const V *__restrict__ val, const Xt *__restrict__ xc, Xt *__restrict__ x,
                          const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    V s = 0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += val[p] * (V)xc[col[p]];
    x[i] = (Xt)((V)x[i] + s);
}

// Coarsest level: x = A_L^{-1} b with the column-major inverse, in FP64.
template <class Bt, class Yt>
__global__ void k_coarse_gemv(int32_t n, const double *__restrict__ inv, const Bt *__restrict__ b,
                              Yt *__restrict__ y, const int32_t *done) {
    if (done && *done) return;
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int32_t c = 0; c < n; ++c) s += inv[(int64_t)c * n + i] * (double)b[c];
    y[i] = (Yt)s;
}

template <class X>
__global__ void k_zero(X *x, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = (X)0;
}

template <class Xt, class Yt>
__global__ void k_convert(const Xt *__restrict__ x, Yt *__restrict__ y, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (Yt)x[i];
}

// Bytes one launch of a CSR pass touches (values, columns, row pointers).
double csr_bytes(int64_t n, int64_t nnz, int vbytes) { return (double)nnz * (vbytes + 4) + 4.0 * (n + 1); }

template <class V>
struct LevelOps {
    static const V *aval(const Level &L);
    static const V *pval(const Level &L);
    static const V *rval(const Level &L);
    static const V *mval(const Level &L);
};
template <>
struct LevelOps<double> {
    static const double *aval(const Level &L) { return L.A.val.p; }
    static const double *pval(const Level &L) { return L.P.val.p; }
    static const double *rval(const Level &L) { return L.R.val.p; }
    static const double *mval(const Level &L) { return L.M.p; }
};
template <>
struct LevelOps<float> {
    static const float *aval(const Level &L) { return L.A.val32.p; }
    static const float *pval(const Level &L) { return L.P.val32.p; }
    static const float *rval(const Level &L) { return L.R.val32.p; }
    static const float *mval(const Level &L) { return L.M32.p; }
};

// One V-cycle on level l.  `b` is the right-hand side (type Bt), the result
// goes to `out` (type Zt) when given, else into one of the level's own
// buffers, whose address is returned.  V = value type of the hierarchy (also
// the type of all internal vectors).
template <class V, class Bt, class Zt>
void *vcycle_level(amg_hierarchy *H, int l, const Bt *b, Zt *out, const int32_t *done, hipStream_t s) {
    Level &Lv = H->L[l];
    const int32_t n = Lv.A.n;
    const unsigned g = blocks_for(n);
    const int vb = (int)sizeof(V);
    if (l == H->nlev - 1) {
        Zt *y = out ? out : reinterpret_cast<Zt *>(Lv.vx.p);
        ProfScope ps(K_COARSE_SOLVE, (double)n * n * 8 + n * (double)(sizeof(Bt) + sizeof(Zt)), s);
        hipLaunchKernelGGL((k_coarse_gemv<Bt, Zt>), dim3(blocks_for(n, 1, 64)), dim3(64), 0, s, n, H->inv.p, b, y, done);
        return y;
    }
    const int32_t *ar = Lv.A.rowptr.p, *ac = Lv.A.col.p;
    const V *av = LevelOps<V>::aval(Lv), *M = LevelOps<V>::mval(Lv);
    const double abytes = csr_bytes(n, Lv.A.nnz, vb);
    V *x = reinterpret_cast<V *>(Lv.vx.p);
    V *t = reinterpret_cast<V *>(Lv.vt.p);
    const int npre = H->prm.npre, npost = H->prm.npost;

    // pre-smoothing
    if (npre == 0) {
        hipLaunchKernelGGL((k_zero<V>), dim3(g), dim3(kBlock), 0, s, x, (int64_t)n, done);
    } else {
        ProfScope ps(K_SMOOTH_FIRST, npre >= 2 ? abytes + n * (double)(sizeof(Bt) + 2 * vb) : n * (double)(sizeof(Bt) + 2 * vb), s);
        hipLaunchKernelGGL((k_smooth_first<V, Bt, V>), dim3(g), dim3(kBlock), 0, s, n, ar, ac, av, M, b, x,
                           npre >= 2 ? 1 : 0, done);
    }
    for (int k = 2; k < npre; ++k) {
        ProfScope ps(K_SMOOTH, abytes + n * (double)(sizeof(Bt) + 3 * vb), s);
        hipLaunchKernelGGL((k_smooth<V, Bt, V, V>), dim3(g), dim3(kBlock), 0, s, n, ar, ac, av, M, b, x, t, done);
        std::swap(x, t);
    }
    // residual and restriction
    {
        ProfScope ps(K_RESIDUAL, abytes + n * (double)(sizeof(Bt) + 2 * vb), s);
        hipLaunchKernelGGL((k_residual<V, Bt, V, V>), dim3(g), dim3(kBlock), 0, s, n, ar, ac, av, b, x, t, done);
    }
    Level &Nx = H->L[l + 1];
    V *bc = reinterpret_cast<V *>(Nx.vb.p);
    {
        ProfScope ps(K_RESTRICT, csr_bytes(Lv.nc, Lv.R.nnz, vb) + (double)(n + Lv.nc) * vb, s);
        hipLaunchKernelGGL((k_spmv<V, V, V>), dim3(blocks_for(Lv.nc)), dim3(kBlock), 0, s, Lv.nc, Lv.R.rowptr.p,
                           Lv.R.col.p, LevelOps<V>::rval(Lv), t, bc, done);
    }
    V *xc = static_cast<V *>(vcycle_level<V, V, V>(H, l + 1, bc, (V *)nullptr, done, s));
    {
        ProfScope ps(K_PROLONG, csr_bytes(n, Lv.P.nnz, vb) + (double)(2 * n + Lv.nc) * vb, s);
        hipLaunchKernelGGL((k_prolong<V, V>), dim3(g), dim3(kBlock), 0, s, n, Lv.P.rowptr.p, Lv.P.col.p,
                           LevelOps<V>::pval(Lv), xc, x, done);
    }
    // post-smoothing; the last sweep writes the requested output
    for (int k = 0; k < npost; ++k) {
        const bool last = (k == npost - 1);
        ProfScope ps(K_SMOOTH, abytes + n * (double)(sizeof(Bt) + 3 * vb), s);
        if (last && out) {
            hipLaunchKernelGGL((k_smooth<V, Bt, V, Zt>), dim3(g), dim3(kBlock), 0, s, n, ar, ac, av, M, b, x, out, done);
            return out;
        }
        hipLaunchKernelGGL((k_smooth<V, Bt, V, V>), dim3(g), dim3(kBlock), 0, s, n, ar, ac, av, M, b, x, t, done);
        std::swap(x, t);
    }
    if (out) {
        hipLaunchKernelGGL((k_convert<V, Zt>), dim3(g), dim3(kBlock), 0, s, x, out, (int64_t)n, done);
        return out;
    }
    return x;
}

// -------------------------------------------------------------- Krylov ---
constexpr int kKBlock = 256;
constexpr int kKMaxBlocks = 2048;

unsigned kgrid(int64_t n) {
    int64_t b = (n + kKBlock - 1) / kKBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kKMaxBlocks));
}

#define GRID_LOOP(i, n) for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ double row_dot(const CsrView &A, int64_t i, const double *__restrict__ x) {
    double s = 0.0;
    for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
    return s;
}

// r = b - A x; first call also forms ||b|| and the tolerance.
__global__ void __launch_bounds__(kKBlock) k_kr_init(CsrView A, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ rh, double *__restrict__ p,
                                                     double *__restrict__ v, double rtol, int first,
                                                     double *partials, KScalars *ks) {
    double acc[2] = {0.0, 0.0};
    GRID_LOOP(i, A.n) {
        double ri = b[i] - row_dot(A, i, x);
        r[i] = ri;
        if (rh) rh[i] = ri;
        if (p) p[i] = 0.0;
        if (v) v[i] = 0.0;
        acc[0] += b[i] * b[i];
        acc[1] += ri * ri;
    }
    double tot[2];
    if (dev::grid_sum_last<2>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        if (first) {
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
        ks->beta = tot[1];  // (rho / 1) * (1 / 1)
        ks->pending_x = 0;
        if (!dev::finite_nz(tot[1]) && ks->bnorm != 0.0) {
            ks->status = GW_BREAKDOWN;
            ks->done = 1;
        }
    }
}

// CG: rz = r.z; beta = rz_new / rz (or Polak-Ribiere -alpha z.q / rz).
__global__ void __launch_bounds__(kKBlock) k_cg_beta(int64_t n, const double *__restrict__ r,
                                                     const double *__restrict__ z, const double *__restrict__ q,
                                                     int first, double *partials, KScalars *ks) {
    if (ks->done) return;
    double acc[2] = {0.0, 0.0};
    GRID_LOOP(i, n) {
        acc[0] += r[i] * z[i];
        if (!first) acc[1] += z[i] * q[i];
    }
    double tot[2];
    if (dev::grid_sum_last<2>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        double rz_new = tot[0];
        if (first) ks->beta = 0.0;
        else if (ks->flexible) ks->beta = (-ks->alpha * tot[1]) / ks->rz;
        else ks->beta = rz_new / ks->rz;
        ks->rz = rz_new;
    }
}

// p_new = z + beta p_old;  q = A p_new;  alpha = rz / (p_new . q)
__global__ void __launch_bounds__(kKBlock) k_cg_spmv(CsrView A, const double *__restrict__ z,
                                                     const double *__restrict__ p_old, double *__restrict__ p_new,
                                                     double *__restrict__ q, double *partials, KScalars *ks) {
    if (ks->done) return;
    const double beta = ks->beta;
    double acc[1] = {0.0};
    GRID_LOOP(i, A.n) {
        double s = 0.0;
        for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
            int32_t j = A.col[p];
            s += A.val[p] * (z[j] + beta * p_old[j]);
        }
        double pi = z[i] + beta * p_old[i];
        p_new[i] = pi;
        q[i] = s;
        acc[0] += pi * s;
    }
    double tot[1];
    if (dev::grid_sum_last<1>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        ks->pq = tot[0];
        if (!dev::finite_nz(tot[0]) || !isfinite(ks->rz)) {
            ks->status = GW_BREAKDOWN;
            ks->done = 1;
        } else {
            ks->alpha = ks->rz / tot[0];
        }
    }
}

// x += alpha p;  r -= alpha q;  stop when ||r|| <= rtol ||b||
__global__ void __launch_bounds__(kKBlock) k_cg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                       const double *__restrict__ p, const double *__restrict__ q,
                                                       double *partials, KScalars *ks) {
    if (ks->done) return;
    const double alpha = ks->alpha;
    double acc[1] = {0.0};
    GRID_LOOP(i, n) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    double tot[1];
    if (dev::grid_sum_last<1>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        ks->rr = tot[0];
        ks->iters += 1;
        double rn = sqrt(tot[0]);
        if (!isfinite(rn)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
        else if (rn <= ks->tol) { ks->status = GW_OK; ks->done = 1; }
        else if (ks->iters >= ks->maxiter) { ks->status = GW_NOT_CONVERGED; ks->done = 1; }
    }
}

// ||b - A x|| / ||b|| in FP64
__global__ void __launch_bounds__(kKBlock) k_true_res(CsrView A, const double *__restrict__ b,
                                                      const double *__restrict__ x, double *partials, KScalars *ks) {
    double acc[1] = {0.0};
    GRID_LOOP(i, A.n) {
        double ri = b[i] - row_dot(A, i, x);
        acc[0] += ri * ri;
    }
    double tot[1];
    if (dev::grid_sum_last<1>(acc, partials, &ks->counter, tot) && threadIdx.x == 0)
        ks->rel_true = sqrt(tot[0]) / ks->bnorm;
}

// BiCGSTAB: p = r + beta (p - omega v)
__global__ void __launch_bounds__(kKBlock) k_bcg_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                                   const double *__restrict__ v, KScalars *ks) {
    if (ks->done) return;
    const double beta = ks->beta, omega = ks->omega;
    GRID_LOOP(i, n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// v = A p_hat;  alpha = rho / (r_hat . v)
__global__ void __launch_bounds__(kKBlock) k_bcg_v(CsrView A, const double *__restrict__ ph, double *__restrict__ v,
                                                   const double *__restrict__ rh, double *partials, KScalars *ks) {
    if (ks->done) return;
    double acc[1] = {0.0};
    GRID_LOOP(i, A.n) {
        double vi = row_dot(A, i, ph);
        v[i] = vi;
        acc[0] += rh[i] * vi;
    }
    double tot[1];
    if (dev::grid_sum_last<1>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        ks->rv = tot[0];
        if (!dev::finite_nz(tot[0])) { ks->status = GW_BREAKDOWN; ks->done = 1; }
        else ks->alpha = ks->rho / tot[0];
    }
}

// s = r - alpha v; stop (after x += alpha p_hat) when ||s|| <= tol
__global__ void __launch_bounds__(kKBlock) k_bcg_s(int64_t n, const double *__restrict__ r,
                                                   const double *__restrict__ v, double *__restrict__ sv,
                                                   double *partials, KScalars *ks) {
    if (ks->done) return;
    const double alpha = ks->alpha;
    double acc[1] = {0.0};
    GRID_LOOP(i, n) {
        double si = r[i] - alpha * v[i];
        sv[i] = si;
        acc[0] += si * si;
    }
    double tot[1];
    if (dev::grid_sum_last<1>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        ks->ss = tot[0];
        ks->iters += 1;
        double sn = sqrt(tot[0]);
        if (!isfinite(sn)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
        else if (sn <= ks->tol) { ks->status = GW_OK; ks->rr = tot[0]; ks->done = 1; ks->pending_x = 1; }
    }
}

// t = A s_hat;  omega = (t.s) / (t.t)
__global__ void __launch_bounds__(kKBlock) k_bcg_t(CsrView A, const double *__restrict__ sh, double *__restrict__ t,
                                                   const double *__restrict__ sv, double *partials, KScalars *ks) {
    if (ks->done) return;
    double acc[2] = {0.0, 0.0};
    GRID_LOOP(i, A.n) {
        double ti = row_dot(A, i, sh);
        t[i] = ti;
        acc[0] += ti * sv[i];
        acc[1] += ti * ti;
    }
    double tot[2];
    if (dev::grid_sum_last<2>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        ks->ts = tot[0];
        ks->tt = tot[1];
        if (!dev::finite_nz(tot[1])) { ks->status = GW_BREAKDOWN; ks->done = 1; }
        else {
            double om = tot[0] / tot[1];
            if (!dev::finite_nz(om)) { ks->status = GW_BREAKDOWN; ks->done = 1; }
            else ks->omega = om;
        }
    }
}

// x += alpha p_hat + omega s_hat;  r = s - omega t;  then the next rho and
// beta.  After an early stop on ||s|| only x += alpha p_hat is applied.
__global__ void __launch_bounds__(kKBlock) k_bcg_xr(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ ph, const double *__restrict__ sh,
                                                    const double *__restrict__ sv, const double *__restrict__ t,
                                                    const double *__restrict__ rh, double *partials, KScalars *ks) {
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
    double tot[2];
    if (dev::grid_sum_last<2>(acc, partials, &ks->counter, tot) && threadIdx.x == 0) {
        if (pending) {
            ks->pending_x = 0;
            return;
        }
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
    }
}

__global__ void k_spmv_f64(CsrView A, const double *__restrict__ x, double *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < A.n) y[i] = row_dot(A, i, x);
}

void ensure_krylov_workspace(amg_hierarchy *H, int nvec) {
    const size_t n = (size_t)H->L[0].A.n;
    if (H->kvec_count < nvec) {
        H->kvec.alloc(n * nvec);
        H->kvec_count = nvec;
    }
    if (!H->partials.p) H->partials.alloc((size_t)kKMaxBlocks * 2);
    if (!H->ks.p) {
        H->ks.alloc(1);
        H->ks_host = new Pinned(sizeof(KScalars));
    }
}

KScalars read_ks(amg_hierarchy *H, hipStream_t s) {
    GW_HIP(hipMemcpyAsync(H->ks_host->p, H->ks.p, sizeof(KScalars), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    KScalars k;
    std::memcpy(&k, H->ks_host->p, sizeof(KScalars));
    return k;
}

void write_ks(amg_hierarchy *H, const KScalars &k, hipStream_t s) {
    std::memcpy(H->ks_host->p, &k, sizeof(KScalars));
    GW_HIP(hipMemcpyAsync(H->ks.p, H->ks_host->p, sizeof(KScalars), hipMemcpyHostToDevice, s));
    GW_HIP(hipStreamSynchronize(s));
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

void vcycle(amg_hierarchy *H, const double *r, double *z, const int32_t *done, hipStream_t s) {
    if (H->nlev == 0) {
        // preconditioner off: z = r
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks_for(H->L[0].A.n)), dim3(kBlock), 0, s, r, z,
                           (int64_t)H->L[0].A.n, done);
        GW_HIP(hipGetLastError());
        return;
    }
    if (H->mixed()) vcycle_level<float, double, double>(H, 0, r, z, done, s);
    else vcycle_level<double, double, double>(H, 0, r, z, done, s);
    GW_HIP(hipGetLastError());
}

void spmv_f64(const CsrView &A, const double *x, double *y, hipStream_t s) {
    ProfScope ps(K_KRYLOV_SPMV, csr_bytes(A.n, A.nnz, 8) + 16.0 * A.n, s);
    hipLaunchKernelGGL(k_spmv_f64, dim3(blocks_for(A.n)), dim3(kBlock), 0, s, A, x, y);
    GW_HIP(hipGetLastError());
}

int krylov_pcg(amg_hierarchy *H, const double *b, double *x, const amg_solve_params &sp, amg_solve_info *info,
               hipStream_t s) {
    const double t0 = now_ms();
    const CsrView A = view(H->L[0].A);
    const int64_t n = A.n;
    ensure_krylov_workspace(H, 5);
    double *r = H->kvec.p, *z = r + n, *pa = z + n, *pb = pa + n, *q = pb + n;
    KScalars k0{};
    k0.maxiter = std::max(0, sp.maxiter);
    k0.flexible = sp.flexible < 0 ? (H->mixed() ? 1 : 0) : (sp.flexible ? 1 : 0);
    k0.status = GW_NOT_CONVERGED;
    write_ks(H, k0, s);
    fill_f64(x, 0.0, n, s);
    const unsigned g = kgrid(n);
    const double vec = 8.0 * n, abytes = csr_bytes(A.n, A.nnz, 8);
    {
        ProfScope ps(K_KRYLOV_SPMV, abytes + 4 * vec, s);
        hipLaunchKernelGGL(k_kr_init, dim3(g), dim3(kKBlock), 0, s, A, b, x, r, (double *)nullptr, pa,
                           (double *)nullptr, sp.rtol, 1, H->partials.p, H->ks.p);
    }
    KScalars k = read_ks(H, s);
    int restarts = 0;
    if (k.bnorm == 0.0) {
        if (info) *info = {0, GW_OK, 0, 0.0, 0.0, 0.0, now_ms() - t0};
        return GW_OK;
    }
    const int check = std::max(1, sp.check_every);
    int32_t *done = &H->ks.p->done;
    int parity = 0;
    for (;;) {
        if (!k.done) {
            vcycle(H, r, z, done, s);
            {
                ProfScope ps(K_KRYLOV_DOT, 2 * vec, s);
                hipLaunchKernelGGL(k_cg_beta, dim3(g), dim3(kKBlock), 0, s, n, r, z, q, 1, H->partials.p, H->ks.p);
            }
            for (;;) {
                for (int c = 0; c < check; ++c) {
                    double *po = parity ? pb : pa, *pn = parity ? pa : pb;
                    {
                        ProfScope ps(K_KRYLOV_SPMV, abytes + 4 * vec, s);
                        hipLaunchKernelGGL(k_cg_spmv, dim3(g), dim3(kKBlock), 0, s, A, z, po, pn, q, H->partials.p, H->ks.p);
                    }
                    {
                        ProfScope ps(K_KRYLOV_UPDATE, 6 * vec, s);
                        hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(kKBlock), 0, s, n, x, r, pn, q, H->partials.p, H->ks.p);
                    }
                    vcycle(H, r, z, done, s);
                    {
                        ProfScope ps(K_KRYLOV_DOT, 3 * vec, s);
                        hipLaunchKernelGGL(k_cg_beta, dim3(g), dim3(kKBlock), 0, s, n, r, z, q, 0, H->partials.p, H->ks.p);
                    }
                    parity ^= 1;
                }
                GW_HIP(hipGetLastError());
                k = read_ks(H, s);
                if (k.done) break;
            }
        }
        {
            ProfScope ps(K_TRUE_RESIDUAL, abytes + 2 * vec, s);
            hipLaunchKernelGGL(k_true_res, dim3(g), dim3(kKBlock), 0, s, A, b, x, H->partials.p, H->ks.p);
        }
        k = read_ks(H, s);
        if (k.status == GW_BREAKDOWN) break;
        if (k.rel_true <= sp.rtol) { k.status = GW_OK; break; }
        if (k.iters >= k.maxiter || restarts >= 8) { k.status = GW_NOT_CONVERGED; break; }
        ++restarts;
        parity = 0;
        hipLaunchKernelGGL(k_kr_init, dim3(g), dim3(kKBlock), 0, s, A, b, x, r, (double *)nullptr, pa,
                           (double *)nullptr, sp.rtol, 0, H->partials.p, H->ks.p);
        k = read_ks(H, s);
    }
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

int krylov_bicgstab(amg_hierarchy *H, const double *b, double *x, const amg_solve_params &sp,
                    amg_solve_info *info, hipStream_t s) {
    const double t0 = now_ms();
    const CsrView A = view(H->L[0].A);
    const int64_t n = A.n;
    ensure_krylov_workspace(H, 8);
    double *r = H->kvec.p, *rh = r + n, *p = rh + n, *v = p + n, *sv = v + n, *t = sv + n, *ph = t + n,
           *sh = ph + n;
    KScalars k0{};
    k0.maxiter = std::max(0, sp.maxiter);
    k0.status = GW_NOT_CONVERGED;
    write_ks(H, k0, s);
    fill_f64(x, 0.0, n, s);
    const unsigned g = kgrid(n);
    const double vec = 8.0 * n, abytes = csr_bytes(A.n, A.nnz, 8);
    {
        ProfScope ps(K_KRYLOV_SPMV, abytes + 6 * vec, s);
        hipLaunchKernelGGL(k_kr_init, dim3(g), dim3(kKBlock), 0, s, A, b, x, r, rh, p, v, sp.rtol, 1, H->partials.p,
                           H->ks.p);
    }
    KScalars k = read_ks(H, s);
    int restarts = 0;
    if (k.bnorm == 0.0) {
        if (info) *info = {0, GW_OK, 0, 0.0, 0.0, 0.0, now_ms() - t0};
        return GW_OK;
    }
    const int check = std::max(1, sp.check_every);
    int32_t *done = &H->ks.p->done;
    for (;;) {
        while (!k.done) {
            for (int c = 0; c < check; ++c) {
                {
                    ProfScope ps(K_KRYLOV_UPDATE, 4 * vec, s);
                    hipLaunchKernelGGL(k_bcg_p, dim3(g), dim3(kKBlock), 0, s, n, r, p, v, H->ks.p);
                }
                vcycle(H, p, ph, done, s);
                {
                    ProfScope ps(K_KRYLOV_SPMV, abytes + 3 * vec, s);
                    hipLaunchKernelGGL(k_bcg_v, dim3(g), dim3(kKBlock), 0, s, A, ph, v, rh, H->partials.p, H->ks.p);
                }
                {
                    ProfScope ps(K_KRYLOV_UPDATE, 3 * vec, s);
                    hipLaunchKernelGGL(k_bcg_s, dim3(g), dim3(kKBlock), 0, s, n, r, v, sv, H->partials.p, H->ks.p);
                }
                vcycle(H, sv, sh, done, s);
                {
                    ProfScope ps(K_KRYLOV_SPMV, abytes + 3 * vec, s);
                    hipLaunchKernelGGL(k_bcg_t, dim3(g), dim3(kKBlock), 0, s, A, sh, t, sv, H->partials.p, H->ks.p);
                }
                {
                    ProfScope ps(K_KRYLOV_UPDATE, 8 * vec, s);
                    hipLaunchKernelGGL(k_bcg_xr, dim3(g), dim3(kKBlock), 0, s, n, x, r, ph, sh, sv, t, rh, H->partials.p,
                                       H->ks.p);
                }
            }
            GW_HIP(hipGetLastError());
            k = read_ks(H, s);
        }
        {
            ProfScope ps(K_TRUE_RESIDUAL, abytes + 2 * vec, s);
            hipLaunchKernelGGL(k_true_res, dim3(g), dim3(kKBlock), 0, s, A, b, x, H->partials.p, H->ks.p);
        }
        k = read_ks(H, s);
        if (k.status == GW_BREAKDOWN) break;
        if (k.rel_true <= sp.rtol) { k.status = GW_OK; break; }
        if (k.iters >= k.maxiter || restarts >= 8) { k.status = GW_NOT_CONVERGED; break; }
        ++restarts;
        hipLaunchKernelGGL(k_kr_init, dim3(g), dim3(kKBlock), 0, s, A, b, x, r, rh, p, v, sp.rtol, 0, H->partials.p,
                           H->ks.p);
        k = read_ks(H, s);
    }
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

}  // namespace gw
