// Solve phase: the V-cycle (Introduction: restrict the residual, smooth,
// recurse to a direct solve on the coarsest level, interpolate and correct,
// smooth -- only sparse matrix-vector products) and the Krylov methods it
// preconditions: CG for the symmetric flow system and BiCGSTAB for the
// upwind travel-time system (Benchmarking Examples).
//
// Every product kernel is written once against an operator type: OpSell (the
// sliced ELL copy of the level-0 operator, one lane per row, dictionary of
// column offsets in LDS) or OpCsr<G> (G lanes per CSR row, G picked per
// matrix from its mean row length, so the lanes of a wave read consecutive
// entries).  The Krylov scalars live on the device: a product kernel leaves
// per-block partial sums, a one-block finalize kernel adds them in a fixed
// order and forms alpha/beta/omega and the convergence flag; every later
// kernel reads the flag and returns at once, so the host only polls it every
// few iterations.  FP64 throughout the Krylov layer; the hierarchy is FP64 or
// FP32 (mixed mode).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "gw_device.h"
#include "gw_internal.h"
#include "solve_kernels.h"

namespace gw {

namespace {

// ------------------------------------------- kernels of their own ------
// Each launches a body of solve_kernels.h on its own grid.
template <class OP, class V, class Bt, class Yt, int NR>
__global__ void k_smooth_first(int64_t n, OP op, const V *__restrict__ M, const Bt *__restrict__ b,
                               Yt *__restrict__ y, int two, const int32_t *done) {
    smooth_first_body<OP, V, Bt, Yt, NR>(VG::here(), n, op, M, b, y, two, done);
}

template <class OP, class V, class Bt, class Xt, class Yt, int NR>
__global__ void k_smooth(int64_t n, OP op, const V *__restrict__ M, const Bt *__restrict__ b,
                         const Xt *__restrict__ x, Yt *__restrict__ y, const int32_t *done) {
    smooth_body<OP, V, Bt, Xt, Yt, NR>(VG::here(), n, op, M, b, x, y, done);
}

template <class OP, class V, class Bt, class Rt, int NR>
__global__ void k_smooth_res(int64_t n, OP op, const V *__restrict__ M, const Bt *__restrict__ b, V *__restrict__ y,
                             Rt *__restrict__ r, const int32_t *done) {
    smooth_res_body<OP, V, Bt, Rt, NR>(VG::here(), n, op, M, b, y, r, done);
}

template <class OP, class V, class Bt, class Xt, class Rt, int NR>
__global__ void k_residual(int64_t n, OP op, const Bt *__restrict__ b, const Xt *__restrict__ x,
                           Rt *__restrict__ r, const int32_t *done) {
    residual_body<OP, V, Bt, Xt, Rt, NR>(VG::here(), n, op, b, x, r, done);
}

template <class OP, class V, class Xt, class Yt, int NR>
__global__ void k_spmv(int64_t n, OP op, const Xt *__restrict__ x, Yt *__restrict__ y, const int32_t *done) {
    spmv_body<OP, V, Xt, Yt, NR>(VG::here(), n, op, x, y, done);
}

template <class OP, class V, int NR>
__global__ void k_restrict(int64_t n, OP op, const V *__restrict__ t, V *__restrict__ bc, const V *__restrict__ Mc,
                           V *__restrict__ x1, const int32_t *done) {
    restrict_body<OP, V, NR>(VG::here(), n, op, t, bc, Mc, x1, done);
}

template <class OP, class V, class Xt, int NR>
__global__ void k_prolong(int64_t n, OP op, const Xt *__restrict__ xc, Xt *__restrict__ x, const int32_t *done) {
    prolong_body<OP, V, Xt, NR>(VG::here(), n, op, xc, x, done);
}

template <class Bt, class Yt, int NR>
__global__ void k_coarse_gemv(int32_t n, const double *__restrict__ inv, const Bt *__restrict__ b,
                              Yt *__restrict__ y, const int32_t *done) {
    coarse_gemv_body<Bt, Yt, NR>(VG::here(), n, inv, b, y, done);
}

template <class X>
__global__ void k_zero(X *x, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = (X)0;
}

// y = x + z (ILU(0) smoothing step; y may be x)
__global__ void k_add(const double *x, const double *__restrict__ z, double *y, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + z[i];
}

template <class Xt, class Yt>
__global__ void k_convert(const Xt *__restrict__ x, Yt *__restrict__ y, int64_t n, const int32_t *done) {
    if (done && *done) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (Yt)x[i];
}

// One V-cycle on level l for NR right-hand sides (interleaved).  `b` is the
// right-hand side (type Bt), the result goes to `out` (type Zt) when given,
// else into one of the level's own buffers, whose address is returned.  V =
// value type of the hierarchy (also the type of all internal vectors).
// x1_ready: the restriction that formed b also wrote the first sweep from
// x = 0 (x1 = M b) into the level's x buffer.
template <class V, class Bt, class Zt, int NR>
void *vcycle_level(amg_hierarchy *H, int l, const Bt *b, Zt *out, const int32_t *done, hipStream_t s,
                   bool x1_ready = false);


// A level with the ILU(0) smoother (FP64, one right-hand side): each sweep is
// x <- x + (LU)^{-1} (b - A x), the first from x = 0 being x = (LU)^{-1} b.
template <class Zt>
void *vcycle_level_ilu(amg_hierarchy *H, int l, const double *b, Zt *out, const int32_t *done, hipStream_t s) {
    Level &Lv = H->L[l];
    IluData &I = *Lv.ilu;
    const int64_t n = Lv.A.n;
    double *x = reinterpret_cast<double *>(Lv.vx.p);
    double *t = reinterpret_cast<double *>(Lv.vt.p);
    const int npre = H->prm.npre, npost = H->prm.npost;
    const double abytes = op_bytes(Lv, 8);
    auto residual = [&](const double *xin, double *r) {
        ProfScope ps(level_kid(K_RESIDUAL0, l), abytes + n * 24.0, s, true);
        with_level_op<double>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_residual<OP, double, double, double, double, 1>), dim3(grid_rows(n, OP::G)),
                               dim3(kBlock), 0, s, n, op, b, xin, r, done);
        });
    };
    auto step = [&](double *xio, double *dst) {  // dst = x + (LU)^{-1}(b - A x)
        residual(xio, I.r.p);
        ilu_apply(I, I.r.p, I.z.p, done, s);
        hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(kBlock), 0, s, xio, I.z.p, dst, n, done);
    };
    if (npre == 0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n, done);
    } else {
        ilu_apply(I, b, x, done, s);
        for (int k = 1; k < npre; ++k) step(x, x);
    }
    residual(x, t);
    Level &Nx = H->L[l + 1];
    double *bc = reinterpret_cast<double *>(Nx.vb.p);
    const int64_t nc = Lv.nc;
    {
        ProfScope ps(level_kid(K_RESTRICT0, l), csr_bytes(nc, Lv.R.nnz, 8) + (double)(n + nc) * 8, s, true);
        with_csr<double>(Lv.R, Lv.R.val.p, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_spmv<OP, double, double, double, 1>), dim3(grid_rows(nc, OP::G)), dim3(kBlock), 0,
                               s, nc, op, t, bc, done);
        });
    }
    double *xc = static_cast<double *>(vcycle_level<double, double, double, 1>(H, l + 1, bc, (double *)nullptr,
                                                                               done, s));
    {
        ProfScope ps(level_kid(K_PROLONG0, l), csr_bytes(n, Lv.P.nnz, 8) + (double)(2 * n + nc) * 8, s, true);
        with_csr<double>(Lv.P, Lv.P.val.p, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_prolong<OP, double, double, 1>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n,
                               op, xc, x, done);
        });
    }
    for (int k = 0; k < npost; ++k) {
        if (k == npost - 1 && out && std::is_same_v<Zt, double>) {
            step(x, reinterpret_cast<double *>(out));
            return out;
        }
        step(x, x);
    }
    if (out) {
        hipLaunchKernelGGL((k_convert<double, Zt>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, out, n, done);
        return out;
    }
    return x;
}

template <class V, class Bt, class Zt, int NR>
void *vcycle_level(amg_hierarchy *H, int l, const Bt *b, Zt *out, const int32_t *done, hipStream_t s,
                   bool x1_ready) {
    Level &Lv = H->L[l];
    const int64_t n = Lv.A.n;
    const int vb = (int)sizeof(V);
    const double nr = NR;
    if (l == H->nlev - 1) {
        Zt *y = out ? out : reinterpret_cast<Zt *>(Lv.vx.p);
        ProfScope ps(K_COARSE_SOLVE, (double)n * n * 8 + nr * n * (double)(sizeof(Bt) + sizeof(Zt)), s);
        hipLaunchKernelGGL((k_coarse_gemv<Bt, Zt, NR>), dim3(blocks_for(n * dev::kWave)), dim3(kBlock), 0, s,
                           (int32_t)n, H->inv.p, b, y, done);
        return y;
    }
    const V *M = LevelOps<V>::mval(Lv);
    const double abytes = op_bytes(Lv, vb), cabytes = csr_bytes(n, Lv.A.nnz, vb);
    V *x = reinterpret_cast<V *>(Lv.vx.p);
    V *t = reinterpret_cast<V *>(Lv.vt.p);
    const int npre = H->prm.npre, npost = H->prm.npost;
    if constexpr (std::is_same_v<V, double> && std::is_same_v<Bt, double> && NR == 1) {
        if (Lv.ilu) return vcycle_level_ilu<Zt>(H, l, b, out, done, s);
    }

    Level &Nx = H->L[l + 1];
    V *bc = reinterpret_cast<V *>(Nx.vb.p);
    const int64_t nc = Lv.nc;
    // pre-smoothing; sweeps done counts those behind x
    int swept = 0;
    if (x1_ready) {
        swept = 1;  // x1 = M b, written with b by the restriction
    } else if (npre == 0) {
        hipLaunchKernelGGL((k_zero<V>), dim3(blocks_for(n * NR)), dim3(kBlock), 0, s, x, n * NR, done);
    } else if (npre == 1) {
        // the one sweep (x = M b) and the residual in one pass (into t)
        const double vec = n * (double)vb + nr * n * (double)(sizeof(Bt) + 2 * vb);
        ProfScope ps(level_kid(K_RESIDUAL0, l), abytes + vec, s, true, cabytes + vec);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_smooth_res<OP, V, Bt, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n,
                               op, M, b, x, t, done);
        });
        swept = 1;
    } else {
        const double vec = n * (double)vb + nr * n * (double)(sizeof(Bt) + vb);
        ProfScope ps(level_kid(K_SMOOTH_FIRST0, l), (npre >= 2 ? abytes : 0.0) + vec, s, true,
                     (npre >= 2 ? cabytes : 0.0) + vec);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_smooth_first<OP, V, Bt, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n,
                               op, M, b, x, npre >= 2 ? 1 : 0, done);
        });
        swept = npre >= 2 ? 2 : 1;
    }
    auto sweep = [&](auto *xin, auto *yout) {
        using YT = std::remove_pointer_t<decltype(yout)>;
        const double vec = n * (double)vb + nr * n * (double)(sizeof(Bt) + vb + sizeof(YT));
        ProfScope ps(level_kid(K_SMOOTH0, l), abytes + vec, s, true, cabytes + vec);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_smooth<OP, V, Bt, V, YT, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, op,
                               M, b, xin, yout, done);
        });
    };
    for (int k = swept; k < npre; ++k) {
        sweep(x, t);
        std::swap(x, t);
    }
    // residual (formed with the first sweep when that was the only one and
    // came from k_smooth_res) and restriction
    if (!(npre == 1 && !x1_ready)) {
        const double vec = nr * n * (double)(sizeof(Bt) + 2 * vb);
        ProfScope ps(level_kid(K_RESIDUAL0, l), abytes + vec, s, true, cabytes + vec);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_residual<OP, V, Bt, V, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, op,
                               b, x, t, done);
        });
    }
    const bool x1c = restrict_writes_x1(H, l);
    {
        const double x1b = x1c ? nc * (double)vb + nr * nc * (double)vb : 0.0;
        ProfScope ps(level_kid(K_RESTRICT0, l), csr_bytes(nc, Lv.R.nnz, vb) + nr * (double)(n + nc) * vb + x1b, s,
                     true);
        with_csr<V>(Lv.R, LevelOps<V>::rval(Lv), [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_restrict<OP, V, NR>), dim3(grid_rows(nc, OP::G)), dim3(kBlock), 0, s, nc, op, t,
                               bc, x1c ? LevelOps<V>::mval(Nx) : (const V *)nullptr,
                               x1c ? reinterpret_cast<V *>(Nx.vx.p) : (V *)nullptr, done);
        });
    }
    V *xc = static_cast<V *>(vcycle_level<V, V, V, NR>(H, l + 1, bc, (V *)nullptr, done, s, x1c));
    {
        ProfScope ps(level_kid(K_PROLONG0, l), csr_bytes(n, Lv.P.nnz, vb) + nr * (double)(2 * n + nc) * vb, s, true);
        with_csr<V>(Lv.P, LevelOps<V>::pval(Lv), [&](auto op) {
            using OP = decltype(op);
            GW_LAUNCH_TIMED(ps, (k_prolong<OP, V, V, NR>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, op, xc, x,
                               done);
        });
    }
    // post-smoothing; the last sweep writes the requested output
    for (int k = 0; k < npost; ++k) {
        if (k == npost - 1 && out) {
            sweep(x, out);
            return out;
        }
        sweep(x, t);
        std::swap(x, t);
    }
    if (out) {
        hipLaunchKernelGGL((k_convert<V, Zt>), dim3(blocks_for(n * NR)), dim3(kBlock), 0, s, x, out, n * NR, done);
        return out;
    }
    return x;
}

// -------------------------------------------------------------- Krylov ---
template <class OP>
__global__ void __launch_bounds__(kKBlock) k_kr_init(int64_t n, OP op, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ rh, double *__restrict__ p,
                                                     double *__restrict__ v, double *partials) {
    kr_init_body<OP>(VG::here(), n, op, b, x, r, rh, p, v, partials);
}

__global__ void __launch_bounds__(kKBlock) k_cg_dot(int64_t n, const double *__restrict__ r,
                                                    const double *__restrict__ z, const double *__restrict__ q,
                                                    double *partials, const KScalars *ks) {
    cg_dot_body(VG::here(), n, r, z, q, partials, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_cg_spmv(int64_t n, OP op, const double *__restrict__ z,
                                                     const double *__restrict__ p_old, double *__restrict__ p_new,
                                                     double *__restrict__ q, double *partials, const KScalars *ks) {
    cg_spmv_body<OP>(VG::here(), n, op, z, p_old, p_new, q, partials, ks);
}

__global__ void __launch_bounds__(kKBlock) k_cg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                       const double *__restrict__ p, const double *__restrict__ q,
                                                       double *partials, const KScalars *ks) {
    cg_update_body(VG::here(), n, x, r, p, q, partials, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_true_res(int64_t n, OP op, const double *__restrict__ b,
                                                      const double *__restrict__ x, double *partials) {
    true_res_body<OP>(VG::here(), n, op, b, x, partials);
}

__global__ void __launch_bounds__(kKBlock) k_bcg_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                                   const double *__restrict__ v, const KScalars *ks) {
    bcg_p_body(VG::here(), n, r, p, v, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_v(int64_t n, OP op, const double *__restrict__ ph,
                                                   double *__restrict__ v, const double *__restrict__ rh,
                                                   double *partials, const KScalars *ks) {
    bcg_v_body<OP>(VG::here(), n, op, ph, v, rh, partials, ks);
}

__global__ void __launch_bounds__(kKBlock) k_bcg_s(int64_t n, const double *__restrict__ r,
                                                   const double *__restrict__ v, double *__restrict__ sv,
                                                   double *partials, const KScalars *ks) {
    bcg_s_body(VG::here(), n, r, v, sv, partials, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_t(int64_t n, OP op, const double *__restrict__ sh,
                                                   double *__restrict__ t, const double *__restrict__ sv,
                                                   double *partials, const KScalars *ks) {
    bcg_t_body<OP>(VG::here(), n, op, sh, t, sv, partials, ks);
}

__global__ void __launch_bounds__(kKBlock) k_bcg_xr(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ ph, const double *__restrict__ sh,
                                                    const double *__restrict__ sv, const double *__restrict__ t,
                                                    const double *__restrict__ rh, double *partials,
                                                    const KScalars *ks) {
    bcg_xr_body(VG::here(), n, x, r, ph, sh, sv, t, rh, partials, ks);
}

__global__ void __launch_bounds__(kKBlock) k_finalize(int op, unsigned nb, const double *partials, double rtol,
                                                      KScalars *ks) {
    finalize_body(op, nb, partials, rtol, ks);
}

__global__ void __launch_bounds__(kKBlock) k_finalize2(int op, unsigned nb, const double *partials, double rtol,
                                                       KScalars *ks, int mask) {
    finalize2_body(op, nb, partials, rtol, ks, mask);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_kr_init2(int64_t n, OP op, const double *__restrict__ b,
                                                      const double *__restrict__ x, double *__restrict__ r,
                                                      double *__restrict__ rh, double *__restrict__ p,
                                                      double *__restrict__ v, double *partials, int mask) {
    kr_init2_body<OP>(VG::here(), n, op, b, x, r, rh, p, v, partials, mask);
}

__global__ void __launch_bounds__(kKBlock) k_bcg_p2(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                                    const double *__restrict__ v, const KScalars *ks) {
    bcg_p2_body(VG::here(), n, r, p, v, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_v2(int64_t n, OP op, const double *__restrict__ ph,
                                                    double *__restrict__ v, const double *__restrict__ rh,
                                                    double *partials, const KScalars *ks) {
    bcg_v2_body<OP>(VG::here(), n, op, ph, v, rh, partials, ks);
}

__global__ void __launch_bounds__(kKBlock) k_bcg_s2(int64_t n, const double *__restrict__ r,
                                                    const double *__restrict__ v, double *__restrict__ sv,
                                                    double *partials, const KScalars *ks) {
    bcg_s2_body(VG::here(), n, r, v, sv, partials, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_bcg_t2(int64_t n, OP op, const double *__restrict__ sh,
                                                    double *__restrict__ t, const double *__restrict__ sv,
                                                    double *partials, const KScalars *ks) {
    bcg_t2_body<OP>(VG::here(), n, op, sh, t, sv, partials, ks);
}

__global__ void __launch_bounds__(kKBlock) k_bcg_xr2(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ ph, const double *__restrict__ sh,
                                                     const double *__restrict__ sv, const double *__restrict__ t,
                                                     const double *__restrict__ rh, double *partials,
                                                     const KScalars *ks) {
    bcg_xr2_body(VG::here(), n, x, r, ph, sh, sv, t, rh, partials, ks);
}

template <class OP>
__global__ void __launch_bounds__(kKBlock) k_true_res2(int64_t n, OP op, const double *__restrict__ b,
                                                       const double *__restrict__ x, double *partials) {
    true_res2_body<OP>(VG::here(), n, op, b, x, partials);
}

__global__ void k_interleave(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                             double *__restrict__ ab) {
    interleave_body(VG::here(), n, a, b, ab);
}

__global__ void k_split(int64_t n, const double *__restrict__ ab, double *__restrict__ a, double *__restrict__ b) {
    split_body(VG::here(), n, ab, a, b);
}

template <class OP>
__global__ void k_spmv_f64(int64_t n, OP op, const double *__restrict__ x, double *__restrict__ y) {
    OP_PROLOGUE(op)
    GROUP_ROW(OP::G)
    double s = op.row(i, lane, sd_, [&](int32_t j) { return x[j]; });
    if (lane == 0) y[i] = s;
}


static_assert(sizeof(KScalars) <= kHostStageBytes, "Krylov scalars must fit the pinned stage");

// Where a Krylov solve keeps its n-vectors (one after another), its block
// partials (kKMaxBlocks x 4) and its scalar records.  `staged`: the scalars
// travel through the calling thread's pinned stage; otherwise through a
// host variable (a pageable copy: nothing is allocated for it).
struct KWork {
    double *vec;
    double *part;
    KScalars *ks;
    bool staged;
};

KWork hier_work(amg_hierarchy *H) { return KWork{H->kvec.p, H->partials.p, H->ks.p, true}; }

KScalars read_ks(const KWork &W, hipStream_t s) {
    KScalars k;
    if (!W.staged) {
        GW_HIP(hipMemcpyAsync(&k, W.ks, sizeof(KScalars), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        return k;
    }
    void *stage = host_stage();
    GW_HIP(hipMemcpyAsync(stage, W.ks, sizeof(KScalars), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    std::memcpy(&k, stage, sizeof(KScalars));
    return k;
}

void write_ks(const KWork &W, const KScalars &k, hipStream_t s) {
    if (!W.staged) {
        KScalars h = k;
        GW_HIP(hipMemcpyAsync(W.ks, &h, sizeof(KScalars), hipMemcpyHostToDevice, s));
        GW_HIP(hipStreamSynchronize(s));
        return;
    }
    void *stage = host_stage();
    std::memcpy(stage, &k, sizeof(KScalars));
    GW_HIP(hipMemcpyAsync(W.ks, stage, sizeof(KScalars), hipMemcpyHostToDevice, s));
    GW_HIP(hipStreamSynchronize(s));
}

static_assert(3 * sizeof(KScalars) <= kHostStageBytes, "two systems' scalars must fit the pinned stage");

void read_ks3(amg_hierarchy *H, KScalars (&k)[3], hipStream_t s) {
    void *stage = host_stage();
    GW_HIP(hipMemcpyAsync(stage, H->ks.p, 3 * sizeof(KScalars), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    std::memcpy(k, stage, 3 * sizeof(KScalars));
}

void write_ks3(amg_hierarchy *H, const KScalars (&k)[3], hipStream_t s) {
    void *stage = host_stage();
    std::memcpy(stage, k, 3 * sizeof(KScalars));
    GW_HIP(hipMemcpyAsync(H->ks.p, stage, 3 * sizeof(KScalars), hipMemcpyHostToDevice, s));
    GW_HIP(hipStreamSynchronize(s));
}

KScalars read_ks(amg_hierarchy *H, hipStream_t s) { return read_ks(hier_work(H), s); }

void write_ks(amg_hierarchy *H, const KScalars &k, hipStream_t s) { write_ks(hier_work(H), k, s); }

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum BlockKind : int { BLOCK_PCG = 1, BLOCK_BICGSTAB = 2, BLOCK_BICGSTAB2 = 3 };

// Enqueue one block of Krylov iterations on s: `emit(stream)` launches its
// kernels.  With `graph`, the block is captured once per (kind, length,
// parity) on the hierarchy's capture stream, which runs nothing, and the
// instantiated graph is launched on s.  Every kernel reads its scalars and
// the convergence flag from device memory, so a replay after convergence is
// a run of early exits, exactly as the one-by-one launches are.
template <class Emit>
void run_block(amg_hierarchy *H, bool graph, int kind, int check, int parity, hipStream_t s, Emit &&emit) {
    if (!graph) {
        emit(s);
        return;
    }
    hipGraphExec_t ex = nullptr;
    for (const auto &g : H->graphs)
        if (g.kind == kind && g.check == check && g.parity == parity) ex = g.exec;
    if (!ex) {
        if (!H->cap) GW_HIP(hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
        GW_HIP(hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal));
        hipGraph_t g = nullptr;
        try {
            emit(H->cap);
        } catch (...) {
            if (hipStreamEndCapture(H->cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            throw;
        }
        GW_HIP(hipStreamEndCapture(H->cap, &g));
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        GW_HIP(e);
        H->graphs.push_back({kind, check, parity, ex});
    }
    GW_HIP(hipGraphLaunch(ex, s));
}

bool use_graph(const amg_solve_params &sp) { return sp.graph > 0; }

// Host-side helper binding the level-0 operator and the scalar block.
struct Kry {
    amg_hierarchy *H;
    const Level &L0;
    int G;
    int64_t n;
    unsigned g1, gG;  // grids of element-wise and row-product kernels
    double *part;
    KScalars *ks;
    hipStream_t s;
    double rtol;
    double vec, abytes, cabytes;
    const double *shift = nullptr;  // diagonal added to A (OpShift), or none

    Kry(amg_hierarchy *H_, hipStream_t s_, double rtol_) : Kry(H_, hier_work(H_), s_, rtol_) {}
    Kry(amg_hierarchy *H_, const KWork &W, hipStream_t s_, double rtol_) : H(H_), L0(H_->L[0]), s(s_), rtol(rtol_) {
        G = (L0.St.built() || L0.As.built()) ? 1 : L0.A.grp;
        n = L0.A.n;
        g1 = kgrid(n, 1);
        gG = kgrid(n, G);
        part = W.part;
        ks = W.ks;
        vec = 8.0 * n;
        abytes = op_bytes(L0, 8);
        cabytes = csr_bytes(n, L0.A.nnz, 8);
    }
    template <bool SHIFT = false, class F>
    void op(F &&f) const {
        if constexpr (SHIFT) {
            if (L0.St.built()) f(OpShift<OpSten<double>>{sten_op<double>(L0.St, L0.St.c.p), shift});
            else if (L0.As.built()) f(OpShift<OpSell<double>>{OpSell<double>{view(L0.As), L0.As.val.p}, shift});
            else with_csr<double>(L0.A, L0.A.val.p, [&](auto o) { f(OpShift<decltype(o)>{o, shift}); });
        } else {
            if (L0.St.built()) f(sten_op<double>(L0.St, L0.St.c.p));
            else if (L0.As.built()) f(OpSell<double>{view(L0.As), L0.As.val.p});
            else with_csr<double>(L0.A, L0.A.val.p, f);
        }
    }
    void fin(int code, unsigned nb) {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kKBlock), 0, s, code, nb, part, rtol, ks);
    }
    template <bool SHIFT = false>
    void init(const double *b, const double *x, double *r, double *rh, double *p, double *v, bool first) {
        {
            ProfScope ps(K_KRYLOV_SPMV, abytes + 4 * vec + (rh ? 3 * vec : 0), s, false, cabytes + 4 * vec + (rh ? 3 * vec : 0));
            op<SHIFT>([&](auto o) {
                hipLaunchKernelGGL((k_kr_init<decltype(o)>), dim3(gG), dim3(kKBlock), 0, s, n, o, b, x, r, rh, p, v,
                                   part);
            });
        }
        fin(first ? FIN_INIT_FIRST : FIN_INIT_RESTART, gG);
    }
    template <bool SHIFT = false>
    void true_res(const double *b, const double *x) {
        {
            ProfScope ps(K_TRUE_RESIDUAL, abytes + 2 * vec, s, false, cabytes + 2 * vec);
            op<SHIFT>([&](auto o) {
                hipLaunchKernelGGL((k_true_res<decltype(o)>), dim3(gG), dim3(kKBlock), 0, s, n, o, b, x, part);
            });
        }
        fin(FIN_TRUE_RES, gG);
    }
};

}  // namespace

void ensure_krylov_workspace(amg_hierarchy *H, int nvec) {
    const size_t n = (size_t)H->L[0].A.n;
    if (H->kvec_count < nvec) {
        H->drop_graphs();
        H->kvec.alloc(n * nvec);
        H->kvec_count = nvec;
    }
    if (!H->partials.p) H->partials.alloc((size_t)kKMaxBlocks * 4);
    if (!H->ks.p) H->ks.alloc(3);
}

// Level vectors sized for nr interleaved right-hand sides.
void ensure_level_vectors(amg_hierarchy *H, int nr) {
    const size_t es = H->mixed() ? 4 : 8;
    for (int l = 0; l < H->nlev; ++l) {
        Level &Lv = H->L[l];
        const size_t need = (size_t)Lv.A.n * es * nr;
        if (Lv.vx.n >= need) continue;
        H->drop_graphs();
        Lv.vx.alloc(need);
        Lv.vt.alloc(need);
        if (l > 0) Lv.vb.alloc(need);
    }
}

int lane_group_for(double mean_row_len) {
    if (mean_row_len <= 3.0) return 1;
    if (mean_row_len <= 12.0) return 4;
    if (mean_row_len <= 48.0) return 16;
    return 64;
}

// Solve-phase products load 8 entries per lane (4 with 64 lanes) before
// summing: a row gets the fewest lanes G (a power of two) whose 8G slots
// hold 1.4 times the mean row length, so a typical row is one round and the
// wave covers as many rows as possible.  Measured against 1/4/16/64 lanes
// with 4/2/2/1 loads per lane: 8.4M-cell pass 215 -> 172 ms, 1M-cell pass
// 32.0 -> 30.5 ms (level-1 sweeps of ~33-entry rows 15 -> 11.6 us).
int solve_group_for(double mean_row_len) {
    int g = 1;
    while (g < 64 && 8.0 * g < 1.4 * mean_row_len) g *= 2;
    return g;
}

void vcycle(amg_hierarchy *H, const double *r, double *z, const int32_t *done, hipStream_t s) {
    if (H->nlev == 0) {
        // preconditioner off: z = r
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks_for(H->L[0].A.n)), dim3(kBlock), 0, s, r, z,
                           (int64_t)H->L[0].A.n, done);
        GW_HIP(hipGetLastError());
        return;
    }
    if (H->mixed()) vcycle_level<float, double, double, 1>(H, 0, r, z, done, s);
    else vcycle_level<double, double, double, 1>(H, 0, r, z, done, s);
    GW_HIP(hipGetLastError());
}

namespace {


// One V-cycle on two interleaved right-hand sides.
void vcycle2(amg_hierarchy *H, const double *r, double *z, const int32_t *done, hipStream_t s) {
    if (H->nlev == 0) {
        const int64_t n2 = 2 * (int64_t)H->L[0].A.n;
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks_for(n2)), dim3(kBlock), 0, s, r, z, n2, done);
        GW_HIP(hipGetLastError());
        return;
    }
    if (H->mixed()) vcycle_level<float, double, double, 2>(H, 0, r, z, done, s);
    else vcycle_level<double, double, double, 2>(H, 0, r, z, done, s);
    GW_HIP(hipGetLastError());
}

}  // namespace

void spmv_level0(amg_hierarchy *H, const double *x, double *y, hipStream_t s) {
    const Level &L0 = H->L[0];
    const int64_t n = L0.A.n;
    ProfScope ps(K_KRYLOV_SPMV, op_bytes(L0, 8) + 16.0 * n, s, false, csr_bytes(n, L0.A.nnz, 8) + 16.0 * n);
    auto launch = [&](auto o) {
        using OP = decltype(o);
        hipLaunchKernelGGL((k_spmv_f64<OP>), dim3(grid_rows(n, OP::G)), dim3(kBlock), 0, s, n, o, x, y);
    };
    if (L0.St.built()) launch(sten_op<double>(L0.St, L0.St.c.p));
    else if (L0.As.built()) launch(OpSell<double>{view(L0.As), L0.As.val.p});
    else with_csr<double>(L0.A, L0.A.val.p, launch);
    GW_HIP(hipGetLastError());
}

namespace {

// PCG on A (SHIFT false) or on A + diag(shift) with the hierarchy of A as the
// preconditioner (SHIFT true; launched one by one: a captured graph would
// keep the shift pointer of its first call).  W holds six n-vectors, the
// block partials and the scalars; graph replay needs W to be the
// hierarchy's own workspace (the captured blocks keep its addresses).
template <bool SHIFT>
int pcg_impl(amg_hierarchy *H, const KWork &W, const double *shift, const double *b, double *x_out,
             const amg_solve_params &sp, amg_solve_info *info, hipStream_t s) {
    const double t0 = now_ms();
    Kry K(H, W, s, sp.rtol);
    K.shift = shift;
    const int64_t n = K.n;
    // the iterate lives in the workspace (a captured block then serves any
    // output buffer) and is copied out at the end
    double *r = W.vec, *z = r + n, *pa = z + n, *pb = pa + n, *q = pb + n, *x = q + n;
    KScalars k0{};
    k0.maxiter = std::max(0, sp.maxiter);
    k0.flexible = sp.flexible < 0 ? (H->mixed() ? 1 : 0) : (sp.flexible ? 1 : 0);
    k0.status = GW_NOT_CONVERGED;
    write_ks(W, k0, s);
    fill_f64(x, 0.0, n, s);
    K.template init<SHIFT>(b, x, r, nullptr, pa, nullptr, true);
    KScalars k = read_ks(W, s);
    int restarts = 0;
    if (k.bnorm == 0.0) {
        fill_f64(x_out, 0.0, n, s);
        if (info) *info = {0, GW_OK, 0, 0.0, 0.0, 0.0, now_ms() - t0};
        return GW_OK;
    }
    const int check = std::max(1, sp.check_every);
    const bool graph = !SHIFT && use_graph(sp) && W.vec == H->kvec.p;
    int32_t *done = &W.ks->done;
    int parity = 0;
    int cnt = check;  // iterations in the next block
    // check_every iterations: q = A p, alpha, x and r updates with the
    // convergence test, z = M r, beta
    auto block = [&](int parity0) {
        return [&, parity0](hipStream_t cs) {
            Kry Kc(H, W, cs, sp.rtol);
            Kc.shift = shift;
            int par = parity0;
            for (int c = 0; c < cnt; ++c) {
                double *po = par ? pb : pa, *pn = par ? pa : pb;
                {
                    ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 4 * Kc.vec, cs, true, Kc.cabytes + 4 * Kc.vec);
                    Kc.template op<SHIFT>([&](auto o) {
                        GW_LAUNCH_TIMED(ps, (k_cg_spmv<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, z, po,
                                           pn, q, Kc.part, Kc.ks);
                    });
                }
                Kc.fin(FIN_CG_ALPHA, Kc.gG);
                {
                    ProfScope ps(K_KRYLOV_UPDATE, 6 * Kc.vec, cs);
                    hipLaunchKernelGGL(k_cg_update, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, x, r, pn, q, Kc.part,
                                       Kc.ks);
                }
                Kc.fin(FIN_CG_CONV, Kc.g1);
                vcycle(H, r, z, done, cs);
                {
                    ProfScope ps(K_KRYLOV_DOT, 3 * Kc.vec, cs);
                    hipLaunchKernelGGL(k_cg_dot, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, z, q, Kc.part, Kc.ks);
                }
                Kc.fin(FIN_CG_BETA, Kc.g1);
                par ^= 1;
            }
            GW_HIP(hipGetLastError());
        };
    };
    for (;;) {
        if (!k.done) {
            vcycle(H, r, z, done, s);
            {
                ProfScope ps(K_KRYLOV_DOT, 3 * K.vec, s);
                hipLaunchKernelGGL(k_cg_dot, dim3(K.g1), dim3(kKBlock), 0, s, n, r, z, q, K.part, K.ks);
            }
            K.fin(FIN_CG_BETA_FIRST, K.g1);
            PollPlan plan{check, graph};
            cnt = check;
            for (;;) {
                run_block(H, graph, BLOCK_PCG, check, parity, s, block(parity));
                parity ^= cnt & 1;
                k = read_ks(W, s);
                if (k.done) break;
                cnt = plan.next(std::sqrt(k.rr), k.tol, k.iters);
            }
        }
        K.template true_res<SHIFT>(b, x);
        k = read_ks(W, s);
        if (k.status == GW_BREAKDOWN) break;
        if (k.rel_true <= sp.rtol) { k.status = GW_OK; break; }
        if (k.iters >= k.maxiter || restarts >= 8) { k.status = GW_NOT_CONVERGED; break; }
        ++restarts;
        parity = 0;
        K.template init<SHIFT>(b, x, r, nullptr, pa, nullptr, false);
        k = read_ks(W, s);
    }
    copy_bytes(x_out, x, sizeof(double) * (size_t)n, s);
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

}  // namespace

int krylov_pcg(amg_hierarchy *H, const double *b, double *x_out, const amg_solve_params &sp, amg_solve_info *info,
               hipStream_t s) {
    ensure_krylov_workspace(H, 6);
    return pcg_impl<false>(H, hier_work(H), nullptr, b, x_out, sp, info, s);
}

int krylov_pcg_shifted(amg_hierarchy *H, const double *shift, const double *b, double *x_out,
                       const amg_solve_params &sp, amg_solve_info *info, hipStream_t s) {
    ensure_krylov_workspace(H, 6);
    return pcg_impl<true>(H, hier_work(H), shift, b, x_out, sp, info, s);
}

// PCG with a workspace the caller provides (six n-vectors, kKMaxBlocks x 4
// block partials, one scalar record), scalars read through a host variable;
// launched one kernel at a time.
int krylov_pcg_in(amg_hierarchy *H, double *vec, double *part, KScalars *ks, const double *b, double *x_out,
                  const amg_solve_params &sp, amg_solve_info *info, hipStream_t s) {
    static_assert(kKMaxBlocks == kKrylovMaxBlocks, "partials of the caller's workspace");
    amg_solve_params one = sp;
    one.graph = 0;
    return pcg_impl<false>(H, KWork{vec, part, ks, false}, nullptr, b, x_out, one, info, s);
}

int krylov_bicgstab(amg_hierarchy *H, const double *b, double *x_out, const amg_solve_params &sp,
                    amg_solve_info *info, hipStream_t s) {
    const double t0 = now_ms();
    ensure_krylov_workspace(H, 9);
    Kry K(H, s, sp.rtol);
    const int64_t n = K.n;
    double *r = H->kvec.p, *rh = r + n, *p = rh + n, *v = p + n, *sv = v + n, *t = sv + n, *ph = t + n,
           *sh = ph + n, *x = sh + n;
    KScalars k0{};
    k0.maxiter = std::max(0, sp.maxiter);
    k0.status = GW_NOT_CONVERGED;
    write_ks(H, k0, s);
    fill_f64(x, 0.0, n, s);
    K.init(b, x, r, rh, p, v, true);
    KScalars k = read_ks(H, s);
    int restarts = 0;
    if (k.bnorm == 0.0) {
        fill_f64(x_out, 0.0, n, s);
        if (info) *info = {0, GW_OK, 0, 0.0, 0.0, 0.0, now_ms() - t0};
        return GW_OK;
    }
    const int check = std::max(1, sp.check_every);
    const bool graph = use_graph(sp);
    int32_t *done = &H->ks.p->done;
    int cnt = check;  // iterations in the next block
    // cnt iterations of right-preconditioned BiCGSTAB
    auto block = [&](hipStream_t cs) {
        Kry Kc(H, cs, sp.rtol);
        for (int c = 0; c < cnt; ++c) {
            {
                ProfScope ps(K_KRYLOV_UPDATE, 4 * Kc.vec, cs);
                hipLaunchKernelGGL(k_bcg_p, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, p, v, Kc.ks);
            }
            vcycle(H, p, ph, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * Kc.vec, cs, true, Kc.cabytes + 3 * Kc.vec);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_v<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, ph, v, rh,
                                       Kc.part, Kc.ks);
                });
            }
            Kc.fin(FIN_BCG_ALPHA, Kc.gG);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 3 * Kc.vec, cs);
                hipLaunchKernelGGL(k_bcg_s, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, v, sv, Kc.part, Kc.ks);
            }
            Kc.fin(FIN_BCG_S, Kc.g1);
            vcycle(H, sv, sh, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * Kc.vec, cs, true, Kc.cabytes + 3 * Kc.vec);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_t<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, sh, t, sv,
                                       Kc.part, Kc.ks);
                });
            }
            Kc.fin(FIN_BCG_OMEGA, Kc.gG);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 8 * Kc.vec, cs);
                hipLaunchKernelGGL(k_bcg_xr, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, x, r, ph, sh, sv, t, rh, Kc.part,
                                   Kc.ks);
            }
            Kc.fin(FIN_BCG_XR, Kc.g1);
        }
        GW_HIP(hipGetLastError());
    };
    for (;;) {
        PollPlan plan{check, graph};
        cnt = check;
        while (!k.done) {
            run_block(H, graph, BLOCK_BICGSTAB, check, 0, s, block);
            k = read_ks(H, s);
            cnt = plan.next(std::sqrt(k.rr), k.tol, k.iters);
        }
        K.true_res(b, x);
        k = read_ks(H, s);
        if (k.status == GW_BREAKDOWN) break;
        if (k.rel_true <= sp.rtol) { k.status = GW_OK; break; }
        if (k.iters >= k.maxiter || restarts >= 8) { k.status = GW_NOT_CONVERGED; break; }
        ++restarts;
        K.init(b, x, r, rh, p, v, false);
        k = read_ks(H, s);
    }
    copy_bytes(x_out, x, sizeof(double) * (size_t)n, s);
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

int krylov_bicgstab2(amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1,
                     const amg_solve_params &sp, amg_solve_info info[2], hipStream_t s) {
    if (H->prm.smoother == GW_SMOOTHER_ILU0) {
        // the substitution sweeps take one right-hand side: one system at a time
        const int s0 = krylov_bicgstab(H, b0, x0, sp, &info[0], s);
        const int s1 = krylov_bicgstab(H, b1, x1, sp, &info[1], s);
        return std::max(s0, s1);
    }
    const double t0 = now_ms();
    ensure_krylov_workspace(H, 20);
    ensure_level_vectors(H, 2);
    Kry K(H, s, sp.rtol);
    const int64_t n = K.n, n2 = 2 * n;
    double *b = H->kvec.p, *r = b + n2, *rh = r + n2, *p = rh + n2, *v = p + n2, *sv = v + n2, *t = sv + n2,
           *ph = t + n2, *sh = ph + n2, *x = sh + n2;
    double *part = K.part;
    KScalars *ks = K.ks;
    const double vec2 = 2 * K.vec;
    auto fin2 = [&](hipStream_t cs, int code, unsigned nb, int mask) {
        hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(kKBlock), 0, cs, code, nb, part, sp.rtol, ks, mask);
    };
    auto init2 = [&](int mask, bool first) {
        {
            ProfScope ps(K_KRYLOV_SPMV, K.abytes + 7 * vec2, s, false, K.cabytes + 7 * vec2);
            K.op([&](auto o) {
                hipLaunchKernelGGL((k_kr_init2<decltype(o)>), dim3(K.gG), dim3(kKBlock), 0, s, n, o, b, x, r, rh, p,
                                   v, part, mask);
            });
        }
        fin2(s, first ? FIN_INIT_FIRST : FIN_INIT_RESTART, K.gG, mask);
    };
    hipLaunchKernelGGL(k_interleave, dim3(K.g1), dim3(kKBlock), 0, s, n, b0, b1, b);
    KScalars kk[3] = {};
    kk[0].maxiter = kk[1].maxiter = std::max(0, sp.maxiter);
    kk[0].status = kk[1].status = GW_NOT_CONVERGED;
    write_ks3(H, kk, s);
    fill_f64(x, 0.0, n2, s);
    init2(3, true);
    read_ks3(H, kk, s);
    bool final[2] = {false, false};
    int restarts[2] = {0, 0}, status[2] = {GW_NOT_CONVERGED, GW_NOT_CONVERGED};
    bool zero_rhs = false;
    for (int k = 0; k < 2; ++k) {
        if (kk[k].bnorm != 0.0) continue;
        // b = 0: x = 0, nothing to iterate
        final[k] = true;
        status[k] = GW_OK;
        kk[k].done = 1;
        kk[k].iters = 0;
        kk[k].rr = 0.0;
        kk[k].rel_true = 0.0;
        zero_rhs = true;
    }
    if (zero_rhs) {
        kk[2].done = kk[0].done && kk[1].done;
        write_ks3(H, kk, s);
    }
    const int check = std::max(1, sp.check_every);
    const bool graph = use_graph(sp);
    const int32_t *done = &ks[2].done;
    int cnt = check;  // iterations in the next block
    auto block = [&](hipStream_t cs) {
        Kry Kc(H, cs, sp.rtol);
        for (int c = 0; c < cnt; ++c) {
            {
                ProfScope ps(K_KRYLOV_UPDATE, 4 * vec2, cs);
                hipLaunchKernelGGL(k_bcg_p2, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, p, v, ks);
            }
            vcycle2(H, p, ph, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * vec2, cs, true, Kc.cabytes + 3 * vec2);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_v2<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, ph, v, rh,
                                       part, ks);
                });
            }
            fin2(cs, FIN_BCG_ALPHA, Kc.gG, 3);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 3 * vec2, cs);
                hipLaunchKernelGGL(k_bcg_s2, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, r, v, sv, part, ks);
            }
            fin2(cs, FIN_BCG_S, Kc.g1, 3);
            vcycle2(H, sv, sh, done, cs);
            {
                ProfScope ps(K_KRYLOV_SPMV, Kc.abytes + 3 * vec2, cs, true, Kc.cabytes + 3 * vec2);
                Kc.op([&](auto o) {
                    GW_LAUNCH_TIMED(ps, (k_bcg_t2<decltype(o)>), dim3(Kc.gG), dim3(kKBlock), 0, cs, n, o, sh, t, sv,
                                       part, ks);
                });
            }
            fin2(cs, FIN_BCG_OMEGA, Kc.gG, 3);
            {
                ProfScope ps(K_KRYLOV_UPDATE, 8 * vec2, cs);
                hipLaunchKernelGGL(k_bcg_xr2, dim3(Kc.g1), dim3(kKBlock), 0, cs, n, x, r, ph, sh, sv, t, rh, part, ks);
            }
            fin2(cs, FIN_BCG_XR, Kc.g1, 3);
        }
        GW_HIP(hipGetLastError());
    };
    for (;;) {
        // the block ends when the slower of the running systems is predicted
        // to converge
        PollPlan plan[2] = {{check, graph}, {check, graph}};
        cnt = check;
        while (!kk[2].done) {
            run_block(H, graph, BLOCK_BICGSTAB2, check, 0, s, block);
            read_ks3(H, kk, s);
            int c2 = 1;
            for (int q = 0; q < 2; ++q) {
                const int cq = plan[q].next(std::sqrt(kk[q].rr), kk[q].tol, kk[q].iters);
                if (!kk[q].done) c2 = std::max(c2, cq);
            }
            cnt = c2;
        }
        {
            ProfScope ps(K_TRUE_RESIDUAL, K.abytes + 2 * vec2, s, false, K.cabytes + 2 * vec2);
            K.op([&](auto o) {
                hipLaunchKernelGGL((k_true_res2<decltype(o)>), dim3(K.gG), dim3(kKBlock), 0, s, n, o, b, x, part);
            });
        }
        fin2(s, FIN_TRUE_RES, K.gG, 3);
        read_ks3(H, kk, s);
        int mask = 0;
        for (int k = 0; k < 2; ++k) {
            if (final[k]) continue;
            const KScalars &q = kk[k];
            if (q.status == GW_BREAKDOWN) { status[k] = GW_BREAKDOWN; final[k] = true; continue; }
            if (q.rel_true <= sp.rtol) { status[k] = GW_OK; final[k] = true; continue; }
            if (q.iters >= q.maxiter || restarts[k] >= 8) { status[k] = GW_NOT_CONVERGED; final[k] = true; continue; }
            ++restarts[k];
            mask |= 1 << k;
        }
        if (!mask) break;
        init2(mask, false);
        read_ks3(H, kk, s);
    }
    hipLaunchKernelGGL(k_split, dim3(K.g1), dim3(kKBlock), 0, s, n, x, x0, x1);
    GW_HIP(hipGetLastError());
    const double ms = now_ms() - t0;
    for (int k = 0; k < 2; ++k) {
        if (!info) break;
        const KScalars &q = kk[k];
        info[k].iters = q.iters;
        info[k].status = status[k];
        info[k].restarts = restarts[k];
        info[k].rel_res = q.bnorm != 0.0 ? std::sqrt(q.rr) / q.bnorm : 0.0;
        info[k].rel_res_true = q.bnorm != 0.0 ? q.rel_true : 0.0;
        info[k].setup_ms = 0.0;
        info[k].solve_ms = ms;
    }
    if (status[0] == GW_BREAKDOWN || status[1] == GW_BREAKDOWN) return GW_BREAKDOWN;
    if (status[0] != GW_OK || status[1] != GW_OK) return GW_NOT_CONVERGED;
    return GW_OK;
}

}  // namespace gw
