// C ABI entry points (include/gwamg.h): argument checks, hierarchy
// lifetime, and the host-side sequencing of assembly, setup and solves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <memory>

#include "gw_internal.h"

using namespace gw;

void amg_hierarchy::drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

amg_hierarchy::~amg_hierarchy() {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
}

size_t amg_hierarchy::bytes() const {
    size_t b = lu.bytes() + inv.bytes() + piv.bytes() + kvec.bytes() + partials.bytes() + ks.bytes();
    for (int l = 0; l < nlev || (l == 0 && !L.empty()); ++l) b += L[l].bytes();
    return b;
}

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void check_grid(const gw_grid *g) {
    GW_REQUIRE(g, "null grid");
    GW_REQUIRE(g->nx > 0 && g->ny > 0 && g->nz > 0, "grid sizes must be positive");
    GW_REQUIRE((int64_t)g->nx * g->ny * g->nz < ((int64_t)1 << 30), "grid exceeds 2^30 cells");
    GW_REQUIRE(g->dx > 0 && g->dy > 0 && g->dz > 0 && std::isfinite(g->dx) && std::isfinite(g->dy) &&
                   std::isfinite(g->dz),
               "grid spacings must be positive and finite");
}

int64_t nnz7(const gw_grid *g) {
    int64_t n = (int64_t)g->nx * g->ny * g->nz;
    return 7 * n - 2 * ((int64_t)g->nx * g->ny + (int64_t)g->ny * g->nz + (int64_t)g->nx * g->nz);
}

void check_params(const amg_params *p) {
    GW_REQUIRE(p, "null amg_params");
    GW_REQUIRE(p->smoother >= GW_SMOOTHER_JACOBI && p->smoother <= GW_SMOOTHER_ILU0, "unknown smoother");
    GW_REQUIRE(p->precision == GW_PRECISION_FP64 || p->precision == GW_PRECISION_MIXED, "unknown precision");
    GW_REQUIRE(p->coarsening == GW_COARSEN_SA || p->coarsening == GW_COARSEN_RS, "unknown coarsening");
    GW_REQUIRE(!(p->smoother == GW_SMOOTHER_ILU0 && p->precision == GW_PRECISION_MIXED),
               "the ILU(0) smoother needs the FP64 hierarchy");
    GW_REQUIRE(p->npre >= 0 && p->npost >= 0 && p->npre <= 16 && p->npost <= 16, "sweeps must be in [0, 16]");
    GW_REQUIRE(p->n_coarse >= 1 && p->max_levels >= 1, "n_coarse and max_levels must be positive");
    GW_REQUIRE(p->eps_strong >= 0 && std::isfinite(p->eps_strong), "eps_strong must be >= 0");
    GW_REQUIRE(std::isfinite(p->omega), "omega must be finite");
}

void finish(hipStream_t s) {
    GW_HIP(hipStreamSynchronize(s));
    if (prof_on()) prof_flush();
}

// Hierarchy of a device CSR (copied), as amg_setup documents.  sym_pattern:
// -1 probes whether the level-0 pattern is symmetric; 0 takes the general
// path (A^T formed explicitly), which is correct for any pattern.
amg_hierarchy *setup_hierarchy(const gw_csr *A, const amg_params *prm, hipStream_t s, int sym_pattern = -1) {
    GW_REQUIRE(A && A->rowptr && A->col && A->val, "amg_setup: null matrix");
    GW_REQUIRE(A->n > 0 && A->nnz >= A->n && A->nnz < INT32_MAX, "amg_setup: bad matrix size");
    check_params(prm);
    std::unique_ptr<amg_hierarchy> H(new amg_hierarchy());
    int dev = 0;
    GW_HIP(hipGetDevice(&dev));
    H->device = dev;
    H->prm = *prm;
    H->sym_pattern = sym_pattern;
    H->L.resize(33);
    Level &L0 = H->L[0];
    L0.A.alloc(A->n, A->n, A->nnz);
    copy_bytes(L0.A.rowptr.p, A->rowptr, sizeof(int32_t) * ((size_t)A->n + 1), s);
    copy_bytes(L0.A.col.p, A->col, sizeof(int32_t) * (size_t)A->nnz, s);
    copy_bytes(L0.A.val.p, A->val, sizeof(double) * (size_t)A->nnz, s);
    {
        DBuf<double> diag(A->n);
        DBuf<int32_t> bad(1);
        fill_i32(bad.p, 0, 1, s);
        launch_csr_check(view(L0.A), diag.p, bad.p, s);
        int32_t hb = 0;
        GW_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        if (hb & 1) fail(GW_EINVAL, "amg_setup: CSR structure invalid (row pointers, column range or order)");
        if (hb & 2) fail(GW_EINVAL, "amg_setup: a diagonal entry is missing or not positive");
        if (hb & 4) fail(GW_EINVAL, "amg_setup: non-finite matrix value");
    }
    if (prm->smoother == GW_SMOOTHER_NONE) {
        H->nlev = 0;
        H->L[0].A.grp = solve_group_for(A->n ? (double)A->nnz / (double)A->n : 0.0);
        const char *sell_env = std::getenv("GWAMG_SELL");
        if (!(sell_env && std::atoi(sell_env) == 0)) build_sell(H.get(), 0, false, s);
        GW_HIP(hipStreamSynchronize(s));
        return H.release();
    }
    CoarseJob coarse;  // after H: waits for the side stream before H is freed
    for (int l = 0;; ++l) {
        bool coarsest = false;
        build_level(H.get(), l, s, &coarsest);
        if (coarsest) {
            start_coarsest(H.get(), l, s, coarse);
            H->nlev = l + 1;
            break;
        }
    }
    {
        // the prolongator weights, kept on the device during the build
        double *stage = static_cast<double *>(host_stage());
        static_assert(33 * sizeof(double) <= kHostStageBytes, "one weight per level fits the pinned stage");
        for (int l = 0; l + 1 < H->nlev; ++l)
            GW_HIP(hipMemcpyAsync(stage + l, H->L[l].omega_dev.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        for (int l = 0; l + 1 < H->nlev; ++l) H->L[l].omega_p = stage[l];
    }
    const size_t es = H->mixed() ? 4 : 8;
    auto mean = [](const Csr &M) { return M.n ? (double)M.nnz / (double)M.n : 0.0; };
    for (int l = 0; l < std::max(H->nlev, 1); ++l) {
        Level &Lv = H->L[l];
        Lv.A.grp = solve_group_for(mean(Lv.A));
        Lv.P.grp = solve_group_for(mean(Lv.P));
        Lv.R.grp = solve_group_for(mean(Lv.R));
    }
    if (const char *e = std::getenv("GWAMG_G0")) {
        int g = std::atoi(e);
        if (g >= 1 && g <= 64 && (g & (g - 1)) == 0) H->L[0].A.grp = g;
    }
    // Level-0 products (smoother, residual, Krylov) run on the sliced ELL
    // copy unless GWAMG_SELL=0 keeps them on the CSR kernels.
    const char *sell_env = std::getenv("GWAMG_SELL");
    if (!(sell_env && std::atoi(sell_env) == 0)) build_sell(H.get(), 0, H->mixed() && H->nlev > 1, s);
    for (int l = 0; l < H->nlev; ++l) {
        Level &Lv = H->L[l];
        if (l < H->nlev - 1) {
            if (prm->smoother == GW_SMOOTHER_ILU0) {
                build_ilu0(H.get(), l, s);
            } else {
                make_smoother(H.get(), l, s);
                if (H->mixed()) convert_level_fp32(H.get(), l, s);
            }
        }
        const size_t n = (size_t)Lv.A.n;
        Lv.vx.alloc(n * es);
        Lv.vt.alloc(n * es);
        if (l > 0) Lv.vb.alloc(n * es);
    }
    finish_coarsest(coarse, s);
    GW_HIP(hipStreamSynchronize(s));
    return H.release();
}

// Steps of Eq. 2 from h0: the hierarchy of C serves every step whose
// storage term passes the reuse criterion (shifted PCG); otherwise a
// hierarchy of C + S/dt is built, and kept while dt does not change.
int transient_run(const gw_grid &g, const Csr &C, const double *b, const double *Ss, const double *h0,
                  const double *dt, int32_t nsteps, double delta, const amg_params &prm, const amg_solve_params &sp,
                  double *h, double *h_steps, gw_step_info *info, hipStream_t s) {
    const int64_t n = C.n;
    const double vol = (g.dx * g.dy) * g.dz;
    const CsrView Cv = view(C);
    DBuf<double> shift(n), rhs(n), hcur(n), At_val((size_t)C.nnz);
    copy_bytes(hcur.p, h0, sizeof(double) * (size_t)n, s);
    auto setup = [&](const double *val) {
        const gw_csr A{(int32_t)n, C.nnz, C.rowptr.p, C.col.p, val};
        return std::unique_ptr<amg_hierarchy>(setup_hierarchy(&A, &prm, s));
    };
    double t0 = 0.0;
    std::unique_ptr<amg_hierarchy> HC;  // hierarchy of C, built at the first step that may keep it
    std::unique_ptr<amg_hierarchy> HT;  // hierarchy of C + S/dt for the last rebuilt dt
    double dt_cached = 0.0;
    int worst = GW_OK;
    for (int32_t k = 0; k < nsteps; ++k) {
        gw_step_info st{};
        storage_shift(n, Ss, vol, dt[k], shift.p, s);
        st.ratio = shift_ratio(Cv, shift.p, s);
        storage_rhs(n, b, shift.p, hcur.p, rhs.p, s);
        amg_solve_info si{};
        int rc;
        if (st.ratio < delta) {
            st.reused = 1;
            if (!HC) {
                t0 = now_ms();
                HC = setup(C.val.p);
                st.setup_ms = now_ms() - t0;
            }
            rc = krylov_pcg_shifted(HC.get(), shift.p, rhs.p, hcur.p, sp, &si, s);
        } else {
            if (!HT || dt[k] != dt_cached) {
                HT.reset();
                add_diagonal(Cv, shift.p, At_val.p, s);
                t0 = now_ms();
                HT = setup(At_val.p);
                st.setup_ms = now_ms() - t0;
                dt_cached = dt[k];
                st.reused = 0;
            } else {
                st.reused = 2;
            }
            rc = krylov_pcg(HT.get(), rhs.p, hcur.p, sp, &si, s);
        }
        st.status = rc;
        st.iters = si.iters;
        st.rel_res_true = si.rel_res_true;
        st.solve_ms = si.solve_ms;
        if (h_steps) copy_bytes(h_steps + k * n, hcur.p, sizeof(double) * (size_t)n, s);
        if (info) info[k] = st;
        if (rc == GW_BREAKDOWN) {
            worst = rc;
            break;
        }
        if (rc != GW_OK) worst = rc;
    }
    copy_bytes(h, hcur.p, sizeof(double) * (size_t)n, s);
    GW_HIP(hipStreamSynchronize(s));
    return worst;
}


}  // namespace

extern "C" {

const char *gw_version(void) { return "gwamg 0.1.0 gfx950"; }

int64_t fv_nnz(const gw_grid *grid) {
    if (!grid || grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0) return -1;
    return nnz7(grid);
}

int64_t tt_nnz_bound(const gw_grid *grid) { return fv_nnz(grid); }

int fv_assemble(const gw_grid *grid, const double *K, const gw_bc *bc, const gw_well *wells, int32_t nwells,
                int32_t *rowptr, int32_t *col, double *val, double *b, void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(K && bc && rowptr && col && val && b, "fv_assemble: null pointer");
        GW_REQUIRE(nwells == 0 || wells, "fv_assemble: null wells");
        GW_REQUIRE(std::isfinite(bc->h_west) && std::isfinite(bc->h_east), "fv_assemble: non-finite head");
        GW_REQUIRE(nnz7(grid) < INT32_MAX, "fv_assemble: matrix exceeds 2^31 nonzeros");
        hipStream_t s = as_stream(stream);
        DBuf<int32_t> bad(1);
        fill_i32(bad.p, 0, 1, s);
        launch_fv_assemble(*grid, K, *bc, wells, nwells, rowptr, col, val, b, bad.p, s);
        int32_t hb = 0;
        GW_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        finish(s);
        if (hb) fail(GW_EINVAL, "fv_assemble: conductivity must be positive and finite");
        return GW_OK;
    });
}

int darcy_flux(const gw_grid *grid, const double *K, const gw_bc *bc, const double *h, double *qx, double *qy,
               double *qz, void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(K && bc && h && qx && qy && qz, "darcy_flux: null pointer");
        hipStream_t s = as_stream(stream);
        launch_darcy(*grid, K, *bc, h, qx, qy, qz, s);
        finish(s);
        return GW_OK;
    });
}

int amg_setup(const gw_csr *A, const amg_params *params, amg_hierarchy **H, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H, "amg_setup: null output");
        *H = nullptr;
        hipStream_t s = as_stream(stream);
        *H = setup_hierarchy(A, params, s);
        finish(s);
        return GW_OK;
    });
}

int amg_vcycle(amg_hierarchy *H, const double *r, double *z, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H && r && z, "amg_vcycle: null pointer");
        hipStream_t s = as_stream(stream);
        vcycle(H, r, z, nullptr, s);
        finish(s);
        return GW_OK;
    });
}

int amg_spmv(amg_hierarchy *H, const double *x, double *y, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H && x && y, "amg_spmv: null pointer");
        hipStream_t s = as_stream(stream);
        spmv_level0(H, x, y, s);
        finish(s);
        return GW_OK;
    });
}

void check_solve(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp) {
    GW_REQUIRE(H && b && x && sp, "solve: null pointer");
    GW_REQUIRE(sp->rtol >= 0 && std::isfinite(sp->rtol), "solve: rtol must be >= 0");
    GW_REQUIRE(sp->maxiter >= 0, "solve: maxiter must be >= 0");
    GW_REQUIRE(sp->graph >= -1 && sp->graph <= 1, "solve: graph must be -1, 0 or 1");
}

int amg_solve_pcg(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp, amg_solve_info *info,
                  void *stream) {
    return guarded([&] {
        check_solve(H, b, x, sp);
        hipStream_t s = as_stream(stream);
        int st = krylov_pcg(H, b, x, *sp, info, s);
        finish(s);
        return st;
    });
}

int amg_solve_pcg_noalloc(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp,
                          amg_solve_info *info, void *stream) {
    return guarded([&] {
        check_solve(H, b, x, sp);
        GW_REQUIRE(sp->graph <= 0, "amg_solve_pcg_noalloc: graph replay allocates graph objects; pass graph <= 0");
        GW_REQUIRE(!prof_on(), "amg_solve_pcg_noalloc: kernel timing is on (it creates events)");
        hipStream_t s = as_stream(stream);
        int st = pcg_noalloc(H, b, x, *sp, info, s);
        finish(s);
        return st;
    });
}

int amg_solve_bicgstab(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp,
                       amg_solve_info *info, void *stream) {
    return guarded([&] {
        check_solve(H, b, x, sp);
        hipStream_t s = as_stream(stream);
        int st = krylov_bicgstab(H, b, x, *sp, info, s);
        finish(s);
        return st;
    });
}

int amg_solve_bicgstab_pair(amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1,
                            const amg_solve_params *sp, amg_solve_info info[2], void *stream) {
    return guarded([&] {
        check_solve(H, b0, x0, sp);
        GW_REQUIRE(b1 && x1, "solve: null pointer");
        GW_REQUIRE(x0 != x1, "amg_solve_bicgstab_pair: x0 and x1 must be different buffers");
        hipStream_t s = as_stream(stream);
        int st = krylov_bicgstab2(H, b0, b1, x0, x1, *sp, info, s);
        finish(s);
        return st;
    });
}

int amg_solve_pcg_batch(amg_hierarchy *const *H, const double *const *b, double *const *x, int32_t nsys,
                        const amg_solve_params *sp, amg_solve_info *info, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H && b && x && sp, "amg_solve_pcg_batch: null pointer");
        GW_REQUIRE(nsys >= 1 && nsys <= 256, "amg_solve_pcg_batch: nsys must be in [1, 256]");
        for (int32_t j = 0; j < nsys; ++j) check_solve(H[j], b[j], x[j], sp);
        hipStream_t s = as_stream(stream);
        int st = krylov_pcg_batch(H, b, x, nsys, *sp, info, s);
        finish(s);
        return st;
    });
}

int amg_solve_bicgstab_pair_batch(amg_hierarchy *const *H, const double *const *b0, const double *const *b1,
                                  double *const *x0, double *const *x1, int32_t nsys, const amg_solve_params *sp,
                                  amg_solve_info *info, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H && b0 && b1 && x0 && x1 && sp, "amg_solve_bicgstab_pair_batch: null pointer");
        GW_REQUIRE(nsys >= 1 && nsys <= 256, "amg_solve_bicgstab_pair_batch: nsys must be in [1, 256]");
        for (int32_t j = 0; j < nsys; ++j) {
            check_solve(H[j], b0[j], x0[j], sp);
            GW_REQUIRE(b1[j] && x1[j], "amg_solve_bicgstab_pair_batch: null pointer");
            GW_REQUIRE(x0[j] != x1[j], "amg_solve_bicgstab_pair_batch: x0 and x1 must be different buffers");
        }
        hipStream_t s = as_stream(stream);
        int st = krylov_bicgstab2_batch(H, b0, b1, x0, x1, nsys, *sp, info, s);
        finish(s);
        return st;
    });
}

int amg_hierarchy_info(const amg_hierarchy *H, amg_level_info *out, int32_t max_levels, int32_t *nlevels,
                       size_t *bytes) {
    return guarded([&] {
        GW_REQUIRE(H, "amg_hierarchy_info: null hierarchy");
        const int nl = std::max(H->nlev, 1);
        if (nlevels) *nlevels = H->nlev;
        if (bytes) *bytes = H->bytes();
        for (int l = 0; l < nl && l < max_levels && out; ++l) {
            const Level &Lv = H->L[l];
            amg_level_info &o = out[l];
            o.n = Lv.A.n;
            o.nnz = Lv.A.nnz;
            o.nc = Lv.nc;
            o.nnz_p = Lv.P.nnz;
            o.nnz_s = Lv.nnz_s;
            o.mis_rounds = Lv.mis_rounds;
            o.omega_p = Lv.omega_p;
            o.bytes = Lv.bytes() + (l == H->nlev - 1 ? H->lu.bytes() + H->inv.bytes() + H->piv.bytes() : 0);
            o.slice_rows = Lv.As.built() ? 1 << Lv.As.cshift : 0;
            o.nnz_sliced = Lv.As.built() ? Lv.As.nnz_padded : 0;
            o.stencil_offsets = Lv.St.K;
        }
        return GW_OK;
    });
}

int amg_level_export(const amg_hierarchy *H, int32_t level, int32_t *a_rowptr, int32_t *a_col, double *a_val,
                     int32_t *agg, double *M, int32_t *p_rowptr, int32_t *p_col, double *p_val, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H, "amg_level_export: null hierarchy");
        GW_REQUIRE(level >= 0 && level < std::max(H->nlev, 1), "amg_level_export: level out of range");
        hipStream_t s = as_stream(stream);
        const Level &Lv = H->L[level];
        const bool coarsest = level == H->nlev - 1 || H->nlev == 0;
        if (a_rowptr) copy_bytes(a_rowptr, Lv.A.rowptr.p, Lv.A.rowptr.bytes(), s);
        if (a_col) copy_bytes(a_col, Lv.A.col.p, Lv.A.col.bytes(), s);
        if (a_val) copy_bytes(a_val, Lv.A.val.p, Lv.A.val.bytes(), s);
        if (!coarsest) {
            if (agg) copy_bytes(agg, Lv.agg.p, Lv.agg.bytes(), s);
            if (M) copy_bytes(M, Lv.M.p, Lv.M.bytes(), s);
            if (p_rowptr) copy_bytes(p_rowptr, Lv.P.rowptr.p, Lv.P.rowptr.bytes(), s);
            if (p_col) copy_bytes(p_col, Lv.P.col.p, Lv.P.col.bytes(), s);
            if (p_val) copy_bytes(p_val, Lv.P.val.p, Lv.P.val.bytes(), s);
        }
        finish(s);
        return GW_OK;
    });
}

int amg_coarse_export(const amg_hierarchy *H, double *lu, int32_t *piv, double *inv, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H && H->nlev > 0, "amg_coarse_export: no coarse level");
        hipStream_t s = as_stream(stream);
        if (lu) copy_bytes(lu, H->lu.p, H->lu.bytes(), s);
        if (piv) copy_bytes(piv, H->piv.p, H->piv.bytes(), s);
        if (inv) copy_bytes(inv, H->inv.p, H->inv.bytes(), s);
        finish(s);
        return GW_OK;
    });
}

int amg_ilu_export(const amg_hierarchy *H, int32_t level, double *lu, void *stream) {
    return guarded([&] {
        GW_REQUIRE(H && lu, "amg_ilu_export: null pointer");
        GW_REQUIRE(level >= 0 && level < H->nlev && H->L[level].ilu, "amg_ilu_export: level has no ILU(0) factors");
        hipStream_t s = as_stream(stream);
        copy_bytes(lu, H->L[level].ilu->lu.p, H->L[level].ilu->lu.bytes(), s);
        finish(s);
        return GW_OK;
    });
}

void amg_free(amg_hierarchy *H) { delete H; }

int tt_assemble(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
                const gw_zone *zone, int32_t *rowptr, int32_t *col, double *val, double *b_tau, double *b_c,
                int64_t *nnz, int64_t *n_identity, void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(qx && qy && qz && rowptr && col && val && b_tau && b_c, "tt_assemble: null pointer");
        GW_REQUIRE(std::isfinite(phi) && phi > 0, "tt_assemble: porosity must be positive");
        hipStream_t s = as_stream(stream);
        gw_zone z = zone ? *zone : gw_zone{0, grid->ny, 0, grid->nz};
        const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
        DBuf<int64_t> total(1);
        DBuf<int32_t> nid(1);
        fill_i32(nid.p, 0, 1, s);
        fill_i32(rowptr, 0, 1, s);
        launch_tt_count(*grid, qx, qy, qz, rowptr + 1, s);
        scan_inclusive_i32(rowptr + 1, n, total.p, s);
        launch_tt_fill(*grid, qx, qy, qz, phi, z, rowptr, col, val, b_tau, b_c, nid.p, s);
        int64_t hn = 0;
        int32_t hi = 0;
        GW_HIP(hipMemcpyAsync(&hn, total.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GW_HIP(hipMemcpyAsync(&hi, nid.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        finish(s);
        if (nnz) *nnz = hn;
        if (n_identity) *n_identity = hi;
        return GW_OK;
    });
}

int tt_solve(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
             const gw_zone *zone, const amg_params *params, const amg_solve_params *sp, double *tau, double *c,
             amg_solve_info info[2], void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(qx && qy && qz && params && sp && tau && c, "tt_solve: null pointer");
        hipStream_t s = as_stream(stream);
        const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
        const double t0 = now_ms();
        Csr A;
        A.alloc((int32_t)n, (int32_t)n, nnz7(grid));
        DBuf<double> bt(n), bc(n);
        int64_t nnz = 0, nid = 0;
        int rc = tt_assemble(grid, qx, qy, qz, phi, zone, A.rowptr.p, A.col.p, A.val.p, bt.p, bc.p, &nnz, &nid,
                             stream);
        if (rc != GW_OK) fail(rc, gw_last_error());
        gw_csr view_{(int32_t)n, nnz, A.rowptr.p, A.col.p, A.val.p};
        // an upwind row holds only inflow neighbours, so a_ij and a_ji are
        // not both stored: no probe for a symmetric pattern
        std::unique_ptr<amg_hierarchy> H(setup_hierarchy(&view_, params, s, 0));
        A = Csr();
        const double setup_ms = now_ms() - t0;
        GW_REQUIRE(tau != c, "tt_solve: tau and c must be different buffers");
        amg_solve_info ii[2] = {};
        const int st = krylov_bicgstab2(H.get(), bt.p, bc.p, tau, c, *sp, ii, s);
        finish(s);
        ii[0].setup_ms = ii[1].setup_ms = setup_ms;
        if (info) {
            info[0] = ii[0];
            info[1] = ii[1];
        }
        return st;
    });
}

int tt_sweep(const gw_csr *A, int32_t nrhs, const double *b, double *x, int32_t *n_levels, void *stream) {
    return guarded([&] {
        GW_REQUIRE(A && A->rowptr && A->col && A->val && b && x, "tt_sweep: null pointer");
        GW_REQUIRE(A->n > 0 && A->nnz >= A->n && A->nnz < INT32_MAX, "tt_sweep: bad matrix size");
        GW_REQUIRE(nrhs >= 1 && nrhs <= 64, "tt_sweep: nrhs must be in [1, 64]");
        GW_REQUIRE(b != x, "tt_sweep: b and x must be different buffers");
        hipStream_t s = as_stream(stream);
        const CsrView V{A->n, A->n, A->nnz, A->rowptr, A->col, A->val};
        {
            DBuf<double> diag(A->n);
            DBuf<int32_t> bad(1);
            fill_i32(bad.p, 0, 1, s);
            launch_csr_check(V, diag.p, bad.p, s);
            int32_t *stage = static_cast<int32_t *>(host_stage());
            GW_HIP(hipMemcpyAsync(stage, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            GW_HIP(hipStreamSynchronize(s));
            const int32_t hb = stage[0];
            if (hb & 1) fail(GW_EINVAL, "tt_sweep: CSR structure invalid (row pointers, column range or order)");
            if (hb & 2) fail(GW_EINVAL, "tt_sweep: a diagonal entry is missing or not positive");
            if (hb & 4) fail(GW_EINVAL, "tt_sweep: non-finite matrix value");
        }
        int32_t lev = 0;
        const int64_t solved = upwind_sweep(V, nrhs, b, x, &lev, s);
        finish(s);
        if (n_levels) *n_levels = lev;
        if (solved != A->n) fail(GW_BREAKDOWN, "tt_sweep: the inflow graph has a cycle (not an upwind matrix)");
        return GW_OK;
    });
}

int tt_solve_direct(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
                    const gw_zone *zone, double *tau, double *c, int32_t *n_levels, void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(qx && qy && qz && tau && c, "tt_solve_direct: null pointer");
        GW_REQUIRE(tau != c, "tt_solve_direct: tau and c must be different buffers");
        hipStream_t s = as_stream(stream);
        const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
        Csr A;
        A.alloc((int32_t)n, (int32_t)n, nnz7(grid));
        DBuf<double> b2((size_t)n * 2), x2((size_t)n * 2);
        int64_t nnz = 0, nid = 0;
        int rc = tt_assemble(grid, qx, qy, qz, phi, zone, A.rowptr.p, A.col.p, A.val.p, b2.p, b2.p + n, &nnz, &nid,
                             stream);
        if (rc != GW_OK) fail(rc, gw_last_error());
        const CsrView V{(int32_t)n, (int32_t)n, nnz, A.rowptr.p, A.col.p, A.val.p};
        int32_t lev = 0;
        const int64_t solved = grid_sweep(*grid, V, 2, b2.p, x2.p, &lev, s);
        copy_bytes(tau, x2.p, sizeof(double) * (size_t)n, s);
        copy_bytes(c, x2.p + n, sizeof(double) * (size_t)n, s);
        finish(s);
        if (n_levels) *n_levels = lev;
        if (solved != n) fail(GW_BREAKDOWN, "tt_solve_direct: the inflow graph has a cycle");
        return GW_OK;
    });
}

int tt_delineate(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
                 const gw_zone *zones, int32_t nzones, const gw_well *wells, int32_t nwells, double *out,
                 int32_t n_levels[2], void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(qx && qy && qz && out, "tt_delineate: null pointer");
        GW_REQUIRE(std::isfinite(phi) && phi > 0, "tt_delineate: porosity must be positive");
        GW_REQUIRE(nzones >= 0 && (nzones == 0 || zones), "tt_delineate: bad zone list");
        GW_REQUIRE(nwells >= 0 && nwells <= 64 && (nwells == 0 || wells), "tt_delineate: at most 64 wells");
        int32_t n_inj = 0, n_prod = 0;
        for (int32_t z = 0; z < nzones; ++z) {
            const gw_zone &Z = zones[z];
            GW_REQUIRE(Z.j0 >= 0 && Z.j0 <= Z.j1 && Z.j1 <= grid->ny && Z.k0 >= 0 && Z.k0 <= Z.k1 &&
                           Z.k1 <= grid->nz,
                       "tt_delineate: zone outside the x = 0 face");
        }
        for (int32_t k = 0; k < nwells; ++k) {
            const gw_well &w = wells[k];
            GW_REQUIRE(w.ix >= 0 && w.ix < grid->nx && w.iy >= 0 && w.iy < grid->ny && w.iz >= 0 &&
                           w.iz < grid->nz && std::isfinite(w.q),
                       "tt_delineate: well outside the grid or rate not finite");
            n_inj += w.q < 0;
            n_prod += w.q > 0;
        }
        GW_REQUIRE(1 + nzones + n_inj <= 64 && 1 + n_prod <= 64, "tt_delineate: at most 64 fields per direction");
        hipStream_t s = as_stream(stream);
        const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
        Csr A;
        A.alloc((int32_t)n, (int32_t)n, nnz7(grid));
        int32_t lev[2] = {0, 0};
        int64_t solved[2] = {0, 0};
        delineate(*grid, qx, qy, qz, phi, zones, nzones, wells, nwells, A, out, lev, solved, s);
        finish(s);
        if (n_levels) {
            n_levels[0] = lev[0];
            n_levels[1] = lev[1];
        }
        if (solved[0] != n || solved[1] != n) fail(GW_BREAKDOWN, "tt_delineate: the inflow graph has a cycle");
        return GW_OK;
    });
}

int amg_solve_pcg_shifted(amg_hierarchy *H, const double *shift, const double *b, double *x,
                          const amg_solve_params *sp, amg_solve_info *info, void *stream) {
    return guarded([&] {
        check_solve(H, b, x, sp);
        GW_REQUIRE(shift, "amg_solve_pcg_shifted: null shift");
        hipStream_t s = as_stream(stream);
        int st = krylov_pcg_shifted(H, shift, b, x, *sp, info, s);
        finish(s);
        return st;
    });
}

int flow_transient(const gw_grid *grid, const double *K, const gw_bc *bc, const gw_well *wells, int32_t nwells,
                   const double *Ss, const double *h0, const double *dt, int32_t nsteps, double delta,
                   const amg_params *params, const amg_solve_params *sp, double *h, double *h_steps,
                   gw_step_info *info, void *stream) {
    return guarded([&] {
        check_grid(grid);
        GW_REQUIRE(K && bc && Ss && h0 && dt && params && sp && h, "flow_transient: null pointer");
        GW_REQUIRE(nwells == 0 || wells, "flow_transient: null wells");
        GW_REQUIRE(nsteps >= 1, "flow_transient: nsteps must be >= 1");
        GW_REQUIRE(std::isfinite(delta) && delta >= 0, "flow_transient: delta must be >= 0");
        for (int32_t k = 0; k < nsteps; ++k)
            GW_REQUIRE(std::isfinite(dt[k]) && dt[k] > 0, "flow_transient: time steps must be positive");
        GW_REQUIRE(params->smoother != GW_SMOOTHER_NONE, "flow_transient: needs an AMG smoother");
        check_params(params);
        GW_REQUIRE(sp->rtol >= 0 && sp->maxiter >= 0, "flow_transient: bad solve parameters");
        GW_REQUIRE(nnz7(grid) < INT32_MAX, "flow_transient: matrix exceeds 2^31 nonzeros");
        hipStream_t s = as_stream(stream);
        const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
        Csr C;
        C.alloc((int32_t)n, (int32_t)n, nnz7(grid));
        DBuf<double> b(n);
        DBuf<int32_t> bad(1);
        fill_i32(bad.p, 0, 1, s);
        launch_fv_assemble(*grid, K, *bc, wells, nwells, C.rowptr.p, C.col.p, C.val.p, b.p, bad.p, s);
        int32_t *stage = static_cast<int32_t *>(host_stage());
        GW_HIP(hipMemcpyAsync(stage, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        if (stage[0]) fail(GW_EINVAL, "flow_transient: conductivity must be positive and finite");
        const int st = transient_run(*grid, C, b.p, Ss, h0, dt, nsteps, delta, *params, *sp, h, h_steps, info, s);
        finish(s);
        return st;
    });
}

}  // extern "C"
