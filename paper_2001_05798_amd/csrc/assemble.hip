// Problem assembly on the device: the 7-point finite-difference flow matrix
// (Benchmarking Examples: M-matrix from 5/7-point stencils), Darcy face
// fluxes, and the first-order upwind matrix of the forward travel-time
// equation v.grad(tau) = phi (Eq. 1) with its two right-hand sides.
//
// Built with -ffp-contract=off: every transmissibility and diagonal sum is
// formed with the same operations in the same order whatever the backend, so
// the matrix is bit-reproducible (the aggregation downstream depends on exact
// comparisons of these values).
#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

struct GridD {
    int32_t nx, ny, nz;
    double gx, gy, gz;  // face area / centre distance per direction
};

GridD grid_d(const gw_grid &g) {
    return {g.nx, g.ny, g.nz, (g.dy * g.dz) / g.dx, (g.dx * g.dz) / g.dy, (g.dx * g.dy) / g.dz};
}

// Harmonic-mean transmissibility; `ka` is the cell with the lower flat index
// so both rows of a face get the same bits.
__device__ __forceinline__ double face_t(double geo, double ka, double kb) {
    return geo * ((2.0 * ka * kb) / (ka + kb));
}

// Number of stored entries of all cells before cell (i,j,k): every cell has
// 7 slots minus one per missing neighbour.
__device__ __forceinline__ int64_t fv_row_start(const GridD &g, int64_t c, int32_t i, int32_t j, int32_t k) {
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const int64_t rows_before = (int64_t)k * g.ny + j;
    int64_t miss = 0;
    miss += rows_before + (i > 0 ? 1 : 0);                                  // i' == 0
    miss += rows_before;                                                    // i' == nx-1
    miss += (int64_t)k * g.nx + (j > 0 ? g.nx : i);                         // j' == 0
    miss += (int64_t)k * g.nx + (j == g.ny - 1 ? i : 0);                    // j' == ny-1
    miss += (k > 0) ? sxy : c;                                              // k' == 0
    miss += (k == g.nz - 1) ? c - (int64_t)(g.nz - 1) * sxy : 0;            // k' == nz-1
    return 7 * c - miss;
}

__global__ void k_fv_assemble(GridD g, const double *__restrict__ K, double hw, double he,
                              int32_t *__restrict__ rowptr, int32_t *__restrict__ col,
                              double *__restrict__ val, double *__restrict__ b, int32_t *bad) {
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const int64_t n = sxy * g.nz;
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int32_t i = (int32_t)(c % g.nx);
    const int32_t j = (int32_t)((c / g.nx) % g.ny);
    const int32_t k = (int32_t)(c / sxy);
    const double kc = K[c];
    if (!(kc > 0.0) || !isfinite(kc)) atomicOr(bad, 1);
    // faces in the order -z, -y, -x, +x, +y, +z (ascending neighbour index)
    bool has[6] = {k > 0, j > 0, i > 0, i < g.nx - 1, j < g.ny - 1, k < g.nz - 1};
    int64_t nb[6] = {c - sxy, c - g.nx, c - 1, c + 1, c + g.nx, c + sxy};
    const double geo[6] = {g.gz, g.gy, g.gx, g.gx, g.gy, g.gz};
    double t[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!has[f]) { t[f] = 0.0; continue; }
        double kn = K[nb[f]];
        t[f] = (f < 3) ? face_t(geo[f], kn, kc) : face_t(geo[f], kc, kn);
    }
    double diag = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f)
        if (has[f]) diag = diag + t[f];
    double rhs = 0.0;
    if (i == 0) {
        double tb = g.gx * (2.0 * kc);
        diag = diag + tb;
        rhs = rhs + tb * hw;
    }
    if (i == g.nx - 1) {
        double tb = g.gx * (2.0 * kc);
        diag = diag + tb;
        rhs = rhs + tb * he;
    }
    int64_t p = fv_row_start(g, c, i, j, k);
    rowptr[c] = (int32_t)p;
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (has[f]) { col[p] = (int32_t)nb[f]; val[p] = -t[f]; ++p; }
    col[p] = (int32_t)c;
    val[p] = diag;
    ++p;
#pragma unroll
    for (int f = 3; f < 6; ++f)
        if (has[f]) { col[p] = (int32_t)nb[f]; val[p] = -t[f]; ++p; }
    if (c == n - 1) rowptr[n] = (int32_t)p;
    b[c] = rhs;
}

constexpr int kMaxWells = 64;
struct WellList {
    int32_t n;
    int64_t cell[kMaxWells];
    double q[kMaxWells];
};

// Point sinks, applied in list order (one thread: the order of repeated
// subtractions on one cell is part of the definition).
__global__ void k_apply_wells(WellList w, double *b) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int32_t k = 0; k < w.n; ++k) b[w.cell[k]] = b[w.cell[k]] - w.q[k];
}

// Face fluxes, positive along +x/+y/+z.  One thread per face, the three face
// families concatenated.
__global__ void k_darcy(GridD g, const double *__restrict__ K, double hw, double he,
                        const double *__restrict__ h, double *__restrict__ qx, double *__restrict__ qy,
                        double *__restrict__ qz) {
    const int64_t nfx = (int64_t)(g.nx + 1) * g.ny * g.nz;
    const int64_t nfy = (int64_t)g.nx * (g.ny + 1) * g.nz;
    const int64_t nfz = (int64_t)g.nx * g.ny * (g.nz + 1);
    const int64_t sxy = (int64_t)g.nx * g.ny;
    int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f < nfx) {
        int32_t i = (int32_t)(f % (g.nx + 1));
        int64_t row = f / (g.nx + 1);  // j + ny*k
        int64_t c = i + g.nx * row;
        double q;
        if (i == 0) q = (g.gx * (2.0 * K[c])) * (hw - h[c]);
        else if (i == g.nx) q = (g.gx * (2.0 * K[c - 1])) * (h[c - 1] - he);
        else q = face_t(g.gx, K[c - 1], K[c]) * (h[c - 1] - h[c]);
        qx[f] = q;
        return;
    }
    f -= nfx;
    if (f < nfy) {
        int32_t i = (int32_t)(f % g.nx);
        int32_t j = (int32_t)((f / g.nx) % (g.ny + 1));
        int64_t k = f / ((int64_t)g.nx * (g.ny + 1));
        int64_t c = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        double q = 0.0;
        if (j > 0 && j < g.ny) q = face_t(g.gy, K[c - g.nx], K[c]) * (h[c - g.nx] - h[c]);
        qy[f] = q;
        return;
    }
    f -= nfy;
    if (f < nfz) {
        int64_t k = f / sxy;
        int64_t c = f;
        double q = 0.0;
        if (k > 0 && k < g.nz) q = face_t(g.gz, K[c - sxy], K[c]) * (h[c - sxy] - h[c]);
        qz[f] = q;
    }
}

// Inflow of each face of cell c (order -z, -y, -x, +x, +y, +z): |q| when the
// flux enters the cell, else 0.
struct Inflow {
    double in[6];
    bool interior[6];
    int64_t nb[6];
};

__device__ __forceinline__ void cell_inflow(const GridD &g, const double *qx, const double *qy,
                                            const double *qz, int64_t c, int32_t i, int32_t j,
                                            int32_t k, Inflow &F) {
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const int64_t fxw = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
    const int64_t fys = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
    double qin[6];
    qin[0] = qz[c];
    qin[1] = qy[fys];
    qin[2] = qx[fxw];
    qin[3] = -qx[fxw + 1];
    qin[4] = -qy[fys + g.nx];
    qin[5] = -qz[c + sxy];
    F.interior[0] = k > 0;        F.nb[0] = c - sxy;
    F.interior[1] = j > 0;        F.nb[1] = c - g.nx;
    F.interior[2] = i > 0;        F.nb[2] = c - 1;
    F.interior[3] = i < g.nx - 1; F.nb[3] = c + 1;
    F.interior[4] = j < g.ny - 1; F.nb[4] = c + g.nx;
    F.interior[5] = k < g.nz - 1; F.nb[5] = c + sxy;
#pragma unroll
    for (int f = 0; f < 6; ++f) F.in[f] = qin[f] > 0.0 ? qin[f] : 0.0;
}

__global__ void k_tt_count(GridD g, const double *__restrict__ qx, const double *__restrict__ qy,
                           const double *__restrict__ qz, int32_t *__restrict__ rowlen) {
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const int64_t n = sxy * g.nz;
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n) return;
    Inflow F;
    cell_inflow(g, qx, qy, qz, c, (int32_t)(c % g.nx), (int32_t)((c / g.nx) % g.ny), (int32_t)(c / sxy), F);
    int32_t len = 1;
#pragma unroll
    for (int f = 0; f < 6; ++f) len += (F.interior[f] && F.in[f] > 0.0) ? 1 : 0;
    rowlen[c] = len;  // an identity row (no inflow at all) also has length 1
}

__global__ void k_tt_fill(GridD g, const double *__restrict__ qx, const double *__restrict__ qy,
                          const double *__restrict__ qz, double phi, double vol, gw_zone z,
                          const int32_t *__restrict__ rowptr, int32_t *__restrict__ col,
                          double *__restrict__ val, double *__restrict__ bt, double *__restrict__ bc,
                          int32_t *n_ident) {
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const int64_t n = sxy * g.nz;
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int32_t i = (int32_t)(c % g.nx), j = (int32_t)((c / g.nx) % g.ny), k = (int32_t)(c / sxy);
    Inflow F;
    cell_inflow(g, qx, qy, qz, c, i, j, k, F);
    double diag = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) diag = diag + F.in[f];
    double b1 = phi * vol, b2 = 0.0;
    if (i == 0 && j >= z.j0 && j < z.j1 && k >= z.k0 && k < z.k1) b2 = F.in[2];
    int64_t p = rowptr[c];
    if (!(diag > 0.0)) {
        atomicAdd(n_ident, 1);
        col[p] = (int32_t)c;
        val[p] = 1.0;
        b1 = 0.0;
        b2 = 0.0;
    } else {
#pragma unroll
        for (int f = 0; f < 3; ++f)
            if (F.interior[f] && F.in[f] > 0.0) { col[p] = (int32_t)F.nb[f]; val[p] = -F.in[f]; ++p; }
        col[p] = (int32_t)c;
        val[p] = diag;
        ++p;
#pragma unroll
        for (int f = 3; f < 6; ++f)
            if (F.interior[f] && F.in[f] > 0.0) { col[p] = (int32_t)F.nb[f]; val[p] = -F.in[f]; ++p; }
    }
    bt[c] = b1;
    bc[c] = b2;
}

}  // namespace

void launch_fv_assemble(const gw_grid &g, const double *K, const gw_bc &bc, const gw_well *wells,
                        int nwells, int32_t *rowptr, int32_t *col, double *val, double *b,
                        int32_t *bad, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    GW_REQUIRE(nwells >= 0 && nwells <= kMaxWells, "fv_assemble: at most 64 wells");
    WellList wl{};
    wl.n = nwells;
    for (int w = 0; w < nwells; ++w) {
        const gw_well &x = wells[w];
        GW_REQUIRE(x.ix >= 0 && x.ix < g.nx && x.iy >= 0 && x.iy < g.ny && x.iz >= 0 && x.iz < g.nz,
                   "fv_assemble: well outside the grid");
        GW_REQUIRE(std::isfinite(x.q), "fv_assemble: non-finite well rate");
        wl.cell[w] = x.ix + (int64_t)g.nx * (x.iy + (int64_t)g.ny * x.iz);
        wl.q[w] = x.q;
    }
    {
        ProfScope ps(K_FV_ASSEMBLE, (double)n * 8 * 2 + (double)(7 * n) * 12 + 4.0 * n, s);
        hipLaunchKernelGGL(k_fv_assemble, dim3(blocks_for(n)), dim3(kBlock), 0, s, grid_d(g), K,
                           bc.h_west, bc.h_east, rowptr, col, val, b, bad);
    }
    if (nwells > 0) hipLaunchKernelGGL(k_apply_wells, dim3(1), dim3(64), 0, s, wl, b);
    GW_HIP(hipGetLastError());
}

void launch_darcy(const gw_grid &g, const double *K, const gw_bc &bc, const double *h, double *qx,
                  double *qy, double *qz, hipStream_t s) {
    const int64_t nf = (int64_t)(g.nx + 1) * g.ny * g.nz + (int64_t)g.nx * (g.ny + 1) * g.nz +
                       (int64_t)g.nx * g.ny * (g.nz + 1);
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    ProfScope ps(K_DARCY, (double)nf * 8 + (double)n * 16, s);
    hipLaunchKernelGGL(k_darcy, dim3(blocks_for(nf)), dim3(kBlock), 0, s, grid_d(g), K, bc.h_west,
                       bc.h_east, h, qx, qy, qz);
    GW_HIP(hipGetLastError());
}

void launch_tt_count(const gw_grid &g, const double *qx, const double *qy, const double *qz,
                     int32_t *rowlen, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    ProfScope ps(K_TT_ASSEMBLE, (double)n * (8 * 6 + 4), s);
    hipLaunchKernelGGL(k_tt_count, dim3(blocks_for(n)), dim3(kBlock), 0, s, grid_d(g), qx, qy, qz, rowlen);
    GW_HIP(hipGetLastError());
}

void launch_tt_fill(const gw_grid &g, const double *qx, const double *qy, const double *qz,
                    double phi, const gw_zone &z, const int32_t *rowptr, int32_t *col, double *val,
                    double *bt, double *bc, int32_t *n_ident, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    ProfScope ps(K_TT_ASSEMBLE, (double)n * (8 * 6 + 4 + 16 + 4 * 12), s);
    hipLaunchKernelGGL(k_tt_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, grid_d(g), qx, qy, qz, phi,
                       (g.dx * g.dy) * g.dz, z, rowptr, col, val, bt, bc, n_ident);
    GW_HIP(hipGetLastError());
}

}  // namespace gw
