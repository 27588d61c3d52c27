// Direct solution of the upwind travel-time system by one sweep in flow
// order.  Each row of the advective upwind matrix couples cell i only to its
// inflow neighbours, and water flows from higher to lower head (Darcy's law),
// so the system is triangular in the order of decreasing head: every cell can
// be solved exactly as soon as its inflow neighbours are (the Results find a
// direct method best for the transport equations; Eq. 1 for the system).
//
// The sweep is level-synchronous (Kahn's topological order): a frontier of
// cells whose inflow neighbours are all solved is solved at once, each cell
// then counts down its downstream neighbours, and those reaching zero form
// the next frontier.  Frontiers are small (about a thousand cells on a 1M-cell
// field, over more than a thousand levels), so the sweep runs in one
// workgroup, with a barrier between levels instead of a kernel launch.  A cell
// is solved with the operations of the sequential sweep in decreasing-head
// order, in the same order: the result equals it bit for bit.
#include <algorithm>

#include "gw_device.h"
#include "gw_internal.h"

namespace gw {

namespace {

// Inflow count of each row (off-diagonal entries) and, per column, the number
// of rows it feeds.
__global__ void k_sw_count(CsrView A, int32_t *__restrict__ indeg, int32_t *__restrict__ dcnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t c = 0;
    for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
        const int32_t j = A.col[p];
        if (j == (int32_t)i) continue;
        ++c;
        atomicAdd(&dcnt[j + 1], 1);
    }
    indeg[i] = c;
}

// Downstream lists: for each column j, the rows i with an entry (i, j).
__global__ void k_sw_fill(CsrView A, const int32_t *__restrict__ drow, int32_t *__restrict__ dfill,
                          int32_t *__restrict__ dcol) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
        const int32_t j = A.col[p];
        if (j == (int32_t)i) continue;
        dcol[drow[j] + atomicAdd(&dfill[j], 1)] = (int32_t)i;
    }
}

__global__ void k_sw_flag(int64_t n, const int32_t *__restrict__ indeg, int32_t *__restrict__ flag) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) flag[i] = indeg[i] == 0 ? 1 : 0;
}

// Cells without inflow, in ascending order: the first frontier.
__global__ void k_sw_first(int64_t n, const int32_t *__restrict__ flag, int32_t *__restrict__ q) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t before = i > 0 ? flag[i - 1] : 0;  // inclusive scan of the flags
    if (flag[i] != before) q[before] = (int32_t)i;
}

constexpr int kSweepThreads = 1024;

// Work copies for one run of a stored schedule: the count-downs (and the
// spare counters behind them), the first frontier and its size.
__global__ void k_sweep_prep(int64_t n, const int32_t *__restrict__ indeg0, const int32_t *__restrict__ q0,
                             const int64_t *__restrict__ first, int32_t *__restrict__ indeg, int32_t *__restrict__ qa,
                             int64_t *out, const int32_t *done) {
    if (done && *done) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n + kSweepThreads) indeg[i] = indeg0[i];
    if (i < *first) qa[i] = q0[i];
    if (i == 0) out[0] = *first;
}
constexpr int kQueueLds = 6144;  // frontier entries kept in LDS per buffer
constexpr int kRowFast = 7;      // rows and downstream lists up to this length (a 7-point stencil): one batch of loads

// x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii for the nrhs systems, with the
// off-diagonal terms subtracted in the row's order.
__device__ __forceinline__ void solve_row_slow(const CsrView &A, int32_t i, int32_t p0, int32_t p1, int32_t nrhs,
                                               const double *__restrict__ b, double *x) {
    const int64_t n = A.n;
    for (int32_t k = 0; k < nrhs; ++k) {
        double s = b[k * n + i], d = 0.0;
        for (int32_t p = p0; p < p1; ++p) {
            const int32_t j = A.col[p];
            if (j == i) d = A.val[p];
            else s = s - A.val[p] * x[k * n + j];
        }
        x[k * n + i] = s / d;
    }
}

// The same for a row of at most kRowFast entries whose column indices and
// values are already in registers (padding entries repeat the last one): the
// inflow values of two systems at a time are fetched in one batch of
// independent loads before the ordered arithmetic.
__device__ __forceinline__ void solve_row_fast(int64_t n, int32_t i, const int32_t (&cj)[kRowFast],
                                               const double (&cv)[kRowFast], int32_t len, int32_t nrhs,
                                               const double *__restrict__ b, double *x) {
    // the diagonal entry, and which entries are inflow terms (selects, not
    // branches: a term outside the row is computed and dropped)
    double d = 0.0;
    bool use[kRowFast];
#pragma unroll
    for (int e = 0; e < kRowFast; ++e) {
        const bool in_row = e < len;
        d = (in_row && cj[e] == i) ? cv[e] : d;
        use[e] = in_row && cj[e] != i;
    }
    int32_t k = 0;
    for (; k + 1 < nrhs; k += 2) {
        const double *x0 = x + k * n, *x1 = x0 + n;
        double s0 = b[k * n + i], s1 = b[(k + 1) * n + i];
        double v0[kRowFast], v1[kRowFast];
#pragma unroll
        for (int e = 0; e < kRowFast; ++e) {
            v0[e] = x0[cj[e]];
            v1[e] = x1[cj[e]];
        }
#pragma unroll
        for (int e = 0; e < kRowFast; ++e) {
            const double t0 = s0 - cv[e] * v0[e], t1 = s1 - cv[e] * v1[e];
            s0 = use[e] ? t0 : s0;
            s1 = use[e] ? t1 : s1;
        }
        x[k * n + i] = s0 / d;
        x[(k + 1) * n + i] = s1 / d;
    }
    if (k < nrhs) {
        const double *x0 = x + k * n;
        double s0 = b[k * n + i];
        double v0[kRowFast];
#pragma unroll
        for (int e = 0; e < kRowFast; ++e) v0[e] = x0[cj[e]];
#pragma unroll
        for (int e = 0; e < kRowFast; ++e) {
            const double t0 = s0 - cv[e] * v0[e];
            s0 = use[e] ? t0 : s0;
        }
        x[k * n + i] = s0 / d;
    }
}

// The whole sweep in one workgroup.  x, b: nrhs systems of n values each;
// out[0] holds the size of the first frontier (in qg0) on entry, the number
// of cells solved on exit, and out[1] the number of levels.
//
// Every level solves its frontier and counts down the downstream cells; those
// reaching zero are appended to the next frontier, whose first kQueueLds
// entries live in LDS and the rest in qg0/qg1.  One barrier per level: the
// append counters rotate over three slots, so a counter is cleared two levels
// after it was last read and one level before it is next used.  The loop
// ends with an empty frontier: all cells solved, or the rest lies downstream
// of a cycle of the inflow graph (then fewer than n cells are counted).
__global__ void __launch_bounds__(kSweepThreads) k_sweep(CsrView A, int32_t *__restrict__ indeg,
                                                         const int32_t *__restrict__ drow,
                                                         const int32_t *__restrict__ dcol, int32_t nrhs,
                                                         const double *__restrict__ b, double *x, int32_t *qg0,
                                                         int32_t *qg1, int64_t *out, const int32_t *done) {
    if (done && *done) return;
    __shared__ int32_t lq[2][kQueueLds];
    __shared__ int32_t cnt[3];
    const int64_t n = A.n;
    const int32_t first = (int32_t)out[0];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    for (int32_t t = threadIdx.x; t < first && t < kQueueLds; t += blockDim.x) lq[0][t] = qg0[t];
    __syncthreads();
    int32_t size = first, lev = 0;
    int64_t total = 0;
    while (size > 0) {
        const int cb = lev & 1, nb = cb ^ 1;
        const int32_t *gcur = cb ? qg1 : qg0;
        int32_t *gnxt = cb ? qg0 : qg1;
        int32_t *app = &cnt[lev % 3];
        if (threadIdx.x == 0) cnt[(lev + 1) % 3] = 0;
        for (int32_t t = threadIdx.x; t < size; t += blockDim.x) {
            const int32_t i = t < kQueueLds ? lq[cb][t] : gcur[t];
            const int32_t p0 = A.rowptr[i], p1 = A.rowptr[i + 1];
            const int32_t d0 = drow[i], d1 = drow[i + 1];
            const int32_t len = p1 - p0, dl = d1 - d0;
            if (len > 0 && len <= kRowFast && dl <= kRowFast) {
                // one batch: the row, the downstream cells; then the count-downs
                // (a padding lane decrements this thread's own spare counter)
                // and the inflow values, all in flight together
                int32_t cj[kRowFast], dj[kRowFast], last[kRowFast];
                double cv[kRowFast];
#pragma unroll
                for (int e = 0; e < kRowFast; ++e) {
                    const int32_t p = p0 + (e < len ? e : len - 1);
                    cj[e] = A.col[p];
                    cv[e] = A.val[p];
                    dj[e] = dcol[dl > 0 ? d0 + (e < dl ? e : dl - 1) : 0];
                }
                const int64_t spare = n + threadIdx.x;
#pragma unroll
                for (int e = 0; e < kRowFast; ++e) last[e] = atomicSub(&indeg[e < dl ? (int64_t)dj[e] : spare], 1);
                solve_row_fast(n, i, cj, cv, len, nrhs, b, x);
#pragma unroll
                for (int e = 0; e < kRowFast; ++e) {
                    if (e < dl && last[e] == 1) {
                        const int32_t pos = atomicAdd(app, 1);
                        if (pos < kQueueLds) lq[nb][pos] = dj[e];
                        else gnxt[pos] = dj[e];
                    }
                }
            } else {
                solve_row_slow(A, i, p0, p1, nrhs, b, x);
                for (int32_t q = d0; q < d1; ++q) {
                    const int32_t k2 = dcol[q];
                    if (atomicSub(&indeg[k2], 1) == 1) {
                        const int32_t pos = atomicAdd(app, 1);
                        if (pos < kQueueLds) lq[nb][pos] = k2;
                        else gnxt[pos] = k2;
                    }
                }
            }
        }
        __syncthreads();
        total += size;
        size = *app;
        ++lev;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = total;
        out[1] = lev;
    }
}


// ---------------------------------------------------- dual delineation --

constexpr int kMaxSweepWells = 64;

// A CSR whose values the well terms modify in place.
struct CsrViewMut {
    int32_t n;
    const int32_t *rowptr, *col;
    double *val;
};

__global__ void k_negate(const double *__restrict__ a, double *__restrict__ out, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) out[i] = -a[i];
}

// Indicator right-hand side of one zone of the x = 0 face: the inflow through
// the face, for the face cells inside the zone (the other entries are zero
// already).  One thread per cell of the face.
__global__ void k_zone_rhs(int32_t nx, int32_t ny, int32_t nz, const double *__restrict__ qx, gw_zone z,
                           double *__restrict__ b) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)ny * nz) return;
    const int32_t j = (int32_t)(t % ny), k = (int32_t)(t / ny);
    if (j < z.j0 || j >= z.j1 || k < z.k0 || k >= z.k1) return;
    const double q = qx[(int64_t)(nx + 1) * (j + (int64_t)ny * k)];
    b[(int64_t)nx * (j + (int64_t)ny * k)] = q > 0.0 ? q : 0.0;
}

struct WellTerms {
    int32_t n;
    int64_t cell[kMaxSweepWells];
    double rate[kMaxSweepWells];   // |q|
    int32_t block[kMaxSweepWells]; // right-hand side that receives |q| at the cell
};

// Wells that bound the system, in list order (one thread: repeated additions
// on one cell are ordered): each adds |q| to its cell's diagonal; a cell that
// was assembled as an identity row (b_tau = 0) first becomes a regular row
// with diagonal 0 and b_tau = phi V.
__global__ void k_well_terms(CsrViewMut A, double *bt, double phi_v, WellTerms w, double *rhs) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t n = A.n;
    for (int32_t k = 0; k < w.n; ++k) {
        const int64_t c = w.cell[k];
        int32_t p = A.rowptr[c];
        while (p + 1 < A.rowptr[c + 1] && A.col[p] != (int32_t)c) ++p;
        if (bt[c] == 0.0) {
            A.val[p] = 0.0;
            bt[c] = phi_v;
        }
        A.val[p] = A.val[p] + w.rate[k];
        rhs[w.block[k] * n + c] = w.rate[k];
    }
}

// ------------------------------------------------- sweep on a 7-point grid --
// On a grid the neighbours of a cell are fixed offsets, so a row is stored as
// one 64-byte record: the matrix entries of the six faces (zero where the face
// brings no inflow), the diagonal, and two 6-bit masks: the faces with
// inflow (the row's off-diagonal entries) and the faces with outflow (the
// cells downstream).  The right-hand sides and solutions of a cell are
// interleaved, so one load returns a neighbour's values of two systems.  A
// sweep step then reads one record line, one value pair per inflow face, and
// counts down the outflow faces: about a third of the memory requests of the
// general sweep.

struct alignas(64) GridRow {
    double v[6];  // faces -z, -y, -x, +x, +y, +z: ascending column order
    double diag;
    int32_t in_mask, out_mask;
};

struct FaceOffsets {
    int64_t d[6];
};

__device__ __forceinline__ FaceOffsets face_offsets(int32_t nx, int32_t ny) {
    const int64_t sxy = (int64_t)nx * ny;
    return {{-sxy, -(int64_t)nx, -1, 1, nx, sxy}};
}

// Records from an assembled upwind CSR (columns ascending): the face of an
// entry is found from the cell coordinates, so grids with a dimension of one
// cell (where two offsets coincide) are handled too.
__global__ void k_grid_rows(CsrView A, int32_t nx, int32_t ny, GridRow *__restrict__ rows,
                            int32_t *__restrict__ indeg) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= A.n) return;
    const int64_t sxy = (int64_t)nx * ny;
    const int32_t i = (int32_t)(c % nx), j = (int32_t)((c / nx) % ny), k = (int32_t)(c / sxy);
    GridRow r;
#pragma unroll
    for (int f = 0; f < 6; ++f) r.v[f] = 0.0;
    r.diag = 0.0;
    r.in_mask = 0;
    r.out_mask = 0;
    for (int32_t p = A.rowptr[c]; p < A.rowptr[c + 1]; ++p) {
        const int64_t col = A.col[p];
        if (col == c) {
            r.diag = A.val[p];
            continue;
        }
        const int32_t ci = (int32_t)(col % nx), cj = (int32_t)((col / nx) % ny), ck = (int32_t)(col / sxy);
        int f;
        if (ck != k) f = ck < k ? 0 : 5;
        else if (cj != j) f = cj < j ? 1 : 4;
        else f = ci < i ? 2 : 3;
        r.v[f] = A.val[p];
        r.in_mask |= 1 << f;
    }
    rows[c] = r;
    indeg[c] = __popc(r.in_mask);
}

// Outflow faces: face f of cell c feeds its neighbour when the neighbour's
// opposite face (5 - f) is an inflow face.
__global__ void k_grid_out(int64_t n, int32_t nx, int32_t ny, GridRow *__restrict__ rows) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t sxy = (int64_t)nx * ny;
    const int32_t nz = (int32_t)(n / sxy);
    const int32_t i = (int32_t)(c % nx), j = (int32_t)((c / nx) % ny), k = (int32_t)(c / sxy);
    const bool has[6] = {k > 0, j > 0, i > 0, i < nx - 1, j < ny - 1, k < nz - 1};
    const FaceOffsets o = face_offsets(nx, ny);
    int32_t m = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f)
        if (has[f] && ((rows[c + o.d[f]].in_mask >> (5 - f)) & 1)) m |= 1 << f;
    rows[c].out_mask = m;
}

// Right-hand sides from nrhs blocks of n values to nrp interleaved values per
// cell (the padding system is zero), and solutions back.
__global__ void k_interleave_rhs(int64_t n, int32_t nrhs, int32_t nrp, const double *__restrict__ b,
                                 double *__restrict__ bi) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * nrp) return;
    const int64_t c = t / nrp;
    const int32_t k = (int32_t)(t % nrp);
    bi[t] = k < nrhs ? b[k * n + c] : 0.0;
}

__global__ void k_split_sol(int64_t n, int32_t nrhs, int32_t nrp, const double *__restrict__ xi,
                            double *__restrict__ x) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    const int32_t k = (int32_t)(t / n);
    const int64_t c = t % n;
    x[t] = xi[c * nrp + k];
}

// The level-synchronous sweep of k_sweep on grid records; nrp (even) systems
// interleaved per cell, solved two at a time with the same record.
__global__ void __launch_bounds__(kSweepThreads) k_sweep_grid(int64_t n, int32_t nx, int32_t ny,
                                                              const GridRow *__restrict__ rows,
                                                              int32_t *__restrict__ indeg, int32_t nrp,
                                                              const double *__restrict__ bi, double *xi,
                                                              int32_t *qg0, int32_t *qg1, int64_t *out) {
    __shared__ int32_t lq[2][kQueueLds];
    __shared__ int32_t cnt[3];
    const FaceOffsets o = face_offsets(nx, ny);
    const int32_t first = (int32_t)out[0];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    for (int32_t t = threadIdx.x; t < first && t < kQueueLds; t += blockDim.x) lq[0][t] = qg0[t];
    __syncthreads();
    int32_t size = first, lev = 0;
    int64_t total = 0;
    while (size > 0) {
        const int cb = lev & 1, nb = cb ^ 1;
        const int32_t *gcur = cb ? qg1 : qg0;
        int32_t *gnxt = cb ? qg0 : qg1;
        int32_t *app = &cnt[lev % 3];
        if (threadIdx.x == 0) cnt[(lev + 1) % 3] = 0;
        for (int32_t t = threadIdx.x; t < size; t += blockDim.x) {
            const int64_t c = t < kQueueLds ? lq[cb][t] : gcur[t];
            const GridRow r = rows[c];
            // count-downs first: they do not wait for the solve.  All six are
            // issued unconditionally, a face without outflow decrementing this
            // thread's spare counter, so that none waits for another.
            const int64_t spare = n + threadIdx.x;
            int32_t last[6];
#pragma unroll
            for (int f = 0; f < 6; ++f)
                last[f] = atomicSub(&indeg[(r.out_mask >> f) & 1 ? c + o.d[f] : spare], 1);
            for (int32_t k = 0; k < nrp; k += 2) {
                const double2 bb = *reinterpret_cast<const double2 *>(bi + c * nrp + k);
                // only the inflow faces are fetched (masked lanes issue no request)
                double2 xv[6];
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    xv[f] = make_double2(0.0, 0.0);
                    if ((r.in_mask >> f) & 1) xv[f] = *reinterpret_cast<const double2 *>(xi + (c + o.d[f]) * nrp + k);
                }
                double s0 = bb.x, s1 = bb.y;
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const double t0 = s0 - r.v[f] * xv[f].x, t1 = s1 - r.v[f] * xv[f].y;
                    const bool use = (r.in_mask >> f) & 1;
                    s0 = use ? t0 : s0;
                    s1 = use ? t1 : s1;
                }
                *reinterpret_cast<double2 *>(xi + c * nrp + k) = make_double2(s0 / r.diag, s1 / r.diag);
            }
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                if (((r.out_mask >> f) & 1) && last[f] == 1) {
                    const int32_t pos = atomicAdd(app, 1);
                    const int32_t d = (int32_t)(c + o.d[f]);
                    if (pos < kQueueLds) lq[nb][pos] = d;
                    else gnxt[pos] = d;
                }
            }
        }
        __syncthreads();
        total += size;
        size = *app;
        ++lev;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = total;
        out[1] = lev;
    }
}

}  // namespace

int64_t upwind_sweep(const CsrView &A, int32_t nrhs, const double *b, double *x, int32_t *levels,
                     hipStream_t s) {
    const int64_t n = A.n;
    // indeg: one count-down per cell, then one spare counter per sweep thread
    DBuf<int32_t> indeg((size_t)n + kSweepThreads), drow((size_t)n + 1), dfill(n), flag(n), q0(n), q1(n);
    DBuf<int32_t> dcol((size_t)std::max<int64_t>(A.nnz - n, 1));
    DBuf<int64_t> total(1), out(2);
    {
        // rows read twice (count, fill), lists written, frontier flags
        ProfScope ps(K_SWEEP_LISTS, 2.0 * ((double)(n + 1) * 4 + (double)A.nnz * 4) + (double)A.nnz * 8 + n * 24.0,
                     s);
        fill_i32(drow.p, 0, n + 1, s);
        fill_i32(dfill.p, 0, n, s);
        fill_i32(indeg.p + n, INT32_MAX, kSweepThreads, s);
        hipLaunchKernelGGL(k_sw_count, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, indeg.p, drow.p);
        scan_inclusive_i32(drow.p + 1, n, total.p, s);
        hipLaunchKernelGGL(k_sw_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, drow.p, dfill.p, dcol.p);
        hipLaunchKernelGGL(k_sw_flag, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, indeg.p, flag.p);
        scan_inclusive_i32(flag.p, n, out.p, s);
        hipLaunchKernelGGL(k_sw_first, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, flag.p, q0.p);
        GW_HIP(hipGetLastError());
    }
    {
        // the operator, the right-hand sides and the solution once each
        ProfScope ps(K_SWEEP, (double)(n + 1) * 4 + (double)A.nnz * 12 + (double)n * nrhs * 16, s);
        hipLaunchKernelGGL(k_sweep, dim3(1), dim3(kSweepThreads), 0, s, A, indeg.p, drow.p, dcol.p, nrhs, b, x,
                           q0.p, q1.p, out.p, (const int32_t *)nullptr);
        GW_HIP(hipGetLastError());
    }
    int64_t *stage = static_cast<int64_t *>(host_stage());
    GW_HIP(hipMemcpyAsync(stage, out.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    if (levels) *levels = (int32_t)stage[1];
    return stage[0];
}

void sweep_plan(TriPlan &P, hipStream_t s) {
    const CsrView A = view(P.M);
    const int64_t n = A.n;
    P.indeg0.alloc((size_t)n + kSweepThreads);
    P.drow.alloc((size_t)n + 1);
    P.dcol.alloc((size_t)std::max<int64_t>(A.nnz - n, 1));
    P.q0.alloc((size_t)std::max<int64_t>(n, 1));
    P.first.alloc(1);
    P.indeg.alloc((size_t)n + kSweepThreads);
    P.qa.alloc((size_t)std::max<int64_t>(n, 1));
    P.qb.alloc((size_t)std::max<int64_t>(n, 1));
    P.out.alloc(2);
    DBuf<int32_t> dfill(n), flag(n);
    DBuf<int64_t> total(1);
    ProfScope ps(K_SWEEP_LISTS, 2.0 * ((double)(n + 1) * 4 + (double)A.nnz * 4) + (double)A.nnz * 8 + n * 24.0, s);
    fill_i32(P.drow.p, 0, n + 1, s);
    fill_i32(dfill.p, 0, n, s);
    fill_i32(P.indeg0.p + n, INT32_MAX, kSweepThreads, s);
    hipLaunchKernelGGL(k_sw_count, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, P.indeg0.p, P.drow.p);
    scan_inclusive_i32(P.drow.p + 1, n, total.p, s);
    hipLaunchKernelGGL(k_sw_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, P.drow.p, dfill.p, P.dcol.p);
    hipLaunchKernelGGL(k_sw_flag, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, P.indeg0.p, flag.p);
    scan_inclusive_i32(flag.p, n, P.first.p, s);
    hipLaunchKernelGGL(k_sw_first, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, flag.p, P.q0.p);
    GW_HIP(hipGetLastError());
}

void sweep_run(TriPlan &P, const double *b, double *x, const int32_t *done, hipStream_t s) {
    const CsrView A = view(P.M);
    const int64_t n = A.n;
    ProfScope ps(K_SWEEP, (double)(n + 1) * 4 + (double)A.nnz * 12 + (double)n * 16, s);
    hipLaunchKernelGGL(k_sweep_prep, dim3(blocks_for(n + kSweepThreads)), dim3(kBlock), 0, s, n, P.indeg0.p, P.q0.p,
                       P.first.p, P.indeg.p, P.qa.p, P.out.p, done);
    hipLaunchKernelGGL(k_sweep, dim3(1), dim3(kSweepThreads), 0, s, A, P.indeg.p, P.drow.p, P.dcol.p, 1, b, x, P.qa.p,
                       P.qb.p, P.out.p, done);
    GW_HIP(hipGetLastError());
}

int64_t grid_sweep(const gw_grid &g, const CsrView &A, int32_t nrhs, const double *b, double *x, int32_t *levels,
                   hipStream_t s) {
    const int64_t n = A.n;
    const int32_t nrp = (nrhs + 1) & ~1;
    DBuf<GridRow> rows(n);
    // count-downs of the cells, then one spare counter per sweep thread
    DBuf<int32_t> indeg((size_t)n + kSweepThreads), flag(n), q0(n), q1(n);
    DBuf<double> bi((size_t)n * nrp), xi((size_t)n * nrp);
    DBuf<int64_t> out(2);
    {
        // CSR read once, records written and read back, frontier flags
        ProfScope ps(K_SWEEP_LISTS, (double)(n + 1) * 4 + (double)A.nnz * 12 + n * (64.0 * 3 + 16),
                     s);
        fill_i32(indeg.p + n, INT32_MAX, kSweepThreads, s);
        hipLaunchKernelGGL(k_grid_rows, dim3(blocks_for(n)), dim3(kBlock), 0, s, A, g.nx, g.ny, rows.p, indeg.p);
        hipLaunchKernelGGL(k_grid_out, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, g.nx, g.ny, rows.p);
        hipLaunchKernelGGL(k_sw_flag, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, indeg.p, flag.p);
        scan_inclusive_i32(flag.p, n, out.p, s);
        hipLaunchKernelGGL(k_sw_first, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, flag.p, q0.p);
        hipLaunchKernelGGL(k_interleave_rhs, dim3(blocks_for(n * nrp)), dim3(kBlock), 0, s, n, nrhs, nrp, b,
                           bi.p);
        GW_HIP(hipGetLastError());
    }
    {
        ProfScope ps(K_SWEEP, (double)n * (64.0 + 16.0 * nrp), s);
        hipLaunchKernelGGL(k_sweep_grid, dim3(1), dim3(kSweepThreads), 0, s, n, g.nx, g.ny, rows.p, indeg.p, nrp,
                           bi.p, xi.p, q0.p, q1.p, out.p);
        GW_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_split_sol, dim3(blocks_for(n * nrhs)), dim3(kBlock), 0, s, n, nrhs, nrp, xi.p, x);
    GW_HIP(hipGetLastError());
    int64_t *stage = static_cast<int64_t *>(host_stage());
    GW_HIP(hipMemcpyAsync(stage, out.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    if (levels) *levels = (int32_t)stage[1];
    return stage[0];
}

void delineate(const gw_grid &g, const double *qx, const double *qy, const double *qz, double phi,
               const gw_zone *zones, int32_t nzones, const gw_well *wells, int32_t nwells, Csr &A, double *out,
               int32_t levels[2], int64_t solved[2], hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const double phi_v = phi * ((g.dx * g.dy) * g.dz);
    WellTerms inj{}, prod{};
    int32_t n_inj = 0, n_prod = 0;
    for (int32_t k = 0; k < nwells; ++k) {
        const gw_well &w = wells[k];
        const int64_t c = w.ix + (int64_t)g.nx * (w.iy + (int64_t)g.ny * w.iz);
        if (w.q < 0) {
            inj.cell[inj.n] = c;
            inj.rate[inj.n] = -w.q;
            inj.block[inj.n] = 1 + nzones + n_inj++;
            ++inj.n;
        } else if (w.q > 0) {
            prod.cell[prod.n] = c;
            prod.rate[prod.n] = w.q;
            prod.block[prod.n] = 1 + n_prod++;
            ++prod.n;
        }
    }
    const int32_t nf = 1 + nzones + n_inj, nb = 1 + n_prod;
    const int64_t fluxes[3] = {(int64_t)(g.nx + 1) * g.ny * g.nz, (int64_t)g.nx * (g.ny + 1) * g.nz,
                               (int64_t)g.nx * g.ny * (g.nz + 1)};
    DBuf<double> rhs((size_t)n * std::max(nf, nb)), scratch(n);
    DBuf<int64_t> nnz(1);
    DBuf<int32_t> nid(1);
    for (int dir = 0; dir < 2; ++dir) {
        const double *q[3] = {qx, qy, qz};
        DBuf<double> rq[3];
        if (dir == 1) {
            for (int a = 0; a < 3; ++a) {
                rq[a].alloc((size_t)fluxes[a]);
                hipLaunchKernelGGL(k_negate, dim3(blocks_for(fluxes[a])), dim3(kBlock), 0, s, q[a], rq[a].p,
                                   fluxes[a]);
                q[a] = rq[a].p;
            }
        }
        const int32_t nr = dir == 0 ? nf : nb;
        fill_f64(rhs.p + n, 0.0, n * (nr - 1), s);
        fill_i32(nid.p, 0, 1, s);
        fill_i32(A.rowptr.p, 0, 1, s);
        const gw_zone all{0, g.ny, 0, g.nz};
        launch_tt_count(g, q[0], q[1], q[2], A.rowptr.p + 1, s);
        scan_inclusive_i32(A.rowptr.p + 1, n, nnz.p, s);
        launch_tt_fill(g, q[0], q[1], q[2], phi, all, A.rowptr.p, A.col.p, A.val.p, rhs.p, scratch.p, nid.p, s);
        if (dir == 0) {
            for (int32_t z = 0; z < nzones; ++z)
                hipLaunchKernelGGL(k_zone_rhs, dim3(blocks_for((int64_t)g.ny * g.nz)), dim3(kBlock), 0, s, g.nx,
                                   g.ny, g.nz, q[0], zones[z], rhs.p + (1 + z) * n);
        }
        const WellTerms &wt = dir == 0 ? inj : prod;
        if (wt.n) {
            const CsrViewMut M{(int32_t)n, A.rowptr.p, A.col.p, A.val.p};
            hipLaunchKernelGGL(k_well_terms, dim3(1), dim3(64), 0, s, M, rhs.p, phi_v, wt, rhs.p);
        }
        GW_HIP(hipGetLastError());
        int64_t *stage = static_cast<int64_t *>(host_stage());
        GW_HIP(hipMemcpyAsync(stage, nnz.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GW_HIP(hipStreamSynchronize(s));
        const CsrView V{(int32_t)n, (int32_t)n, stage[0], A.rowptr.p, A.col.p, A.val.p};
        solved[dir] = grid_sweep(g, V, nr, rhs.p, out + (dir == 0 ? 0 : nf * n), &levels[dir], s);
    }
}

}  // namespace gw
