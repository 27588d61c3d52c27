/*
 * gwref.c -- plain FP64 CPU oracle for the groundwater AMG-Krylov path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (Sbai & Larabi, "On Solving Groundwater Flow and Transport
 * Models with Algebraic Multigrid Preconditioning"):
 *   - the cell-centred finite-difference head equation whose 7-point matrix is
 *     an M-matrix (Benchmarking Examples section);
 *   - a smoothed-aggregation AMG hierarchy: setup phase, then V-cycle built of
 *     sparse matrix-vector products with a direct solve on the coarsest level
 *     (Introduction, description of the two AMG phases);
 *   - AMG-preconditioned CG for flow and BiCGSTAB for the travel-time system
 *     (Benchmarking Examples; Results, Groundwater Flow / Transport Problems);
 *   - Darcy face fluxes and the steady forward travel-time equation v.grad(tau)
 *     = phi with tau = 0 on inflow boundaries (Eq. 1), discretised by first-order
 *     upwinding; the same matrix serves a second right-hand side (Introduction,
 *     dual delineation: all its equations share one matrix).
 *
 * The paper names smoothed aggregation but gives none of its constants; the
 * readings used here (strength threshold, MIS-2 rule, tie-breaks, prolongator
 * smoothing weight, summation orders, stopping rules) are the project's own,
 * listed in the design notes, and the HIP path is written from the same list.
 *
 * Every floating-point sum in the setup runs left to right in the order stated
 * next to it, and the file is compiled with -ffp-contract=off so no product is
 * fused into an add: the setup results are then bit-reproducible.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_OK 0
#define REF_NOT_CONVERGED 1
#define REF_BREAKDOWN 2
#define REF_EINVAL (-1)
#define REF_SINGULAR (-3)

#define SM_JACOBI 0
#define SM_SPAI0 1
#define SM_NONE 2
#define SM_ILU0 3

#define ST_OUT 0u
#define ST_UNDECIDED 1u
#define ST_ROOT 2u

#define REF_MAX_LEVELS 32
#define REF_MAX_DENSE 2048

typedef struct {
    int32_t n, ncols;
    int64_t nnz;
    int32_t *rowptr, *col;
    double *val;
} rcsr;

typedef struct {
    double eps_strong;   /* epsilon_0 of the strength test                */
    int32_t smoother;    /* SM_JACOBI | SM_SPAI0 | SM_NONE | SM_ILU0      */
    double omega;        /* Jacobi damping                                 */
    int32_t npre, npost; /* smoothing sweeps                               */
    int32_t n_coarse;    /* stop coarsening at or below this size          */
    int32_t max_levels;
    uint64_t seed;       /* MIS-2 / PMIS hash seed                         */
    int32_t coarsening;  /* CO_SA | CO_RS                                  */
} ref_params;

#define CO_SA 0
#define CO_RS 1

typedef struct {
    rcsr A;
    rcsr P, R;          /* empty on the coarsest level                    */
    int32_t *agg;       /* aggregate of each row, -1 = removed node        */
    int32_t *state;     /* final MIS-2 state                               */
    int32_t nc;         /* number of aggregates                            */
    double *M;          /* smoother diagonal                               */
    double *ilu;        /* ILU(0) factors on A's pattern (SM_ILU0): L below
                           the diagonal (unit diagonal implied), U on and
                           above it                                        */
    int32_t *dpos;      /* position of each row's diagonal entry           */
    double omega_p;     /* prolongator smoothing weight                    */
    int64_t nnz_s;      /* strength-graph edges                            */
    int32_t mis_rounds;
} ref_level;

typedef struct {
    int nlevels;
    ref_params prm;
    ref_level L[REF_MAX_LEVELS];
    int32_t nd;         /* coarsest size (dense)                           */
    double *lu;         /* row-major LU factors of the coarsest matrix     */
    int32_t *piv;
    double *work[REF_MAX_LEVELS][3];
} ref_hier;

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s ? s : 1);
    if (!p) abort();
    return p;
}

static void csr_alloc(rcsr *A, int32_t n, int32_t ncols, int64_t nnz) {
    A->n = n;
    A->ncols = ncols;
    A->nnz = nnz;
    A->rowptr = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    A->col = (int32_t *)xcalloc((size_t)nnz, sizeof(int32_t));
    A->val = (double *)xcalloc((size_t)nnz, sizeof(double));
}

static void csr_free(rcsr *A) {
    free(A->rowptr);
    free(A->col);
    free(A->val);
    memset(A, 0, sizeof(*A));
}

/* ------------------------------------------------------------------------ */
/* Finite-difference flow assembly (Benchmarking Examples: 5-/7-point       */
/* stencils giving an M-matrix).                                             */
/* ------------------------------------------------------------------------ */

/* nnz of the 7-point matrix: every cell couples to itself and to each
 * existing neighbour; Dirichlet faces only change the diagonal. */
int64_t ref_fv_nnz(int32_t nx, int32_t ny, int32_t nz) {
    int64_t n = (int64_t)nx * ny * nz;
    return 7 * n - 2 * ((int64_t)nx * ny + (int64_t)ny * nz + (int64_t)nx * nz);
}

/* Harmonic-mean face transmissibility between two cells.  ka is the cell with
 * the lower flat index so the value is computed once per face. */
static double face_t(double geo, double ka, double kb) {
    return geo * ((2.0 * ka * kb) / (ka + kb));
}

/* Assemble A h = b.  Fixed heads sit on the x = 0 and x = L faces, at half a
 * cell from the boundary cell centre (T_b = geo * 2K).  Other faces are
 * no-flow.  Wells are point sinks: b -= Q.  Columns ascend; the diagonal is
 * the sum of the six face terms in the order -z, -y, -x, +x, +y, +z, then the
 * west and east Dirichlet terms. */
int ref_fv_assemble(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                    const double *K, double hw, double he,
                    const int32_t *well_ijk, const double *well_q, int32_t nwells,
                    int32_t *rowptr, int32_t *col, double *val, double *b) {
    const double gx = (dy * dz) / dx, gy = (dx * dz) / dy, gz = (dx * dy) / dz;
    const int64_t sxy = (int64_t)nx * ny;
    int64_t p = 0;
    int64_t n = sxy * nz;
    for (int64_t c = 0; c < n; ++c) {
        if (!(K[c] > 0.0) || !isfinite(K[c])) return REF_EINVAL;
    }
    rowptr[0] = 0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t c = i + nx * ((int64_t)j + (int64_t)ny * k);
                double kc = K[c];
                double t[6];
                int64_t nb[6];
                int has[6];
                /* -z, -y, -x, +x, +y, +z */
                has[0] = k > 0;      nb[0] = c - sxy;
                has[1] = j > 0;      nb[1] = c - nx;
                has[2] = i > 0;      nb[2] = c - 1;
                has[3] = i < nx - 1; nb[3] = c + 1;
                has[4] = j < ny - 1; nb[4] = c + nx;
                has[5] = k < nz - 1; nb[5] = c + sxy;
                const double geo[6] = {gz, gy, gx, gx, gy, gz};
                for (int f = 0; f < 6; ++f) {
                    if (!has[f]) { t[f] = 0.0; continue; }
                    double kn = K[nb[f]];
                    t[f] = (f < 3) ? face_t(geo[f], kn, kc) : face_t(geo[f], kc, kn);
                }
                double diag = 0.0;
                for (int f = 0; f < 6; ++f)
                    if (has[f]) diag = diag + t[f];
                double rhs = 0.0;
                if (i == 0) {
                    double tb = gx * (2.0 * kc);
                    diag = diag + tb;
                    rhs = rhs + tb * hw;
                }
                if (i == nx - 1) {
                    double tb = gx * (2.0 * kc);
                    diag = diag + tb;
                    rhs = rhs + tb * he;
                }
                for (int32_t w = 0; w < nwells; ++w)
                    if (well_ijk[3 * w] == i && well_ijk[3 * w + 1] == j && well_ijk[3 * w + 2] == k)
                        rhs = rhs - well_q[w];
                /* lower neighbours, diagonal, upper neighbours: ascending */
                for (int f = 0; f < 3; ++f)
                    if (has[f]) { col[p] = (int32_t)nb[f]; val[p] = -t[f]; ++p; }
                col[p] = (int32_t)c; val[p] = diag; ++p;
                for (int f = 3; f < 6; ++f)
                    if (has[f]) { col[p] = (int32_t)nb[f]; val[p] = -t[f]; ++p; }
                rowptr[c + 1] = (int32_t)p;
                b[c] = rhs;
            }
    return REF_OK;
}

/* Darcy face fluxes q = T (h_upper_index_side ...): positive along +x/+y/+z.
 * qx has (nx+1)*ny*nz entries, face i of row (j,k) at i + (nx+1)*(j + ny*k):
 * interior T*(h[i-1]-h[i]); west T_b*(hw-h[0]); east T_b*(h[nx-1]-he).
 * qy, qz likewise, zero on the no-flow faces. */
void ref_darcy_flux(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                    const double *K, double hw, double he, const double *h,
                    double *qx, double *qy, double *qz) {
    const double gx = (dy * dz) / dx, gy = (dx * dz) / dy, gz = (dx * dy) / dz;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i <= nx; ++i) {
                int64_t f = i + (int64_t)(nx + 1) * (j + (int64_t)ny * k);
                int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
                double q;
                if (i == 0) q = (gx * (2.0 * K[c])) * (hw - h[c]);
                else if (i == nx) q = (gx * (2.0 * K[c - 1])) * (h[c - 1] - he);
                else q = face_t(gx, K[c - 1], K[c]) * (h[c - 1] - h[c]);
                qx[f] = q;
            }
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j <= ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t f = i + (int64_t)nx * (j + (int64_t)(ny + 1) * k);
                int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
                double q = 0.0;
                if (j > 0 && j < ny) q = face_t(gy, K[c - nx], K[c]) * (h[c - nx] - h[c]);
                qy[f] = q;
            }
    const int64_t sxy = (int64_t)nx * ny;
    for (int32_t k = 0; k <= nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t f = i + (int64_t)nx * (j + (int64_t)ny * k);
                int64_t c = f;
                double q = 0.0;
                if (k > 0 && k < nz) q = face_t(gz, K[c - sxy], K[c]) * (h[c - sxy] - h[c]);
                qz[f] = q;
            }
}

/* ------------------------------------------------------------------------ */
/* Upwind travel-time system (Eq. 1, advective form).                         */
/* Row i:  sum_in |q_f| tau_i - sum_{interior inflow faces} |q_f| tau_up = phi*V_i */
/* Inflow boundary faces carry tau = 0 and add nothing to b_tau.  The second */
/* right-hand side is the inflow indicator of a source zone, a window        */
/* [j0,j1) x [k0,k1) of the x = 0 face:  b_c,i = |q| on that face of cell i  */
/* when it is an inflow face inside the window.  Its solution c_i is the     */
/* fraction of the water in cell i that entered through the zone.  A row     */
/* with no inflow face becomes an identity row with zero right-hand sides.   */
/* Face order for the diagonal sum and for columns: -z, -y, -x, +x, +y, +z.  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double in[6];      /* |q| of each face if it is an inflow face, else 0 */
    int interior[6];   /* face has a neighbour cell                        */
    int64_t nb[6];
} tt_faces;

static void tt_cell_faces(int32_t nx, int32_t ny, int32_t nz, const double *qx, const double *qy,
                          const double *qz, int32_t i, int32_t j, int32_t k, tt_faces *F) {
    int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
    int64_t sxy = (int64_t)nx * ny;
    int64_t fxw = i + (int64_t)(nx + 1) * (j + (int64_t)ny * k), fxe = fxw + 1;
    int64_t fys = i + (int64_t)nx * (j + (int64_t)(ny + 1) * k), fyn = fys + nx;
    int64_t fzb = c, fzt = c + sxy;
    /* flux into the cell across each face */
    double qin[6];
    qin[0] = qz[fzb];   /* -z face: +z flux enters */
    qin[1] = qy[fys];
    qin[2] = qx[fxw];
    qin[3] = -qx[fxe];  /* +x face: -x flux enters */
    qin[4] = -qy[fyn];
    qin[5] = -qz[fzt];
    F->interior[0] = k > 0;      F->nb[0] = c - sxy;
    F->interior[1] = j > 0;      F->nb[1] = c - nx;
    F->interior[2] = i > 0;      F->nb[2] = c - 1;
    F->interior[3] = i < nx - 1; F->nb[3] = c + 1;
    F->interior[4] = j < ny - 1; F->nb[4] = c + nx;
    F->interior[5] = k < nz - 1; F->nb[5] = c + sxy;
    for (int f = 0; f < 6; ++f) F->in[f] = qin[f] > 0.0 ? qin[f] : 0.0;
}

int64_t ref_tt_nnz(int32_t nx, int32_t ny, int32_t nz, const double *qx, const double *qy,
                   const double *qz) {
    int64_t nnz = 0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                tt_faces F;
                tt_cell_faces(nx, ny, nz, qx, qy, qz, i, j, k, &F);
                nnz += 1;
                for (int f = 0; f < 6; ++f)
                    if (F.interior[f] && F.in[f] > 0.0) nnz += 1;
            }
    return nnz;
}

int64_t ref_tt_assemble(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                        const double *qx, const double *qy, const double *qz, double phi,
                        const int32_t *zone, int32_t *rowptr, int32_t *col, double *val,
                        double *b_tau, double *b_c) {
    int64_t p = 0, n_ident = 0;
    const double vol = (dx * dy) * dz;
    rowptr[0] = 0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
                tt_faces F;
                tt_cell_faces(nx, ny, nz, qx, qy, qz, i, j, k, &F);
                double diag = 0.0;
                for (int f = 0; f < 6; ++f) diag = diag + F.in[f];
                double bt = phi * vol, bc = 0.0;
                if (i == 0 && j >= zone[0] && j < zone[1] && k >= zone[2] && k < zone[3]) bc = F.in[2];
                if (!(diag > 0.0)) {
                    diag = 1.0; bt = 0.0; bc = 0.0; ++n_ident;
                    col[p] = (int32_t)c; val[p] = diag; ++p;
                } else {
                    for (int f = 0; f < 3; ++f)
                        if (F.interior[f] && F.in[f] > 0.0) { col[p] = (int32_t)F.nb[f]; val[p] = -F.in[f]; ++p; }
                    col[p] = (int32_t)c; val[p] = diag; ++p;
                    for (int f = 3; f < 6; ++f)
                        if (F.interior[f] && F.in[f] > 0.0) { col[p] = (int32_t)F.nb[f]; val[p] = -F.in[f]; ++p; }
                }
                rowptr[c + 1] = (int32_t)p;
                b_tau[c] = bt;
                b_c[c] = bc;
            }
    return n_ident;
}

/* Exact direct solve of the upwind system by one sweep.  An upstream cell j of
 * i has q_ji > 0, i.e. h_j > h_i, so visiting cells by descending head (ties by
 * index) visits every upstream cell first: the matrix is triangular in that
 * order and forward substitution is the exact solution. */
static const double *g_sort_h;
static int cmp_desc_head(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double hi = g_sort_h[i], hj = g_sort_h[j];
    if (hi > hj) return -1;
    if (hi < hj) return 1;
    return (i < j) ? -1 : (i > j);
}

void ref_tt_sweep(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                  const double *b, const double *h, double *x) {
    int64_t *order = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    g_sort_h = h;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_desc_head);
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = order[t];
        double s = b[i], d = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] == i) d = val[p];
            else s = s - val[p] * x[col[p]];
        }
        x[i] = s / d;
    }
    free(order);
}

/* ------------------------------------------------------------------------ */
/* Sparse helpers                                                            */
/* ------------------------------------------------------------------------ */

/* y = A x, each row summed in ascending column order */
static void spmv(const rcsr *A, const double *x, double *y) {
    for (int32_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) s = s + A->val[p] * x[A->col[p]];
        y[i] = s;
    }
}

static double dot(int32_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

/* Transpose; rows of the result list the source rows in ascending order, so
 * columns come out sorted. */
static void transpose(const rcsr *A, rcsr *T) {
    csr_alloc(T, A->ncols, A->n, A->nnz);
    for (int64_t p = 0; p < A->nnz; ++p) T->rowptr[A->col[p] + 1]++;
    for (int32_t i = 0; i < T->n; ++i) T->rowptr[i + 1] += T->rowptr[i];
    int32_t *fill = (int32_t *)xcalloc((size_t)T->n, sizeof(int32_t));
    for (int32_t i = 0; i < A->n; ++i)
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            int32_t j = A->col[p];
            int32_t q = T->rowptr[j] + fill[j]++;
            T->col[q] = i;
            T->val[q] = A->val[p];
        }
    free(fill);
}

static double diag_of(const rcsr *A, int32_t i) {
    for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
        if (A->col[p] == i) return A->val[p];
    return 0.0;
}

/* Validate: square, sorted unique columns in range, positive finite diagonal,
 * finite values. */
int ref_csr_check(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val) {
    if (n <= 0 || rowptr[0] != 0) return REF_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return REF_EINVAL;
        int found = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n) return REF_EINVAL;
            if (p > rowptr[i] && col[p] <= col[p - 1]) return REF_EINVAL;
            if (!isfinite(val[p])) return REF_EINVAL;
            if (col[p] == i) { found = 1; if (!(val[p] > 0.0)) return REF_EINVAL; }
        }
        if (!found) return REF_EINVAL;
    }
    return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Smoothed-aggregation setup (Introduction: the setup phase builds the grid */
/* hierarchy and the transfer operators automatically by nodal aggregation; */
/* Results: smoothed aggregation is the variant used for coarsening).        */
/* ------------------------------------------------------------------------ */

/* MurmurHash3 32-bit finalizer (Appleby). */
static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

static uint32_t level_salt(uint64_t seed, int32_t level) {
    return fmix32((uint32_t)seed ^ fmix32((uint32_t)(seed >> 32) + 0x9E3779B9u * (uint32_t)(level + 1)));
}

/* Priority key of node i: (state rank, hash, index), lexicographic.  OUT nodes
 * carry the lowest key 0; ROOT outranks UNDECIDED.  Requires i < 2^30. */
static uint64_t mis_key(uint32_t state, uint32_t salt, int32_t i) {
    if (state == ST_OUT) return 0;
    return ((uint64_t)state << 62) | ((uint64_t)fmix32((uint32_t)i ^ salt) << 30) | (uint64_t)i;
}

typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t *rowptr, *col;
    double *w;
} rgraph;

/* Strength of connection, symmetrised:  {i,j} strong  <=>
 *   a_ij*a_ij > eps2*(a_ii*a_jj)  or  a_ji*a_ji > eps2*(a_ii*a_jj).
 * Builds the strength graph S (no self loops, weight max(|a_ij|,|a_ji|)) and
 * marks which stored entries of A are strong. */
static void strength(const rcsr *A, const rcsr *At, double eps2, rgraph *S, uint8_t *strongA) {
    int32_t n = A->n;
    double *d = (double *)xcalloc((size_t)n, sizeof(double));
    for (int32_t i = 0; i < n; ++i) d[i] = diag_of(A, i);
    S->n = n;
    S->rowptr = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    int64_t cap = A->nnz + At->nnz;
    S->col = (int32_t *)xcalloc((size_t)cap, sizeof(int32_t));
    S->w = (double *)xcalloc((size_t)cap, sizeof(double));
    int64_t q = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t pa = A->rowptr[i], ea = A->rowptr[i + 1];
        int32_t pt = At->rowptr[i], et = At->rowptr[i + 1];
        while (pa < ea || pt < et) {
            int32_t ja = pa < ea ? A->col[pa] : INT32_MAX;
            int32_t jt = pt < et ? At->col[pt] : INT32_MAX;
            int32_t j = ja < jt ? ja : jt;
            double aij = 0.0, aji = 0.0;
            int32_t posa = -1;
            if (ja == j) { aij = A->val[pa]; posa = pa; ++pa; }
            if (jt == j) { aji = At->val[pt]; ++pt; }
            if (j == i) { if (posa >= 0) strongA[posa] = 0; continue; }
            double dd = d[i] * d[j];
            int s = (aij * aij > eps2 * dd) || (aji * aji > eps2 * dd);
            if (posa >= 0) strongA[posa] = (uint8_t)s;
            if (s) {
                S->col[q] = j;
                S->w[q] = fabs(aij) > fabs(aji) ? fabs(aij) : fabs(aji);
                ++q;
            }
        }
        S->rowptr[i + 1] = (int32_t)q;
    }
    S->nnz = q;
    free(d);
}

/* Distance-2 maximal independent set by synchronous rounds.  Each round:
 *   m1_i = max(key_i, max_{j in S(i)} key_j)
 *   m2_i = max(m1_i, max_{j in S(i)} m1_j)
 *   UNDECIDED i with m2_i == key_i becomes ROOT;
 *   UNDECIDED i whose m2_i has ROOT rank becomes OUT.
 * Nodes with no strong neighbour are removed (OUT from the start). */
static int32_t mis2(const rgraph *S, uint64_t seed, int32_t level, uint32_t *state) {
    int32_t n = S->n;
    uint32_t salt = level_salt(seed, level);
    uint64_t *m1 = (uint64_t *)xcalloc((size_t)n, sizeof(uint64_t));
    int64_t undecided = 0;
    for (int32_t i = 0; i < n; ++i) {
        state[i] = (S->rowptr[i + 1] > S->rowptr[i]) ? ST_UNDECIDED : ST_OUT;
        undecided += state[i] == ST_UNDECIDED;
    }
    int32_t rounds = 0;
    while (undecided > 0) {
        ++rounds;
        for (int32_t i = 0; i < n; ++i) {
            uint64_t m = mis_key(state[i], salt, i);
            for (int32_t p = S->rowptr[i]; p < S->rowptr[i + 1]; ++p) {
                uint64_t kj = mis_key(state[S->col[p]], salt, S->col[p]);
                if (kj > m) m = kj;
            }
            m1[i] = m;
        }
        undecided = 0;
        for (int32_t i = 0; i < n; ++i) {
            if (state[i] != ST_UNDECIDED) continue;
            uint64_t m = m1[i];
            for (int32_t p = S->rowptr[i]; p < S->rowptr[i + 1]; ++p)
                if (m1[S->col[p]] > m) m = m1[S->col[p]];
            /* state[i] is only read for i itself below and in the next round,
             * and m1 already holds every key this round needs */
            if (m == mis_key(ST_UNDECIDED, salt, i)) state[i] = ST_ROOT;
            else if ((m >> 62) == ST_ROOT) state[i] = ST_OUT;
            else ++undecided;
        }
    }
    free(m1);
    return rounds;
}

/* Aggregates from the MIS-2 roots.
 *   ids: roots numbered in ascending node order;
 *   pass 1: a non-root with a strong root neighbour joins it (unique);
 *   pass 2: a node still unassigned joins the pass-1-assigned strong neighbour
 *           with the largest weight, ties to the smaller aggregate id;
 *           pass 2 reads pass-1 assignments only.
 * Returns the number of aggregates. */
static int32_t aggregate(const rgraph *S, const uint32_t *state, int32_t *agg) {
    int32_t n = S->n, nc = 0;
    int32_t *agg1 = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) agg1[i] = (state[i] == ST_ROOT) ? nc++ : -1;
    int32_t *root_id = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    memcpy(root_id, agg1, (size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) {
        if (state[i] == ST_ROOT) continue;
        for (int32_t p = S->rowptr[i]; p < S->rowptr[i + 1]; ++p)
            if (state[S->col[p]] == ST_ROOT) { agg1[i] = root_id[S->col[p]]; break; }
    }
    for (int32_t i = 0; i < n; ++i) {
        agg[i] = agg1[i];
        if (agg1[i] >= 0 || S->rowptr[i + 1] == S->rowptr[i]) continue;
        double best_w = -1.0;
        int32_t best = -1;
        for (int32_t p = S->rowptr[i]; p < S->rowptr[i + 1]; ++p) {
            int32_t a = agg1[S->col[p]];
            if (a < 0) continue;
            double w = S->w[p];
            if (w > best_w || (w == best_w && a < best)) { best_w = w; best = a; }
        }
        agg[i] = best;
    }
    free(agg1);
    free(root_id);
    return nc;
}

/* Smoothed prolongator P = (I - omega_P D_F^{-1} A_F) P_tent with unit P_tent.
 *   A_F: diagonal plus strong off-diagonals, weak off-diagonals lumped onto the
 *        diagonal  dF_i = a_ii + sum_{weak j, ascending} a_ij  (A_F 1 = A 1);
 *   d_i = dF_i if dF_i > 0 else a_ii;
 *   omega_P = (4/3) / rho,  rho = max_i (sum_j |a_ij|, ascending j) / a_ii, the
 *   Gershgorin bound of D^{-1} A on the unfiltered matrix (the same bound on
 *   A_F degenerates on rows where lumping nearly cancels the diagonal);
 *   P_iI = [agg(i) == I] - (omega_P / d_i) * (sum_{j: agg(j)=I, ascending} aF_ij).
 * Rows of removed nodes are empty; columns ascend. */
static double smooth_prolongator(const rcsr *A, const uint8_t *strongA, const int32_t *agg,
                                 int32_t nc, rcsr *P) {
    int32_t n = A->n;
    double *dF = (double *)xcalloc((size_t)n, sizeof(double));
    double *d = (double *)xcalloc((size_t)n, sizeof(double));
    double rho = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double aii = diag_of(A, i);
        double s = aii;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
            if (A->col[p] != i && !strongA[p]) s = s + A->val[p];
        dF[i] = s;
        d[i] = s > 0.0 ? s : aii;
    }
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) s = s + fabs(A->val[p]);
        double r = s / diag_of(A, i);
        if (r > rho) rho = r;
    }
    const double omega = (4.0 / 3.0) / rho;

    /* row lengths: distinct aggregates in the filtered row */
    int32_t *cnt = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    int32_t *tmp_a = (int32_t *)xcalloc(64, sizeof(int32_t));
    int32_t tmp_cap = 64;
    for (int32_t i = 0; i < n; ++i) {
        if (agg[i] < 0) continue;
        int32_t m = 0;
        int32_t len = A->rowptr[i + 1] - A->rowptr[i];
        if (len > tmp_cap) { tmp_cap = len; tmp_a = (int32_t *)realloc(tmp_a, (size_t)tmp_cap * sizeof(int32_t)); }
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            int32_t j = A->col[p];
            if (j != i && !strongA[p]) continue;
            int32_t a = agg[j];
            if (a < 0) continue;
            int dup = 0;
            for (int32_t t = 0; t < m; ++t) dup |= tmp_a[t] == a;
            if (!dup) tmp_a[m++] = a;
        }
        cnt[i + 1] = m;
    }
    int64_t nnz = 0;
    for (int32_t i = 0; i < n; ++i) nnz += cnt[i + 1];
    csr_alloc(P, n, nc, nnz);
    for (int32_t i = 0; i < n; ++i) P->rowptr[i + 1] = P->rowptr[i] + cnt[i + 1];
    for (int32_t i = 0; i < n; ++i) {
        if (agg[i] < 0) continue;
        int32_t m = 0;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            int32_t j = A->col[p];
            if (j != i && !strongA[p]) continue;
            int32_t a = agg[j];
            if (a < 0) continue;
            int dup = 0;
            for (int32_t t = 0; t < m; ++t) dup |= tmp_a[t] == a;
            if (!dup) tmp_a[m++] = a;
        }
        /* ascending aggregate ids (insertion sort; rows are short) */
        for (int32_t t = 1; t < m; ++t) {
            int32_t v = tmp_a[t], u = t - 1;
            while (u >= 0 && tmp_a[u] > v) { tmp_a[u + 1] = tmp_a[u]; --u; }
            tmp_a[u + 1] = v;
        }
        const double coef = omega / d[i];
        int32_t base = P->rowptr[i];
        for (int32_t t = 0; t < m; ++t) {
            int32_t I = tmp_a[t];
            double s = 0.0;
            for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
                int32_t j = A->col[p];
                if (j != i && !strongA[p]) continue;
                if (agg[j] != I) continue;
                double af = (j == i) ? dF[i] : A->val[p];
                s = s + af;
            }
            double delta = (agg[i] == I) ? 1.0 : 0.0;
            P->col[base + t] = I;
            P->val[base + t] = delta - coef * s;
        }
    }
    free(tmp_a);
    free(cnt);
    free(dF);
    free(d);
    return omega;
}

/* C = A B (Gustavson).  Entry (i,J) = sum over k in A's row i, ascending, of
 * a_ik * b_kJ, accumulated left to right from 0.  Columns ascend; entries
 * that cancel to zero are kept. */
static void spgemm(const rcsr *A, const rcsr *B, rcsr *C) {
    int32_t n = A->n, m = B->ncols;
    double *acc = (double *)xcalloc((size_t)m, sizeof(double));
    int32_t *mark = (int32_t *)xcalloc((size_t)m, sizeof(int32_t));
    for (int32_t J = 0; J < m; ++J) mark[J] = -1;
    int32_t *list = (int32_t *)xcalloc((size_t)m, sizeof(int32_t));
    /* symbolic */
    int32_t *rp = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) {
        int32_t cnt = 0;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            int32_t k = A->col[p];
            for (int32_t q = B->rowptr[k]; q < B->rowptr[k + 1]; ++q) {
                int32_t J = B->col[q];
                if (mark[J] != i) { mark[J] = i; ++cnt; }
            }
        }
        rp[i + 1] = rp[i] + cnt;
    }
    csr_alloc(C, n, m, rp[n]);
    memcpy(C->rowptr, rp, ((size_t)n + 1) * sizeof(int32_t));
    free(rp);
    for (int32_t J = 0; J < m; ++J) mark[J] = -1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t cnt = 0;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            int32_t k = A->col[p];
            double a = A->val[p];
            for (int32_t q = B->rowptr[k]; q < B->rowptr[k + 1]; ++q) {
                int32_t J = B->col[q];
                if (mark[J] != i) { mark[J] = i; acc[J] = 0.0; list[cnt++] = J; }
                acc[J] = acc[J] + a * B->val[q];
            }
        }
        /* ascending columns (insertion sort of a short list) */
        for (int32_t t = 1; t < cnt; ++t) {
            int32_t v = list[t], u = t - 1;
            while (u >= 0 && list[u] > v) { list[u + 1] = list[u]; --u; }
            list[u + 1] = v;
        }
        for (int32_t t = 0; t < cnt; ++t) {
            C->col[C->rowptr[i] + t] = list[t];
            C->val[C->rowptr[i] + t] = acc[list[t]];
        }
    }
    free(acc);
    free(mark);
    free(list);
}

/* Dense LU with partial pivoting (LAPACK getrf semantics: first row with the
 * largest |pivot|), row-major, in place. */
static int dense_lu(int32_t n, double *a, int32_t *piv) {
    for (int32_t k = 0; k < n; ++k) {
        int32_t p = k;
        double amax = fabs(a[(int64_t)k * n + k]);
        for (int32_t i = k + 1; i < n; ++i) {
            double v = fabs(a[(int64_t)i * n + k]);
            if (v > amax) { amax = v; p = i; }
        }
        piv[k] = p;
        if (amax == 0.0) return REF_SINGULAR;
        if (p != k)
            for (int32_t j = 0; j < n; ++j) {
                double t = a[(int64_t)k * n + j];
                a[(int64_t)k * n + j] = a[(int64_t)p * n + j];
                a[(int64_t)p * n + j] = t;
            }
        double akk = a[(int64_t)k * n + k];
        for (int32_t i = k + 1; i < n; ++i) {
            double l = a[(int64_t)i * n + k] / akk;
            a[(int64_t)i * n + k] = l;
            for (int32_t j = k + 1; j < n; ++j)
                a[(int64_t)i * n + j] = a[(int64_t)i * n + j] - l * a[(int64_t)k * n + j];
        }
    }
    return REF_OK;
}

static void dense_lu_solve(int32_t n, const double *lu, const int32_t *piv, const double *b, double *x) {
    for (int32_t i = 0; i < n; ++i) x[i] = b[i];
    for (int32_t k = 0; k < n; ++k)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int32_t i = 0; i < n; ++i) {
        double s = x[i];
        for (int32_t j = 0; j < i; ++j) s = s - lu[(int64_t)i * n + j] * x[j];
        x[i] = s;
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int32_t j = i + 1; j < n; ++j) s = s - lu[(int64_t)i * n + j] * x[j];
        x[i] = s / lu[(int64_t)i * n + i];
    }
}

/* Smoother diagonal: Jacobi  M_i = omega / a_ii;  SPAI0  M_i = a_ii / sum_j a_ij^2
 * (ascending j). */
static void smoother_diag(const rcsr *A, const ref_params *prm, double *M) {
    for (int32_t i = 0; i < A->n; ++i) {
        double aii = diag_of(A, i);
        if (prm->smoother == SM_SPAI0) {
            double s = 0.0;
            for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) s = s + A->val[p] * A->val[p];
            M[i] = aii / s;
        } else {
            M[i] = prm->omega / aii;
        }
    }
}

/* ILU(0): the incomplete LU factorization on A's own pattern (Results: the
 * relaxation used throughout).  Row by row in ascending order, and in each
 * row over its lower entries k in ascending column order: l_ik = a_ik / u_kk,
 * then a_ij = a_ij - l_ik u_kj for every later entry j of row i that row k
 * also holds.  Returns REF_SINGULAR for a zero pivot. */
static int ilu0(const rcsr *A, double *ilu, int32_t *dpos) {
    memcpy(ilu, A->val, (size_t)A->nnz * sizeof(double));
    for (int32_t i = 0; i < A->n; ++i) {
        dpos[i] = -1;
        for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
            if (A->col[p] == i) dpos[i] = p;
        if (dpos[i] < 0) return REF_SINGULAR;
    }
    for (int32_t i = 0; i < A->n; ++i) {
        const int32_t e = A->rowptr[i + 1];
        for (int32_t p = A->rowptr[i]; p < e && A->col[p] < i; ++p) {
            const int32_t k = A->col[p];
            const double ukk = ilu[dpos[k]];
            if (ukk == 0.0) return REF_SINGULAR;
            const double lik = ilu[p] / ukk;
            ilu[p] = lik;
            int32_t r = dpos[k] + 1;
            const int32_t ek = A->rowptr[k + 1];
            for (int32_t q = p + 1; q < e; ++q) {
                const int32_t j = A->col[q];
                while (r < ek && A->col[r] < j) ++r;
                if (r < ek && A->col[r] == j) ilu[q] = ilu[q] - lik * ilu[r];
            }
        }
        if (ilu[dpos[i]] == 0.0) return REF_SINGULAR;
    }
    return REF_OK;
}

/* t <- (LU)^{-1} t in place: forward substitution with the unit lower factor,
 * then backward substitution with U, each row's terms in column order. */
static void ilu_solve(const rcsr *A, const double *ilu, const int32_t *dpos, double *t) {
    for (int32_t i = 0; i < A->n; ++i) {
        double s = t[i];
        for (int32_t p = A->rowptr[i]; p < dpos[i]; ++p) s = s - ilu[p] * t[A->col[p]];
        t[i] = s;
    }
    for (int32_t i = A->n - 1; i >= 0; --i) {
        double s = t[i];
        for (int32_t p = dpos[i] + 1; p < A->rowptr[i + 1]; ++p) s = s - ilu[p] * t[A->col[p]];
        t[i] = s / ilu[dpos[i]];
    }
}

/* ---------------------------------------------------------------------- */
/* Ruge-Stueben coarsening (the paper's other AMG variant): classical       */
/* strength, a PMIS C/F splitting and direct interpolation.                 */
/* ---------------------------------------------------------------------- */

/* S_i = { j != i : -a_ij >= theta * max_{k != i} (-a_ik) }, the points i
 * depends on strongly (empty when row i has no negative off-diagonal). */
static void strength_rs(const rcsr *A, double theta, rcsr *S) {
    int32_t n = A->n;
    int64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        cnt = 0;
        for (int32_t i = 0; i < n; ++i) {
            double mx = 0.0;
            for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                if (A->col[p] != i && -A->val[p] > mx) mx = -A->val[p];
            if (pass == 1) S->rowptr[i] = (int32_t)cnt;
            if (mx > 0.0)
                for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                    if (A->col[p] != i && -A->val[p] >= theta * mx) {
                        if (pass == 1) { S->col[cnt] = A->col[p]; S->val[cnt] = 1.0; }
                        ++cnt;
                    }
        }
        if (pass == 0) csr_alloc(S, n, n, cnt);
    }
    S->rowptr[n] = (int32_t)cnt;
}

#define CF_UND 0
#define CF_C 1
#define CF_F 2

/* Weight of point i: the number of points that depend on it strongly, plus
 * a hash fraction in [0, 1) (24 bits of fmix32(i ^ salt)); ties by index. */
static int pmis_beats(double wi, int32_t i, double wj, int32_t j) { return wi > wj || (wi == wj && i > j); }

/* PMIS: a point with no dependents is F; then in rounds, an undecided point
 * whose weight beats every undecided neighbour of the symmetrised strength
 * graph becomes C, and an undecided point that depends strongly on a C point
 * becomes F.  Returns the number of rounds. */
static int32_t pmis(const rcsr *S, const rcsr *St, uint64_t seed, int32_t level, int32_t *cf) {
    int32_t n = S->n;
    uint32_t salt = level_salt(seed, level);
    double *w = (double *)xcalloc((size_t)n, sizeof(double));
    int32_t *newc = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) {
        int32_t dep = St->rowptr[i + 1] - St->rowptr[i];
        w[i] = (double)dep + (double)(fmix32((uint32_t)i ^ salt) >> 8) * (1.0 / 16777216.0);
        cf[i] = dep == 0 ? CF_F : CF_UND;
    }
    int32_t rounds = 0;
    for (;;) {
        int any = 0;
        for (int32_t i = 0; i < n; ++i) any |= cf[i] == CF_UND;
        if (!any) break;
        ++rounds;
        for (int32_t i = 0; i < n; ++i) {
            newc[i] = 0;
            if (cf[i] != CF_UND) continue;
            int best = 1;
            for (int32_t p = S->rowptr[i]; p < S->rowptr[i + 1] && best; ++p) {
                int32_t j = S->col[p];
                if (cf[j] == CF_UND && !pmis_beats(w[i], i, w[j], j)) best = 0;
            }
            for (int32_t p = St->rowptr[i]; p < St->rowptr[i + 1] && best; ++p) {
                int32_t j = St->col[p];
                if (cf[j] == CF_UND && !pmis_beats(w[i], i, w[j], j)) best = 0;
            }
            newc[i] = best;
        }
        for (int32_t i = 0; i < n; ++i)
            if (newc[i]) cf[i] = CF_C;
        for (int32_t i = 0; i < n; ++i) {
            if (cf[i] != CF_UND) continue;
            for (int32_t p = S->rowptr[i]; p < S->rowptr[i + 1]; ++p)
                if (cf[S->col[p]] == CF_C) { cf[i] = CF_F; break; }
        }
    }
    free(w);
    free(newc);
    return rounds;
}

/* Direct interpolation.  C points are numbered in ascending order; a C
 * point's row of P is 1 at its own number.  For an F point i with strong C
 * neighbours C_i: d = a_ii + (positive off-diagonals, lumped), alpha =
 * (sum of negative off-diagonals) / (sum of a_ij over C_i), and
 * P_ij = -(alpha * a_ij) / d for j in C_i (all sums in column order).  An F
 * point without strong C neighbours has an empty row. */
static int32_t interp_direct(const rcsr *A, const rcsr *S, const int32_t *cf, int32_t *cidx, rcsr *P) {
    int32_t n = A->n, nc = 0;
    for (int32_t i = 0; i < n; ++i) cidx[i] = cf[i] == CF_C ? nc++ : -1;
    int64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        cnt = 0;
        for (int32_t i = 0; i < n; ++i) {
            if (pass == 1) P->rowptr[i] = (int32_t)cnt;
            if (cf[i] == CF_C) {
                if (pass == 1) { P->col[cnt] = cidx[i]; P->val[cnt] = 1.0; }
                ++cnt;
                continue;
            }
            double d = 0.0, neg = 0.0, sc = 0.0;
            int32_t q = S->rowptr[i];
            for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
                int32_t j = A->col[p];
                double a = A->val[p];
                if (j == i) { d = d + a; continue; }
                if (a > 0.0) { d = d + a; continue; }
                neg = neg + a;
                while (q < S->rowptr[i + 1] && S->col[q] < j) ++q;
                if (q < S->rowptr[i + 1] && S->col[q] == j && cf[j] == CF_C) sc = sc + a;
            }
            if (sc == 0.0) continue;
            double alpha = neg / sc;
            q = S->rowptr[i];
            for (int32_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
                int32_t j = A->col[p];
                if (j == i || A->val[p] > 0.0) continue;
                while (q < S->rowptr[i + 1] && S->col[q] < j) ++q;
                if (q < S->rowptr[i + 1] && S->col[q] == j && cf[j] == CF_C) {
                    if (pass == 1) { P->col[cnt] = cidx[j]; P->val[cnt] = -(alpha * A->val[p]) / d; }
                    ++cnt;
                }
            }
        }
        if (pass == 0) csr_alloc(P, n, nc, cnt);
    }
    P->rowptr[n] = (int32_t)cnt;
    return nc;
}

static void copy_csr(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, rcsr *A) {
    csr_alloc(A, n, n, rowptr[n]);
    memcpy(A->rowptr, rowptr, ((size_t)n + 1) * sizeof(int32_t));
    memcpy(A->col, col, (size_t)rowptr[n] * sizeof(int32_t));
    memcpy(A->val, val, (size_t)rowptr[n] * sizeof(double));
}

static void make_coarsest(ref_hier *H, int l, int *status) {
    ref_level *L = &H->L[l];
    H->nlevels = l + 1;
    H->nd = L->A.n;
    if (H->nd > REF_MAX_DENSE) { *status = REF_EINVAL; return; }
    int32_t n = H->nd;
    H->lu = (double *)xcalloc((size_t)n * n, sizeof(double));
    H->piv = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = L->A.rowptr[i]; p < L->A.rowptr[i + 1]; ++p)
            H->lu[(int64_t)i * n + L->A.col[p]] = L->A.val[p];
    *status = dense_lu(n, H->lu, H->piv);
}

void ref_amg_free(ref_hier *H);

/* Build the hierarchy.  Level l stops being refined when n_l <= n_coarse or
 * l reaches max_levels-1; a candidate coarse level is dropped (level l becomes
 * the coarsest) if it has no aggregates or fails to shrink below 0.9 n_l.
 * The strength threshold halves per level: eps2_l = eps^2 * 0.25^l. */
ref_hier *ref_amg_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                        const ref_params *prm, int *status) {
    *status = REF_OK;
    if (ref_csr_check(n, rowptr, col, val) != REF_OK) { *status = REF_EINVAL; return NULL; }
    ref_hier *H = (ref_hier *)xcalloc(1, sizeof(ref_hier));
    H->prm = *prm;
    copy_csr(n, rowptr, col, val, &H->L[0].A);
    if (prm->smoother == SM_NONE) { H->nlevels = 0; return H; }
    int maxl = prm->max_levels < 1 ? 1 : (prm->max_levels > REF_MAX_LEVELS ? REF_MAX_LEVELS : prm->max_levels);
    double eps2 = prm->eps_strong * prm->eps_strong;
    for (int l = 0;; ++l) {
        ref_level *L = &H->L[l];
        int32_t nl = L->A.n;
        if (nl <= prm->n_coarse || l == maxl - 1) { make_coarsest(H, l, status); break; }
        if (prm->coarsening == CO_RS) {
            rcsr S, St;
            strength_rs(&L->A, prm->eps_strong, &S);
            transpose(&S, &St);
            L->nnz_s = S.nnz;
            int32_t *cf = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
            L->mis_rounds = pmis(&S, &St, prm->seed, l, cf);
            L->agg = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
            L->state = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
            for (int32_t i = 0; i < nl; ++i) L->state[i] = cf[i];
            L->nc = interp_direct(&L->A, &S, cf, L->agg, &L->P);
            free(cf);
            csr_free(&S);
            csr_free(&St);
            if (L->nc == 0 || (double)L->nc > 0.9 * (double)nl) {
                csr_free(&L->P);
                memset(&L->P, 0, sizeof(L->P));
                make_coarsest(H, l, status);
                break;
            }
            L->M = (double *)xcalloc((size_t)nl, sizeof(double));
            if (prm->smoother == SM_ILU0) {
                L->ilu = (double *)xcalloc((size_t)L->A.nnz, sizeof(double));
                L->dpos = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
                if (ilu0(&L->A, L->ilu, L->dpos) != REF_OK) { *status = REF_SINGULAR; H->nlevels = l + 1; break; }
            } else {
                smoother_diag(&L->A, prm, L->M);
            }
            L->omega_p = 0.0;
            transpose(&L->P, &L->R);
            rcsr AP;
            spgemm(&L->A, &L->P, &AP);
            spgemm(&L->R, &AP, &H->L[l + 1].A);
            csr_free(&AP);
            continue;
        }
        rcsr At;
        transpose(&L->A, &At);
        uint8_t *strongA = (uint8_t *)xcalloc((size_t)L->A.nnz, 1);
        rgraph S;
        strength(&L->A, &At, eps2, &S, strongA);
        csr_free(&At);
        L->nnz_s = S.nnz;
        uint32_t *state = (uint32_t *)xcalloc((size_t)nl, sizeof(uint32_t));
        L->mis_rounds = mis2(&S, prm->seed, l, state);
        L->agg = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
        L->state = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
        for (int32_t i = 0; i < nl; ++i) L->state[i] = (int32_t)state[i];
        L->nc = aggregate(&S, state, L->agg);
        free(state);
        free(S.rowptr); free(S.col); free(S.w);
        if (L->nc == 0 || (double)L->nc > 0.9 * (double)nl) {
            free(strongA);
            make_coarsest(H, l, status);
            break;
        }
        L->M = (double *)xcalloc((size_t)nl, sizeof(double));
        if (prm->smoother == SM_ILU0) {
            L->ilu = (double *)xcalloc((size_t)L->A.nnz, sizeof(double));
            L->dpos = (int32_t *)xcalloc((size_t)nl, sizeof(int32_t));
            if (ilu0(&L->A, L->ilu, L->dpos) != REF_OK) {
                free(strongA);
                *status = REF_SINGULAR;
                H->nlevels = l + 1;
                break;
            }
        } else {
            smoother_diag(&L->A, prm, L->M);
        }
        L->omega_p = smooth_prolongator(&L->A, strongA, L->agg, L->nc, &L->P);
        free(strongA);
        transpose(&L->P, &L->R);
        rcsr AP;
        spgemm(&L->A, &L->P, &AP);
        spgemm(&L->R, &AP, &H->L[l + 1].A);
        csr_free(&AP);
        eps2 = eps2 * 0.25;
    }
    for (int l = 0; l < H->nlevels; ++l) {
        int32_t nl = H->L[l].A.n;
        for (int t = 0; t < 3; ++t) H->work[l][t] = (double *)xcalloc((size_t)nl, sizeof(double));
    }
    return H;
}

void ref_amg_free(ref_hier *H) {
    if (!H) return;
    for (int l = 0; l < REF_MAX_LEVELS; ++l) {
        ref_level *L = &H->L[l];
        free(L->ilu);
        free(L->dpos);
        csr_free(&L->A); csr_free(&L->P); csr_free(&L->R);
        free(L->agg); free(L->state); free(L->M);
        for (int t = 0; t < 3; ++t) free(H->work[l][t]);
    }
    free(H->lu);
    free(H->piv);
    free(H);
}

/* ---- hierarchy introspection for the tests ---- */
int ref_hier_nlevels(const ref_hier *H) { return H->nlevels; }
void ref_hier_level_sizes(const ref_hier *H, int l, int32_t *n, int64_t *nnz, int32_t *nc,
                          int64_t *nnz_p, double *omega_p, int32_t *rounds, int64_t *nnz_s) {
    const ref_level *L = &H->L[l];
    *n = L->A.n; *nnz = L->A.nnz; *nc = L->nc; *nnz_p = L->P.nnz;
    *omega_p = L->omega_p; *rounds = L->mis_rounds; *nnz_s = L->nnz_s;
}
/* ILU(0) factors of level l (A's pattern), when the smoother is SM_ILU0. */
int ref_hier_level_ilu(const ref_hier *H, int l, double *ilu) {
    const ref_level *L = &H->L[l];
    if (!L->ilu) return REF_EINVAL;
    memcpy(ilu, L->ilu, (size_t)L->A.nnz * sizeof(double));
    return REF_OK;
}

void ref_hier_level_copy(const ref_hier *H, int l, int32_t *a_rowptr, int32_t *a_col, double *a_val,
                         int32_t *agg, int32_t *state, double *M, int32_t *p_rowptr, int32_t *p_col,
                         double *p_val) {
    const ref_level *L = &H->L[l];
    memcpy(a_rowptr, L->A.rowptr, ((size_t)L->A.n + 1) * sizeof(int32_t));
    memcpy(a_col, L->A.col, (size_t)L->A.nnz * sizeof(int32_t));
    memcpy(a_val, L->A.val, (size_t)L->A.nnz * sizeof(double));
    int coarsest = (l == H->nlevels - 1);
    if (agg && L->agg) memcpy(agg, L->agg, (size_t)L->A.n * sizeof(int32_t));
    if (state && L->state) memcpy(state, L->state, (size_t)L->A.n * sizeof(int32_t));
    if (M && L->M) memcpy(M, L->M, (size_t)L->A.n * sizeof(double));
    if (!coarsest && p_rowptr) {
        memcpy(p_rowptr, L->P.rowptr, ((size_t)L->P.n + 1) * sizeof(int32_t));
        memcpy(p_col, L->P.col, (size_t)L->P.nnz * sizeof(int32_t));
        memcpy(p_val, L->P.val, (size_t)L->P.nnz * sizeof(double));
    }
}
void ref_hier_coarse_copy(const ref_hier *H, double *lu, int32_t *piv) {
    memcpy(lu, H->lu, (size_t)H->nd * H->nd * sizeof(double));
    memcpy(piv, H->piv, (size_t)H->nd * sizeof(int32_t));
}

/* ------------------------------------------------------------------------ */
/* V-cycle (Introduction: restrict the residual, smooth, recurse down to a   */
/* direct solve on the coarsest level, interpolate and correct, smooth).     */
/* Level l < L:  x = 0;  npre sweeps x <- x + M (b - A x);                    */
/*   b_c = R (b - A x);  x_c = V_{l+1}(b_c);  x <- x + P x_c;  npost sweeps.   */
/* ------------------------------------------------------------------------ */

static void smooth_sweeps(const ref_level *L, const double *b, double *x, double *t, int sweeps) {
    int32_t n = L->A.n;
    for (int s = 0; s < sweeps; ++s) {
        spmv(&L->A, x, t);
        if (L->ilu) {
            /* x <- x + (LU)^{-1} (b - A x) */
            for (int32_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
            ilu_solve(&L->A, L->ilu, L->dpos, t);
            for (int32_t i = 0; i < n; ++i) x[i] = x[i] + t[i];
        } else {
            for (int32_t i = 0; i < n; ++i) x[i] = x[i] + L->M[i] * (b[i] - t[i]);
        }
    }
}

static void vcycle_level(ref_hier *H, int l, const double *b, double *x) {
    ref_level *L = &H->L[l];
    int32_t n = L->A.n;
    if (l == H->nlevels - 1) { dense_lu_solve(H->nd, H->lu, H->piv, b, x); return; }
    double *t = H->work[l][0];
    double *bc = H->work[l + 1][1];
    double *xc = H->work[l + 1][2];
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    smooth_sweeps(L, b, x, t, H->prm.npre);
    spmv(&L->A, x, t);
    for (int32_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    spmv(&L->R, t, bc);
    vcycle_level(H, l + 1, bc, xc);
    spmv(&L->P, xc, t);
    for (int32_t i = 0; i < n; ++i) x[i] = x[i] + t[i];
    smooth_sweeps(L, b, x, t, H->prm.npost);
}

/* z = V(r); identity when the preconditioner is off. */
void ref_vcycle(ref_hier *H, const double *r, double *z) {
    if (H->nlevels == 0) { memcpy(z, r, (size_t)H->L[0].A.n * sizeof(double)); return; }
    vcycle_level(H, 0, r, z);
}

/* ------------------------------------------------------------------------ */
/* Krylov solvers.  x0 = 0.  Stop at the first iteration with                */
/* ||r||_2 <= rtol ||b||_2 (recursive residual); then the true residual b - A x */
/* is formed and, if it is above rtol, the method restarts from x with that  */
/* residual.  b = 0 returns x = 0.                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t iters;
    int32_t status;
    int32_t restarts;
    double rel_res;       /* last recursive residual / ||b|| */
    double rel_res_true;  /* ||b - A x|| / ||b||             */
} ref_info;

#define MAX_RESTARTS 8

static int finite_nz(double v) { return isfinite(v) && v != 0.0; }

/* PCG (flex = 0) or flexible CG with the Polak-Ribiere beta (flex = 1).
 * When dirs is not null, the search directions p_0, p_1, ... of the first
 * cycle (before any restart) are copied into dirs[k*n .. k*n+n-1], at most
 * max_dirs of them, and their count is stored in *ndirs (a test hook: the
 * iteration itself is the same with or without it). */
static int pcg_run(ref_hier *H, const double *b, double *x, double rtol, int32_t maxiter, int flex,
                   ref_info *info, double *dirs, int32_t max_dirs, int32_t *ndirs) {
    const rcsr *A = &H->L[0].A;
    int32_t n = A->n;
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(n, b, b));
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    if (bnorm == 0.0) return REF_OK;
    double *r = (double *)xcalloc((size_t)n, sizeof(double));
    double *z = (double *)xcalloc((size_t)n, sizeof(double));
    double *p = (double *)xcalloc((size_t)n, sizeof(double));
    double *q = (double *)xcalloc((size_t)n, sizeof(double));
    double *rold = (double *)xcalloc((size_t)n, sizeof(double));
    int status = REF_NOT_CONVERGED;
    const double tol = rtol * bnorm;
    for (;;) {
        spmv(A, x, q);
        for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        ref_vcycle(H, r, z);
        for (int32_t i = 0; i < n; ++i) p[i] = z[i];
        if (dirs && info->restarts == 0 && *ndirs < max_dirs)
            memcpy(dirs + (size_t)(*ndirs)++ * (size_t)n, p, (size_t)n * sizeof(double));
        double rz = dot(n, r, z);
        int inner = REF_NOT_CONVERGED;
        while (info->iters < maxiter) {
            spmv(A, p, q);
            double pq = dot(n, p, q);
            if (!finite_nz(pq) || !isfinite(rz)) { inner = REF_BREAKDOWN; break; }
            double alpha = rz / pq;
            for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            if (flex) memcpy(rold, r, (size_t)n * sizeof(double));
            for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            info->iters++;
            double rn = sqrt(dot(n, r, r));
            info->rel_res = rn / bnorm;
            if (!isfinite(rn)) { inner = REF_BREAKDOWN; break; }
            if (rn <= tol) { inner = REF_OK; break; }
            ref_vcycle(H, r, z);
            double beta, rz_new = dot(n, r, z);
            if (flex) {
                double s = 0.0;
                for (int32_t i = 0; i < n; ++i) s = s + z[i] * (r[i] - rold[i]);
                beta = s / rz;
            } else {
                beta = rz_new / rz;
            }
            rz = rz_new;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            if (dirs && info->restarts == 0 && *ndirs < max_dirs)
                memcpy(dirs + (size_t)(*ndirs)++ * (size_t)n, p, (size_t)n * sizeof(double));
        }
        spmv(A, x, q);
        for (int32_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
        info->rel_res_true = sqrt(dot(n, q, q)) / bnorm;
        if (inner == REF_BREAKDOWN) { status = REF_BREAKDOWN; break; }
        if (info->rel_res_true <= rtol) { status = REF_OK; break; }
        if (info->iters >= maxiter || info->restarts >= MAX_RESTARTS) { status = REF_NOT_CONVERGED; break; }
        info->restarts++;
    }
    info->status = status;
    free(r); free(z); free(p); free(q); free(rold);
    return status;
}

int ref_pcg(ref_hier *H, const double *b, double *x, double rtol, int32_t maxiter, int flex,
            ref_info *info) {
    return pcg_run(H, b, x, rtol, maxiter, flex, info, NULL, 0, NULL);
}

/* ref_pcg that also records the search directions (test hook, see pcg_run). */
int ref_pcg_dirs(ref_hier *H, const double *b, double *x, double rtol, int32_t maxiter, int flex,
                 ref_info *info, double *dirs, int32_t max_dirs, int32_t *ndirs) {
    *ndirs = 0;
    return pcg_run(H, b, x, rtol, maxiter, flex, info, dirs, max_dirs, ndirs);
}

/* Right-preconditioned BiCGSTAB (van der Vorst 1992).
 *   r_hat = r0;  rho_prev = alpha = omega = 1;  v = p = 0
 *   loop:  rho = r_hat.r;  beta = (rho/rho_prev)(alpha/omega);  p = r + beta (p - omega v)
 *          p_hat = V(p);  v = A p_hat;  alpha = rho / (r_hat.v);  s = r - alpha v
 *          if ||s|| <= tol:  x += alpha p_hat; stop
 *          s_hat = V(s);  t = A s_hat;  omega = (t.s)/(t.t)
 *          x += alpha p_hat + omega s_hat;  r = s - omega t;  stop if ||r|| <= tol
 * Breakdown when rho, r_hat.v, t.t or omega is zero or not finite. */
int ref_bicgstab(ref_hier *H, const double *b, double *x, double rtol, int32_t maxiter, ref_info *info) {
    const rcsr *A = &H->L[0].A;
    int32_t n = A->n;
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(n, b, b));
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    if (bnorm == 0.0) return REF_OK;
    double *r = (double *)xcalloc((size_t)n, sizeof(double));
    double *rh = (double *)xcalloc((size_t)n, sizeof(double));
    double *p = (double *)xcalloc((size_t)n, sizeof(double));
    double *v = (double *)xcalloc((size_t)n, sizeof(double));
    double *s = (double *)xcalloc((size_t)n, sizeof(double));
    double *t = (double *)xcalloc((size_t)n, sizeof(double));
    double *ph = (double *)xcalloc((size_t)n, sizeof(double));
    double *sh = (double *)xcalloc((size_t)n, sizeof(double));
    const double tol = rtol * bnorm;
    int status = REF_NOT_CONVERGED;
    for (;;) {
        spmv(A, x, t);
        for (int32_t i = 0; i < n; ++i) { r[i] = b[i] - t[i]; rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
        double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
        int inner = REF_NOT_CONVERGED;
        while (info->iters < maxiter) {
            double rho = dot(n, rh, r);
            if (!finite_nz(rho)) { inner = REF_BREAKDOWN; break; }
            double beta = (rho / rho_prev) * (alpha / omega);
            for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            ref_vcycle(H, p, ph);
            spmv(A, ph, v);
            double rv = dot(n, rh, v);
            if (!finite_nz(rv)) { inner = REF_BREAKDOWN; break; }
            alpha = rho / rv;
            for (int32_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            info->iters++;
            double sn = sqrt(dot(n, s, s));
            if (!isfinite(sn)) { inner = REF_BREAKDOWN; break; }
            if (sn <= tol) {
                for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
                info->rel_res = sn / bnorm;
                inner = REF_OK;
                break;
            }
            ref_vcycle(H, s, sh);
            spmv(A, sh, t);
            double tt = dot(n, t, t);
            if (!finite_nz(tt)) { inner = REF_BREAKDOWN; break; }
            omega = dot(n, t, s) / tt;
            if (!finite_nz(omega)) { inner = REF_BREAKDOWN; break; }
            for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i] + omega * sh[i];
            for (int32_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
            double rn = sqrt(dot(n, r, r));
            info->rel_res = rn / bnorm;
            if (!isfinite(rn)) { inner = REF_BREAKDOWN; break; }
            if (rn <= tol) { inner = REF_OK; break; }
            rho_prev = rho;
        }
        spmv(A, x, t);
        for (int32_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
        info->rel_res_true = sqrt(dot(n, t, t)) / bnorm;
        if (inner == REF_BREAKDOWN) { status = REF_BREAKDOWN; break; }
        if (info->rel_res_true <= rtol) { status = REF_OK; break; }
        if (info->iters >= maxiter || info->restarts >= MAX_RESTARTS) { status = REF_NOT_CONVERGED; break; }
        info->restarts++;
    }
    info->status = status;
    free(r); free(rh); free(p); free(v); free(s); free(t); free(ph); free(sh);
    return status;
}

/* y = A x with the hierarchy's level-0 matrix (test helper). */
void ref_spmv(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, const double *x,
              double *y) {
    rcsr A = {n, n, rowptr[n], (int32_t *)rowptr, (int32_t *)col, (double *)val};
    spmv(&A, x, y);
}

/* MIS-2 priority keys of UNDECIDED nodes at `level` (test helper). */
void ref_mis2_keys(int32_t n, uint64_t seed, int32_t level, uint64_t *keys) {
    uint32_t salt = level_salt(seed, level);
    for (int32_t i = 0; i < n; ++i) keys[i] = mis_key(ST_UNDECIDED, salt, i);
}
