/*
 * gwamg.h -- C ABI of the MI355X (gfx950) groundwater AMG-Krylov library.
 *
 * Method: Sbai & Larabi, "On Solving Groundwater Flow and Transport Models
 * with Algebraic Multigrid Preconditioning".  A steady confined flow solve
 * (finite-difference 7-point M-matrix, CG preconditioned by smoothed-
 * aggregation AMG), then the steady forward travel-time equation on the
 * resulting Darcy velocities (Eq. 1, BiCGSTAB preconditioned by AMG), whose
 * matrix serves several right-hand sides of the dual delineation.
 *
 * Conventions for every entry point
 *   - Pointers marked [device] are HIP device pointers on the current device;
 *     [host] pointers are ordinary host memory.  The caller owns every buffer
 *     it passes and keeps it alive until the call returns (queue requests:
 *     until queue_poll reports the ticket finished).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work of the call is ordered on it.  Calls that must read back sizes or
 *     convergence flags block until their work is done; the others only
 *     enqueue.
 *   - Cell (i,j,k) of an nx x ny x nz grid has flat index i + nx*(j + ny*k).
 *   - Every function returns a status (GW_OK = 0) and never throws; on error
 *     gw_last_error() returns a thread-local message.
 *   - Calls on one amg_hierarchy must not overlap (hierarchies hold their
 *     solve workspace).  The queue functions are thread safe.
 */
#ifndef GWAMG_H
#define GWAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GW_OK 0
#define GW_NOT_CONVERGED 1 /* x holds the last iterate, info is filled      */
#define GW_BREAKDOWN 2     /* a Krylov scalar became zero or non-finite      */
#define GW_PENDING 3       /* queue_poll: the request is not finished yet    */
#define GW_EINVAL (-1)     /* bad size, null pointer, K <= 0 or NaN, unsorted
                              or non-square CSR, missing/non-positive diagonal */
#define GW_ENOMEM (-2)     /* device allocation failed / request > budget    */
#define GW_SINGULAR (-3)   /* zero pivot in the coarsest-level LU            */
#define GW_EDEVICE (-4)    /* HIP runtime error                              */
#define GW_EAGAIN (-5)     /* queue full                                     */

enum { GW_SMOOTHER_JACOBI = 0, GW_SMOOTHER_SPAI0 = 1, GW_SMOOTHER_NONE = 2, GW_SMOOTHER_ILU0 = 3 };
enum { GW_PRECISION_FP64 = 0, GW_PRECISION_MIXED = 1 };
enum { GW_COARSEN_SA = 0, GW_COARSEN_RS = 1 };

/* ---- plain data --------------------------------------------------------- */

/* Uniform grid; nz = 1 is a 2D slab of thickness dz. */
typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } gw_grid;

/* Square CSR matrix, sorted unique columns, diagonal stored. [device] */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *rowptr; /* n+1 */
    const int32_t *col;    /* nnz */
    const double *val;     /* nnz */
} gw_csr;

/* Point sink in cell (ix,iy,iz): q > 0 pumps q m^3/s out of the aquifer. */
typedef struct { int32_t ix, iy, iz; double q; } gw_well;

/* Fixed heads on the x = 0 and x = L faces; every other face is no-flow. */
typedef struct { double h_west, h_east; } gw_bc;

/* Source window [j0,j1) x [k0,k1) on the x = 0 face: its inflow indicator is
 * the second travel-time right-hand side. */
typedef struct { int32_t j0, j1, k0, k1; } gw_zone;

/* AMG parameters.
 *   eps_strong  strength threshold eps_0 (halved every level under SA) [0.08]
 *   smoother    GW_SMOOTHER_*; NONE disables the preconditioner; ILU0 [SPAI0]
 *               is the paper's relaxation (incomplete LU on each level's
 *               pattern, applied by level-scheduled substitutions: a
 *               baseline, FP64 only, pair solves run one system at a time)
 *   omega       damping of the Jacobi smoother                       [2/3]
 *   npre/npost  smoothing sweeps before/after the coarse correction  [2/2]
 *   n_coarse    a level of at most this many rows is the coarsest    [500]
 *   max_levels  level cap                                            [20]
 *   precision   FP64, or MIXED = FP32 hierarchy inside FP64 Krylov   [FP64]
 *   seed        seed of the MIS-2 hash priorities (of the PMIS weights
 *               under RS)
 *   coarsening  GW_COARSEN_SA: smoothed aggregation on MIS-2 aggregates [SA]
 *               (Figs. 1 and 3, CG/AMG/SA); GW_COARSEN_RS: classical
 *               Ruge-Stueben (the figures' other AMG, CG/AMG/RS, kept as
 *               a baseline): strong set S_i = { j : -a_ij >= eps_strong
 *               max_k -a_ik } with eps_strong kept on every level, a PMIS
 *               C/F splitting (weight: number of dependents plus a 24-bit
 *               hash fraction, ties by index; a point with no dependents
 *               is F) and direct interpolation from the strong C neighbours
 *               (positive off-diagonals lumped into the diagonal); the
 *               level's aggregate array then holds each C point's coarse
 *               index and -1 for F points, and omega_P is 0 */
typedef struct {
    double eps_strong;
    int32_t smoother;
    double omega;
    int32_t npre, npost;
    int32_t n_coarse, max_levels;
    int32_t precision;
    uint64_t seed;
    int32_t coarsening;
} amg_params;

/* rtol: stop when ||r||_2 <= rtol ||b||_2.  check_every: iterations between
 * two reads of the device convergence flag.  flexible: for amg_solve_pcg,
 * 1 = flexible CG (Polak-Ribiere beta), 0 = standard PCG, -1 = flexible
 * exactly when the hierarchy is MIXED.  graph: 1 = the check_every
 * iterations between two flag reads are captured once as a HIP graph (kept
 * with the hierarchy, freed by amg_free) and replayed with one launch;
 * 0 or -1 (default) = kernels are launched one by one, which measured
 * slightly faster on a 1M-cell pass (capture included; the kernels are not
 * small enough for the graph's dispatch savings to pay).  Both modes run the
 * same kernels in the same order: results are identical.  Launches inside a
 * graph are not event-timed by gw_prof_enable. */
typedef struct {
    double rtol;
    int32_t maxiter;
    int32_t check_every;
    int32_t flexible;
    int32_t graph;
} amg_solve_params;

typedef struct {
    int32_t iters;        /* Krylov iterations over all restarts          */
    int32_t status;       /* GW_OK, GW_NOT_CONVERGED or GW_BREAKDOWN       */
    int32_t restarts;     /* restarts after a true-residual check failed   */
    double rel_res;       /* recursive residual / ||b|| at exit            */
    double rel_res_true;  /* ||b - A x|| / ||b|| in FP64 at exit           */
    double setup_ms;      /* hierarchy setup time (tt_solve, queue)        */
    double solve_ms;      /* wall time of this solve                       */
} amg_solve_info;

typedef struct {
    int32_t n;            /* rows of A_l                                   */
    int64_t nnz;          /* nonzeros of A_l                               */
    int32_t nc;           /* aggregates (rows of A_{l+1}), 0 on coarsest   */
    int64_t nnz_p;        /* nonzeros of P_l                               */
    int64_t nnz_s;        /* edges of the strength graph                   */
    int32_t mis_rounds;   /* MIS-2 rounds                                  */
    double omega_p;       /* prolongator smoothing weight                  */
    size_t bytes;         /* device bytes held for this level              */
    int32_t slice_rows;   /* rows per slice of the sliced copy the solve
                             kernels read (64, 32, 16 or 8), 0: none       */
    int64_t nnz_sliced;   /* entries the sliced copy stores, padding
                             included (each slice as wide as its longest
                             row)                                          */
    int32_t stencil_offsets; /* positive column offsets of the stencil
                             copy the solve kernels read instead of the
                             sliced copy (1-3: 3-, 5- and 7-point
                             operators), symmetric (values equal to their
                             mirrors bit for bit) or one-sided (upwind: one
                             negative value per face), 0: none            */
} amg_level_info;

typedef struct amg_hierarchy amg_hierarchy;
typedef struct gw_queue gw_queue;

/* ---- library ------------------------------------------------------------ */

const char *gw_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char *gw_last_error(void);
/* Release cached device memory held by the library's pool. */
int gw_trim(void);

/* ---- flow assembly (Benchmarking Examples: 7-point finite differences
 *      giving an M-matrix) -------------------------------------------------- */

/* Number of nonzeros of the flow matrix of `grid`:
 * 7n - 2(nx ny + ny nz + nx nz). */
int64_t fv_nnz(const gw_grid *grid);

/* Assemble A h = b.  Face transmissibility T = (A_f/d) 2 K_a K_b/(K_a+K_b);
 * fixed-head faces add T_b = (A_f/d) 2 K to the diagonal and T_b h to b;
 * wells subtract q from b.  K [device] n; wells [host] nwells (<= 64);
 * rowptr [device] n+1, col/val [device] fv_nnz(grid), b [device] n.
 * EINVAL for a K that is not positive and finite. */
int fv_assemble(const gw_grid *grid, const double *K, const gw_bc *bc, const gw_well *wells,
                int32_t nwells, int32_t *rowptr, int32_t *col, double *val, double *b, void *stream);

/* Darcy face fluxes, positive along +x/+y/+z (the velocity of Eq. 1 times
 * the face area).  qx [device] (nx+1) ny nz, face i of row (j,k) at
 * i + (nx+1)(j + ny k); qy [device] nx (ny+1) nz; qz [device] nx ny (nz+1).
 * Faces on no-flow boundaries are 0. */
int darcy_flux(const gw_grid *grid, const double *K, const gw_bc *bc, const double *h,
               double *qx, double *qy, double *qz, void *stream);

/* ---- AMG (Introduction: setup phase, then V-cycle of sparse products with
 *      a direct solve on the coarsest level) ------------------------------- */

/* Build the hierarchy of A [device].  The hierarchy copies what it needs; A
 * may be freed when the call returns.  Blocks for the level sizes.
 * EINVAL: invalid CSR, or coarsening stalled above 2048 rows;
 * SINGULAR: zero pivot in the coarsest LU. */
int amg_setup(const gw_csr *A, const amg_params *params, amg_hierarchy **H, void *stream);

/* Apply one V-cycle z = V(r) (the preconditioner).  r, z [device] n. */
int amg_vcycle(amg_hierarchy *H, const double *r, double *z, void *stream);

/* y = A x with the level-0 operator of H.  x, y [device] n. */
int amg_spmv(amg_hierarchy *H, const double *x, double *y, void *stream);

/* AMG-preconditioned CG (flow, symmetric), x0 = 0.  b, x [device] n. */
int amg_solve_pcg(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp,
                  amg_solve_info *info, void *stream);

/* amg_solve_pcg for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, the same kernels and results bit for bit, but the Krylov
 * workspace (six n-vectors, block partials, the scalar record) is a
 * statically sized array of device memory (6 x 8 x GW_NOALLOC_MAX_ROWS
 * bytes + 64 KiB, ~48 MiB) that the HIP runtime places on a device with
 * the code object holding it, at this entry point's first call there, and
 * keeps until the process ends; the scalars travel through a host variable
 * instead of a pinned stage.  The call allocates nothing: no hipMalloc,
 * hipFree, pinned or pool allocation, no graph.  H
 * must come from amg_setup (which allocated the hierarchy); b, x [device] n,
 * caller-owned.  EINVAL when n > GW_NOALLOC_MAX_ROWS, when sp->graph > 0
 * (graph objects are allocations) or while kernel timing is on
 * (gw_prof_enable creates events).  Every call on one device shares that
 * device's array, and each call initialises everything it reads there:
 * calls that overlap on one device (other host threads, other streams) race
 * on it and must be serialised by the caller. */
#define GW_NOALLOC_MAX_ROWS 1048576
int amg_solve_pcg_noalloc(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp,
                          amg_solve_info *info, void *stream);

/* AMG right-preconditioned BiCGSTAB (nonsymmetric), x0 = 0. */
int amg_solve_bicgstab(amg_hierarchy *H, const double *b, double *x, const amg_solve_params *sp,
                       amg_solve_info *info, void *stream);

/* Two systems with the same matrix, A x0 = b0 and A x1 = b1 (the travel time
 * and the source-zone fraction share the upwind matrix: Benchmarking
 * Examples, Eq. 1, and the Results' travel-time runs), solved by BiCGSTAB in
 * lockstep: each product reads the matrix and the hierarchy once for both,
 * each system keeps its own scalars, stopping test and restarts, and gets
 * exactly the iterates amg_solve_bicgstab gives it alone.  b0, b1, x0, x1
 * [device] n each; x0 and x1 must not overlap.  info [host] 2 entries
 * (solve_ms is the wall time of the pair in both).
 * Returns GW_BREAKDOWN if either system broke down, else GW_NOT_CONVERGED if
 * either did not converge, else GW_OK. */
int amg_solve_bicgstab_pair(amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1,
                            const amg_solve_params *sp, amg_solve_info info[2], void *stream);

/* Shared launches for many solves (the Discussion's setups kept for many
 * solves; the serving loop's batches): nsys independent systems, each with
 * its own hierarchy H[j] (all distinct, from amg_setup, with the same
 * precision and the same pre- and post-sweep counts, both >= 1, and a
 * diagonal smoother), solved together so that every kernel step is one
 * launch for all of them per operator type instead of one per system.  Each
 * launch runs every system's kernel on the grid it would have alone, so each
 * system gets exactly the iterates, iteration count, stopping decision and
 * restarts of amg_solve_pcg / amg_solve_bicgstab_pair on its own (bit for
 * bit); a system that has converged skips the remaining launches.  H, b, x,
 * b0, b1, x0, x1 [host] arrays of nsys pointers; the vectors they point to
 * [device] n_j each.  info [host] nsys entries (the pair: 2 nsys, systems
 * 2j and 2j+1 of hierarchy j); solve_ms is the batch's wall time.  graph = 1
 * replays each block of check_every iterations of the whole batch as one
 * captured HIP graph.  nsys in [1, 256].  Returns the worst status
 * (BREAKDOWN, then NOT_CONVERGED); EINVAL for mismatched hierarchies. */
int amg_solve_pcg_batch(amg_hierarchy *const *H, const double *const *b, double *const *x, int32_t nsys,
                        const amg_solve_params *sp, amg_solve_info *info, void *stream);
int amg_solve_bicgstab_pair_batch(amg_hierarchy *const *H, const double *const *b0, const double *const *b1,
                                  double *const *x0, double *const *x1, int32_t nsys, const amg_solve_params *sp,
                                  amg_solve_info *info, void *stream);

/* Per-level statistics; `out` [host] holds max_levels entries. */
int amg_hierarchy_info(const amg_hierarchy *H, amg_level_info *out, int32_t max_levels,
                       int32_t *nlevels, size_t *bytes);

/* Copy level l into caller buffers [device] sized from amg_hierarchy_info:
 * A_l (rowptr n+1, col/val nnz), the aggregate map agg (n, -1 = removed),
 * the smoother diagonal M (n), and P_l (rowptr n+1, col/val nnz_p).  Any
 * pointer may be NULL.  On the coarsest level agg, M and P are not written. */
int amg_level_export(const amg_hierarchy *H, int32_t level, int32_t *a_rowptr, int32_t *a_col,
                     double *a_val, int32_t *agg, double *M, int32_t *p_rowptr, int32_t *p_col,
                     double *p_val, void *stream);

/* Coarsest level: LU factors (row-major nd x nd, unit lower L below the
 * diagonal), pivot rows (LAPACK getrf order) and the inverse used by the
 * V-cycle (row-major nd x nd).  [device]; any may be NULL. */
int amg_coarse_export(const amg_hierarchy *H, double *lu, int32_t *piv, double *inv, void *stream);

/* ILU(0) factors of level l (smoother GW_SMOOTHER_ILU0), on A_l's pattern:
 * L below the diagonal (unit diagonal implied), U on and above it.
 * lu [device] nnz of A_l.  EINVAL for a level without them. */
int amg_ilu_export(const amg_hierarchy *H, int32_t level, double *lu, void *stream);

void amg_free(amg_hierarchy *H);

/* ---- transient flow (Eq. 2) -------------------------------------------- */

/* PCG on (A + diag(shift)) x = b, preconditioned by the V-cycle of H built
 * for A: the setup of the conductance matrix kept for the fully implicit
 * time steps of Eq. 2, whose matrix adds S_i V_i / dt to the diagonal.  The
 * Discussion after Eq. 2 keeps it while S_i V_i / dt < delta C_ii for all i.
 * shift, b, x [device] n.  Launched one kernel at a time (graph ignored). */
int amg_solve_pcg_shifted(amg_hierarchy *H, const double *shift, const double *b, double *x,
                          const amg_solve_params *sp, amg_solve_info *info, void *stream);

typedef struct {
    int32_t status;       /* of the step's solve                          */
    int32_t iters;
    int32_t reused;       /* 1: setup of C (built once, at the first step
                             that meets the criterion); 2: setup of C + S/dt
                             of an earlier step with the same dt; 0: built
                             for this step                                 */
    double ratio;         /* max_i S_i V_i / (dt C_ii)                     */
    double rel_res_true;
    double setup_ms;      /* setup done in this step (C's at its first use) */
    double solve_ms;
} gw_step_info;

/* Fully implicit steps of Eq. 2 from h0: (C + S/dt_k) h^{k+1} =
 * b + (S/dt_k) h^k, with C and b assembled as fv_assemble does (fixed-head
 * faces and wells held constant) and S_i = Ss_i V_i.  The hierarchy of C
 * serves every step with max_i S_i V_i / (dt_k C_ii) < delta (shifted PCG);
 * other steps build a hierarchy of C + S/dt_k, kept while dt does not
 * change.  K, Ss, h0 [device] n; dt [host] nsteps; h [device] n receives
 * the last heads; h_steps [device] nsteps x n or NULL receives every step;
 * info [host] nsteps or NULL.  Returns the worst step status (stops at a
 * breakdown). */
int flow_transient(const gw_grid *grid, const double *K, const gw_bc *bc, const gw_well *wells, int32_t nwells,
                   const double *Ss, const double *h0, const double *dt, int32_t nsteps, double delta,
                   const amg_params *params, const amg_solve_params *sp, double *h, double *h_steps,
                   gw_step_info *info, void *stream);

/* ---- travel time (Eq. 1) ------------------------------------------------ */

/* Upper bound of the travel-time matrix nonzeros (= fv_nnz). */
int64_t tt_nnz_bound(const gw_grid *grid);

/* Assemble the first-order upwind matrix of v.grad(tau) = phi:
 * A_ii = sum of |q| over the inflow faces of cell i, A_ij = -|q| for each
 * interior inflow face from neighbour j; b_tau = phi V_i; b_c = |q| on the
 * x = 0 inflow face of cells inside `zone` (NULL = whole face).  Rows with no
 * inflow become identity rows with zero right-hand sides.  rowptr/col/val
 * [device] sized n+1 / tt_nnz_bound; b_tau, b_c [device] n.  Returns the
 * actual nnz and the number of identity rows [host]. */
int tt_assemble(const gw_grid *grid, const double *qx, const double *qy, const double *qz,
                double phi, const gw_zone *zone, int32_t *rowptr, int32_t *col, double *val,
                double *b_tau, double *b_c, int64_t *nnz, int64_t *n_identity, void *stream);

/* Assemble, build one AMG hierarchy, and solve both right-hand sides with
 * BiCGSTAB on it (the dual-delineation matrix is shared by its equations).
 * tau, c [device] n; info [host] 2 entries (setup_ms is filled in both). */
int tt_solve(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
             const gw_zone *zone, const amg_params *params, const amg_solve_params *sp, double *tau,
             double *c, amg_solve_info info[2], void *stream);

/* Exact direct solve of an upwind system (Eq. 1 discretised as tt_assemble
 * does, or the reversed-flow system of the backward travel time).  Each
 * off-diagonal entry (i, j) of such a matrix couples cell i to an inflow
 * neighbour j, and water enters a cell only from cells of higher head, so
 * the matrix is triangular in the order of decreasing head; the paper's
 * Results prefer a direct method for the transport systems, and this one
 * costs a single pass.  Cells are solved level by level in a topological
 * order of the inflow graph (a cell as soon as all its inflow neighbours
 * are), each as forward substitution does it: x_i = (b_i - sum_j a_ij x_j) /
 * a_ii with the off-diagonal terms subtracted in the row's column order.
 * A [device] square CSR with ascending columns and a positive diagonal;
 * b, x [device] nrhs blocks of n values each (system k in [k n, (k+1) n)),
 * 1 <= nrhs <= 64; n_levels [host] or NULL receives the number of levels.
 * EINVAL for a malformed matrix; BREAKDOWN when the inflow graph has a cycle
 * (then only the cells upstream of no cycle are written). */
int tt_sweep(const gw_csr *A, int32_t nrhs, const double *b, double *x, int32_t *n_levels, void *stream);

/* tt_assemble followed by tt_sweep on both right-hand sides: the direct
 * counterpart of tt_solve.  tau, c [device] n; n_levels as in tt_sweep. */
int tt_solve_direct(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
                    const gw_zone *zone, double *tau, double *c, int32_t *n_levels, void *stream);

/* The full dual delineation (Introduction: N_i + N_p + 2 steady advection
 * equations; Eq. 1 and its reversed-flow form), each field exact by the
 * sweep.  Forward, on q: the travel time tau_f, then one indicator per
 * source, i.e. each zone of the x = 0 face (right-hand side: the inflow
 * through that face) and each injection well (q < 0).  Backward, on -q: the
 * travel time tau_b to an outlet, then the capture indicator of each
 * production well (q > 0).  A well bounds the system in which water crosses
 * it inwards: it adds |q| to its cell's diagonal (a cell without face inflow
 * becoming a regular row with b_tau = phi V) and gives its indicator the
 * right-hand side |q| at that cell; wells are applied in list order.
 * zones [host] nzones; wells [host] nwells <= 64; out [device]
 * (2 + nzones + n_injection + n_production) blocks of n values, in the order
 * above (forward blocks first); n_levels [host] 2 entries or NULL.  At most
 * 64 fields per direction.  BREAKDOWN if a system is not an upwind one. */
int tt_delineate(const gw_grid *grid, const double *qx, const double *qy, const double *qz, double phi,
                 const gw_zone *zones, int32_t nzones, const gw_well *wells, int32_t nwells, double *out,
                 int32_t n_levels[2], void *stream);

/* ---- kernel timing (HIP events around launches, for roofline reports) --- */

typedef struct {
    char name[32];
    int64_t launches;
    double ms;            /* summed event time                            */
    double bytes;         /* summed algorithmic HBM bytes, operators in the
                             format the kernel reads (sliced copy or CSR)  */
    double bytes_csr;     /* the same with every operator pass counted as a
                             CSR pass: nnz (value + 4-byte column)
                             + 4 (n + 1)                                   */
} gw_kernel_stat;

/* on = 1 starts recording (and clears the table), 0 stops. */
int gw_prof_enable(int32_t on);
/* Record only the kernel class `name` (a name gw_prof_read reports), so the
 * event pairs cost nothing elsewhere; NULL or "" records every class. */
int gw_prof_select(const char *name);
/* Copy up to max entries [host]; *n receives the number of kernels. */
int gw_prof_read(gw_kernel_stat *out, int32_t max, int32_t *n);

/* ---- serving: continuous batching of flow + travel-time requests -------- */

typedef struct {
    gw_grid grid;
    const double *K;         /* [host] n, read during the request        */
    gw_bc bc;
    const gw_well *wells;    /* [host] nwells                            */
    int32_t nwells;
    double phi;
    gw_zone zone;
    amg_params flow_params;
    amg_params tt_params;
    amg_solve_params solve;
    double *h_out;           /* [host] n or NULL                          */
    double *tau_out;         /* [host] n or NULL                          */
    double *c_out;           /* [host] n or NULL                          */
    double t_arrival;        /* seconds on the queue clock; < 0 = now     */
} gw_request;

typedef struct {
    int32_t status;
    amg_solve_info flow;
    amg_solve_info tt[2];
    double t_arrival, t_start, t_done; /* seconds on the queue clock      */
    size_t bytes_reserved;             /* admission footprint             */
    char error[160];                   /* message when status < 0         */
    int32_t setup_reused;              /* 1: flow hierarchy from the cache */
    size_t bytes_used;                 /* device bytes the request held at its
                                          larger phase (flow: K, CSR, vectors,
                                          hierarchy; travel time: K, h, fluxes,
                                          CSR, vectors, hierarchy); setup
                                          temporaries not included         */
} gw_result;

/* hbm_budget_bytes: device memory the queue may reserve for requests in
 * flight; max_slots: requests that may run at once. */
int queue_create(size_t hbm_budget_bytes, int32_t max_slots, gw_queue **q);
/* Seconds since the queue was created (the clock of t_arrival). */
double queue_clock(const gw_queue *q);
/* Enqueue; EAGAIN when 4096 requests wait; ENOMEM when the request alone
 * exceeds the budget.  The request is copied; its buffers are not. */
int queue_submit(gw_queue *q, const gw_request *req, uint64_t *ticket);
/* GW_PENDING while queued or running; otherwise the final status, with
 * `res` filled; a finished ticket is forgotten after it is returned. */
int queue_poll(gw_queue *q, uint64_t ticket, gw_result *res);
/* Block until every submitted request is finished. */
int queue_drain(gw_queue *q);

/* Keep up to max_entries flow hierarchies after their requests (0, the
 * default, frees each one at the end of its request).  A request whose
 * conductance field, grid, boundary heads and flow AMG parameters equal a
 * cached one's takes that hierarchy instead of a new setup: wells change
 * only the right-hand side, so the matrix, and the hierarchy built from it,
 * are the same (the Discussion's setup caching, applied across requests such
 * as a sensitivity analysis on well rates).  The match compares two 64-bit
 * hashes of those inputs.  A cached hierarchy serves one request at a time;
 * cached bytes count against the HBM budget and the least recently used
 * idle entry is freed when a waiting request does not fit. */
int queue_set_setup_cache(gw_queue *q, int32_t max_entries);
/* Shared launches for the solves of the running requests (off by default:
 * max_batch = 1; with max_batch > 1, window_us = 0 and one solver stream
 * are the defaults of the other two arguments): a request's flow solve
 * and its travel-time pair go to the queue's solver thread, whose engines
 * (one for flow CG, one for travel-time pairs) run the iterations of every
 * solve they hold -- up to max_batch, with the same precision, sweeps and
 * stopping parameters -- in shared launches (one launch per kernel step for
 * all of them, as amg_solve_pcg_batch / amg_solve_bicgstab_pair_batch); a
 * solve joins at the next block of iterations and leaves as soon as it is
 * final, and its result is bit for bit the one of a solve of its own.  With
 * window_us > 0 an idle solver waits up to that long for the solves of the
 * other running requests before its first block (it starts as soon as every
 * running request has one waiting).  streams: solver threads, each with its
 * own stream and engines (raised, never lowered, by a call).  max_batch = 1:
 * each request solves on its own slot stream, which measured faster on one
 * MI355X (the slots' small kernels already overlap on its four hardware
 * queues; a shared launch adds two dependent loads to every kernel and
 * serializes the systems' steps on one stream).  EINVAL for max_batch outside
 * [1, 256], window_us outside [0, 1e7] or streams outside [1, 16]. */
int queue_set_batch(gw_queue *q, int32_t max_batch, double window_us, int32_t streams);
/* Blocks of iterations the solver threads ran for two or more solves at
 * once, and the solves they have taken, since the queue was created. */
int queue_stats(const gw_queue *q, uint64_t *shared_blocks, uint64_t *solves);
void queue_destroy(gw_queue *q);

#ifdef __cplusplus
}
#endif

#endif /* GWAMG_H */
