"""CPU oracle for the groundwater AMG-Krylov path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never touches it:
the HIP path and the oracle share no code, headers or helpers.

The arithmetic lives in ``gwref.c`` (plain loops, FP64, compiled with
``-ffp-contract=off``); this module marshals numpy arrays through ctypes, and
adds the well terms and indicator right-hand sides of the dual delineation
(a handful of additions, in plain numpy, at the end of this file).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gwref.c")
_LIB = os.path.join(_HERE, "libgwref.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
EINVAL, SINGULAR = -1, -3
JACOBI, SPAI0, NONE, ILU0 = 0, 1, 2, 3
SA, RS = 0, 1
CF_UND, CF_C, CF_F = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no fused multiply-add)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Params(C.Structure):
    _fields_ = [("eps_strong", C.c_double), ("smoother", C.c_int32), ("omega", C.c_double),
                ("npre", C.c_int32), ("npost", C.c_int32), ("n_coarse", C.c_int32),
                ("max_levels", C.c_int32), ("seed", C.c_uint64), ("coarsening", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("restarts", C.c_int32),
                ("rel_res", C.c_double), ("rel_res_true", C.c_double)]


_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def _declare(L):
    L.ref_fv_nnz.restype = C.c_int64
    L.ref_fv_nnz.argtypes = [C.c_int32] * 3
    L.ref_fv_assemble.restype = C.c_int
    L.ref_fv_assemble.argtypes = [C.c_int32] * 3 + [C.c_double] * 3 + [_f64p, C.c_double, C.c_double,
                                  C.c_void_p, C.c_void_p, C.c_int32, _i32p, _i32p, _f64p, _f64p]
    L.ref_darcy_flux.restype = None
    L.ref_darcy_flux.argtypes = [C.c_int32] * 3 + [C.c_double] * 3 + [_f64p, C.c_double, C.c_double,
                                 _f64p, _f64p, _f64p, _f64p]
    L.ref_tt_nnz.restype = C.c_int64
    L.ref_tt_nnz.argtypes = [C.c_int32] * 3 + [_f64p] * 3
    L.ref_tt_assemble.restype = C.c_int64
    L.ref_tt_assemble.argtypes = [C.c_int32] * 3 + [C.c_double] * 3 + [_f64p] * 3 + [C.c_double,
                                  _i32p, _i32p, _i32p, _f64p, _f64p, _f64p]
    L.ref_tt_sweep.restype = None
    L.ref_tt_sweep.argtypes = [C.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
    L.ref_csr_check.restype = C.c_int
    L.ref_csr_check.argtypes = [C.c_int32, _i32p, _i32p, _f64p]
    L.ref_amg_setup.restype = C.c_void_p
    L.ref_amg_setup.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.POINTER(_Params), C.POINTER(C.c_int)]
    L.ref_amg_free.restype = None
    L.ref_amg_free.argtypes = [C.c_void_p]
    L.ref_hier_nlevels.restype = C.c_int
    L.ref_hier_nlevels.argtypes = [C.c_void_p]
    L.ref_hier_level_sizes.restype = None
    L.ref_hier_level_sizes.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    L.ref_hier_level_ilu.restype = C.c_int
    L.ref_hier_level_ilu.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    L.ref_hier_level_copy.restype = None
    L.ref_hier_level_copy.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 9
    L.ref_hier_coarse_copy.restype = None
    L.ref_hier_coarse_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.ref_vcycle.restype = None
    L.ref_vcycle.argtypes = [C.c_void_p, _f64p, _f64p]
    L.ref_pcg.restype = C.c_int
    L.ref_pcg.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int32, C.c_int, C.POINTER(_Info)]
    L.ref_pcg_dirs.restype = C.c_int
    L.ref_pcg_dirs.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int32, C.c_int, C.POINTER(_Info),
                               C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    L.ref_bicgstab.restype = C.c_int
    L.ref_bicgstab.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int32, C.POINTER(_Info)]
    L.ref_mis2_keys.restype = None
    L.ref_mis2_keys.argtypes = [C.c_int32, C.c_uint64, C.c_int32, C.c_void_p]
    L.ref_spmv.restype = None
    L.ref_spmv.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclasses.dataclass
class Csr:
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    ncols: int = -1

    @property
    def n(self) -> int:
        return len(self.rowptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        nc = self.n if self.ncols < 0 else self.ncols
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, nc))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


@dataclasses.dataclass
class AmgParams:
    """Smoothed-aggregation parameters (their meaning is given in gwref.c)."""
    eps_strong: float = 0.08
    smoother: int = SPAI0
    omega: float = 2.0 / 3.0
    npre: int = 2
    npost: int = 2
    n_coarse: int = 500
    max_levels: int = 20
    seed: int = 0x5EED
    coarsening: int = 0  # SA, or RS (Ruge-Stueben: eps_strong is then its theta)

    def _c(self) -> _Params:
        return _Params(self.eps_strong, self.smoother, self.omega, self.npre, self.npost,
                       self.n_coarse, self.max_levels, self.seed, self.coarsening)


@dataclasses.dataclass
class SolveInfo:
    iters: int
    status: int
    restarts: int
    rel_res: float
    rel_res_true: float


# --------------------------------------------------------------------------
# flow assembly and Darcy flux
# --------------------------------------------------------------------------

def fv_nnz(nx: int, ny: int, nz: int) -> int:
    return int(_L().ref_fv_nnz(nx, ny, nz))


def _wells(wells) -> Tuple[Optional[np.ndarray], Optional[np.ndarray], int]:
    if not wells:
        return None, None, 0
    ijk = np.array([[w.ix, w.iy, w.iz] for w in wells], dtype=np.int32).reshape(-1)
    q = np.array([w.q for w in wells], dtype=np.float64)
    return ijk, q, len(wells)


def fv_assemble(problem) -> Tuple[Csr, np.ndarray]:
    g = problem.grid
    n = g.n
    nnz = fv_nnz(g.nx, g.ny, g.nz)
    rowptr = np.zeros(n + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    b = np.zeros(n, np.float64)
    ijk, q, nw = _wells(problem.wells)
    K = np.ascontiguousarray(problem.K, dtype=np.float64)
    rc = _L().ref_fv_assemble(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, K, problem.h_west, problem.h_east,
                              _p(ijk) if nw else None, _p(q) if nw else None, nw, rowptr, col, val, b)
    if rc != OK:
        raise ValueError(f"fv_assemble: invalid input (status {rc})")
    return Csr(rowptr, col, val), b


def darcy_flux(problem, h: np.ndarray):
    g = problem.grid
    qx = np.zeros((g.nx + 1) * g.ny * g.nz)
    qy = np.zeros(g.nx * (g.ny + 1) * g.nz)
    qz = np.zeros(g.nx * g.ny * (g.nz + 1))
    _L().ref_darcy_flux(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, np.ascontiguousarray(problem.K),
                        problem.h_west, problem.h_east, np.ascontiguousarray(h, dtype=np.float64),
                        qx, qy, qz)
    return qx, qy, qz


# --------------------------------------------------------------------------
# travel time (Eq. 1)
# --------------------------------------------------------------------------

def full_zone(grid) -> Tuple[int, int, int, int]:
    return (0, grid.ny, 0, grid.nz)


def tt_assemble(grid, qx, qy, qz, phi: float, zone: Optional[Sequence[int]] = None):
    """Upwind travel-time matrix and its two right-hand sides.

    ``zone`` = (j0, j1, k0, k1) is the source window on the x = 0 face whose
    inflow indicator is the second right-hand side (default: the whole face).
    """
    z = np.array(full_zone(grid) if zone is None else zone, dtype=np.int32)
    L = _L()
    nnz = int(L.ref_tt_nnz(grid.nx, grid.ny, grid.nz, qx, qy, qz))
    n = grid.n
    rowptr = np.zeros(n + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    bt = np.zeros(n)
    bc = np.zeros(n)
    n_ident = L.ref_tt_assemble(grid.nx, grid.ny, grid.nz, grid.dx, grid.dy, grid.dz, qx, qy, qz,
                                float(phi), z, rowptr, col, val, bt, bc)
    return Csr(rowptr, col, val), bt, bc, int(n_ident)


def tt_sweep(A: Csr, b: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Exact solve of the upwind system by one sweep in descending-head order."""
    x = np.zeros(A.n)
    _L().ref_tt_sweep(A.n, A.rowptr, A.col, A.val, np.ascontiguousarray(b, dtype=np.float64),
                      np.ascontiguousarray(h, dtype=np.float64), x)
    return x


# --------------------------------------------------------------------------
# AMG hierarchy, V-cycle and Krylov solvers
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Level:
    A: Csr
    agg: Optional[np.ndarray]
    state: Optional[np.ndarray]
    M: Optional[np.ndarray]
    P: Optional[Csr]
    nc: int
    omega_p: float
    mis_rounds: int
    nnz_s: int


class Hierarchy:
    def __init__(self, A: Csr, params: AmgParams = AmgParams()):
        self.A = A
        self.params = params
        st = C.c_int(0)
        prm = params._c()
        self._h = _L().ref_amg_setup(A.n, A.rowptr, A.col, A.val, C.byref(prm), C.byref(st))
        self.status = st.value
        if not self._h:
            raise ValueError(f"amg_setup: invalid matrix (status {st.value})")
        if st.value != OK:
            _L().ref_amg_free(self._h)
            self._h = None
            raise ArithmeticError(f"amg_setup failed with status {st.value}")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ref_amg_free(h)
            self._h = None

    @property
    def nlevels(self) -> int:
        return int(_L().ref_hier_nlevels(self._h))

    def level_ilu(self, l: int) -> np.ndarray:
        """ILU(0) factors of level l on its matrix's pattern (smoother ILU0)."""
        lv = self.level(l)
        out = np.zeros(lv.A.nnz)
        if _L().ref_hier_level_ilu(self._h, l, _p(out)) != OK:
            raise ValueError("no ILU(0) factors on this level")
        return out

    def level(self, l: int) -> Level:
        L = _L()
        n, nnz, nc, nnzp = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int64()
        om, rounds, nnzs = C.c_double(), C.c_int32(), C.c_int64()
        L.ref_hier_level_sizes(self._h, l, C.byref(n), C.byref(nnz), C.byref(nc), C.byref(nnzp),
                               C.byref(om), C.byref(rounds), C.byref(nnzs))
        n, nnz, nc, nnzp = n.value, nnz.value, nc.value, nnzp.value
        coarsest = l == self.nlevels - 1
        ar = np.zeros(n + 1, np.int32)
        ac = np.zeros(nnz, np.int32)
        av = np.zeros(nnz, np.float64)
        agg = np.zeros(n, np.int32)
        state = np.zeros(n, np.int32)
        M = np.zeros(n, np.float64)
        pr = np.zeros(n + 1, np.int32)
        pc = np.zeros(max(nnzp, 1), np.int32)
        pv = np.zeros(max(nnzp, 1), np.float64)
        L.ref_hier_level_copy(self._h, l, _p(ar), _p(ac), _p(av), _p(agg), _p(state), _p(M),
                              None if coarsest else _p(pr), _p(pc), _p(pv))
        P = None if coarsest else Csr(pr, pc[:nnzp], pv[:nnzp], nc)
        return Level(Csr(ar, ac, av), None if coarsest else agg, None if coarsest else state,
                     None if coarsest else M, P, nc, om.value, rounds.value, nnzs.value)

    def coarse_lu(self) -> Tuple[np.ndarray, np.ndarray]:
        nd = self.level(self.nlevels - 1).A.n
        lu = np.zeros((nd, nd))
        piv = np.zeros(nd, np.int32)
        _L().ref_hier_coarse_copy(self._h, _p(lu), _p(piv))
        return lu, piv

    def vcycle(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros(self.A.n)
        _L().ref_vcycle(self._h, np.ascontiguousarray(r, dtype=np.float64), z)
        return z

    def complexity(self) -> Tuple[float, float]:
        """(operator complexity sum nnz_l / nnz_0, grid complexity sum n_l / n_0)."""
        lv = [self.level(l) for l in range(self.nlevels)]
        return (sum(x.A.nnz for x in lv) / lv[0].A.nnz, sum(x.A.n for x in lv) / lv[0].A.n)


def pcg(H: Hierarchy, b: np.ndarray, rtol: float = 1e-8, maxiter: int = 1000,
        flexible: bool = False) -> Tuple[np.ndarray, SolveInfo]:
    x = np.zeros(H.A.n)
    info = _Info()
    _L().ref_pcg(H._h, np.ascontiguousarray(b, dtype=np.float64), x, rtol, maxiter,
                 1 if flexible else 0, C.byref(info))
    return x, SolveInfo(info.iters, info.status, info.restarts, info.rel_res, info.rel_res_true)


def pcg_directions(H: Hierarchy, b: np.ndarray, rtol: float = 1e-8, maxiter: int = 1000,
                   flexible: bool = False, max_dirs: int = 64):
    """pcg() that also returns its search directions p_0, p_1, ... (rows)."""
    n = H.A.n
    x = np.zeros(n)
    dirs = np.zeros((max_dirs, n))
    nd = C.c_int32(0)
    info = _Info()
    _L().ref_pcg_dirs(H._h, np.ascontiguousarray(b, dtype=np.float64), x, rtol, maxiter,
                      1 if flexible else 0, C.byref(info), _p(dirs), max_dirs, C.byref(nd))
    return x, SolveInfo(info.iters, info.status, info.restarts, info.rel_res, info.rel_res_true), dirs[:nd.value]


def bicgstab(H: Hierarchy, b: np.ndarray, rtol: float = 1e-8,
             maxiter: int = 1000) -> Tuple[np.ndarray, SolveInfo]:
    x = np.zeros(H.A.n)
    info = _Info()
    _L().ref_bicgstab(H._h, np.ascontiguousarray(b, dtype=np.float64), x, rtol, maxiter, C.byref(info))
    return x, SolveInfo(info.iters, info.status, info.restarts, info.rel_res, info.rel_res_true)


def spmv(A: Csr, x: np.ndarray) -> np.ndarray:
    y = np.zeros(A.n)
    _L().ref_spmv(A.n, A.rowptr, A.col, A.val, np.ascontiguousarray(x, dtype=np.float64), y)
    return y


def mis2_keys(n: int, seed: int, level: int) -> np.ndarray:
    """Priority keys the MIS-2 rounds give UNDECIDED nodes on `level`."""
    k = np.zeros(n, np.uint64)
    _L().ref_mis2_keys(n, seed, level, _p(k))
    return k


def csr_check(A: Csr) -> int:
    return int(_L().ref_csr_check(A.n, A.rowptr, A.col, A.val))


# --------------------------------------------------------------------------
# whole path: flow solve, Darcy fluxes, travel time with two right-hand sides
# --------------------------------------------------------------------------

@dataclasses.dataclass
class FlowResult:
    A: Csr
    b: np.ndarray
    h: np.ndarray
    info: SolveInfo
    H: Hierarchy


def solve_flow(problem, params: AmgParams = AmgParams(), rtol: float = 1e-8,
               maxiter: int = 1000, flexible: bool = False) -> FlowResult:
    A, b = fv_assemble(problem)
    H = Hierarchy(A, params)
    h, info = pcg(H, b, rtol, maxiter, flexible)
    return FlowResult(A, b, h, info, H)


@dataclasses.dataclass
class TravelTimeResult:
    A: Csr
    b_tau: np.ndarray
    b_c: np.ndarray
    tau: np.ndarray
    c: np.ndarray
    info: List[SolveInfo]
    n_identity: int
    H: Hierarchy


def solve_travel_time(grid, qx, qy, qz, phi: float, params: AmgParams = AmgParams(),
                      rtol: float = 1e-8, maxiter: int = 1000,
                      zone: Optional[Sequence[int]] = None) -> TravelTimeResult:
    A, bt, bc, nid = tt_assemble(grid, qx, qy, qz, phi, zone)
    H = Hierarchy(A, params)
    tau, i1 = bicgstab(H, bt, rtol, maxiter)
    c, i2 = bicgstab(H, bc, rtol, maxiter)
    return TravelTimeResult(A, bt, bc, tau, c, [i1, i2], nid, H)


# --------------------------------------------------------------------------
# Dual delineation: the full set of steady advection problems
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Delineation:
    forward: np.ndarray    # [1 + n_sources, n]: tau_f, then one indicator per source
    backward: np.ndarray   # [1 + n_production, n]: tau_b, then one capture indicator per well
    A_forward: Csr
    A_backward: Csr
    rhs_forward: List[np.ndarray]
    rhs_backward: List[np.ndarray]


def _well_terms(grid, A: Csr, bt: np.ndarray, phi: float, wells) -> List[np.ndarray]:
    """Wells that bound this system, in list order: each adds its rate |q| to
    the outflow balance of its cell (the diagonal) and gives an indicator
    right-hand side |q| at that cell.  A cell without face inflow was
    assembled as an identity row; its first well turns it into a regular row
    (diagonal 0 + |q|, b_tau = phi V).  A and bt are modified in place."""
    phi_v = phi * ((grid.dx * grid.dy) * grid.dz)
    rhs = []
    for w in wells:
        c = w.ix + grid.nx * (w.iy + grid.ny * w.iz)
        lo, hi = int(A.rowptr[c]), int(A.rowptr[c + 1])
        p = lo + int(np.nonzero(A.col[lo:hi] == c)[0][0])
        if bt[c] == 0.0:
            A.val[p] = 0.0
            bt[c] = phi_v
        A.val[p] = A.val[p] + abs(w.q)
        b = np.zeros(grid.n)
        b[c] = abs(w.q)
        rhs.append(b)
    return rhs


def dual_delineation(grid, qx, qy, qz, phi: float, h: np.ndarray, zones: Sequence[Sequence[int]],
                     wells: Sequence) -> Delineation:
    """The steady advection problems of the dual delineation (Introduction;
    Eq. 1 and its reversed-flow counterpart), each solved exactly by the sweep.

    Forward, on the flow field q: the travel time tau_f (zero where water
    enters) and one indicator per source: each zone (j0, j1, k0, k1) of the
    x = 0 face, whose right-hand side is the inflow through that face, then
    each injection well (q < 0).  Backward, on the reversed field -q: the
    travel time tau_b to an outlet (life expectancy, zero where water leaves)
    and the capture indicator of each production well (q > 0).  A well is a
    boundary of the system in which water crosses it inwards: injection wells
    of the forward one, production wells of the backward one.
    """
    inj = [w for w in wells if w.q < 0]
    prod = [w for w in wells if w.q > 0]
    Af, btf, _, _ = tt_assemble(grid, qx, qy, qz, phi)
    west = qx.reshape(grid.nz, grid.ny, grid.nx + 1)[:, :, 0]
    west_in = np.where(west > 0.0, west, 0.0)
    rhs_f = [btf]
    for (j0, j1, k0, k1) in zones:
        b = np.zeros((grid.nz, grid.ny, grid.nx))
        b[k0:k1, j0:j1, 0] = west_in[k0:k1, j0:j1]
        rhs_f.append(b.reshape(-1))
    rhs_f += _well_terms(grid, Af, btf, phi, inj)
    Ab, btb, _, _ = tt_assemble(grid, -qx, -qy, -qz, phi)
    rhs_b = [btb] + _well_terms(grid, Ab, btb, phi, prod)
    fwd = np.stack([tt_sweep(Af, b, h) for b in rhs_f])
    bwd = np.stack([tt_sweep(Ab, b, -h) for b in rhs_b])
    return Delineation(fwd, bwd, Af, Ab, rhs_f, rhs_b)


# --------------------------------------------------------------------------
# Transient flow (Eq. 2) and the setup-reuse criterion
# --------------------------------------------------------------------------

def storage_shift(grid, Ss: np.ndarray, dt: float) -> np.ndarray:
    """Diagonal of S / dt in Eq. 2: S_i V_i / dt (specific storage times cell
    volume, over the time step)."""
    vol = (grid.dx * grid.dy) * grid.dz
    return (np.asarray(Ss, dtype=np.float64) * vol) / dt


def reuse_ratio(A: Csr, shift: np.ndarray) -> float:
    """max_i shift_i / C_ii: a setup built for C may be kept for C + S/dt
    while this stays below the small factor delta (Discussion, after Eq. 2)."""
    d = A.to_scipy().diagonal()
    return float(np.max(shift / d))


@dataclasses.dataclass
class TransientResult:
    heads: List[np.ndarray]     # h^1 .. h^N
    ratios: List[float]
    reuse: List[bool]


def transient_flow(problem, Ss: np.ndarray, h0: np.ndarray, dts: Sequence[float],
                   delta: float = 0.01) -> TransientResult:
    """Fully implicit steps of Eq. 2, (C + S/dt) h^{n+1} = Q^{n+1} with
    Q^{n+1} = b + (S/dt) h^n (b: fixed-head faces and wells of the steady
    system), each solved directly; the reuse decision is reported beside."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    A, b = fv_assemble(problem)
    C = A.to_scipy().tocsr()
    h = np.array(h0, dtype=np.float64)
    heads, ratios, reuse = [], [], []
    for dt in dts:
        s = storage_shift(problem.grid, Ss, dt)
        ratio = reuse_ratio(A, s)
        rhs = b + s * h
        h = sla.spsolve((C + sp.diags(s)).tocsc(), rhs)
        heads.append(h)
        ratios.append(ratio)
        reuse.append(ratio < delta)
    return TransientResult(heads, ratios, reuse)
