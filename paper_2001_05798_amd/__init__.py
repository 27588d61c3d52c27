"""Python binding of libgwamg (gfx950 groundwater AMG-Krylov library).

Argument marshalling only: every step runs in the HIP library behind the C
ABI declared in ``include/gwamg.h``.  Device buffers are PyTorch tensors on
the current HIP device; the stream is torch's current stream unless one is
given.  Importing fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwamg.so")

OK, NOT_CONVERGED, BREAKDOWN, PENDING = 0, 1, 2, 3
EINVAL, ENOMEM, SINGULAR, EDEVICE, EAGAIN = -1, -2, -3, -4, -5
SMOOTHER_JACOBI, SMOOTHER_SPAI0, SMOOTHER_NONE, SMOOTHER_ILU0 = 0, 1, 2, 3
PRECISION_FP64, PRECISION_MIXED = 0, 1
COARSEN_SA, COARSEN_RS = 0, 1
TT_EPS_STRONG = 0.25
NOALLOC_MAX_ROWS = 1048576  # GW_NOALLOC_MAX_ROWS

STATUS_NAMES = {OK: "OK", NOT_CONVERGED: "NOT_CONVERGED", BREAKDOWN: "BREAKDOWN", PENDING: "PENDING",
                EINVAL: "EINVAL", ENOMEM: "ENOMEM", SINGULAR: "SINGULAR", EDEVICE: "EDEVICE",
                EAGAIN: "EAGAIN"}


class GwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# --------------------------------------------------------------- structs --
class GwGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class GwCsr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class GwWell(C.Structure):
    _fields_ = [("ix", C.c_int32), ("iy", C.c_int32), ("iz", C.c_int32), ("q", C.c_double)]


class GwBc(C.Structure):
    _fields_ = [("h_west", C.c_double), ("h_east", C.c_double)]


class GwZone(C.Structure):
    _fields_ = [("j0", C.c_int32), ("j1", C.c_int32), ("k0", C.c_int32), ("k1", C.c_int32)]


class AmgParamsC(C.Structure):
    _fields_ = [("eps_strong", C.c_double), ("smoother", C.c_int32), ("omega", C.c_double),
                ("npre", C.c_int32), ("npost", C.c_int32), ("n_coarse", C.c_int32),
                ("max_levels", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("coarsening", C.c_int32)]


class SolveParamsC(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxiter", C.c_int32), ("check_every", C.c_int32),
                ("flexible", C.c_int32), ("graph", C.c_int32)]


class SolveInfoC(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("restarts", C.c_int32),
                ("rel_res", C.c_double), ("rel_res_true", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double)]


class StepInfoC(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("reused", C.c_int32), ("ratio", C.c_double),
                ("rel_res_true", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


class LevelInfoC(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("nc", C.c_int32), ("nnz_p", C.c_int64),
                ("nnz_s", C.c_int64), ("mis_rounds", C.c_int32), ("omega_p", C.c_double),
                ("bytes", C.c_size_t), ("slice_rows", C.c_int32), ("nnz_sliced", C.c_int64),
                ("stencil_offsets", C.c_int32)]


class KernelStatC(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("bytes_csr", C.c_double)]


class RequestC(C.Structure):
    _fields_ = [("grid", GwGrid), ("K", C.c_void_p), ("bc", GwBc), ("wells", C.c_void_p),
                ("nwells", C.c_int32), ("phi", C.c_double), ("zone", GwZone),
                ("flow_params", AmgParamsC), ("tt_params", AmgParamsC), ("solve", SolveParamsC),
                ("h_out", C.c_void_p), ("tau_out", C.c_void_p), ("c_out", C.c_void_p),
                ("t_arrival", C.c_double)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("flow", SolveInfoC), ("tt", SolveInfoC * 2),
                ("t_arrival", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("bytes_reserved", C.c_size_t), ("error", C.c_char * 160), ("setup_reused", C.c_int32),
                ("bytes_used", C.c_size_t)]


# ------------------------------------------------------------------ load --
def _load():
    # PyTorch ships its own HIP runtime under the soname libamdhip64.so.7.
    # Loading torch first makes the library bind to that same runtime; the
    # other order would bring a second HIP runtime into the process, and only
    # one of the two can own the device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2001_05798_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "gw_version": (C.c_char_p, []),
        "gw_last_error": (C.c_char_p, []),
        "gw_trim": (C.c_int, []),
        "fv_nnz": (i64, [C.POINTER(GwGrid)]),
        "fv_assemble": (C.c_int, [C.POINTER(GwGrid), vp, C.POINTER(GwBc), vp, i32, vp, vp, vp, vp, vp]),
        "darcy_flux": (C.c_int, [C.POINTER(GwGrid), vp, C.POINTER(GwBc), vp, vp, vp, vp, vp]),
        "amg_setup": (C.c_int, [C.POINTER(GwCsr), C.POINTER(AmgParamsC), C.POINTER(vp), vp]),
        "amg_vcycle": (C.c_int, [vp, vp, vp, vp]),
        "amg_spmv": (C.c_int, [vp, vp, vp, vp]),
        "amg_solve_pcg": (C.c_int, [vp, vp, vp, C.POINTER(SolveParamsC), C.POINTER(SolveInfoC), vp]),
        "amg_solve_bicgstab": (C.c_int, [vp, vp, vp, C.POINTER(SolveParamsC), C.POINTER(SolveInfoC), vp]),
        "amg_solve_bicgstab_pair": (C.c_int, [vp, vp, vp, vp, vp, C.POINTER(SolveParamsC), C.POINTER(SolveInfoC),
                                              vp]),
        "amg_hierarchy_info": (C.c_int, [vp, C.POINTER(LevelInfoC), i32, C.POINTER(i32), C.POINTER(C.c_size_t)]),
        "amg_level_export": (C.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "amg_coarse_export": (C.c_int, [vp, vp, vp, vp, vp]),
        "amg_ilu_export": (C.c_int, [vp, i32, vp, vp]),
        "amg_free": (None, [vp]),
        "tt_nnz_bound": (i64, [C.POINTER(GwGrid)]),
        "tt_assemble": (C.c_int, [C.POINTER(GwGrid), vp, vp, vp, f64, C.POINTER(GwZone), vp, vp, vp, vp, vp,
                                  C.POINTER(i64), C.POINTER(i64), vp]),
        "tt_solve": (C.c_int, [C.POINTER(GwGrid), vp, vp, vp, f64, C.POINTER(GwZone), C.POINTER(AmgParamsC),
                               C.POINTER(SolveParamsC), vp, vp, C.POINTER(SolveInfoC), vp]),
        "tt_sweep": (C.c_int, [C.POINTER(GwCsr), i32, vp, vp, C.POINTER(i32), vp]),
        "tt_solve_direct": (C.c_int, [C.POINTER(GwGrid), vp, vp, vp, f64, C.POINTER(GwZone), vp, vp,
                                      C.POINTER(i32), vp]),
        "amg_solve_pcg_shifted": (C.c_int, [vp, vp, vp, vp, C.POINTER(SolveParamsC), C.POINTER(SolveInfoC), vp]),
        "amg_solve_pcg_noalloc": (C.c_int, [vp, vp, vp, C.POINTER(SolveParamsC), C.POINTER(SolveInfoC), vp]),
        "amg_solve_pcg_batch": (C.c_int, [vp, vp, vp, C.c_int32, C.POINTER(SolveParamsC), C.POINTER(SolveInfoC), vp]),
        "amg_solve_bicgstab_pair_batch": (C.c_int, [vp, vp, vp, vp, vp, C.c_int32, C.POINTER(SolveParamsC),
                                                    C.POINTER(SolveInfoC), vp]),
        "flow_transient": (C.c_int, [C.POINTER(GwGrid), vp, C.POINTER(GwBc), vp, i32, vp, vp, C.POINTER(f64), i32,
                                     f64, C.POINTER(AmgParamsC), C.POINTER(SolveParamsC), vp, vp,
                                     C.POINTER(StepInfoC), vp]),
        "tt_delineate": (C.c_int, [C.POINTER(GwGrid), vp, vp, vp, f64, vp, i32, vp, i32, vp, C.POINTER(i32),
                                   vp]),
        "gw_prof_enable": (C.c_int, [i32]),
        "gw_prof_read": (C.c_int, [C.POINTER(KernelStatC), i32, C.POINTER(i32)]),
        "gw_prof_select": (C.c_int, [C.c_char_p]),
        "queue_create": (C.c_int, [C.c_size_t, i32, C.POINTER(vp)]),
        "queue_clock": (f64, [vp]),
        "queue_submit": (C.c_int, [vp, C.POINTER(RequestC), C.POINTER(C.c_uint64)]),
        "queue_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(ResultC)]),
        "queue_drain": (C.c_int, [vp]),
        "queue_set_setup_cache": (C.c_int, [vp, i32]),
        "queue_set_batch": (C.c_int, [vp, i32, f64, i32]),
        "queue_stats": (C.c_int, [vp, vp, vp]),
        "queue_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()


def lib():
    return _lib


def version() -> str:
    return _lib.gw_version().decode()


def last_error() -> str:
    return _lib.gw_last_error().decode()


def _check(status: int, allow=(OK,)) -> int:
    if status not in allow:
        raise GwError(status, last_error())
    return status


# ------------------------------------------------------------- helpers ---
def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _expect(t, dtype, n: int, name: str):
    import torch
    if t is None:
        return
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {n}")


def grid_c(grid) -> GwGrid:
    return GwGrid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.dx), float(grid.dy), float(grid.dz))


@dataclasses.dataclass
class AmgParams:
    eps_strong: float = 0.08
    smoother: int = SMOOTHER_SPAI0
    omega: float = 2.0 / 3.0
    npre: int = 2
    npost: int = 2
    n_coarse: int = 500
    max_levels: int = 20
    precision: int = PRECISION_FP64
    seed: int = 0x5EED
    coarsening: int = COARSEN_SA

    def c(self) -> AmgParamsC:
        return AmgParamsC(self.eps_strong, self.smoother, self.omega, self.npre, self.npost,
                          self.n_coarse, self.max_levels, self.precision, self.seed, self.coarsening)

    @classmethod
    def flow(cls, **kw) -> "AmgParams":
        """Defaults for the flow system in the benchmark pass: strength
        threshold 0.03 and one pre- and one post-smoothing sweep.  On the
        1M-cell lognormal aquifer (variance 4) setup + CG to 1e-8 take
        11.2 ms against 12.0 ms at (0.08, 1/1) and 12.6 ms at (0.08, 2/2);
        on the 550x500x10 aquifer of variance 10, 45.6 ms against 60.4 ms.
        Thresholds from 0.05 up leave coarse levels of several hundred rows
        whose dense factorization dominates the setup.  The travel-time
        system keeps two sweeps each (1/1 costs it 10 more BiCGSTAB
        iterations)."""
        kw.setdefault("eps_strong", 0.03)
        kw.setdefault("npre", 1)
        kw.setdefault("npost", 1)
        return cls(**kw)

    @classmethod
    def travel_time(cls, **kw) -> "AmgParams":
        """Defaults for the advective travel-time system: a larger strength
        threshold (0.25) keeps aggregates small along streamlines; with the
        flow default (0.08) BiCGSTAB needs 3x more iterations on 1M cells and
        breaks down on the larger served grids."""
        kw.setdefault("eps_strong", TT_EPS_STRONG)
        return cls(**kw)


@dataclasses.dataclass
class SolveParams:
    rtol: float = 1e-8
    maxiter: int = 1000
    check_every: int = 4
    flexible: int = -1
    graph: int = -1

    def c(self) -> SolveParamsC:
        return SolveParamsC(self.rtol, self.maxiter, self.check_every, self.flexible, self.graph)


@dataclasses.dataclass
class SolveInfo:
    iters: int
    status: int
    restarts: int
    rel_res: float
    rel_res_true: float
    setup_ms: float
    solve_ms: float

    @staticmethod
    def of(c: SolveInfoC) -> "SolveInfo":
        return SolveInfo(c.iters, c.status, c.restarts, c.rel_res, c.rel_res_true, c.setup_ms, c.solve_ms)


@dataclasses.dataclass
class StepInfo:
    status: int
    iters: int
    reused: int      # 1 setup of C kept, 2 setup of an earlier equal step, 0 built
    ratio: float     # max_i S_i V_i / (dt C_ii)
    rel_res_true: float
    setup_ms: float
    solve_ms: float


# ----------------------------------------------------------- assembly ----
def fv_nnz(grid) -> int:
    return int(_lib.fv_nnz(C.byref(grid_c(grid))))


def fv_assemble(grid, K, bc: Tuple[float, float], wells: Sequence, rowptr, col, val, b, stream=None) -> None:
    import torch
    g = grid_c(grid)
    n = g.nx * g.ny * g.nz
    nnz = fv_nnz(grid)
    _expect(K, torch.float64, n, "K")
    _expect(rowptr, torch.int32, n + 1, "rowptr")
    _expect(col, torch.int32, nnz, "col")
    _expect(val, torch.float64, nnz, "val")
    _expect(b, torch.float64, n, "b")
    wl = (GwWell * max(1, len(wells)))(*[GwWell(w.ix, w.iy, w.iz, w.q) for w in wells])
    _check(_lib.fv_assemble(C.byref(g), _ptr(K), C.byref(GwBc(*bc)), C.addressof(wl), len(wells),
                            _ptr(rowptr), _ptr(col), _ptr(val), _ptr(b), _stream(stream)))


def darcy_flux(grid, K, bc: Tuple[float, float], h, qx, qy, qz, stream=None) -> None:
    _check(_lib.darcy_flux(C.byref(grid_c(grid)), _ptr(K), C.byref(GwBc(*bc)), _ptr(h), _ptr(qx),
                           _ptr(qy), _ptr(qz), _stream(stream)))


def tt_nnz_bound(grid) -> int:
    return int(_lib.tt_nnz_bound(C.byref(grid_c(grid))))


def tt_assemble(grid, qx, qy, qz, phi: float, zone, rowptr, col, val, b_tau, b_c,
                stream=None) -> Tuple[int, int]:
    nnz, nid = C.c_int64(0), C.c_int64(0)
    z = None if zone is None else C.byref(GwZone(*zone))
    _check(_lib.tt_assemble(C.byref(grid_c(grid)), _ptr(qx), _ptr(qy), _ptr(qz), float(phi), z,
                            _ptr(rowptr), _ptr(col), _ptr(val), _ptr(b_tau), _ptr(b_c),
                            C.byref(nnz), C.byref(nid), _stream(stream)))
    return int(nnz.value), int(nid.value)


def tt_solve(grid, qx, qy, qz, phi: float, zone, params: AmgParams, sp: SolveParams, tau, c,
             stream=None) -> Tuple[int, List[SolveInfo]]:
    info = (SolveInfoC * 2)()
    z = None if zone is None else C.byref(GwZone(*zone))
    st = _check(_lib.tt_solve(C.byref(grid_c(grid)), _ptr(qx), _ptr(qy), _ptr(qz), float(phi), z,
                              C.byref(params.c()), C.byref(sp.c()), _ptr(tau), _ptr(c), info,
                              _stream(stream)), allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return st, [SolveInfo.of(info[0]), SolveInfo.of(info[1])]


def tt_sweep(n: int, rowptr, col, val, b, x, nrhs: int = 1, stream=None) -> int:
    """Exact solve of an upwind system for nrhs right-hand sides (b, x hold
    nrhs blocks of n values).  Returns the number of dependency levels."""
    import torch
    nnz = int(col.numel())
    for t, name, dt, m in ((rowptr, "rowptr", torch.int32, n + 1), (col, "col", torch.int32, nnz),
                           (val, "val", torch.float64, nnz), (b, "b", torch.float64, n * nrhs),
                           (x, "x", torch.float64, n * nrhs)):
        _expect(t, dt, m, name)
    A = GwCsr(int(n), nnz, _ptr(rowptr), _ptr(col), _ptr(val))
    lev = C.c_int32(0)
    _check(_lib.tt_sweep(C.byref(A), int(nrhs), _ptr(b), _ptr(x), C.byref(lev), _stream(stream)))
    return int(lev.value)


def tt_solve_direct(grid, qx, qy, qz, phi: float, zone, tau, c, stream=None) -> int:
    """Assemble the travel-time system and solve both right-hand sides by
    the upwind sweep.  Returns the number of dependency levels."""
    z = None if zone is None else C.byref(GwZone(*zone))
    lev = C.c_int32(0)
    _check(_lib.tt_solve_direct(C.byref(grid_c(grid)), _ptr(qx), _ptr(qy), _ptr(qz), float(phi), z,
                                _ptr(tau), _ptr(c), C.byref(lev), _stream(stream)))
    return int(lev.value)


def delineation_fields(zones: Sequence, wells: Sequence) -> Tuple[int, int]:
    """Number of forward and backward fields tt_delineate writes."""
    return (1 + len(zones) + sum(w.q < 0 for w in wells), 1 + sum(w.q > 0 for w in wells))


def tt_delineate(grid, qx, qy, qz, phi: float, zones: Sequence, wells: Sequence, out,
                 stream=None) -> Tuple[int, int]:
    """The dual delineation's fields by the upwind sweep into out (forward
    fields, then backward ones; see delineation_fields).  Returns the number
    of dependency levels of the forward and backward systems."""
    import torch
    g = grid_c(grid)
    nf, nb = delineation_fields(zones, wells)
    _expect(out, torch.float64, (nf + nb) * g.nx * g.ny * g.nz, "out")
    zl = (GwZone * max(1, len(zones)))(*[GwZone(*z) for z in zones])
    wl = (GwWell * max(1, len(wells)))(*[GwWell(w.ix, w.iy, w.iz, w.q) for w in wells])
    lev = (C.c_int32 * 2)()
    _check(_lib.tt_delineate(C.byref(g), _ptr(qx), _ptr(qy), _ptr(qz), float(phi), C.addressof(zl), len(zones),
                             C.addressof(wl), len(wells), _ptr(out), lev, _stream(stream)))
    return int(lev[0]), int(lev[1])


# ---------------------------------------------------------------- AMG ----
@dataclasses.dataclass
class LevelInfo:
    n: int
    nnz: int
    nc: int
    nnz_p: int
    nnz_s: int
    mis_rounds: int
    omega_p: float
    bytes: int
    slice_rows: int = 0
    nnz_sliced: int = 0
    stencil_offsets: int = 0


class Hierarchy:
    """Owns an amg_hierarchy handle (freed with amg_free)."""

    def __init__(self, handle: int, n: int):
        self._h = C.c_void_p(handle)
        self.n = n
        # held by the object: module globals may already be cleared when a
        # hierarchy is collected at interpreter exit
        self._free = _lib.amg_free

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> Tuple[List[LevelInfo], int]:
        arr = (LevelInfoC * 32)()
        nl, nb = C.c_int32(0), C.c_size_t(0)
        _check(_lib.amg_hierarchy_info(self._h, arr, 32, C.byref(nl), C.byref(nb)))
        k = max(1, nl.value)
        return ([LevelInfo(a.n, a.nnz, a.nc, a.nnz_p, a.nnz_s, a.mis_rounds, a.omega_p, a.bytes, a.slice_rows,
                           a.nnz_sliced, a.stencil_offsets) for a in arr[:k]], int(nb.value))

    @property
    def nlevels(self) -> int:
        nl = C.c_int32(0)
        _check(_lib.amg_hierarchy_info(self._h, None, 0, C.byref(nl), None))
        return nl.value


def amg_setup(n: int, rowptr, col, val, params: AmgParams = AmgParams(), stream=None) -> Hierarchy:
    nnz = int(col.numel())
    A = GwCsr(int(n), nnz, _ptr(rowptr), _ptr(col), _ptr(val))
    h = C.c_void_p(0)
    _check(_lib.amg_setup(C.byref(A), C.byref(params.c()), C.byref(h), _stream(stream)))
    return Hierarchy(h.value, int(n))


def amg_vcycle(H: Hierarchy, r, z, stream=None) -> None:
    _check(_lib.amg_vcycle(H.handle, _ptr(r), _ptr(z), _stream(stream)))


def amg_spmv(H: Hierarchy, x, y, stream=None) -> None:
    _check(_lib.amg_spmv(H.handle, _ptr(x), _ptr(y), _stream(stream)))


def amg_solve_pcg(H: Hierarchy, b, x, sp: SolveParams = SolveParams(), stream=None) -> SolveInfo:
    info = SolveInfoC()
    _check(_lib.amg_solve_pcg(H.handle, _ptr(b), _ptr(x), C.byref(sp.c()), C.byref(info), _stream(stream)),
           allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return SolveInfo.of(info)


def amg_solve_pcg_noalloc(H: Hierarchy, b, x, sp: SolveParams = SolveParams(), stream=None) -> SolveInfo:
    """amg_solve_pcg with the library's static workspace: allocates nothing
    (n <= NOALLOC_MAX_ROWS; calls on one device must not overlap)."""
    info = SolveInfoC()
    _check(_lib.amg_solve_pcg_noalloc(H.handle, _ptr(b), _ptr(x), C.byref(sp.c()), C.byref(info),
                                      _stream(stream)), allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return SolveInfo.of(info)


def _ptr_array(items, conv):
    arr = (C.c_void_p * len(items))()
    for k, it in enumerate(items):
        arr[k] = conv(it)
    return arr


def amg_solve_pcg_batch(Hs: Sequence[Hierarchy], bs, xs, sp: SolveParams = SolveParams(),
                        stream=None) -> List[SolveInfo]:
    """PCG on several hierarchies at once, one launch per kernel step for all
    (each system's iterates equal amg_solve_pcg's)."""
    n = len(Hs)
    if not (len(bs) == len(xs) == n):
        raise ValueError("one b and one x per hierarchy")
    info = (SolveInfoC * n)()
    _check(_lib.amg_solve_pcg_batch(_ptr_array(Hs, lambda h: h.handle), _ptr_array(bs, _ptr),
                                    _ptr_array(xs, _ptr), n, C.byref(sp.c()), info, _stream(stream)),
           allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return [SolveInfo.of(i) for i in info]


def amg_solve_bicgstab_pair_batch(Hs: Sequence[Hierarchy], b0s, b1s, x0s, x1s, sp: SolveParams = SolveParams(),
                                  stream=None) -> Tuple[int, List[Tuple[SolveInfo, SolveInfo]]]:
    """The BiCGSTAB pair on several hierarchies at once (each pair's iterates
    equal amg_solve_bicgstab_pair's).  Returns the worst status and one
    (info0, info1) per hierarchy."""
    n = len(Hs)
    if not (len(b0s) == len(b1s) == len(x0s) == len(x1s) == n):
        raise ValueError("two right-hand sides and two solutions per hierarchy")
    info = (SolveInfoC * (2 * n))()
    st = _lib.amg_solve_bicgstab_pair_batch(_ptr_array(Hs, lambda h: h.handle), _ptr_array(b0s, _ptr),
                                            _ptr_array(b1s, _ptr), _ptr_array(x0s, _ptr), _ptr_array(x1s, _ptr), n,
                                            C.byref(sp.c()), info, _stream(stream))
    _check(st, allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return st, [(SolveInfo.of(info[2 * k]), SolveInfo.of(info[2 * k + 1])) for k in range(n)]


def amg_solve_pcg_shifted(H: Hierarchy, shift, b, x, sp: SolveParams = SolveParams(), stream=None) -> SolveInfo:
    """PCG on (A + diag(shift)) x = b with the hierarchy of A as preconditioner."""
    info = SolveInfoC()
    _check(_lib.amg_solve_pcg_shifted(H.handle, _ptr(shift), _ptr(b), _ptr(x), C.byref(sp.c()), C.byref(info),
                                      _stream(stream)), allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return SolveInfo.of(info)


def flow_transient(grid, K, bc: Tuple[float, float], wells: Sequence, Ss, h0, dts: Sequence[float], h,
                   delta: float = 0.01, params: "AmgParams" = None, sp: SolveParams = SolveParams(),
                   h_steps=None, stream=None) -> Tuple[int, List[StepInfo]]:
    """Fully implicit steps of Eq. 2 with setup reuse; see flow_transient in
    the C header.  Returns the worst status and one StepInfo per step."""
    import torch
    g = grid_c(grid)
    n = g.nx * g.ny * g.nz
    for t, name in ((K, "K"), (Ss, "Ss"), (h0, "h0"), (h, "h")):
        _expect(t, torch.float64, n, name)
    if h_steps is not None:
        _expect(h_steps, torch.float64, n * len(dts), "h_steps")
    params = params if params is not None else AmgParams()
    wl = (GwWell * max(1, len(wells)))(*[GwWell(w.ix, w.iy, w.iz, w.q) for w in wells])
    dt = (C.c_double * len(dts))(*[float(x) for x in dts])
    info = (StepInfoC * len(dts))()
    st = _check(_lib.flow_transient(C.byref(g), _ptr(K), C.byref(GwBc(*bc)), C.addressof(wl), len(wells), _ptr(Ss),
                                    _ptr(h0), dt, len(dts), float(delta), C.byref(params.c()), C.byref(sp.c()),
                                    _ptr(h), _ptr(h_steps), info, _stream(stream)),
                allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return st, [StepInfo(i.status, i.iters, i.reused, i.ratio, i.rel_res_true, i.setup_ms, i.solve_ms)
                for i in info]


def amg_solve_bicgstab(H: Hierarchy, b, x, sp: SolveParams = SolveParams(), stream=None) -> SolveInfo:
    info = SolveInfoC()
    _check(_lib.amg_solve_bicgstab(H.handle, _ptr(b), _ptr(x), C.byref(sp.c()), C.byref(info),
                                   _stream(stream)), allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return SolveInfo.of(info)


def amg_solve_bicgstab_pair(H: Hierarchy, b0, b1, x0, x1, sp: SolveParams = SolveParams(),
                            stream=None) -> Tuple[int, List[SolveInfo]]:
    info = (SolveInfoC * 2)()
    st = _check(_lib.amg_solve_bicgstab_pair(H.handle, _ptr(b0), _ptr(b1), _ptr(x0), _ptr(x1), C.byref(sp.c()),
                                             info, _stream(stream)), allow=(OK, NOT_CONVERGED, BREAKDOWN))
    return st, [SolveInfo.of(info[0]), SolveInfo.of(info[1])]


def amg_level_export(H: Hierarchy, level: int, a_rowptr=None, a_col=None, a_val=None, agg=None, M=None,
                     p_rowptr=None, p_col=None, p_val=None, stream=None) -> None:
    _check(_lib.amg_level_export(H.handle, int(level), _ptr(a_rowptr), _ptr(a_col), _ptr(a_val), _ptr(agg),
                                 _ptr(M), _ptr(p_rowptr), _ptr(p_col), _ptr(p_val), _stream(stream)))


def amg_ilu_export(H: Hierarchy, level: int, lu, stream=None) -> None:
    _check(_lib.amg_ilu_export(H.handle, int(level), _ptr(lu), _stream(stream)))


def amg_coarse_export(H: Hierarchy, lu=None, piv=None, inv=None, stream=None) -> None:
    _check(_lib.amg_coarse_export(H.handle, _ptr(lu), _ptr(piv), _ptr(inv), _stream(stream)))


# ------------------------------------------------------------ profiling --
def prof_enable(on: bool) -> None:
    _check(_lib.gw_prof_enable(1 if on else 0))


def prof_select(name: Optional[str]) -> None:
    _check(_lib.gw_prof_select(name.encode() if name else None))


def prof_read() -> dict:
    arr = (KernelStatC * 64)()
    n = C.c_int32(0)
    _check(_lib.gw_prof_read(arr, 64, C.byref(n)))
    return {a.name.decode(): {"launches": int(a.launches), "ms": float(a.ms), "bytes": float(a.bytes),
                              "bytes_csr": float(a.bytes_csr)}
            for a in arr[:n.value]}


def trim() -> None:
    _check(_lib.gw_trim())


# -------------------------------------------------------------- serving --
@dataclasses.dataclass
class Result:
    status: int
    flow: SolveInfo
    tt: List[SolveInfo]
    t_arrival: float
    t_start: float
    t_done: float
    bytes_reserved: int
    error: str = ""
    setup_reused: int = 0   # 1: the flow hierarchy came from the setup cache
    bytes_used: int = 0     # device bytes held at the request's larger phase

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Queue:
    """Continuous-batching queue of flow + travel-time requests.

    Inputs (K, wells) and outputs (h, tau, c) are host numpy arrays that the
    queue keeps referenced until the ticket's result has been polled.
    """

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4):
        q = C.c_void_p(0)
        _check(_lib.queue_create(C.c_size_t(int(hbm_budget_bytes)), int(max_slots), C.byref(q)))
        self._q = q
        self._keep = {}
        self._destroy = _lib.queue_destroy

    def __del__(self):
        self.close()

    def close(self):
        q = getattr(self, "_q", None)
        if q is not None and q.value:
            self._destroy(q)
            self._q = None
        self._keep = {}

    def clock(self) -> float:
        return float(_lib.queue_clock(self._q))

    def submit(self, problem, flow_params: AmgParams, tt_params: AmgParams, sp: SolveParams,
               zone=None, want=("h", "tau", "c"), t_arrival: float = -1.0):
        import numpy as np
        g = problem.grid
        n = g.n
        K = np.ascontiguousarray(problem.K, dtype=np.float64)
        wl = (GwWell * max(1, len(problem.wells)))(*[GwWell(w.ix, w.iy, w.iz, w.q) for w in problem.wells])
        outs = {k: np.zeros(n) for k in want}
        z = zone if zone is not None else (0, g.ny, 0, g.nz)
        req = RequestC(grid_c(g), K.ctypes.data, GwBc(problem.h_west, problem.h_east), C.addressof(wl),
                       len(problem.wells), float(problem.phi), GwZone(*z), flow_params.c(), tt_params.c(),
                       sp.c(), outs["h"].ctypes.data if "h" in outs else None,
                       outs["tau"].ctypes.data if "tau" in outs else None,
                       outs["c"].ctypes.data if "c" in outs else None, float(t_arrival))
        t = C.c_uint64(0)
        _check(_lib.queue_submit(self._q, C.byref(req), C.byref(t)))
        self._keep[t.value] = (K, wl, outs)
        return t.value

    def poll(self, ticket: int):
        """None while pending; else (Result, outputs dict)."""
        r = ResultC()
        st = _lib.queue_poll(self._q, C.c_uint64(ticket), C.byref(r))
        if st == PENDING:
            return None
        if st == EINVAL and ticket not in self._keep:
            raise GwError(st, last_error())
        K, wl, outs = self._keep.pop(ticket)
        res = Result(r.status, SolveInfo.of(r.flow), [SolveInfo.of(r.tt[0]), SolveInfo.of(r.tt[1])],
                     r.t_arrival, r.t_start, r.t_done, int(r.bytes_reserved), r.error.decode(errors="replace"),
                     int(r.setup_reused), int(r.bytes_used))
        return res, outs

    def drain(self) -> None:
        _check(_lib.queue_drain(self._q))

    def set_batch(self, max_batch: int, window_us: float = 0.0, streams: int = 1) -> None:
        """Solves of the running requests share launches in batches of up to
        max_batch (1: each request solves on its own stream); a batch waits
        up to window_us for other running requests' solves to join; `streams`
        solver threads run batches side by side."""
        _check(_lib.queue_set_batch(self._q, int(max_batch), float(window_us), int(streams)))

    def stats(self) -> Tuple[int, int]:
        """(blocks of iterations run for two or more solves at once, solves taken)."""
        a, b = C.c_uint64(0), C.c_uint64(0)
        _check(_lib.queue_stats(self._q, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def set_setup_cache(self, max_entries: int) -> None:
        """Keep up to max_entries flow hierarchies for later requests with the
        same conductance field, grid, heads and AMG parameters (0: off)."""
        _check(_lib.queue_set_setup_cache(self._q, int(max_entries)))
