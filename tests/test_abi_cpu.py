"""CPU checks of the C ABI: the library loads and exports every function the
header declares; argument validation happens before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwamg.h")
LIB = os.path.join(ROOT, "paper_2001_05798_amd", "libgwamg.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["fv_assemble", "amg_setup", "amg_solve_pcg", "amg_solve_bicgstab", "amg_solve_bicgstab_pair", "tt_solve",
              "tt_sweep", "tt_solve_direct", "tt_delineate", "amg_solve_pcg_shifted", "flow_transient", "amg_ilu_export", "amg_solve_pcg_noalloc",
              "amg_solve_pcg_batch", "amg_solve_bicgstab_pair_batch",
              "queue_submit", "queue_poll", "darcy_flux", "amg_free", "gw_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_validation_without_device():
    # these calls fail on their arguments before touching HIP
    lib = ctypes.CDLL(LIB)
    lib.fv_nnz.restype = ctypes.c_int64
    lib.gw_last_error.restype = ctypes.c_char_p
    lib.gw_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.gw_version()

    class Grid(ctypes.Structure):
        _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                    ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]

    assert lib.fv_nnz(ctypes.byref(Grid(550, 500, 10, 1, 1, 1))) == 18_679_000
    assert lib.fv_nnz(ctypes.byref(Grid(0, 5, 5, 1, 1, 1))) == -1
    rc = lib.fv_assemble(ctypes.byref(Grid(-1, 2, 2, 1, 1, 1)), None, None, None, 0, None, None, None, None, None)
    assert rc == -1 and b"grid" in lib.gw_last_error()
    rc = lib.amg_setup(None, None, None, None)
    assert rc == -1
    assert lib.amg_solve_bicgstab_pair(None, None, None, None, None, None, None, None) == -1
    assert lib.tt_sweep(None, 1, None, None, None, None) == -1
    assert lib.amg_solve_pcg_shifted(None, None, None, None, None, None, None) == -1
    assert lib.amg_solve_pcg_noalloc(None, None, None, None, None, None) == -1
    assert lib.amg_solve_pcg_batch(None, None, None, 1, None, None, None) == -1
    assert lib.amg_solve_bicgstab_pair_batch(None, None, None, None, None, 1, None, None, None) == -1
    assert lib.flow_transient(ctypes.byref(Grid(0, 4, 4, 1, 1, 1)), None, None, None, 0, None, None, None, 1,
                              ctypes.c_double(0.01), None, None, None, None, None, None) == -1
    assert lib.tt_delineate(ctypes.byref(Grid(4, 4, 4, 1, 1, 1)), None, None, None, ctypes.c_double(0.25),
                            None, 0, None, 0, None, None, None) == -1
    assert lib.tt_solve_direct(ctypes.byref(Grid(0, 2, 2, 1, 1, 1)), None, None, None, ctypes.c_double(0.25),
                               None, None, None, None, None) == -1


def _c_layout(struct, field):
    # sizeof and offsetof as the C compiler sees the header
    import subprocess
    import tempfile
    src = (f'#include <stdio.h>\n#include <stddef.h>\n#include "gwamg.h"\n'
           f'int main(void) {{ printf("%zu %zu", sizeof({struct}), offsetof({struct}, {field})); return 0; }}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), int(out[1])


def test_amg_params_layout_and_validation():
    # amg_params as the header lays it out (coarsening last), checked by the
    # library before any device work
    lib = ctypes.CDLL(LIB)
    lib.gw_last_error.restype = ctypes.c_char_p

    class Csr(ctypes.Structure):
        _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                    ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]

    class Params(ctypes.Structure):
        _fields_ = [("eps_strong", ctypes.c_double), ("smoother", ctypes.c_int32), ("omega", ctypes.c_double),
                    ("npre", ctypes.c_int32), ("npost", ctypes.c_int32), ("n_coarse", ctypes.c_int32),
                    ("max_levels", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                    ("coarsening", ctypes.c_int32)]

    import paper_2001_05798_amd as gw
    size, off = _c_layout("amg_params", "coarsening")
    assert ctypes.sizeof(gw.AmgParamsC) == ctypes.sizeof(Params) == size
    assert gw.AmgParamsC.coarsening.offset == Params.coarsening.offset == off
    buf = (ctypes.c_int64 * 8)()
    a = ctypes.addressof(buf)
    A = Csr(2, 2, a, a, a)
    h = ctypes.c_void_p()
    for coarsening, ok in ((2, False), (-1, False)):
        prm = Params(0.25, 1, 2.0 / 3.0, 2, 2, 500, 20, 0, 0x5EED, coarsening)
        assert lib.amg_setup(ctypes.byref(A), ctypes.byref(prm), ctypes.byref(h), None) == -1
        assert b"coarsening" in lib.gw_last_error()
    prm = Params(0.25, 3, 2.0 / 3.0, 2, 2, 500, 20, 1, 0x5EED, 1)   # ILU0 with the FP32 hierarchy
    assert lib.amg_setup(ctypes.byref(A), ctypes.byref(prm), ctypes.byref(h), None) == -1
    assert b"ILU(0)" in lib.gw_last_error()


@pytest.mark.parametrize("struct,cls,field", [
    ("amg_level_info", "LevelInfoC", "stencil_offsets"),
    ("amg_solve_params", "SolveParamsC", None),
    ("amg_solve_info", "SolveInfoC", None),
    ("gw_kernel_stat", "KernelStatC", "bytes_csr"),
    ("gw_result", "ResultC", "bytes_used"),
])
def test_struct_layouts_match_header(struct, cls, field):
    # the binding's ctypes records against the header as the C compiler lays
    # it out: size, and the offset of the last field added
    import paper_2001_05798_amd as gw
    c = getattr(gw, cls)
    last = field or c._fields_[-1][0]
    size, off = _c_layout(struct, last)
    assert ctypes.sizeof(c) == size
    assert getattr(c, last).offset == off
