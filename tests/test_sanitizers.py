"""Host code under sanitizers (CPU): the library is built with the host side
instrumented -- AddressSanitizer with UndefinedBehaviorSanitizer, and
separately ThreadSanitizer (device code is not instrumented) -- and a small
driver (tests/sanitize/driver.cpp) runs argument validation and the serving
queue from two submitting threads against it; each run must finish with
every check passing and no sanitizer report.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.slow

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"  # the sanitizer runtimes of the library's compiler


def _build(tmp, sanitize):
    import importlib.util
    spec = importlib.util.spec_from_file_location("_gw_build", os.path.join(ROOT, "paper_2001_05798_amd", "build.py"))
    bmod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bmod)
    san = ["-Xarch_host", f"-fsanitize={sanitize}", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]

    def compile_one(item):
        src, exact = item
        obj = os.path.join(tmp, src + ".o")
        cmd = [HIPCC] + bmod.COMMON + san + (["-ffp-contract=off"] if exact else ["-ffp-contract=fast"])
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += ["-c", os.path.join(bmod.CSRC, src), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=min(8, len(bmod.SOURCES))) as ex:
        objs = list(ex.map(compile_one, bmod.SOURCES))
    lib = os.path.join(tmp, "libgwamg_san.so")
    subprocess.run([HIPCC, f"--offload-arch={bmod.ARCH}", "-shared", "-fPIC", "-o", lib] + objs
                   + ["-Xarch_host", f"-fsanitize={sanitize}", "-lpthread"], check=True, capture_output=True)
    exe = os.path.join(tmp, "driver")
    subprocess.run([CLANG, "-std=c++17", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
                    lib, "-o", exe, "-lpthread", f"-Wl,-rpath,{tmp}"], check=True, capture_output=True)
    return exe


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
@pytest.mark.parametrize("sanitize", ["address,undefined", "thread"], ids=["asan-ubsan", "tsan"])
def test_host_code_under_sanitizer(tmp_path, sanitize):
    exe = _build(str(tmp_path), sanitize)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "all checks passed" in r.stdout
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in report, report[-4000:]
