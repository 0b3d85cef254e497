"""The library's host-side checks under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU, no GPU calls).

`tests/abi_sanitize_main.cpp` calls the C ABI's size queries and argument
checks (every entry point that takes a context, a batch or network shapes,
with invalid and valid arguments, ragged and degenerate geometries up to the
512^3 benchmark size).  It is linked against the library's host translation
units (`lbm_api.hip`, `lbm_batch.hip`, `wsn_api.hip`) built with the
sanitizers on their host code, and the step launchers of the regular build.
Every call must return before any HIP call; any out-of-bounds access, leak or
undefined integer operation in the layout arithmetic or the checks fails.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1609_09685_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1609_09685_amd", "csrc")
OBJDIR = os.path.join(ROOT, "paper_1609_09685_amd", "_build")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def test_abi_checks_clean_under_sanitizers(tmp_path):
    steps = [os.path.join(OBJDIR, f"step_{lat}_{real}.o") for lat in ("D2Q9", "D3Q19")
             for real in ("float", "double")]
    if shutil.which("hipcc") is None or not os.path.exists(CLANG):
        pytest.skip("ROCm compilers not available")
    if not all(os.path.exists(p) for p in steps):
        pytest.skip("library not built (run __graft_entry__.build())")
    flags = [f"--offload-arch={build.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{build.INCLUDE}", f"-I{CSRC}"]
    for f in SAN:
        flags += ["-Xarch_host", f]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.run(["hipcc", *flags, "-c", "-o", obj, os.path.join(CSRC, src)], check=True,
                       capture_output=True)
        return obj

    with ThreadPoolExecutor(3) as ex:
        objs = list(ex.map(compile_one, ["lbm_api.hip", "lbm_batch.hip", "wsn_api.hip"]))
    drv_o = str(tmp_path / "drv.o")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-Wall", "-Wextra", "-Werror", *SAN,
                    f"-I{build.INCLUDE}", "-c", "-o", drv_o,
                    os.path.join(HERE, "abi_sanitize_main.cpp")], check=True)
    exe = str(tmp_path / "abi_check")
    subprocess.run([CLANG, *SAN, "-o", exe, drv_o, *objs, *steps, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, env=env, timeout=300)
    out = p.stdout.decode()
    assert p.returncode == 0, out[-3000:] + p.stderr.decode()[-3000:]
    assert "failures 0" in out
    assert b"runtime error" not in p.stderr and b"Sanitizer" not in p.stderr
