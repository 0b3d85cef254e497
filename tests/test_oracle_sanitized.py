"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

`tests/oracle_sanitize_main.c` calls every entry point of `oracle/lbm_oracle.c`
(creation, both starts and given fields, BGK and TRT, full and linear
equilibrium, pressure and periodic boundaries, populations in and out,
moments, flux, mass, permeability, the run to steady state, and the
single-node functions) on ragged and degenerate domains.  Built with the
sanitizers, any out-of-bounds access, use of freed memory, leak or undefined
integer operation in the oracle fails the run; its printed results must equal
those of the same program built without them, so the instrumented run is the
oracle's ordinary arithmetic.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "lbm_oracle.c")
MAIN_C = os.path.join(HERE, "oracle_sanitize_main.c")
FLAGS = ["-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "-Wall", "-Wextra"]


@pytest.fixture(scope="module")
def programs(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("oracle_san")
    san, plain = str(d / "oracle_san"), str(d / "oracle_plain")
    subprocess.run(["gcc", *FLAGS, "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", san, MAIN_C, ORACLE_C, "-lm"], check=True)
    subprocess.run(["gcc", *FLAGS, "-o", plain, MAIN_C, ORACLE_C, "-lm"], check=True)
    return san, plain


def _cases():
    rng = np.random.default_rng(7)
    out = []

    def add(Q, shape, frac, tau=0.8, rin=1.001, rout=0.999, linear=0, periodic=0, force=0.0,
            trt=0.0, start=0, steps=3):
        mask = (rng.random(shape) < frac).astype(np.uint8)
        nz, ny, nx = (1,) + shape if len(shape) == 2 else shape
        if periodic:
            rin = rout = 1.0
        head = (f"{Q} {nx} {ny} {nz} {tau!r} {rin!r} {rout!r} {linear} {periodic} {force!r} "
                f"{trt!r} {start} {steps}\n")
        out.append(head.encode() + mask.tobytes())

    for shape in ((1, 1), (1, 2), (2, 1), (3, 7), (5, 33), (4, 64)):
        add(9, shape, 0.3)
        add(9, shape, 0.3, linear=1, start=1)
        add(9, shape, 0.3, trt=0.1875, start=2)
        add(9, shape, 0.3, periodic=1, force=1e-4, start=2)
    for shape in ((1, 1, 1), (1, 1, 3), (2, 3, 1), (3, 4, 5), (4, 3, 9)):
        add(19, shape, 0.4)
        add(19, shape, 0.4, linear=1, trt=0.25, start=2)
        add(19, shape, 0.4, periodic=1, force=1e-5, start=1)
    add(9, (6, 20), 1.0)            # all solid
    add(9, (6, 20), 0.0, steps=10)  # no solid
    add(19, (3, 3, 8), 0.0, periodic=1, force=1e-4)
    return b"".join(out), len(out)


def _run(exe, blob):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    p = subprocess.run([exe], input=blob, capture_output=True, env=env, timeout=300)
    assert p.returncode == 0, p.stderr.decode()[-4000:]
    assert b"runtime error" not in p.stderr and b"Sanitizer" not in p.stderr, p.stderr.decode()
    return p.stdout.decode().splitlines()


def test_oracle_clean_under_sanitizers(programs):
    san, plain = programs
    blob, n = _cases()
    a, b = _run(san, blob), _run(plain, blob)
    assert len(a) == n + 2 and a[0].startswith("node 9") and a[1].startswith("node 19")
    assert a == b
    vals = np.array([[float(v) for v in line.split()[1:]] for line in a[2:]])
    assert np.isfinite(vals[:, :5]).all()


def test_sanitizers_catch_a_planted_overrun(tmp_path):
    """A copy of the oracle whose population array is one value short must fail
    under the sanitizers: the run is not blind to the mistakes it is for."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(ORACLE_C).read()
    old = "o->f = (double *)malloc((size_t)N * Q * sizeof(double));"
    assert old in src
    bad = tmp_path / "lbm_oracle_bad.c"
    bad.write_text(src.replace(old, "o->f = (double *)malloc((size_t)(N * Q - 1) * sizeof(double));"))
    exe = str(tmp_path / "oracle_bad")
    subprocess.run(["gcc", *FLAGS, "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, MAIN_C, str(bad), "-lm"], check=True)
    blob = b"9 5 3 1 0.8 1.001 0.999 0 0 0.0 0.0 0 2\n" + bytes(15)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    p = subprocess.run([exe], input=blob, capture_output=True, env=env, timeout=60)
    assert p.returncode != 0 and b"heap-buffer-overflow" in p.stderr
