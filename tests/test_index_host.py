"""CPU check of the step kernel's index arithmetic (no GPU).

`tests/host_index_check.cpp` runs the functions the GPU step kernel uses to
find its pull sources and its segment stores (`csrc/pull_index.h`) for every
lane of every word, and compares them with the boundary rules applied directly
to an independently built slot map: streaming, halfway bounce-back at solid
sources, mirrors at the symmetric y / z planes, pressure ghosts at the x faces
(the paper's pressure-driven 2D case, Fig. 1 and the first paragraph of the
Results) and the periodic faces of its 3D force-driven case.  It also checks
that no slot read or written leaves the population arrays (capacity from the
library's own lbm_query_sizes), that padding is never read, that the block
stores write every slot once in whole 128-byte lines, and that the LDS staging
index stays inside a block.  The program is built with AddressSanitizer and
UndefinedBehaviorSanitizer, so an out-of-bounds host access or an integer
overflow in this arithmetic also fails the test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1609_09685_amd import lbm
from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1609_09685_amd", "csrc")
SRC = os.path.join(HERE, "host_index_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("idx") / "host_index_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-DLBM_CHECK_MAIN", "-Wall", "-Wextra",
                    "-Werror", f"-I{CSRC}", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", exe, SRC], check=True)
    return exe


def slots_capacity(Q, shape, n_fluid, precision):
    nz, ny, nx = shape
    f_bytes, _ = lbm.query_sizes(Q, nx, ny, nz, n_fluid, precision=precision)
    esize = 8 if precision == "fp64" else 4
    return f_bytes // (Q * esize)


def run_cases(exe, cases):
    """cases: (Q, mask [nz, ny, nx] uint8 1 = solid, precision, periodic)."""
    blob = bytearray()
    for Q, mask, precision, periodic in cases:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.ndim == 2:
            mask = mask[None]
        nz, ny, nx = mask.shape
        ps = slots_capacity(Q, mask.shape, int((mask == 0).sum()), precision)
        esize = 8 if precision == "fp64" else 4
        blob += f"{Q} {nx} {ny} {nz} {esize} {int(periodic)} {ps}\n".encode()
        blob += mask.tobytes()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe], input=bytes(blob), capture_output=True, env=env, timeout=600)
    lines = p.stdout.decode().splitlines()
    assert p.returncode in (0, 1), p.stderr.decode()[-3000:]
    assert len(lines) == len(cases), (lines, p.stderr.decode()[-3000:])
    for (Q, mask, precision, periodic), line in zip(cases, lines):
        parts = line.split(" ", 6)
        errors, checked = int(parts[3]), int(parts[5])
        msg = parts[6] if len(parts) > 6 else ""
        assert errors == 0, (Q, np.shape(mask), precision, periodic, msg)
        n_fluid = int((np.asarray(mask) == 0).sum())
        assert checked == 2 * n_fluid * (Q - 1)   # every direction, two uniform offsets
    assert p.returncode == 0


def random_mask(rng, shape, solid_frac):
    return (rng.random(shape) < solid_frac).astype(np.uint8)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("periodic", [False, True])
def test_d2q9_ragged_and_degenerate(checker, precision, periodic):
    rng = np.random.default_rng(11)
    cases = []
    for nx in (2, 3, 63, 64, 65, 127, 128, 129, 191, 256, 257, 300, 513):
        for ny in (1, 2, 3, 7):
            for frac in (0.0, 0.3, 0.7):
                cases.append((9, random_mask(rng, (ny, nx), frac), precision, periodic))
    # all solid, one fluid node, fluid runs that end on word boundaries
    cases.append((9, np.ones((4, 130), np.uint8), precision, periodic))
    one = np.ones((3, 70), np.uint8)
    one[1, 64] = 0
    cases.append((9, one, precision, periodic))
    runs = np.ones((5, 320), np.uint8)
    runs[:, 60:260] = 0
    cases.append((9, runs, precision, periodic))
    cases.append((9, qsgs_2d(400, 200, 0.74, 3), precision, periodic))
    run_cases(checker, cases)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("periodic", [False, True])
def test_d3q19_ragged_and_degenerate(checker, precision, periodic):
    rng = np.random.default_rng(12)
    cases = []
    for nx in (2, 5, 64, 65, 129, 257, 300):
        for ny, nz in ((1, 1), (1, 3), (3, 1), (2, 2), (4, 5)):
            for frac in (0.0, 0.4):
                cases.append((19, random_mask(rng, (nz, ny, nx), frac), precision, periodic))
    cases.append((19, qsgs_3d(70, 9, 8, 0.6, 1), precision, periodic))
    cases.append((19, qsgs_3d(300, 6, 5, 0.6, 2), precision, periodic))
    run_cases(checker, cases)


@pytest.mark.parametrize("old,new", [
    ("off = cnt * E + ub;", "off = cnt * E + ub + E;"),             # a neighbour slot off by one
    ("count = d1.base + popc64(desc_bits(d1)) - d0.base;",
     "count = d1.base + popc64(desc_bits(d1)) - d0.base + 1u;"),    # one store too many
    ("if (has_next) info |= (pfx_next - (pfx + popc64(mid))) << 16;",
     "if (has_next) info |= (pfx_next - (pfx + popc64(mid))) << 17;"),  # a corrupt record
])
def test_checker_catches_a_planted_slip(checker, tmp_path, old, new):
    """A copy of the index header with one planted mistake must fail: the check
    is not blind to the mistakes it exists to catch."""
    src = open(os.path.join(CSRC, "pull_index.h")).read()
    bad = src.replace(old, new, 1)
    assert bad != src
    d = tmp_path / "csrc"
    d.mkdir()
    (d / "pull_index.h").write_text(bad)
    shutil.copy(os.path.join(CSRC, "lattice.h"), d / "lattice.h")
    exe = str(tmp_path / "bad_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-DLBM_CHECK_MAIN", f"-I{d}", "-o", exe, SRC],
                   check=True)
    mask = random_mask(np.random.default_rng(4), (3, 300), 0.3)   # segment gaps inside rows
    ps = slots_capacity(9, (1, 3, 300), int((mask == 0).sum()), "fp32")
    blob = f"9 300 3 1 4 0 {ps}\n".encode() + mask.tobytes()
    p = subprocess.run([exe], input=blob, capture_output=True, timeout=60)
    assert p.returncode == 1
    assert "errors 0 " not in p.stdout.decode()
