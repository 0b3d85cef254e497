"""The committed rocprofv3 summaries describe the kernel sources as they
stand (CPU): the step-kernel summaries carry the sources' hash, so the
benchmark reports the counter-measured HBM traffic next to its timing."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_step_kernel_profiles_match_sources():
    h = bench.kernel_source_hash()
    for name in ("k_step_d3q19_512_fp32_trace.md", "k_step_d3q19_512_fp32_pmc.md",
                 "k_step_d3q19_512_fp32_sq.md"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            text = f.read()
        m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
        assert m and m.group(1) == h, (name, m and m.group(1), h)
        assert "rocprofv3" in text   # the command that made it


def test_benchmark_reports_profiled_traffic():
    t = bench.profiled_traffic("k_step_d3q19_512_fp32")
    assert t is not None and t > 12_374_874_552   # above the algorithmic bytes


def test_batch_kernel_profiles_match_sources():
    h = bench.kernel_source_hash(bench.BATCH_SOURCES)
    for name in (f"{bench.BATCH_PROFILE}_trace.md", f"{bench.BATCH_PROFILE}_pmc.md"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            text = f.read()
        m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
        assert m and m.group(1) == h, (name, m and m.group(1), h)
        assert "rocprofv3" in text
    t = bench.profiled_traffic(bench.BATCH_PROFILE, bench.BATCH_SOURCES)
    assert t is not None and t > 5_462_684_368   # above the algorithmic bytes
