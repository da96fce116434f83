"""The library's pass sequences run on the host (tests/host_pipeline.cpp): the
loss unit with the fused next-pass chunk maps against the same unit with
separate summary passes, for every compiled bandwidth, with the fusion limit
raised to all of them and the address and undefined-behaviour sanitizers on.
This pins the fused accumulators of the F1, F2, B1 and FS steppers (the chunk
maps of the next pass, Algorithms 2-4) and shows them free of out-of-range
indexing and of reads before writes.  Host code only: no GPU is used."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_fused_maps_equal_separate_summaries_on_host(tmp_path):
    exe = str(tmp_path / "host_pipeline")
    cmd = [HIPCC, "--cuda-host-only", "-O0", "-g", "-std=c++17", "-DBO_KMAX_FUSED=12",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "host_pipeline.cpp"), "-x", "hip", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "KMAX_FUSED 12" in r.stdout and "host pipeline ok" in r.stdout, r.stdout
