"""The library's candidate classification and clipping, compiled for the
host from the same header the kernels use, against the oracle's per-piece
clip (paper sec. 3.2, polyhedron intersection): whether each (triangle,
cell) pair has a piece of positive area, and its two surface integrals,
must agree bit for bit.  The triangles are seeded and include the
degenerate kinds where rounding decides: corners on grid planes and on
quarter points, collinear and repeated corners, tiny and large triangles,
triangles lying in a grid plane.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def harness(tmp_path_factory, oracle):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    oracle._load()  # builds the oracle library if needed
    out = str(tmp_path_factory.mktemp("host_clip") / "clip_vs_oracle")
    cmd = [hipcc, "-O2", "-std=c++17", "-ffp-contract=off",
           "-I", os.path.join(ROOT, "paper_2505_06932_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "tests", "host_clip", "clip_vs_oracle.cpp"),
           "-L", os.path.join(ROOT, "oracle"), "-lftc_oracle", "-Wl,-rpath," + os.path.join(ROOT, "oracle"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_library_clip_matches_oracle_bitwise(harness, seed):
    r = subprocess.run([harness, "200000", str(seed)], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "differences 0" in r.stdout
