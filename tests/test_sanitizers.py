"""Native code under AddressSanitizer and UndefinedBehaviorSanitizer (host
builds only; no GPU is used):
  * the oracle's C source with a driver that runs every native entry point
    on the 32^3 sphere front (cell lists, volume fractions along each axis,
    PPIC with its support, CSF in both modes, interpolation, RK4), its
    checksums equal to those of the ordinary build of the oracle;
  * the host build of the library's candidate classification and clipping
    against the oracle (tests/host_clip), on seeded degenerate-heavy
    triangles.
Any memory error, leak or undefined behaviour fails the test."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2505_06932_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# verify_asan_link_order=0: the environment may preload a library ahead of
# the sanitizer runtime, which the runtime otherwise refuses
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=900, **kw)


def _write_front(path, grid, mesh, U, V, W):
    with open(path, "wb") as f:
        np.array([grid.nx, grid.ny, grid.nz], np.int32).tofile(f)
        np.array([grid.x0, grid.y0, grid.z0, grid.h], np.float64).tofile(f)
        np.array([mesh.nv, mesh.nt], np.int32).tofile(f)
        for a in (mesh.x, mesh.y, mesh.z):
            np.ascontiguousarray(a, np.float64).tofile(f)
        for a in (mesh.t0, mesh.t1, mesh.t2):
            np.ascontiguousarray(a, np.int32).tofile(f)
        for a in (U, V, W):
            np.ascontiguousarray(a, np.float64).reshape(-1).tofile(f)


def _expected(grid, mesh, U, V, W):
    """The driver's checksums from the ordinary oracle build."""
    def s(a):
        a = np.asarray(a, np.float64).ravel()
        return math.fsum(a[~np.isnan(a)])
    cells, off, tris = oracle.cell_lists(grid, mesh)
    out = {"cell_lists": (len(tris), len(cells), int(np.sum(tris, dtype=np.int64)))}
    for axis in range(3):
        a, _ = oracle.volume_fraction(grid, mesh, axis=axis)
        out[f"vf{axis}"] = s(a)
    r = oracle.ppic(grid, mesh, cells)
    out["ppic"] = (s(r["kappa"]), s(r["normal"]), int(r["diag"].sum()))
    sp = oracle.ppic_support(grid, mesh, cells[0])
    out["support"] = (len(sp["tri"]), s(sp["w"]), sp["delta"])
    alpha, _ = oracle.volume_fraction(grid, mesh)
    out["csf"] = s(oracle.csf(grid, alpha, cells, r["kappa"], 1.0))
    bid, kb, _ = oracle.csf_band(grid, alpha, cells, r["kappa"], r["normal"], 1.0)
    out["band"] = (len(bid), s(kb))
    out["interp"] = s(oracle.interp(grid, mesh.x, mesh.y, mesh.z, U, V, W))
    out["rk4"] = s(oracle.advect_rk4(grid, mesh.x, mesh.y, mesh.z, U, V, W, 1e-3))
    return out


def _close(a, b):
    return abs(a - b) <= 1e-12 * max(1.0, abs(b))


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    r = _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
              "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
              os.path.join(ROOT, "oracle", "ftc_oracle.c"), "-lm", "-o", exe])
    assert r.returncode == 0, r.stderr[-3000:]
    grid, mesh, _ = I.make_workload("sphere_32", 0)
    U, V, W = I.psi_face_velocity(grid)
    front = str(tmp_path / "front.bin")
    _write_front(front, grid, mesh, U, V, W)
    r = _run([exe, front], env=SAN_ENV)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    got = {}
    for line in r.stdout.splitlines():
        w = line.split()
        if w[0] == "cell_lists":
            got["cell_lists"] = (int(w[2]), int(w[4]), int(w[6]))
        elif w[0] == "volume_fraction":
            got[f"vf{w[2]}"] = float(w[4])
        elif w[0] == "ppic":
            got["ppic"] = (float(w[2]), float(w[4]), int(w[6]))
        elif w[0] == "ppic_support":
            got["support"] = (int(w[2]), float(w[4]), float(w[6]))
        elif w[0] == "csf":
            got["csf"] = float(w[2])
        elif w[0] == "csf_band":
            got["band"] = (int(w[2]), float(w[4]))
        elif w[0] == "interp":
            got["interp"] = float(w[2])
        elif w[0] == "advect_rk4":
            got["rk4"] = float(w[2])
    exp = _expected(grid, mesh, U, V, W)
    assert set(got) == set(exp)
    for k, v in exp.items():
        g = got[k]
        if isinstance(v, tuple):
            assert all((a == b) if isinstance(b, int) else _close(a, b) for a, b in zip(g, v)), (k, g, v)
        else:
            assert _close(g, v), (k, g, v)


def test_host_clip_under_sanitizers(tmp_path):
    hipcc = next((c for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc") if c and os.path.exists(c)), None)
    if hipcc is None or shutil.which("gcc") is None:
        pytest.skip("hipcc or gcc not available")
    # the oracle's clip compiled with the sanitizers as well
    obj = str(tmp_path / "ftc_oracle.o")
    r = _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-c",
              os.path.join(ROOT, "oracle", "ftc_oracle.c"), "-o", obj])
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "clip_vs_oracle")
    hobj = str(tmp_path / "clip_vs_oracle.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    r = _run([hipcc, "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-omit-frame-pointer", *san,
              "-I", os.path.join(ROOT, "paper_2505_06932_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
              "-I", os.path.join(ROOT, "oracle"), "-c", os.path.join(ROOT, "tests", "host_clip", "clip_vs_oracle.cpp"),
              "-o", hobj])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([hipcc, hobj, obj, *san, "-lm", "-o", exe])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([exe, "20000", "3"], env=SAN_ENV)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "differences 0" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
