#!/usr/bin/env python3
"""Benchmark of the interfacial-cell coupling on one MI355X.

A step is one pass of the whole hot path over one front: cell lists, exact
volume fractions (interfacial cells and the dense field), PPIC curvature,
CSF force on the interfacial cells and vertex-velocity interpolation.  The
default workload is the large surface: a polar surface of revolution
rho(theta) = R (1 - 0.3 cos^2 theta + 0.2 cos^4 theta), R = 0.2, as a
geodesic mesh of 1,997,120 triangles on a 512^3 grid, with stream-function
face velocities and sigma = 1 (--workload picks another).  Inputs are
resident in device memory before timing starts.

Timed region: W warm-up steps, then K steps replayed from a HIP graph of one
step, bracketed by device synchronisation; value = interfacial cells x K /
elapsed seconds.  After it, K eager steps with the library's timing events
(recorded on the launch stream) give the average duration of each call; the
PPIC call's FP64 work per launch over that duration is the roofline figure.
The CPU oracle is then timed on the host (all cores, then one thread) on the
same workload: full cell lists and volume fractions, PPIC and CSF on a
seeded sample of cells scaled to all of them, interpolation of every
vertex; its outputs are compared with the GPU's (lists and volume fractions
in full, curvature and forces on the sample).  One JSON line goes to stdout;
progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interfacial cells/s (volume fraction+PPIC curvature), err vs FP64 oracle"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 128 FLOP/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0

# Algorithmic FP64 operations of the PPIC curvature call (its two kernels
# are timed together): per ring triangle (centre distance), per weighted
# triangle (weight, projection, moments, normal-equation update), per cell
# (vertex normal, frame, 6x6 Cholesky with one refinement step, curvature,
# normal).
FLOP_PER_RING_TRI = 17
FLOP_PER_FIT_TRI = 187
FLOP_PER_CELL = 530


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=None,
                    help="revolution_512 (default), sphere_128, ellipsoids_256, or sh_spheres_128 "
                         "(default with --learned)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of a graph")
    ap.add_argument("--mixed", action="store_true",
                    help="PPIC normal equations formed in single precision and refined in double")
    ap.add_argument("--learned", action="store_true",
                    help="curvature by the trained surrogate with its PPIC fallback (the learned form)")
    ap.add_argument("--bound", type=float, default=None, help="spread bound of the learned form (kappa h units)")
    ap.add_argument("--tune", action="store_true",
                    help="choose the launch shapes with the autotuner (whole-step graph timings) before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="interfacial cells of the oracle's PPIC and CSF sample (all cells if fewer)")
    ap.add_argument("--extras", action="store_true",
                    help="also time the calls outside the step: the paraboloid cell quantities, the CSF band mode, "
                         "the surface-tension face flux, RK4 advection, roughness detection and smoothing")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (the reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2505_06932_amd import ftc
    from paper_2505_06932_amd import inputs as I
    from paper_2505_06932_amd import pipeline

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        copy_calibration(torch)
        return
    K, Wm = args.steps, args.warmup
    if args.workload is None:
        args.workload = "sh_spheres_128" if args.learned else "revolution_512"

    grid, mesh, centre = I.make_workload(args.workload, args.seed)
    U, V, W = I.psi_face_velocity(grid)
    log(f"[bench] workload={args.workload} grid={grid.nx}^3 nv={mesh.nv} nt={mesh.nt}")
    params = ftc.PPICParams(precision=1) if args.mixed else None
    theta = None
    if args.learned:
        from paper_2505_06932_amd import surrogate
        theta = surrogate.load_theta()
    step = pipeline.CouplingStep(grid, mesh, U, V, W, sigma=1.0, params=params, learned=theta, bound=args.bound)
    step.run()
    torch.cuda.synchronize()
    n_if, n_pairs = step.cells.count()
    err = step.cells.last_device_error()
    if err != ftc.FTC_OK:
        raise ftc.FTCError(err, "first step")
    log(f"[bench] interfacial cells={n_if} pieces={n_pairs}")
    tune_table = None
    if args.tune:
        from paper_2505_06932_amd import tune
        chosen, table = tune.autotune(step, log=log)
        tune_table = [{**t.__dict__, "us_per_step": round(ms * 1e3, 1)} for t, ms in table]
        log(f"[bench] tuned shapes: {chosen}")

    # ---------------------------------------------------------------- timed
    launch = "eager" if args.eager else "hip_graph"
    graph = None
    if not args.eager:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step.run()
        torch.cuda.synchronize()

    def one():
        if graph is not None:
            graph.replay()
        else:
            step.run()

    for _ in range(Wm):
        one()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(K):
        one()
    ev1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * elapsed / K
    value = n_if * K / elapsed
    log(f"[bench] {launch}: {ms_per_step * 1e3:.1f} us/step wall, {gpu_ms / K * 1e3:.1f} us/step events, "
        f"{value:.3e} cells/s")
    if step.cells.last_device_error() != ftc.FTC_OK:
        raise RuntimeError("device error latched during the timed steps")

    # ----------------------------------------------------- per-kernel times
    step.cells.set_timing(True)
    used = [k for k in ftc.KERNELS if k != "surrogate" or args.learned]
    sums = {k: 0.0 for k in used}
    for _ in range(K):
        step.run()
        for k in used:
            sums[k] += step.cells.kernel_time(k)
    step.cells.set_timing(False)
    kern_ms = {k: v / K for k, v in sums.items()}
    log("[bench] kernel ms: " + ", ".join(f"{k}={v * 1e3:.1f}us" for k, v in kern_ms.items()))

    res = step.results()
    extras = None
    if args.extras and not args.learned:
        extras = time_extras(step, grid, mesh, res, n_if, K, log)
    if args.learned:
        roofline = learned_roofline(res, kern_ms, n_if)
    else:
        roofline = ppic_roofline(res, kern_ms, args.workload)

    out = {
        "metric": METRIC, "value": value, "unit": "interfacial cells/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ("bf16+f32+f64" if args.learned else ("f32+f64" if args.mixed else "f64")),
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [grid.nx, grid.ny, grid.nz], "triangles": mesh.nt,
                   "vertices": mesh.nv, "interfacial_cells": n_if, "pieces": n_pairs, "seed": args.seed,
                   "launch": launch,
                   "step": "cell_lists+volume_fraction+" + ("learned_curvature" if args.learned else "ppic_curvature")
                           + "+csf_force+interp_vertex_velocity",
                   **({"spread_bound": step.bound, "ppic_fallback_cells": res["n_fallback"]} if args.learned else {}),
                   "shapes": ftc.get_tuning(step.cells).__dict__,
                   **({"autotune": tune_table} if tune_table else {})},
        "gpu_ms_per_step_events": gpu_ms / K,
        "kernel_ms": kern_ms,
        "roofline": roofline,
        **({"extras_ms": extras} if extras else {}),
    }

    # ---------------------------------------------------------- CPU oracle
    if not args.no_cpu_baseline:
        base, errs = cpu_baseline(args, grid, mesh, centre, U, V, W, res, step, theta, n_if)
        out["cpu_baseline"] = base
        out["err_vs_oracle"] = errs
        log(f"[bench] oracle {base['value']:.3e} cells/s on {base['cores']} threads, "
            f"{base['single_thread']['value']:.3e} on one; errors {errs}")
    print(json.dumps(out), flush=True)


def _timed(fn):
    t0 = time.perf_counter()
    r = fn()
    return time.perf_counter() - t0, r


def cpu_baseline(args, grid, mesh, centre, U, V, W, res, step, theta, n_if):
    """The oracle timed on the host, all cores then one thread: full cell
    lists and dense volume fractions, PPIC (or the learned form) and CSF on
    a seeded sample of interfacial cells (its time scaled by n_if / sample),
    interpolation of every vertex; and the GPU's errors against it (lists,
    volume fractions and velocities in full, curvature, normals, decisions
    and forces on the sample)."""
    import numpy as np
    import oracle
    from oracle import surrogate as OS
    log("[bench] timing the CPU oracle")
    rng = np.random.default_rng(args.seed + 12345)
    theta_h = theta.cpu().numpy().astype(np.float64) if args.learned else None
    legs = {}
    for leg, nthreads in (("all", 0), ("single", 1)):
        oracle.set_threads(nthreads)
        cores = oracle.threads()
        t_lists, (cells, offsets, tris) = _timed(lambda: oracle.cell_lists(grid, mesh))
        t_vf, (alpha, _) = _timed(lambda: oracle.volume_fraction(grid, mesh))
        ns = min(len(cells), args.cpu_sample if leg == "all" else max(1, args.cpu_sample // 4))
        samp = np.sort(rng.choice(len(cells), ns, replace=False)) if ns < len(cells) else np.arange(len(cells))
        if args.learned:
            # the surrogate's definition: features, four symmetries, PPIC where not trusted
            def learned():
                F, final = OS.features(grid, mesh, alpha, cells[samp])
                mean, spread = OS.predict(theta_h, F)
                fb = ~final | ~(spread <= step.bound)
                kap = mean / grid.h
                kap[fb] = oracle.ppic(grid, mesh, cells[samp][fb])["kappa"]
                return {"kappa": kap, "status": np.zeros(ns, np.int32), "fallback": fb}
            t_ppic, r = _timed(learned)
        else:
            t_ppic, r = _timed(lambda: oracle.ppic(grid, mesh, cells[samp]))  # always double precision
        t_csf, force = _timed(lambda: oracle.csf(grid, alpha, cells[samp], r["kappa"], 1.0))
        t_interp, u = _timed(lambda: oracle.interp(grid, mesh.x, mesh.y, mesh.z, U, V, W))
        per_step = t_lists + t_vf + (t_ppic + t_csf) * len(cells) / ns + t_interp
        legs[leg] = {"value": len(cells) / per_step, "cores": cores, "sample_cells": int(ns),
                     "s": {"cell_lists": t_lists, "volume_fraction": t_vf, "curvature_sample": t_ppic,
                           "csf_sample": t_csf, "interp": t_interp}}
        log(f"[bench] oracle leg {leg}: {cores} threads, {per_step:.2f} s per step estimated")
        if leg == "all":
            ref = (cells, tris, alpha, samp, r, force, u)
    oracle.set_threads(0)
    a = legs["all"]
    base = {"value": a["value"], "unit": "interfacial cells/s", "cores": a["cores"], "kind": "oracle",
            "sample": f"{args.workload}: full cell lists and dense volume fractions, "
                      f"{'learned curvature' if args.learned else 'PPIC'} and CSF on {a['sample_cells']} seeded "
                      f"interfacial cells of {n_if} (time scaled by {n_if / a['sample_cells']:.1f}), "
                      f"interpolation of all {mesh.nv} vertices; seconds {a['s']}; "
                      f"host nproc={os.cpu_count()}, cpu={_cpu_model()}",
            "single_thread": {"value": legs["single"]["value"], "cores": 1,
                              "sample_cells": legs["single"]["sample_cells"], "s": legs["single"]["s"]}}
    cells, tris, alpha, samp, r, force, u = ref
    ok = r["status"] == 0
    g_k, g_f = res["kappa"][samp], res["force"][samp]
    errs = {
        "cell_lists_identical": bool(np.array_equal(res["cell_ids"], cells) and np.array_equal(res["tri_ids"], tris)),
        "max_abs_alpha": float(np.abs(res["alpha"] - alpha).max()),
        "sample_cells": int(len(samp)),
        "max_rel_kappa": float(np.max(np.abs(g_k[ok] - r["kappa"][ok]) / np.abs(r["kappa"][ok]))),
        "max_rel_force": float(np.abs(g_f[ok] - force[ok]).max() / np.abs(force[ok]).max()),
        "max_rel_velocity": float(np.abs(res["u"] - u).max() / np.abs(u).max()),
    }
    if args.learned:
        # the learned form against the double-precision PPIC oracle, on the sample
        fb_g = (res["status"][samp] & 4) == 0
        errs["fallback_frac"] = float(fb_g.mean())
        errs["fallback_decisions_match_oracle"] = float(np.mean(fb_g == r["fallback"]))
        pp = oracle.ppic(grid, mesh, cells[samp])
        okp = pp["status"] == 0
        rel = np.abs(g_k - pp["kappa"]) / np.abs(pp["kappa"])
        tr = ~fb_g & okp
        if tr.any():
            errs["surrogate_rel_kappa_vs_ppic_q50_q90_q99"] = [float(np.quantile(rel[tr], q)) for q in (0.5, 0.9, 0.99)]
            errs["surrogate_abs_kappa_h_vs_ppic_rms"] = float(np.sqrt(np.mean(((g_k - pp["kappa"])[tr] * grid.h) ** 2)))
    else:
        errs["decisions_identical"] = bool(np.array_equal(res["diag"][samp], r["diag"]))
    # the enclosed volume of a closed mesh does not depend on the reference point
    refp = centre if np.asarray(centre).shape == (3,) else np.zeros(3)
    errs["volume_rel_err"] = float(abs(math.fsum(res["alpha"].ravel()) * grid.h ** 3 / _vpoly(mesh, refp) - 1.0))
    return base, errs


def time_extras(step, grid, mesh, res, n_if, K, log):
    """Average times (ms per call, HIP events on the current stream) of the
    library calls outside the coupling step, on the step's own workspace
    after one plain step, plus the paraboloid's deviation from the
    polyhedral alpha."""
    import numpy as np
    import torch
    from paper_2505_06932_amd import ftc

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    step.run()
    cap = step.cells.cell_capacity
    f64 = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    out = {}
    a_par, k_par, n_par = f64(cap), f64(cap), f64(3 * cap)
    out["paraboloid_alpha"] = timeit(lambda: ftc.paraboloid_cell(step.cells, grid, step.coeff, a_par))
    out["paraboloid_alpha_kappa_normal"] = timeit(
        lambda: ftc.paraboloid_cell(step.cells, grid, step.coeff, a_par, k_par, n_par))
    ok = res["status"] == 0
    dev = np.abs(a_par.cpu().numpy()[:n_if][ok] - res["alpha_if"][ok])
    out["paraboloid_alpha_vs_polyhedral_max"] = float(dev.max())
    out["paraboloid_alpha_vs_polyhedral_median"] = float(np.median(dev))
    bcap = 6 * cap
    bid, kb, bx, by, bz = torch.zeros(bcap, dtype=torch.int32, device="cuda"), f64(bcap), f64(bcap), f64(bcap), \
        f64(bcap)
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    out["csf_band"] = timeit(lambda: ftc.csf_force_band(step.cells, grid, step.alpha, step.kappa, step.nx, step.ny,
                                                        step.nz, step.sigma, bid, kb, bx, by, bz, nb))
    fi, fb = f64(6 * cap), f64(6 * bcap)
    out["surface_tension_flux"] = timeit(lambda: ftc.surface_tension_flux(step.cells, grid, step.alpha, step.kappa, bid,
                                                                          kb, nb, 1.2, 1000.0, step.sigma, fi, fb))
    nv = mesh.nv
    xo, yo, zo = f64(nv), f64(nv), f64(nv)
    out["advect_rk4"] = timeit(lambda: ftc.advect_vertices_rk4(step.cells, grid, step.mesh, step.U, step.V, step.W,
                                                               1e-3, xo, yo, zo))
    gl, rough = f64(nv), f64(nv)
    out["front_roughness"] = timeit(lambda: ftc.front_roughness(step.cells, grid, step.mesh, gl, rough))
    # smoothing of the roughest tenth of the vertices by both measures
    glt, rt = float(torch.quantile(gl, 0.9)), float(torch.quantile(rough, 0.9))
    counts = torch.zeros(3, dtype=torch.int32, device="cuda")
    out["smooth_rough_edges"] = timeit(lambda: ftc.smooth_rough_edges(step.cells, grid, step.mesh, gl, rough, glt, rt,
                                                                      xo, yo, zo, counts))
    cnt = counts.cpu().numpy()
    out["edges_listed"], out["edges_moved"] = int(cnt[0]), int(cnt[1])
    log("[bench] extras: " + ", ".join(f"{k}={v:.4g}" for k, v in out.items()))
    return out


def ppic_roofline(res, kern_ms, workload):
    import numpy as np
    diag = res["diag"]
    flops = float(np.sum(FLOP_PER_RING_TRI * diag[:, 1].astype(np.float64)
                         + FLOP_PER_FIT_TRI * diag[:, 2].astype(np.float64) + FLOP_PER_CELL))
    achieved = flops / (kern_ms["ppic"] * 1e-3) / 1e12
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"ppic_{workload}_traffic.json")
    digest = source_digest(["paper_2505_06932_amd/csrc/ppic.hip", "paper_2505_06932_amd/csrc/ftc_device.hpp"])
    if os.path.exists(tfile):
        with open(tfile) as f:
            t = json.load(f)
        if t.get("source_digest") == digest:
            traffic = t.get("bytes_per_launch")
    return {"kernel": "ppic_curvature: k_ppic_fast8 (or its four-wavefront build k_ppic_fast8_w4 on small fronts) + k_ppic_wide",
            "bound": "alu", "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 5), "traffic": traffic,
            "flop_per_launch": flops, "avg_launch_ms": kern_ms["ppic"], "source_digest": digest}


# Algorithmic bfloat16 matrix-core work of the surrogate per interfacial cell:
# four symmetries x (layer 1 over 60 inputs -- the 30 features as high and low
# bfloat16 parts -- to 64 units, layer 2 64 x 64), 2 FLOP per product term.
FLOP_PER_SURROGATE_CELL = 4 * 2 * (60 * 64 + 64 * 64)
BF16_PEAK_TFLOPS = 2500.0


def learned_roofline(res, kern_ms, n_if):
    flops = float(FLOP_PER_SURROGATE_CELL * n_if)
    ms = kern_ms["surrogate"]
    achieved = flops / (ms * 1e-3) / 1e12
    return {"kernel": "learned_curvature: k_surrogate + PPIC kernels on the fallback cells",
            "bound": "mfma", "achieved": round(achieved, 4), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / BF16_PEAK_TFLOPS, 6), "traffic": None, "flop_per_launch": flops,
            "avg_launch_ms": ms}


COPY_BYTES = 256 << 20


def copy_calibration(torch):
    """Five launches of a plain copy of COPY_BYTES: each reads and writes exactly that many bytes."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 5}), flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _vpoly(mesh, centre):
    import numpy as np
    v = mesh.verts() - centre
    t = mesh.tris()
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return math.fsum(np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0)


if __name__ == "__main__":
    main()
