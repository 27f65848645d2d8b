"""GPU parity of the volume fraction under the fitted paraboloid (paper
sec. 3.2) through the C ABI.  The GPU call is given the oracle's own PPIC
coefficients, so both sides integrate the same paraboloid (the frame normal
comes from the PPIC run on the device, which picks the same closest vertex):
sampled cells within 1e-12.  At full size every cell is checked against the
exact polyhedral alpha to the fit error, and the host-side preconditions."""
import sys

import numpy as np
import pytest

from oracle import paraboloid as PB
from paper_2505_06932_amd import inputs as I

pytestmark = pytest.mark.gpu

ALPHA_TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(name, seed=0):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2505_06932_amd import pipeline
    grid, mesh, _ = I.make_workload(name, seed)
    _say(f"[paraboloid] case={name}/{seed} nv={mesh.nv} nt={mesh.nt}")
    step = pipeline.CouplingStep(grid, mesh)
    step.run()
    return grid, mesh, step


def _cell_gpu(step, grid, coeff_rows, surface=False):
    """Run the GPU call with the given coefficients [n_if, 6] (host):
    alpha, or (alpha, kappa_cell, normal_cell [n, 3])."""
    import torch
    from paper_2505_06932_amd import ftc
    cap = step.cells.cell_capacity
    n = len(coeff_rows)
    co = np.zeros((6, cap))
    co[:, :n] = np.asarray(coeff_rows).T
    dco = torch.from_numpy(co).to("cuda").reshape(-1)
    out = torch.full((cap,), -1.0, dtype=torch.float64, device="cuda")
    kap = torch.full((cap,), -1.0, dtype=torch.float64, device="cuda") if surface else None
    nrm = torch.full((3 * cap,), -1.0, dtype=torch.float64, device="cuda") if surface else None
    ftc.paraboloid_cell(step.cells, grid, dco, out, kap, nrm)
    torch.cuda.synchronize()
    a = out.cpu().numpy()[:n]
    if not surface:
        return a
    return a, kap.cpu().numpy()[:n], nrm.cpu().numpy().reshape(3, cap)[:, :n].T


def _alpha_gpu(step, grid, coeff_rows):
    return _cell_gpu(step, grid, coeff_rows)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name,nsample", [("sphere_32", 48), ("sh_spheres_128", 32)])
def test_paraboloid_alpha_parity(oracle, name, nsample):
    grid, mesh, step = _run(name)
    g = step.results()
    cells, _, _ = oracle.cell_lists(grid, mesh)
    assert np.array_equal(g["cell_ids"][:g["n_if"]], cells)
    r = oracle.ppic(grid, mesh, cells)
    _, _, fn = oracle.frame_normal(grid, mesh, cells)
    ok = np.nonzero(r["status"] == 0)[0]
    ag = _alpha_gpu(step, grid, r["coeff"])
    assert np.all(np.isfinite(ag[ok])) and np.all((ag[ok] >= -1e-15) & (ag[ok] <= 1 + 1e-15))
    pick = np.random.default_rng(11).choice(ok, min(nsample, len(ok)), replace=False)
    # every cell whose frame normal has a zero or tiny component: the faces of
    # that axis are (almost) parallel to n, the ill-conditioned case
    flat = ok[np.abs(fn[ok]).min(1) < 1e-6]
    pick = np.union1d(pick, flat[:16])
    ao = PB.alpha_cells(fn[pick], r["coeff"][pick], grid.h)
    err = np.abs(ag[pick] - ao).max()
    _say(f"[paraboloid] {name}: {len(cells)} cells, {len(pick)} sampled ({min(len(flat), 16)} with a tiny normal "
         f"component), max |alpha_gpu - alpha_oracle| = {err:.2e}")
    assert err <= ALPHA_TOL


@pytest.mark.timeout(300)
def test_paraboloid_surface_parity(oracle):
    """Curvature and normal integrated over each cell's paraboloid patch:
    sampled cells of the 32^3 sphere (and every one with a tiny normal
    component, up to 16) within 1e-10 relative (the curvature bar), normals
    within 1e-10; the volume fractions of the same call (its finer rule in
    the second direction) match the volume-only call within the alpha bar."""
    grid, mesh, step = _run("sphere_32")
    cells, _, _ = oracle.cell_lists(grid, mesh)
    r = oracle.ppic(grid, mesh, cells)
    _, _, fn = oracle.frame_normal(grid, mesh, cells)
    ok = np.nonzero(r["status"] == 0)[0]
    a1 = _cell_gpu(step, grid, r["coeff"])
    a2, kg, ng = _cell_gpu(step, grid, r["coeff"], surface=True)
    assert np.abs(a1 - a2).max() <= ALPHA_TOL
    pick = np.random.default_rng(12).choice(ok, 24, replace=False)
    flat = ok[np.abs(fn[ok]).min(1) < 1e-6]
    pick = np.union1d(pick, flat[:16])
    ko, no = PB.surface_cells(fn[pick], r["coeff"][pick], grid.h)
    assert np.all(np.isfinite(ko))
    kerr = np.abs(kg[pick] - ko) / np.abs(ko)
    nerr = np.abs(ng[pick] - no).max()
    _say(f"[paraboloid] sphere_32 surface: {len(pick)} cells, kappa rel err {kerr.max():.2e}, normal err {nerr:.2e}")
    assert kerr.max() <= 1e-10 and nerr <= 1e-10


def test_paraboloid_alpha_full_size_against_polyhedral():
    """128^3 sphere, the device's own PPIC coefficients: every cell's alpha
    under its paraboloid is within the fit error of the exact polyhedral
    alpha, and the two total volumes agree to the same order."""
    import torch
    from paper_2505_06932_amd import ftc
    grid, mesh, step = _run("sphere_128")
    out = torch.empty_like(step.alpha_if)
    kap = torch.empty_like(step.alpha_if)
    nrm = torch.empty(3 * step.cells.cell_capacity, dtype=torch.float64, device="cuda")
    ftc.paraboloid_cell(step.cells, grid, step.coeff, out, kap, nrm)
    g = step.results()
    n = g["n_if"]
    ap = out.cpu().numpy()[:n]
    ok = g["status"] == 0
    assert ok.mean() > 0.99
    d = np.abs(ap[ok] - g["alpha_if"][ok])
    _say(f"[paraboloid] sphere_128: |alpha_par - alpha_poly| max {d.max():.2e} median {np.median(d):.2e}")
    assert d.max() < 1e-2 and np.median(d) < 1e-3
    # the curvature averaged over the patch stays close to the same fit's
    # curvature at the frame origin (the noisy front spreads both around 2/R)
    kc = kap.cpu().numpy()[:n][ok]
    fin = np.isfinite(kc)
    rel = np.abs(kc[fin] / g["kappa"][ok][fin] - 1)
    _say(f"[paraboloid] sphere_128: kappa_cell finite {fin.mean():.4f}, |kappa_cell / kappa_origin - 1| median "
         f"{np.median(rel):.2e} q99 {np.quantile(rel, 0.99):.2e}")
    assert fin.mean() > 0.99 and np.median(rel) < 0.02


def test_paraboloid_alpha_preconditions():
    """FTC_EINVAL after a new build without PPIC, and after the learned
    curvature (which runs PPIC for its fallback cells only)."""
    import torch
    from paper_2505_06932_amd import ftc
    grid, mesh, step = _run("sphere_32")
    out = torch.empty_like(step.alpha_if)
    ftc.paraboloid_cell(step.cells, grid, step.coeff, out)
    ftc.build_cell_lists(step.cells, grid, step.mesh)
    with pytest.raises(ftc.FTCError):
        ftc.paraboloid_cell(step.cells, grid, step.coeff, out)
    torch.cuda.synchronize()


def test_failed_fits_give_nan(oracle):
    """A cell whose coefficients are NaN (a failed fit) gets NaN for alpha,
    curvature and normal; its neighbours in the list are unaffected."""
    grid, mesh, step = _run("sphere_32")
    cells, _, _ = oracle.cell_lists(grid, mesh)
    r = oracle.ppic(grid, mesh, cells)
    co = r["coeff"].copy()
    a0, k0, n0 = _cell_gpu(step, grid, co, surface=True)
    bad = [3, 400, len(co) - 1]
    co[bad] = np.nan
    a1, k1, n1 = _cell_gpu(step, grid, co, surface=True)
    assert np.all(np.isnan(a1[bad])) and np.all(np.isnan(k1[bad])) and np.all(np.isnan(n1[bad]))
    keep = np.setdiff1d(np.arange(len(co)), bad)
    assert np.array_equal(a1[keep], a0[keep]) and np.array_equal(k1[keep], k0[keep], equal_nan=True)
    assert np.array_equal(n1[keep], n0[keep], equal_nan=True)


@pytest.mark.timeout(900)
def test_paraboloid_parity_many_cells_perturbed_spheres(oracle):
    """Perturbed spheres on 128^3 (non-convex patches, larger kappa h): the
    volume fraction, the curvature and the normal integrated over the patch,
    on 1,000 seeded cells plus every cell whose frame normal has a tiny
    component, against the oracle (run in a pool of CPU processes): alpha
    within 1e-12, curvature within 1e-10 relative, normal within 1e-10; cells
    whose patch misses the cell are NaN on both sides."""
    grid, mesh, step = _run("sh_spheres_128")
    cells, _, _ = oracle.cell_lists(grid, mesh)
    g = step.results()
    assert np.array_equal(g["cell_ids"][:g["n_if"]], cells)
    r = oracle.ppic(grid, mesh, cells)
    _, _, fn = oracle.frame_normal(grid, mesh, cells)
    ok = np.nonzero(r["status"] == 0)[0]
    pick = np.random.default_rng(13).choice(ok, min(1000, len(ok)), replace=False)
    flat = ok[np.abs(fn[ok]).min(1) < 1e-6]
    pick = np.union1d(pick, flat)
    ag, kg, ng = _cell_gpu(step, grid, r["coeff"], surface=True)
    ao = PB.map_cells("alpha", fn[pick], r["coeff"][pick], grid.h)
    ko, no = PB.map_cells("surface", fn[pick], r["coeff"][pick], grid.h)
    aerr = np.abs(ag[pick] - ao).max()
    miss = np.isnan(ko)
    assert np.array_equal(np.isnan(kg[pick]), miss)
    kerr = (np.abs(kg[pick] - ko) / np.abs(ko))[~miss]
    nerr = np.abs(ng[pick] - no)[~miss].max()
    _say(f"[paraboloid] sh_spheres_128: {len(cells)} cells, {len(pick)} checked ({len(flat)} with a tiny normal "
         f"component, {int(miss.sum())} patches outside their cell): alpha {aerr:.2e}, kappa rel {kerr.max():.2e}, "
         f"normal {nerr:.2e}")
    ne = np.abs(ng[pick] - no).max(1)
    for q in np.argsort(-np.nan_to_num(ne))[:4]:
        c = pick[q]
        _say(f"[paraboloid]   cell {c} (id {cells[c]}): normal err {ne[q]:.2e} kappa rel "
             f"{abs(kg[c] - ko[q]) / abs(ko[q]):.2e} frame n {fn[c].tolist()} coeff {r['coeff'][c].tolist()} "
             f"gpu n {ng[c].tolist()} oracle n {no[q].tolist()}")
    assert aerr <= ALPHA_TOL
    assert kerr.max() <= 1e-10 and nerr <= 1e-10
