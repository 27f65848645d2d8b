"""Pins for the oracle's surface-tension face flux (paper sec. 3.3,
Eq. mwi_disc): the force balance against the pressure term of the same
flux, a slab worked by hand, mirror antisymmetry, and zero curvature."""
import numpy as np
import pytest

from oracle import balanced as B
from paper_2505_06932_amd import inputs as I

SIGMA = 0.07


def _sphere(oracle):
    g, m, _ = I.make_workload("sphere_32", 1)
    cells, _, _ = oracle.cell_lists(g, m)
    alpha, _ = oracle.volume_fraction(g, m)
    r = oracle.ppic(g, m, cells)
    bid, kb, _ = oracle.csf_band(g, alpha, cells, r["kappa"], r["normal"], 1.0)
    return g, np.asarray(alpha).reshape(-1), np.asarray(cells), r, bid, kb


def _faces(g, ids):
    """(P, Q, d) of the six faces of each cell, in slot order."""
    st = (1, g.nx, g.nx * g.ny)
    out = []
    for c in np.asarray(ids).tolist():
        for d in range(3):
            out.append((c - st[d], c, d))
            out.append((c, c + st[d], d))
    return out


def _pressure_term(g, p, rho, faces):
    """The pressure term of the flux, (p_Q - p_P)/h - rho*_f/2 (grad p_P /
    rho_P + grad p_Q / rho_Q) . n_f, with central-difference gradients and
    the harmonic face density (sec. 2), written out here on its own."""
    st = (1, g.nx, g.nx * g.ny)
    out = np.empty(len(faces))
    for i, (P, Q, d) in enumerate(faces):
        gP = (p[P + st[d]] - p[P - st[d]]) / (2 * g.h)
        gQ = (p[Q + st[d]] - p[Q - st[d]]) / (2 * g.h)
        rf = 2 * rho[P] * rho[Q] / (rho[P] + rho[Q])
        out[i] = (p[Q] - p[P]) / g.h - rf / 2 * (gP / rho[P] + gQ / rho[Q])
    return out


@pytest.mark.parametrize("rho_a,rho_b", [(1.0, 1.0), (1.0, 1000.0), (850.0, 1.2)])
def test_force_balance_with_constant_curvature(oracle, rho_a, rho_b):
    """With one curvature k0 in every interfacial and band cell, the
    surface-tension term equals the pressure term of the same flux for the
    Laplace pressure p = sigma k0 alpha, face by face: the force balance of
    the discretisation (sec. 3.3)."""
    g, alpha, cells, r, bid, kb = _sphere(oracle)
    k0 = 8.0
    fi, fb = B.surface_tension_face_flux(g, alpha, cells, np.full(len(cells), k0), bid, np.full(len(bid), k0),
                                         rho_a, rho_b, SIGMA)
    rho = rho_a + alpha * (rho_b - rho_a)
    ref_i = _pressure_term(g, SIGMA * k0 * alpha, rho, _faces(g, cells)).reshape(-1, 6)
    ref_b = _pressure_term(g, SIGMA * k0 * alpha, rho, _faces(g, bid)).reshape(-1, 6)
    scale = SIGMA * k0 / g.h
    assert np.abs(fi - ref_i).max() <= 1e-13 * scale
    assert np.abs(fb - ref_b).max() <= 1e-13 * scale
    # the term is not trivially zero: interfacial faces carry the jump
    assert np.abs(fi).max() > 0.1 * scale


def _slab():
    """alpha depends on i only: 0 for i <= 3, 0.3 at i = 4, 1 for i >= 5, in
    a 10^3 grid.  Interfacial cells (4, j, k) for j, k in 2..7; the band is
    their face neighbours that are not interfacial."""
    g = I.Grid(10, 10, 10, 0.0, 0.0, 0.0, 0.1)
    a = np.zeros((g.nz, g.ny, g.nx))
    a[:, :, 4] = 0.3
    a[:, :, 5:] = 1.0
    lin = lambda i, j, k: i + g.nx * (j + g.ny * k)
    cells = sorted(lin(4, j, k) for j in range(2, 8) for k in range(2, 8))
    cs = set(cells)
    band = set()
    for c in cells:
        for s in (1, -1, g.nx, -g.nx, g.nx * g.ny, -g.nx * g.ny):
            if c + s not in cs:
                band.add(c + s)
    return g, a.reshape(-1), np.array(cells), np.array(sorted(band)), lin


def test_slab_by_hand():
    """Curvature 2 in every interfacial and band cell, sigma / h = 1.
    Face (4|5) along x, interior j, k: kbar 2, g_4 = 1/(2h), g_5 = 0.7/(2h),
    rho*/2 (1/rho_4 + 0.7/rho_5) = (rho_5 + 0.7 rho_4)/(rho_4 + rho_5), so
    Phi = 1.4 - (rho_5 + 0.7 rho_4)/(rho_4 + rho_5).  Face (3|4):
    Phi = 0.6 - (0.3 rho_4 + rho_3)/(rho_3 + rho_4).  Face (2|3) (cell 2 is
    outside the band): Phi = -0.15.  Faces along y inside the slab: 0."""
    g, a, cells, band, lin = _slab()
    sigma = g.h
    ra, rb = 1.0, 1000.0
    fi, fb = B.surface_tension_face_flux(g, a, cells, np.full(len(cells), 2.0), band, np.full(len(band), 2.0),
                                         ra, rb, sigma)
    rows_i = {c: k for k, c in enumerate(cells.tolist())}
    rows_b = {c: k for k, c in enumerate(band.tolist())}
    r3, r4, r5 = ra, ra + 0.3 * (rb - ra), rb
    c4 = lin(4, 5, 5)
    assert fi[rows_i[c4], 1] == pytest.approx(1.4 - (r5 + 0.7 * r4) / (r4 + r5), rel=1e-14)
    assert fi[rows_i[c4], 0] == pytest.approx(0.6 - (0.3 * r4 + r3) / (r3 + r4), rel=1e-14)
    assert fb[rows_b[lin(3, 5, 5)], 0] == pytest.approx(-0.15, rel=1e-14)
    assert fi[rows_i[c4], 2] == 0.0 and fi[rows_i[c4], 3] == 0.0
    # equal densities: 1.4 - 0.85 and 0.6 - 0.65
    fi1, _ = B.surface_tension_face_flux(g, a, cells, np.full(len(cells), 2.0), band, np.full(len(band), 2.0),
                                         5.0, 5.0, sigma)
    assert fi1[rows_i[c4], 1] == pytest.approx(0.55, rel=1e-14)
    assert fi1[rows_i[c4], 0] == pytest.approx(-0.05, rel=1e-13)


def test_mirror_antisymmetry(oracle):
    """Reflecting the fields in x (i -> nx-1-i) flips the sign of every
    x-face value and swaps the two x slots; y and z faces keep their values.
    PPIC curvatures, density ratio 1000."""
    g, alpha, cells, r, bid, kb = _sphere(oracle)
    nx, ny, nz = g.nx, g.ny, g.nz
    a3 = alpha.reshape(nz, ny, nx)
    am = a3[:, :, ::-1].reshape(-1)

    def mirror(ids):
        ids = np.asarray(ids)
        i, j, k = ids % nx, (ids // nx) % ny, ids // (nx * ny)
        return (nx - 1 - i) + nx * (j + ny * k)

    ci, cb = mirror(cells), mirror(bid)
    oi, ob = np.argsort(ci), np.argsort(cb)
    f0i, f0b = B.surface_tension_face_flux(g, alpha, cells, r["kappa"], bid, kb, 1.0, 1000.0, SIGMA)
    f1i, f1b = B.surface_tension_face_flux(g, am, ci[oi], r["kappa"][oi], cb[ob], kb[ob], 1.0, 1000.0, SIGMA)
    for f0, f1, o in ((f0i, f1i, oi), (f0b, f1b, ob)):
        g0 = f0[o]
        assert np.array_equal(f1[:, 0], -g0[:, 1]) and np.array_equal(f1[:, 1], -g0[:, 0])
        assert np.array_equal(f1[:, 2:], g0[:, 2:])


def test_zero_curvature_gives_zero(oracle):
    g, alpha, cells, r, bid, kb = _sphere(oracle)
    fi, fb = B.surface_tension_face_flux(g, alpha, cells, np.zeros(len(cells)), bid, np.zeros(len(bid)), 1.0, 10.0,
                                         SIGMA)
    assert not fi.any() and not fb.any()


def test_slab_face_curvature_is_the_mean_of_the_carrying_cells():
    """Curvature 2 in the interfacial cells and 4 in the band, equal
    densities, sigma / h = 1.  Face (4|5): kbar_f = 3, so
    Phi = 3 * 0.7 - (2 * 0.5 + 4 * 0.35) / 2 = 0.9.  Face (2|3): only
    cell 3 carries a curvature, kbar_f = 4, alpha is equal on both sides,
    Phi = -(4 * 0.15) / 2 = -0.3."""
    g, a, cells, band, lin = _slab()
    fi, fb = B.surface_tension_face_flux(g, a, cells, np.full(len(cells), 2.0), band, np.full(len(band), 4.0),
                                         3.0, 3.0, g.h)
    rows_i = {c: k for k, c in enumerate(cells.tolist())}
    rows_b = {c: k for k, c in enumerate(band.tolist())}
    assert fi[rows_i[lin(4, 5, 5)], 1] == pytest.approx(0.9, rel=1e-14)
    assert fb[rows_b[lin(5, 5, 5)], 0] == fi[rows_i[lin(4, 5, 5)], 1]
    assert fb[rows_b[lin(3, 5, 5)], 0] == pytest.approx(-0.3, rel=1e-14)
