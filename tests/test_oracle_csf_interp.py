"""Pins for the oracle's CSF source (paper Eq. csf) and the
divergence-preserving interpolation (paper sec. 3.1)."""
import math

import numpy as np
import pytest

from paper_2505_06932_amd import inputs as I


# ------------------------------------------------------------------ CSF
def test_csf_is_sigma_kappa_central_gradient(oracle):
    """Element-wise sigma * kappa * grad(alpha) with a central difference;
    on a linear alpha ramp the gradient is exact."""
    g = I.Grid(10, 9, 8, 0.0, 0.0, 0.0, 0.1)
    z, y, x = np.indices((g.nz, g.ny, g.nx)) * g.h
    alpha = 0.3 * x - 0.7 * y + 0.2 * z + 0.1
    ids = np.array([1 + g.nx * (1 + g.ny * 1), 5 + g.nx * (4 + g.ny * 3), 8 + g.nx * (7 + g.ny * 6)])
    kap = np.array([1.5, -2.0, 0.25])
    f = oracle.csf(g, alpha, ids, kap, 0.072)
    ref = 0.072 * kap[:, None] * np.array([0.3, -0.7, 0.2])[None, :]
    assert np.abs(f - ref).max() <= 1e-14


# ------------------------------------------------------------ BAND mode
def _lin(g, i, j, k):
    return i + g.nx * (j + g.ny * k)


def test_band_set_is_face_neighbours_minus_interfacial(oracle):
    """The band is exactly the cells sharing a face with an interfacial
    cell and not interfacial, in ascending linear id (set computed here by
    brute force over the 6 face offsets)."""
    g, m, c = I.make_workload("sphere_32", 1)
    cells, _, _ = oracle.cell_lists(g, m)
    alpha, _ = oracle.volume_fraction(g, m)
    r = oracle.ppic(g, m, cells)
    bid, kb, f = oracle.csf_band(g, alpha, cells, r["kappa"], r["normal"], 1.0)
    cs = set(int(x) for x in cells)
    ref = set()
    for cl in cs:
        i, j, k = cl % g.nx, (cl // g.nx) % g.ny, cl // (g.nx * g.ny)
        for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            n = _lin(g, i + di, j + dj, k + dk)
            if n not in cs:
                ref.add(n)
    assert list(bid) == sorted(ref)
    # on a sphere every kappa is near 2/R, so every weighted mean is too
    assert np.all(np.abs(kb * 0.25 / 2 - 1) < 0.02)


def test_band_weighted_mean_by_hand(oracle):
    """Two interfacial cells Q1 = (4,4,4) with kappa 1, Q2 = (5,4,4) with
    kappa 3, both with normal +z.  Band cell P = (4,4,5) (above Q1): offsets
    s1 = (0,0,-1), s2 = (1,0,-1), weights 1 and 1/sqrt(2).  Band cell
    (3,4,4) (beside Q1): only Q1 is a neighbour... and Q2 is not (two cells
    away); its weight |s.n| = 0, so the plain mean, 1."""
    g = I.Grid(10, 10, 10, 0.0, 0.0, 0.0, 0.1)
    cells = np.array([_lin(g, 4, 4, 4), _lin(g, 5, 4, 4)])
    kap = np.array([1.0, 3.0])
    nrm = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    alpha = np.zeros((g.nz, g.ny, g.nx))
    bid, kb, f = oracle.csf_band(g, alpha, cells, kap, nrm, 1.0)
    got = dict(zip(bid.tolist(), kb.tolist()))
    w2 = 1 / math.sqrt(2)
    assert got[_lin(g, 4, 4, 5)] == pytest.approx((1 + 3 * w2) / (1 + w2), rel=1e-15)
    assert got[_lin(g, 5, 4, 5)] == pytest.approx((3 + 1 * w2) / (1 + w2), rel=1e-15)
    assert got[_lin(g, 3, 4, 4)] == 1.0
    assert got[_lin(g, 6, 4, 4)] == 3.0
    # (4,5,4) touches both by an edge or face, all in the plane z = const:
    # every weight vanishes, plain mean of 1 and 3
    assert got[_lin(g, 4, 5, 4)] == 2.0
    assert len(bid) == 10  # 6 + 6 face neighbours minus the two cells themselves
    assert np.all(f == 0.0)  # alpha is flat


def test_band_constant_curvature_and_nan_handling(oracle):
    """A constant curvature field is reproduced (weighted mean of equal
    values); a NaN curvature is left out, and a band cell whose only
    interfacial neighbour has NaN curvature gets NaN; the source is
    sigma kappa_bar times the central gradient."""
    g, m, c = I.make_workload("sphere_32", 2)
    cells, _, _ = oracle.cell_lists(g, m)
    alpha, _ = oracle.volume_fraction(g, m)
    r = oracle.ppic(g, m, cells)
    kap = np.full(len(cells), 3.25)
    bid, kb, f = oracle.csf_band(g, alpha, cells, kap, r["normal"], 0.5)
    # a weighted mean of at most 26 equal values: within (2 n + 2) unit
    # roundoffs of the value
    assert np.all(np.abs(kb - 3.25) <= 54 * 2.0 ** -53 * 3.25)
    a = alpha.reshape(-1)
    gx = (a[bid + 1] - a[bid - 1]) / (2 * g.h)
    gy = (a[bid + g.nx] - a[bid - g.nx]) / (2 * g.h)
    gz = (a[bid + g.nx * g.ny] - a[bid - g.nx * g.ny]) / (2 * g.h)
    assert np.array_equal(f, 0.5 * kb[:, None] * np.stack([gx, gy, gz], 1))
    g2 = I.Grid(8, 8, 8, 0.0, 0.0, 0.0, 0.125)
    one = np.array([_lin(g2, 3, 3, 3)])
    bid2, kb2, _ = oracle.csf_band(g2, np.zeros((8, 8, 8)), one, np.array([np.nan]), np.array([[0.0, 0, 1]]), 1.0)
    assert len(bid2) == 6 and np.all(np.isnan(kb2))
    two = np.array([_lin(g2, 3, 3, 3), _lin(g2, 3, 3, 4)])
    bid3, kb3, _ = oracle.csf_band(g2, np.zeros((8, 8, 8)), two, np.array([np.nan, 2.0]),
                                   np.array([[0.0, 0, 1], [0.0, 0, 1]]), 1.0)
    got = dict(zip(bid3.tolist(), kb3.tolist()))
    assert got[_lin(g2, 3, 3, 5)] == 2.0       # above the finite one
    assert math.isnan(got[_lin(g2, 3, 3, 2)])  # below the NaN one, the finite one two cells away
    assert got[_lin(g2, 4, 3, 3)] == 2.0       # beside the NaN one, diagonal to the finite one


def test_csf_sphere_force_points_inward_with_magnitude(oracle):
    """On a sphere the CSF force in interfacial cells points to the centre;
    summed over all cells, sum |S| h^3 over interfacial cells stays within the
    expected range of sigma * kappa * area (only part of grad alpha sits in
    interfacial cells)."""
    g, m, c = I.make_workload("sphere_32", 0)
    alpha, isif = oracle.volume_fraction(g, m)
    cells = np.flatnonzero(isif.ravel())
    r = oracle.ppic(g, m, cells)
    f = oracle.csf(g, alpha, cells, r["kappa"], 1.0)
    n = g.nx
    ctr = np.stack([(cells % n + 0.5), ((cells // n) % n + 0.5), (cells // (n * n) + 0.5)], 1) * g.h
    rad = (ctr - c) / np.linalg.norm(ctr - c, axis=1, keepdims=True)
    mag = np.linalg.norm(f, axis=1)
    big = mag > 0.2 * mag.max()
    assert np.all(np.einsum("ij,ij->i", f[big], rad[big]) < 0)
    R = 0.25
    total = mag.sum() * g.h ** 3
    assert 0.3 * (2 / R) * 4 * math.pi * R * R < total < 1.2 * (2 / R) * 4 * math.pi * R * R


# ------------------------------------------------------------ interpolation
GRID = I.Grid(12, 11, 10, -0.2, 0.1, 0.3, 0.07)


def _interior_points(grid, n, rng):
    lo = np.array([grid.x0, grid.y0, grid.z0]) + 1.0 * grid.h
    hi = np.array([grid.x0 + (grid.nx - 1) * grid.h, grid.y0 + (grid.ny - 1) * grid.h,
                   grid.z0 + (grid.nz - 1) * grid.h])
    return lo + (hi - lo) * rng.uniform(0, 1, (n, 3))


def test_uniform_field_exact(oracle):
    rng = np.random.default_rng(0)
    u0 = np.array([0.3, -1.7, 2.2])
    U, V, W = I.uniform_face_velocity(GRID, u0)
    p = _interior_points(GRID, 500, rng)
    u = oracle.interp(GRID, p[:, 0], p[:, 1], p[:, 2], U, V, W)
    assert np.abs(u - u0).max() <= 4e-16 * np.abs(u0).max()


@pytest.mark.parametrize("seed", range(3))
def test_affine_field_exact(oracle, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=3)
    B = rng.normal(size=(3, 3))
    U, V, W = I.affine_face_velocity(GRID, c, B)
    p = _interior_points(GRID, 500, rng)
    u = oracle.interp(GRID, p[:, 0], p[:, 1], p[:, 2], U, V, W)
    ref = c[None, :] + p @ B.T
    assert np.abs(u - ref).max() <= 1e-13


@pytest.mark.parametrize("seed", range(3))
def test_divergence_equals_discrete_cell_divergence(oracle, seed):
    """d(u)/dx + d(v)/dy + d(w)/dz of the interpolant, anywhere in a cell, is
    the cell's discrete divergence.  Derivatives by central differences, exact
    here because the polynomial is at most quadratic in each coordinate."""
    rng = np.random.default_rng(seed)
    U = rng.normal(size=(GRID.nz, GRID.ny, GRID.nx + 1))
    V = rng.normal(size=(GRID.nz, GRID.ny + 1, GRID.nx))
    W = rng.normal(size=(GRID.nz + 1, GRID.ny, GRID.nx))
    h = GRID.h
    for _ in range(40):
        ijk = rng.integers(1, [GRID.nx - 1, GRID.ny - 1, GRID.nz - 1])
        i, j, k = ijk
        lo = np.array([GRID.x0 + i * h, GRID.y0 + j * h, GRID.z0 + k * h])
        p = lo + h * rng.uniform(0.2, 0.8, 3)
        s = 0.1 * h
        div = 0.0
        for d in range(3):
            e = np.zeros(3)
            e[d] = s
            up = oracle.interp_in_cell(GRID, ijk, p + e, U, V, W)
            um = oracle.interp_in_cell(GRID, ijk, p - e, U, V, W)
            div += (up[d] - um[d]) / (2 * s)
        ddiv = (U[k, j, i + 1] - U[k, j, i] + V[k, j + 1, i] - V[k, j, i] + W[k + 1, j, i] - W[k, j, i]) / h
        assert abs(div - ddiv) <= 1e-9 * max(1.0, abs(ddiv))


def test_normal_component_continuous_across_faces(oracle):
    rng = np.random.default_rng(9)
    U = rng.normal(size=(GRID.nz, GRID.ny, GRID.nx + 1))
    V = rng.normal(size=(GRID.nz, GRID.ny + 1, GRID.nx))
    W = rng.normal(size=(GRID.nz + 1, GRID.ny, GRID.nx))
    h = GRID.h
    for _ in range(30):
        i, j, k = rng.integers(1, [GRID.nx - 2, GRID.ny - 2, GRID.nz - 2])
        lo = np.array([GRID.x0 + i * h, GRID.y0 + j * h, GRID.z0 + k * h])
        for d in range(3):
            p = lo + h * rng.uniform(0.1, 0.9, 3)
            p[d] = lo[d] + h  # the upper face of (i, j, k)
            nxt = np.array([i, j, k])
            nxt[d] += 1
            a = oracle.interp_in_cell(GRID, (i, j, k), p, U, V, W)
            b = oracle.interp_in_cell(GRID, nxt, p, U, V, W)
            assert abs(a[d] - b[d]) <= 1e-13


def test_psi_field_second_order_and_divergence_free(oracle):
    """On the face-averaged stream-function field the interpolant converges
    to the continuous velocity at second order, and its cell divergence is
    zero to rounding."""
    errs = []
    rng = np.random.default_rng(4)
    p0 = rng.uniform(0.2, 0.8, (400, 3))
    for n in (32, 64, 128):
        g = I.Grid(n, n, n, 0.0, 0.0, 0.0, 1.0 / n)
        U, V, W = I.psi_face_velocity(g)
        u = oracle.interp(g, p0[:, 0], p0[:, 1], p0[:, 2], U, V, W)
        ex = np.stack(I.psi_velocity_exact(p0[:, 0], p0[:, 1], p0[:, 2]), 1)
        errs.append(np.abs(u - ex).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 1.7), (errs, order)


def test_outside_margin_rejected(oracle):
    U, V, W = I.uniform_face_velocity(GRID, [1, 0, 0])
    with pytest.raises(oracle.OracleError):
        oracle.interp(GRID, np.array([GRID.x0 + 0.5 * GRID.h]), np.array([0.5]), np.array([0.6]), U, V, W)
