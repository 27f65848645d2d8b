"""Pins for the oracle's volume fraction under the local paraboloid (paper
sec. 3.2): the exact plane-cube volume, closed forms for an axis-aligned
paraboloid and a parabolic cylinder (with kinks), the complement rule, cube
symmetries, and agreement with the exact polyhedral alpha on a sphere up to
the fit error."""
import itertools
import math

import numpy as np
import pytest

from oracle import paraboloid as PB
from paper_2505_06932_amd import inputs as I

EZ = np.array([0.0, 0.0, 1.0])


def _plane_cube_volume(g, d):
    """|{q in [0,1]^3 : g.q < d}| by inclusion-exclusion over the corners
    (every g_k non-zero): sum_v (-1)^|v| max(0, d - g.v)^3 / (6 g0 g1 g2),
    after reflecting the axes with g_k < 0."""
    g = np.array(g, dtype=np.float64)
    d = float(d)
    for k in range(3):
        if g[k] < 0.0:
            d -= g[k]
            g[k] = -g[k]
    s = 0.0
    for v in itertools.product((0, 1), repeat=3):
        s += (-1) ** sum(v) * max(0.0, d - float(np.dot(g, v))) ** 3
    return s / (6.0 * g[0] * g[1] * g[2])


def test_plane_matches_inclusion_exclusion():
    rng = np.random.default_rng(3)
    for _ in range(8):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        t1, t2 = PB.duff_frame(n)
        b1, b2, b3 = rng.uniform(-0.4, 0.4), rng.normal() * 0.3, rng.normal() * 0.3
        got = PB.alpha_unit(n, t1, t2, (b1, b2, b3, 0.0, 0.0, 0.0))
        # liquid: n.p - b1 - b2 t1.p - b3 t2.p < 0, i.e. g.p < b1; p = q - 1/2
        g = n - b2 * t1 - b3 * t2
        ref = _plane_cube_volume(g, b1 + 0.5 * g.sum())
        assert got == pytest.approx(ref, abs=1e-13)


def test_duff_frame_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(4)
    for n in [EZ, -EZ, np.array([0.0, 0.6, 0.8]), *(v / np.linalg.norm(v) for v in rng.normal(size=(5, 3)))]:
        t1, t2 = PB.duff_frame(n)
        R = np.stack([t1, t2, n])
        assert np.abs(R @ R.T - np.eye(3)).max() < 1e-15
        assert np.dot(np.cross(t1, t2), n) == pytest.approx(1.0, abs=1e-15)


def test_aligned_paraboloid_inside_the_slab():
    """n = e_z (frame e_x, e_y): the surface stays inside -1/2 < z < 1/2, so
    alpha = integral of (P + 1/2) over the square = b1 + 1/2 + (b4 + b6)/12."""
    t1, t2 = PB.duff_frame(EZ)
    assert np.array_equal(t1, [1.0, 0.0, 0.0]) and np.array_equal(t2, [0.0, 1.0, 0.0])
    b = (0.05, 0.1, -0.2, 0.3, 0.25, -0.1)
    assert PB.alpha_unit(EZ, t1, t2, b) == pytest.approx(0.55 + 0.2 / 12, abs=1e-14)


def test_parabolic_cylinder_with_kinks():
    """zeta = -0.6 + 2 xi^2: the chord length is max(0, 2x^2 - 0.1), zero for
    |x| < sqrt(0.05); alpha = 2 [1/12 - 0.05 - (2/3) x0^3 + 0.1 x0]."""
    t1, t2 = PB.duff_frame(EZ)
    x0 = math.sqrt(0.05)
    ref = 2 * (1 / 12 - 0.05 - 2 / 3 * x0 ** 3 + 0.1 * x0)
    assert PB.alpha_unit(EZ, t1, t2, (-0.6, 0, 0, 2.0, 0, 0)) == pytest.approx(ref, abs=1e-14)
    # the same along eta
    assert PB.alpha_unit(EZ, t1, t2, (-0.6, 0, 0, 0, 0, 2.0)) == pytest.approx(ref, abs=1e-14)


def _random_case(rng):
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    t1, t2 = PB.duff_frame(n)
    b = (rng.uniform(-0.4, 0.4), rng.normal() * 0.3, rng.normal() * 0.3, rng.normal() * 0.2, rng.normal() * 0.2,
         rng.normal() * 0.2)
    return n, t1, t2, b


def test_complement():
    """Above the paraboloid is below the one with normal -n and coefficients
    -b in the same tangents: the two fractions add up to 1."""
    rng = np.random.default_rng(5)
    for _ in range(4):
        n, t1, t2, b = _random_case(rng)
        a = PB.alpha_unit(n, t1, t2, b)
        c = PB.alpha_unit(-n, t1, t2, tuple(-v for v in b))
        assert a + c == pytest.approx(1.0, abs=1e-13)


def test_cube_symmetries():
    """Rotating (or reflecting) the paraboloid by a symmetry of the cube
    leaves alpha unchanged."""
    rng = np.random.default_rng(6)
    n, t1, t2, b = _random_case(rng)
    a0 = PB.alpha_unit(n, t1, t2, b)
    for perm, signs in (((1, 2, 0), (1, 1, 1)), ((2, 1, 0), (-1, 1, 1)), ((0, 1, 2), (1, -1, -1))):
        S = np.zeros((3, 3))
        for r, (c, s) in enumerate(zip(perm, signs)):
            S[r, c] = s
        assert PB.alpha_unit(S @ n, S @ t1, S @ t2, b) == pytest.approx(a0, abs=1e-14)


def test_same_volume_with_the_chord_along_each_axis():
    """A cell of the 32^3 sphere whose nested quadrature needs the slice-area
    kinks: the volume computed with the inner chord along z, x and y (axes
    permuted) agrees to 1e-14."""
    n = np.array([-0.65645707, -0.26770795, -0.70526347])
    n /= np.linalg.norm(n)
    t1, t2 = PB.duff_frame(n)
    b = (0.372184277, -0.0388448336, 0.00384352669, -0.0632620764, -0.000286374076, -0.0634228759)
    vals = []
    for perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        S = np.eye(3)[list(perm)]
        vals.append(PB.alpha_unit(S @ n, S @ t1, S @ t2, b))
    assert max(vals) - min(vals) < 1e-14


def test_sphere_cells_close_to_exact_alpha(oracle):
    """On the 32^3 sphere the paraboloid of each cell's PPIC fit bounds almost
    the same volume as the polyhedral front: sampled cells agree with the
    exact polyhedral alpha to the fit error (well under 1e-2), which a wrong
    frame, unit or sign would not."""
    g, m, _ = I.make_workload("sphere_32", 1)
    cells, _, _ = oracle.cell_lists(g, m)
    alpha, _ = oracle.volume_fraction(g, m)
    r = oracle.ppic(g, m, cells)
    _, _, fn = oracle.frame_normal(g, m, cells)
    pick = np.random.default_rng(7).choice(len(cells), 24, replace=False)
    ap = PB.alpha_cells(fn[pick], r["coeff"][pick], g.h)
    ex = np.asarray(alpha).reshape(-1)[np.asarray(cells)[pick]]
    err = np.abs(ap - ex)
    assert err.max() < 1e-2 and np.median(err) < 2e-3


# ------------------------------------------------------------ surface integrals
def _plane_section_area(g, d):
    """Area of {g.q = d} inside [0,1]^3: |g| times the derivative in d of the
    inclusion-exclusion volume, sum_v (-1)^|v| max(0, d - g.v)^2 / (2 g0 g1 g2)."""
    g = np.array(g, dtype=np.float64)
    d = float(d)
    gn = np.linalg.norm(g)
    for k in range(3):
        if g[k] < 0.0:
            d -= g[k]
            g[k] = -g[k]
    s = 0.0
    for v in itertools.product((0, 1), repeat=3):
        s += (-1) ** sum(v) * max(0.0, d - float(np.dot(g, v))) ** 2
    return gn * s / (2.0 * g[0] * g[1] * g[2])


def test_plane_patch_area_normal_and_zero_curvature():
    rng = np.random.default_rng(8)
    for _ in range(5):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        t1, t2 = PB.duff_frame(n)
        b1, b2, b3 = rng.uniform(-0.3, 0.3), rng.normal() * 0.3, rng.normal() * 0.3
        area, K, N = PB.surface_unit(n, t1, t2, (b1, b2, b3, 0.0, 0.0, 0.0))
        g = n - b2 * t1 - b3 * t2
        assert area == pytest.approx(_plane_section_area(g, b1 + 0.5 * g.sum()), abs=1e-12)
        assert K == 0.0
        Nw = N[0] * t1 + N[1] * t2 + N[2] * n
        assert np.abs(Nw / np.linalg.norm(Nw) - g / np.linalg.norm(g)).max() < 1e-13


def test_aligned_paraboloid_surface_integrals(oracle):
    """n = e_z and a surface inside the slab: R is the unit square, so the
    area and K are plain double integrals over it (no kinks), with the
    curvature at each point taken from the PPIC oracle's curvature of the
    paraboloid re-expanded about that point (Taylor coefficients P, P_xi,
    P_eta and the unchanged second-order ones).  The normal integral is
    (-b1, -b2, 1) by the symmetry of the square."""
    from scipy import integrate
    t1, t2 = PB.duff_frame(EZ)
    b = (0.05, 0.1, -0.2, 0.3, 0.25, -0.1)
    area, K, N = PB.surface_unit(EZ, t1, t2, b)

    def taylor(x, y):
        p = b[0] + b[1] * x + b[2] * y + b[3] * x * x + b[4] * x * y + b[5] * y * y
        px, py = b[1] + 2 * b[3] * x + b[4] * y, b[2] + b[4] * x + 2 * b[5] * y
        return p, px, py

    def w(x, y):
        _, px, py = taylor(x, y)
        return math.sqrt(1 + px * px + py * py)

    def kw(x, y):
        p, px, py = taylor(x, y)
        return oracle.kappa_of([p, px, py, b[3], b[4], b[5]]) * w(x, y)

    ref_k = integrate.dblquad(lambda y, x: kw(x, y), -0.5, 0.5, -0.5, 0.5, epsabs=1e-14, epsrel=1e-14)[0]
    ref_a = integrate.dblquad(lambda y, x: w(x, y), -0.5, 0.5, -0.5, 0.5, epsabs=1e-14, epsrel=1e-14)[0]
    assert K == pytest.approx(ref_k, abs=1e-12)
    assert area == pytest.approx(ref_a, abs=1e-12)
    assert np.abs(N - np.array([-0.1, 0.2, 1.0])).max() < 1e-13


def test_surface_integrals_under_cube_symmetries():
    rng = np.random.default_rng(9)
    n, t1, t2, b = _random_case(rng)
    a0, k0, n0 = PB.surface_unit(n, t1, t2, b)
    for perm, signs in (((1, 2, 0), (1, 1, 1)), ((2, 1, 0), (-1, 1, 1))):
        S = np.zeros((3, 3))
        for r, (c, s) in enumerate(zip(perm, signs)):
            S[r, c] = s
        a1, k1, n1 = PB.surface_unit(S @ n, S @ t1, S @ t2, b)
        assert a1 == pytest.approx(a0, abs=1e-12) and k1 == pytest.approx(k0, abs=1e-12)
        assert np.abs(n1 - n0).max() < 1e-12  # local components: the frame moved with the cube


def test_sphere_cell_curvature_close_to_frame_curvature(oracle):
    """On the 32^3 sphere the curvature averaged over each cell's paraboloid
    patch stays within a few per cent of the fit's curvature at the frame
    origin (both near 2/R = 8), and the averaged normal within a few degrees
    of the fitted normal."""
    g, m, _ = I.make_workload("sphere_32", 1)
    cells, _, _ = oracle.cell_lists(g, m)
    r = oracle.ppic(g, m, cells)
    _, _, fn = oracle.frame_normal(g, m, cells)
    pick = np.random.default_rng(10).choice(len(cells), 12, replace=False)
    kc, nc = PB.surface_cells(fn[pick], r["coeff"][pick], g.h)
    assert np.all(np.abs(kc / r["kappa"][pick] - 1) < 0.05)
    assert np.all(np.einsum("ij,ij->i", nc, r["normal"][pick]) > np.cos(np.radians(5)))


def test_unconverged_quadrature_raises():
    """The oracle's quadratures fail loudly: an integral that QUADPACK cannot
    bring within the stated error bound (here a kink it is not told about,
    with a single subinterval allowed) raises instead of returning a value."""
    with pytest.raises(PB.QuadratureError):
        PB._quad(lambda x: abs(x - 0.3), -0.5, 0.5, epsabs=1e-14, epsrel=1e-14, limit=1)
    # told about the kink, the same integral is exact
    assert abs(PB._quad(lambda x: abs(x - 0.3), -0.5, 0.5, points=[0.3], epsabs=1e-14, epsrel=1e-14)
               - (0.8 ** 2 + 0.2 ** 2) / 2) < 1e-15
