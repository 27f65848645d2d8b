"""Volume fraction under the local paraboloid (paper section 3.2: alpha is the
volume of the intersection of the cell with the region below the fitted
paraboloid, over the cell volume): the plain CPU definition the GPU kernel is
checked against.  Test infrastructure only.

The paraboloid is the one the PPIC fit returns for a cell: in the frame
(t1, t2, n) with origin at the cell centre x_c, local coordinates
xi = t1.(x - x_c), eta = t2.(x - x_c), zeta = n.(x - x_c), the surface is
zeta = a1 + a2 xi + a3 eta + a4 xi^2 + a5 xi eta + a6 eta^2 (world units),
and the liquid (alpha = 1 side, n points out of it) lies below it.  The frame
is the PPIC frame: n the area-weighted normal of the front vertex closest to
the cell centre, (t1, t2) the branchless orthonormal basis of Duff et al.
(JCGT 2017) completing it.

Definition used here, written out directly: in cell units p = (x - x_c)/h,
the cell is the cube [-1/2, 1/2]^3 and the liquid is F(p) < 0 with
F(p) = n.p - Pc(t1.p, t2.p), Pc the paraboloid in cell units
(a1/h, a2, a3, a4 h, a5 h, a6 h).  Then

    alpha = integral over x in [-1/2, 1/2] of
            integral over y in [-1/2, 1/2] of |{z in [-1/2, 1/2] : F < 0}| dy dx,

the inner length from the two roots of the quadratic F(x, y, .) in z.  Both
integrals are adaptive Gauss-Kronrod quadratures (scipy's QUADPACK); the
inner one is told the y at which its integrand has a kink (F(x, y, -+1/2) =
0, or a double root in z), the outer one the x at which those kink curves
meet the cube edges, each other, or turn along y; all are roots of
quadratics.  Accurate to about 1e-15 on the unit cube.

Every quadrature here goes through _quad, which fails loudly: QUADPACK's own
estimate of the absolute error of each integral must not exceed
QUAD_ERR_BOUND (1e-13 in cell units, an order below the 1e-12 to which the
GPU's alpha is compared), or else the same integral over a refined
partition must agree with it within that bound; otherwise the oracle
raises QuadratureError instead of returning an unconverged value.
"""
from __future__ import annotations

import os

import numpy as np
from scipy import integrate

TOL = 1e-14
QUAD_ERR_BOUND = 1e-13


class QuadratureError(RuntimeError):
    """A quadrature of this oracle did not reach its stated accuracy."""


def _quad(f, a, b, points=None, **kw):
    """integrate.quad with its error estimate checked: the value, or
    QuadratureError.  QUADPACK stopping short of `tol` because of round-off
    (its return code 2) is accepted when the estimate stays in bound.  Its
    estimate is pessimistic where the integrand is itself a quadrature
    (noise at the 1e-16 level between nearby abscissae), so an estimate above
    the bound is checked once more: the integral is recomputed as the sum of
    separate quadratures over the breakpoint intervals, each split at its
    midpoint, and the value is accepted only if both results are finite and
    agree within QUAD_ERR_BOUND."""
    pts = sorted(p for p in (points or []) if a < p < b)
    r = integrate.quad(f, a, b, points=pts or None, full_output=1, **kw)
    val, err = r[0], r[1]
    if np.isfinite(val) and err <= QUAD_ERR_BOUND:
        return val
    cuts = [a] + pts + [b]
    fine = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        fine += [lo, 0.5 * (lo + hi)]
    fine.append(b)
    check = 0.0
    for lo, hi in zip(fine[:-1], fine[1:]):
        if hi > lo:
            check += integrate.quad(f, lo, hi, full_output=1, **kw)[0]
    if np.isfinite(val) and np.isfinite(check) and abs(check - val) <= QUAD_ERR_BOUND:
        return val
    msg = r[3] if len(r) > 3 else ""
    raise QuadratureError(f"quadrature over [{a}, {b}] gave {val!r} with error estimate {err:.3e} and "
                          f"{check!r} over a refined partition (bound {QUAD_ERR_BOUND:.0e}): {msg}")


def duff_frame(n):
    """Tangents (t1, t2) completing the unit vector n to a right-handed
    orthonormal frame, by the branchless construction of Duff et al."""
    n = np.asarray(n, dtype=np.float64)
    s = np.copysign(1.0, n[2])
    a = -1.0 / (s + n[2])
    b = n[0] * n[1] * a
    return (np.array([1.0 + s * n[0] * n[0] * a, s * b, -s * n[0]]),
            np.array([b, s + n[1] * n[1] * a, -n[1]]))


def _roots(qa, qb, qc):
    """Real roots of qa t^2 + qb t + qc (the linear case too)."""
    if qa == 0.0:
        return [-qc / qb] if qb != 0.0 else []
    d = qb * qb - 4.0 * qa * qc
    if d < 0.0:
        return []
    q = -0.5 * (qb + np.copysign(np.sqrt(d), qb))
    out = [q / qa]
    if q != 0.0:
        out.append(qc / q)
    return out


class _Quadric:
    """F(p) = p^T M p + g.p + f0 for the paraboloid in cell units."""

    def __init__(self, n, t1, t2, b):
        b1, b2, b3, b4, b5, b6 = (float(v) for v in b)
        n, t1, t2 = (np.asarray(v, dtype=np.float64) for v in (n, t1, t2))
        self.M = -(b4 * np.outer(t1, t1) + 0.5 * b5 * (np.outer(t1, t2) + np.outer(t2, t1)) + b6 * np.outer(t2, t2))
        self.g = n - b2 * t1 - b3 * t2
        self.f0 = -b1

    def z_coeffs(self, x, y):
        """F(x, y, z) = A z^2 + B z + C."""
        M, g = self.M, self.g
        A = M[2, 2]
        B = 2.0 * (M[0, 2] * x + M[1, 2] * y) + g[2]
        C = M[0, 0] * x * x + 2.0 * M[0, 1] * x * y + M[1, 1] * y * y + g[0] * x + g[1] * y + self.f0
        return A, B, C

    def z_length(self, x, y):
        """|{z in [-1/2, 1/2] : F(x, y, z) < 0}|."""
        A, B, C = self.z_coeffs(x, y)
        cuts = sorted([-0.5, 0.5] + [r for r in _roots(A, B, C) if -0.5 < r < 0.5])
        s = 0.0
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            zm = 0.5 * (lo + hi)
            if (A * zm + B) * zm + C < 0.0:
                s += hi - lo
        return s

    def y_kinks(self, x):
        """y in (-1/2, 1/2) where the z-length may have a kink: F(x, y, -+1/2)
        = 0, or F(x, y, .) has a double root."""
        M, g = self.M, self.g
        out = []
        for z in (-0.5, 0.5):
            out += _roots(M[1, 1], 2.0 * M[0, 1] * x + 2.0 * M[1, 2] * z + g[1],
                          M[0, 0] * x * x + M[2, 2] * z * z + 2.0 * M[0, 2] * x * z + g[0] * x + g[2] * z + self.f0)
        A = M[2, 2]
        b1, b0 = 2.0 * M[1, 2], 2.0 * M[0, 2] * x + g[2]
        c2, c1, c0 = M[1, 1], 2.0 * M[0, 1] * x + g[1], M[0, 0] * x * x + g[0] * x + self.f0
        out += _roots(b1 * b1 - 4.0 * A * c2, 2.0 * b1 * b0 - 4.0 * A * c1, b0 * b0 - 4.0 * A * c0)
        return sorted(v for v in out if -0.5 < v < 0.5)


    def x_kinks(self):
        """x in (-1/2, 1/2) where the area of the slice x = const may have a
        kink: where the curves of y_kinks meet the edges y = -+1/2, have a
        tangent along y, or meet each other.  Each is a root of a quadratic
        in x:
          * F = 0 on a cube edge along x (y, z = -+1/2);
          * a double root in z on a face y = -+1/2;
          * F(x, ., z0) = 0 (z0 = -+1/2) tangent along y;
          * the double-root curve tangent along y;
          * the double root at z0 (F = dF/dz = 0 there);
          * F(x, y, -1/2) = F(x, y, 1/2) = 0 (then dF/dz vanishes at z = 0)."""
        M, g, f0 = self.M, self.g, self.f0
        A = M[2, 2]
        out = []
        for y in (-0.5, 0.5):
            for z in (-0.5, 0.5):
                out += _roots(M[0, 0], 2 * M[0, 1] * y + 2 * M[0, 2] * z + g[0],
                              M[1, 1] * y * y + 2 * M[1, 2] * y * z + M[2, 2] * z * z + g[1] * y + g[2] * z + f0)
            # B = 2 M02 x + (2 M12 y + g2), C = M00 x^2 + (2 M01 y + g0) x + (M11 y^2 + g1 y + f0)
            p1, p0 = 2 * M[0, 2], 2 * M[1, 2] * y + g[2]
            c2, c1, c0 = M[0, 0], 2 * M[0, 1] * y + g[0], M[1, 1] * y * y + g[1] * y + f0
            out += _roots(p1 * p1 - 4 * A * c2, 2 * p1 * p0 - 4 * A * c1, p0 * p0 - 4 * A * c0)
        # F(x, y, z0) = M11 y^2 + (2 M01 x + 2 M12 z0 + g1) y + (M00 x^2 + (2 M02 z0 + g0) x + M22 z0^2 + g2 z0 + f0)
        for z in (-0.5, 0.5):
            u1, u0 = 2 * M[0, 1], 2 * M[1, 2] * z + g[1]
            w2, w1, w0 = M[0, 0], 2 * M[0, 2] * z + g[0], M[2, 2] * z * z + g[2] * z + f0
            out += _roots(u1 * u1 - 4 * M[1, 1] * w2, 2 * u1 * u0 - 4 * M[1, 1] * w1, u0 * u0 - 4 * M[1, 1] * w0)
        # double-root curve D(x, y) = B^2 - 4 A C = Dy2 y^2 + Dy1(x) y + Dy0(x)
        b1 = 2 * M[1, 2]
        Dy2 = b1 * b1 - 4 * A * M[1, 1]
        # Dy1 = 2 b1 (2 M02 x + g2) - 4 A (2 M01 x + g1) = e1 x + e0
        e1, e0 = 4 * b1 * M[0, 2] - 8 * A * M[0, 1], 2 * b1 * g[2] - 4 * A * g[1]
        # Dy0 = (2 M02 x + g2)^2 - 4 A (M00 x^2 + g0 x + f0) = d2 x^2 + d1 x + d0
        d2, d1, d0 = 4 * M[0, 2] ** 2 - 4 * A * M[0, 0], 4 * M[0, 2] * g[2] - 4 * A * g[0], g[2] ** 2 - 4 * A * f0
        out += _roots(e1 * e1 - 4 * Dy2 * d2, 2 * e1 * e0 - 4 * Dy2 * d1, e0 * e0 - 4 * Dy2 * d0)
        # dF/dz = 2 A z + 2 M02 x + 2 M12 y + g2 = 0 at z = zc, together with F(x, y, zc) = 0
        for zc in (-0.5, 0.5, 0.0):
            k0 = 2 * A * zc + g[2]
            if M[1, 2] != 0.0:
                al, be = -k0 / (2 * M[1, 2]), -M[0, 2] / M[1, 2]  # y = al + be x
                qa = M[0, 0] + 2 * M[0, 1] * be + M[1, 1] * be * be
                qb = 2 * M[0, 1] * al + 2 * M[1, 1] * al * be + 2 * M[0, 2] * zc + 2 * M[1, 2] * zc * be + g[0] + g[1] * be
                qc = M[1, 1] * al * al + 2 * M[1, 2] * al * zc + M[2, 2] * zc * zc + g[1] * al + g[2] * zc + f0
                out += _roots(qa, qb, qc)
            elif M[0, 2] != 0.0:
                out.append(-k0 / (2 * M[0, 2]))
        return sorted(v for v in out if -0.5 < v < 0.5)


def alpha_unit(n, t1, t2, b, tol: float = TOL) -> float:
    """Liquid fraction of the cube [-1/2, 1/2]^3 below the paraboloid
    zeta = b1 + b2 xi + b3 eta + b4 xi^2 + b5 xi eta + b6 eta^2 in the frame
    (t1, t2, n) (all in cell units)."""
    Q = _Quadric(n, t1, t2, b)

    def area(x):
        pts = Q.y_kinks(x)
        return _quad(lambda y: Q.z_length(x, y), -0.5, 0.5, points=pts or None, epsabs=tol, epsrel=tol, limit=200)

    return _quad(area, -0.5, 0.5, points=Q.x_kinks() or None, epsabs=tol, epsrel=tol, limit=400)


def cell_units(coeff, h):
    """PPIC coefficients (world units, origin at the cell centre) in cell units."""
    a1, a2, a3, a4, a5, a6 = (float(v) for v in coeff)
    return (a1 / h, a2, a3, a4 * h, a5 * h, a6 * h)


def alpha_cells(frame_normals, coeffs, h, tol: float = TOL):
    """alpha under the PPIC paraboloid of each listed cell: frame_normals [n, 3]
    (the PPIC frame normal of each cell), coeffs [n, 6] (world units, origin
    at the cell centre)."""
    out = np.empty(len(coeffs))
    for i, (nv, co) in enumerate(zip(np.asarray(frame_normals), np.asarray(coeffs))):
        t1, t2 = duff_frame(nv)
        out[i] = alpha_unit(nv, t1, t2, cell_units(co, h), tol)
    return out


# ----------------------------------------------------------------------------
# Surface integrals over the part of the paraboloid inside the cell (paper
# section 3.2: the cell's curvature and normal are integrated over the
# surface of the paraboloid within the cell).
#
# The surface is the graph zeta = P(xi, eta); with W = sqrt(1 + P_xi^2 +
# P_eta^2), dA = W dxi deta, the unit normal (pointing away from the liquid,
# +zeta side) is (-P_xi, -P_eta, 1) / W in the frame, and the mean curvature
# (kappa = 2H, positive for a sphere seen from outside) is
#   kappa = -[(1 + P_eta^2) P_xixi - 2 P_xi P_eta P_xieta + (1 + P_xi^2) P_etaeta] / W^3.
# Over the set R of (xi, eta) whose surface point lies in the cube:
#   area = int_R W,  K = int_R kappa W,  N = int_R (-P_xi, -P_eta, 1);
# kappa_cell = K / area, normal_cell = N / |N| (in world axes).  The integrals
# are nested adaptive quadratures over the disc |(xi, eta)| <= sqrt(3)/2 that
# holds R; the inner one is told the eta at which the surface point crosses a
# face plane (roots of quadratics), the outer one the xi at which the surface
# crosses a cube edge or its curve on a face turns along eta.

def _surface_kinks_xi(n, t1, t2, b):
    """xi where the slice R cap {xi = const} changes its structure: the surface
    crossing one of the 12 cube edges, and points of its curve on a face
    plane with a tangent along eta (where the curve's tangent has no
    component along t1)."""
    Q = _Quadric(n, t1, t2, b)
    M, g, f0 = Q.M, Q.g, Q.f0
    t1 = np.asarray(t1, dtype=np.float64)
    out = []
    # edges: x = e0 + s d, d a unit axis, |s| <= 1/2; F quadratic in s
    for ax in range(3):
        d = np.zeros(3)
        d[ax] = 1.0
        o1, o2 = [k for k in range(3) if k != ax]
        for w1 in (-0.5, 0.5):
            for w2 in (-0.5, 0.5):
                e0 = np.zeros(3)
                e0[o1], e0[o2] = w1, w2
                qa = d @ M @ d
                qb = 2.0 * (e0 @ M @ d) + g @ d
                qc = e0 @ M @ e0 + g @ e0 + f0
                for s in _roots(qa, qb, qc):
                    if -0.5 <= s <= 0.5:
                        out.append(float(t1 @ (e0 + s * d)))
    # face curves x_k = w: F = 0 and t1 . (grad F x e_k) = 0 (grad F = 2 M x + g),
    # the second linear in x: c . x + c0 = 0 with c = 2 M^T (e_k x t1) ... written out:
    for k in range(3):
        ek = np.zeros(3)
        ek[k] = 1.0
        u = np.cross(ek, t1)  # t1 . (v x e_k) = v . (e_k x t1)
        c = 2.0 * M @ u
        c0 = g @ u
        o1, o2 = [m for m in range(3) if m != k]
        for w in (-0.5, 0.5):
            # on the face: x = w e_k + y e_o1 + z e_o2; linear: c_o1 y + c_o2 z + (c_k w + c0) = 0
            A1, A2, A0 = c[o1], c[o2], c[k] * w + c0
            if A2 != 0.0:
                # z = al + be y
                al, be = -A0 / A2, -A1 / A2
                base = w * ek + al * np.eye(3)[o2]
                dirv = np.eye(3)[o1] + be * np.eye(3)[o2]
            elif A1 != 0.0:
                base = w * ek + (-A0 / A1) * np.eye(3)[o1]
                dirv = np.eye(3)[o2]
            else:
                continue
            qa = dirv @ M @ dirv
            qb = 2.0 * (base @ M @ dirv) + g @ dirv
            qc = base @ M @ base + g @ base + f0
            for s in _roots(qa, qb, qc):
                x = base + s * dirv
                if abs(x[o1]) <= 0.5 and abs(x[o2]) <= 0.5:
                    out.append(float(t1 @ x))
    R = np.sqrt(3.0) / 2.0
    return sorted(v for v in out if -R < v < R)


def surface_unit(n, t1, t2, b, tol: float = 1e-13):
    """(area, K, N_local[3]) over the part of the paraboloid in the cube
    [-1/2, 1/2]^3, cell units, frame (t1, t2, n)."""
    b0, b1, b2, b3, b4, b5 = (float(v) for v in b)
    n, t1, t2 = (np.asarray(v, dtype=np.float64) for v in (n, t1, t2))
    R = np.sqrt(3.0) / 2.0

    def inside(xi, eta):
        z = b0 + b1 * xi + b2 * eta + b3 * xi * xi + b4 * xi * eta + b5 * eta * eta
        x = xi * t1 + eta * t2 + z * n
        return bool(np.all(np.abs(x) <= 0.5))

    def eta_kinks(xi):
        # x_k = xi t1_k + eta t2_k + P n_k = w: quadratic in eta
        out = []
        for k in range(3):
            for w in (-0.5, 0.5):
                qa = b5 * n[k]
                qb = t2[k] + (b2 + b4 * xi) * n[k]
                qc = xi * t1[k] + (b0 + b1 * xi + b3 * xi * xi) * n[k] - w
                out += _roots(qa, qb, qc)
        return sorted(v for v in out if -R < v < R)

    def integrand(xi, eta, what):
        px = b1 + 2 * b3 * xi + b4 * eta
        pe = b2 + b4 * xi + 2 * b5 * eta
        if what == 0:
            return np.sqrt(1 + px * px + pe * pe)
        if what == 1:
            w2 = 1 + px * px + pe * pe
            return -((1 + pe * pe) * 2 * b3 - 2 * px * pe * b4 + (1 + px * px) * 2 * b5) / w2
        return (-px, -pe, 1.0)[what - 2]

    def slice_integral(xi, what):
        cuts = [-R] + eta_kinks(xi) + [R]
        s = 0.0
        for a, c in zip(cuts[:-1], cuts[1:]):
            if c <= a or not inside(xi, 0.5 * (a + c)):
                continue
            s += _quad(lambda e: integrand(xi, e, what), a, c, epsabs=tol, epsrel=tol, limit=200)
        return s

    pts = _surface_kinks_xi(n, t1, t2, b)
    vals = [_quad(lambda x: slice_integral(x, what), -R, R, points=pts or None, epsabs=tol, epsrel=tol, limit=400)
            for what in range(5)]
    return vals[0], vals[1], np.array(vals[2:])


def surface_cells(frame_normals, coeffs, h, tol: float = 1e-13):
    """(kappa_cell [n], normal_cell [n, 3]) of each listed cell: the
    area-weighted mean curvature (world units) and the normalised integral of
    the unit normal (world axes) over its paraboloid inside the cell; NaN
    where the paraboloid misses the cell."""
    kap = np.empty(len(coeffs))
    nrm = np.empty((len(coeffs), 3))
    for i, (nv, co) in enumerate(zip(np.asarray(frame_normals), np.asarray(coeffs))):
        t1, t2 = duff_frame(nv)
        area, K, N = surface_unit(nv, t1, t2, cell_units(co, h), tol)
        if area > 0.0:
            kap[i] = K / area / h
            Nw = N[0] * t1 + N[1] * t2 + N[2] * np.asarray(nv)
            nrm[i] = Nw / np.linalg.norm(Nw)
        else:
            kap[i] = np.nan
            nrm[i] = np.nan
    return kap, nrm


def _pool_chunk(job):
    kind, frame_normals, coeffs, h = job
    if kind == "alpha":
        return alpha_cells(frame_normals, coeffs, h)
    return surface_cells(frame_normals, coeffs, h)


def map_cells(kind, frame_normals, coeffs, h, workers: int = 12):
    """alpha_cells ("alpha") or surface_cells ("surface") of the listed cells,
    computed in a pool of at most `workers` CPU processes (started fresh, so
    they hold none of the caller's state and never touch a GPU); the results
    are those of the serial call, cell by cell."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    frame_normals, coeffs = np.asarray(frame_normals), np.asarray(coeffs)
    n = len(coeffs)
    workers = max(1, min(workers, os.cpu_count() or 1, n))
    parts = [p for p in np.array_split(np.arange(n), 4 * workers) if len(p)]
    jobs = [(kind, frame_normals[p], coeffs[p], h) for p in parts]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_pool_chunk, jobs))
    if kind == "alpha":
        return np.concatenate(res)
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])
