"""Independent checks that pin the oracle to mathematics, not to itself.

Everything here is written separately from ``oracle/`` (different algorithms
where possible) and uses no code from the HIP library.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


# --------------------------------------------------------------------------
# enclosed volume
# --------------------------------------------------------------------------

def polyhedron_volume(verts: np.ndarray, tris: np.ndarray, origin=None) -> float:
    """V = (1/6) sum_t v0 . (v1 x v2) over the closed outward mesh, with the
    origin shifted to ``origin`` and summed with math.fsum."""
    v = np.asarray(verts, dtype=np.float64)
    if origin is not None:
        v = v - np.asarray(origin, dtype=np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    return math.fsum(np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0)


# --------------------------------------------------------------------------
# convex polyhedron clipping (cube cut by half-spaces)
# --------------------------------------------------------------------------

def _cube_faces(lo, h):
    lo = np.asarray(lo, dtype=np.float64)
    c = [lo + h * np.array([(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1], dtype=np.float64)
         for k in range(8)]
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    centre = lo + 0.5 * h
    faces = []
    for q in quads:
        f = [c[i] for i in q]
        n = np.cross(f[1] - f[0], f[2] - f[0])
        if np.dot(n, f[0] - centre) < 0:
            f = f[::-1]
        faces.append(f)
    return faces


def _clip_poly(poly, n, d):
    """Keep n.x <= d; return clipped polygon and the points created on the plane."""
    out, onp = [], []
    m = len(poly)
    for e in range(m):
        p, q = poly[e], poly[(e + 1) % m]
        sp, sq = np.dot(n, p) - d, np.dot(n, q) - d
        if sp <= 0:
            out.append(p)
            if sp == 0:
                onp.append(p)
        if (sp < 0 < sq) or (sq < 0 < sp):
            t = sp / (sp - sq)
            r = p + t * (q - p)
            out.append(r)
            onp.append(r)
    return out, onp


def convex_clip_volume(lo, h, planes) -> float:
    """Volume of the cube [lo, lo+h]^3 intersected with the half-spaces
    n . x <= d for (n, d) in ``planes`` (n need not be unit).  Faces are kept
    as polygons; each cut adds a cap polygon ordered by angle on the plane;
    the volume is (1/3) sum over faces of (point . normal) * area."""
    faces = _cube_faces(lo, h)
    for n, d in planes:
        n = np.asarray(n, dtype=np.float64)
        new, cap = [], []
        for f in faces:
            g, onp = _clip_poly(f, n, d)
            cap += onp
            if len(g) >= 3:
                new.append(g)
        if not new:
            return 0.0
        if len(cap) >= 3:
            cap = np.array(cap)
            ctr = cap.mean(axis=0)
            un = n / np.linalg.norm(n)
            e1 = cap[np.argmax(np.linalg.norm(cap - ctr, axis=1))] - ctr
            e1 = e1 - np.dot(e1, un) * un
            if np.linalg.norm(e1) > 0:
                e1 /= np.linalg.norm(e1)
                e2 = np.cross(un, e1)
                ang = np.arctan2((cap - ctr) @ e2, (cap - ctr) @ e1)
                order = np.argsort(ang)
                pts = [cap[i] for i in order]
                # drop duplicates
                uniq = [pts[0]]
                for p in pts[1:]:
                    if np.linalg.norm(p - uniq[-1]) > 1e-15 * h:
                        uniq.append(p)
                if len(uniq) >= 3 and np.linalg.norm(uniq[0] - uniq[-1]) <= 1e-15 * h:
                    uniq.pop()
                if len(uniq) >= 3:
                    new.append(uniq)
        faces = new
    vol = 0.0
    ref = np.asarray(lo, dtype=np.float64) + 0.5 * h
    for f in faces:
        p0 = f[0] - ref
        for j in range(1, len(f) - 1):
            vol += np.dot(p0, np.cross(f[j] - ref, f[j + 1] - ref)) / 6.0
    return vol


def mesh_is_convex(verts, tris, margin=0.0) -> bool:
    """For every triangle plane, all mesh vertices lie on its inner side."""
    v = np.asarray(verts)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    d = np.einsum("ij,ij->i", n, a)
    s = v @ n.T - d[None, :]
    return bool(np.all(s <= margin))


# --------------------------------------------------------------------------
# plane / cube volume (Scardovelli & Zaleski, J. Comput. Phys. 164 (2000))
# --------------------------------------------------------------------------

def plane_cube_volume(m, alpha) -> float:
    """Volume of {x in [0,1]^3 : m . x <= alpha} for m with positive
    components, by inclusion-exclusion over the cube corners."""
    m1, m2, m3 = (float(x) for x in m)

    def F(t):
        return t ** 3 if t > 0 else 0.0

    s = (F(alpha) - F(alpha - m1) - F(alpha - m2) - F(alpha - m3)
         + F(alpha - m1 - m2) + F(alpha - m1 - m3) + F(alpha - m2 - m3)
         - F(alpha - m1 - m2 - m3))
    return s / (6.0 * m1 * m2 * m3)


# --------------------------------------------------------------------------
# polygon clipping of a triangle against a box (membership brute force)
# --------------------------------------------------------------------------

def tri_box_area(tri, lo, hi) -> float:
    """Area of triangle ``tri`` (3x3) inside the closed box [lo, hi]."""
    poly = [np.asarray(p, dtype=np.float64) for p in tri]
    for d in range(3):
        for sgn, bound in ((-1.0, lo[d]), (1.0, hi[d])):
            n = np.zeros(3)
            n[d] = sgn
            poly, _ = _clip_poly(poly, n, sgn * bound)
            if len(poly) < 3:
                return 0.0
    s = np.zeros(3)
    for j in range(1, len(poly) - 1):
        s += np.cross(poly[j] - poly[0], poly[j + 1] - poly[0])
    return 0.5 * float(np.linalg.norm(s))


# --------------------------------------------------------------------------
# exact polynomial integrals over triangles (Fractions)
# --------------------------------------------------------------------------

def _fact(n):
    return math.factorial(n)


def tri_monomial_integral(p0, p1, p2, a: int, b: int) -> Fraction:
    """Exact integral of x^a y^b over the planar triangle (p0, p1, p2) in the
    (x, y) plane, signed by orientation, via the affine map from the
    reference triangle and int_ref s^i t^j = i! j! / (i+j+2)!."""
    x0, y0 = Fraction(p0[0]), Fraction(p0[1])
    ex = (Fraction(p1[0]) - x0, Fraction(p2[0]) - x0)
    ey = (Fraction(p1[1]) - y0, Fraction(p2[1]) - y0)
    jac = ex[0] * ey[1] - ex[1] * ey[0]

    # polynomial in (s, t) as dict {(i, j): coeff}
    def poly_pow(c0, cs, ct, n):
        res = {(0, 0): Fraction(1)}
        for _ in range(n):
            nxt = {}
            for (i, j), v in res.items():
                for (di, dj, c) in ((0, 0, c0), (1, 0, cs), (0, 1, ct)):
                    if c == 0:
                        continue
                    key = (i + di, j + dj)
                    nxt[key] = nxt.get(key, Fraction(0)) + v * c
            res = nxt
        return res

    px = poly_pow(x0, ex[0], ex[1], a)
    py = poly_pow(y0, ey[0], ey[1], b)
    total = Fraction(0)
    for (i1, j1), v1 in px.items():
        for (i2, j2), v2 in py.items():
            i, j = i1 + i2, j1 + j2
            total += v1 * v2 * Fraction(_fact(i) * _fact(j), _fact(i + j + 2))
    return total * jac


def solve_exact(M, b):
    """Gaussian elimination in Fractions."""
    n = len(b)
    A = [list(map(Fraction, row)) + [Fraction(bb)] for row, bb in zip(M, b)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[r][n] / A[r][r] for r in range(n)]
