"""Seeded synthetic inputs for the front-to-fluid-mesh coupling.

This module only *generates* inputs: closed triangulated fronts, uniform
Cartesian grids and staggered face-velocity fields.  It contains none of the
coupling arithmetic (no clipping, no volume fractions, no fits), so both the
HIP library and the CPU oracle can be fed from it without sharing method code.

Conventions (shared by every producer and consumer of these arrays):

* A grid is ``Grid(nx, ny, nz, x0, y0, z0, h)``: cubic cells of edge ``h``,
  cell (i, j, k) covers the half-open box ``[x0+i*h, x0+(i+1)*h) x ...``;
  linear cell id ``i + nx*(j + ny*k)`` (x fastest).
* A mesh is ``Mesh(x, y, z, t0, t1, t2)``: float64 vertex coordinates (SoA) and
  int32 triangle corners, counter-clockwise seen from outside, so the
  triangle normals point out of the enclosed fluid (where the indicator is 1,
  paper section 2, definition of the indicator function).
* Staggered face velocities (paper section 3.1): ``U`` has shape
  ``(nz, ny, nx+1)`` (x-normal faces at ``x0+i*h``), ``V`` has
  ``(nz, ny+1, nx)``, ``W`` has ``(nz+1, ny, nx)``; all C-contiguous, so the
  linear index is x fastest.

The workloads follow the paper's test shapes (spheres, perturbed spheres,
surfaces of revolution; section 4) at the sizes used by the benchmark.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Grid", "Mesh", "icosahedron", "icosphere", "geodesic_sphere",
    "sphere_workload", "polar_revolution_workload", "ellipsoids_workload",
    "sh_spheres_workload", "real_sph_harm",
    "random_rotation", "box_mesh", "tetra_mesh",
    "subdivided_cube_mesh", "psi_face_velocity", "uniform_face_velocity",
    "affine_face_velocity", "mesh_edges_ok", "WORKLOADS",
]


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    x0: float
    y0: float
    z0: float
    h: float

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Mesh:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    t0: np.ndarray
    t1: np.ndarray
    t2: np.ndarray

    @property
    def nv(self) -> int:
        return int(self.x.shape[0])

    @property
    def nt(self) -> int:
        return int(self.t0.shape[0])

    @staticmethod
    def from_arrays(verts: np.ndarray, tris: np.ndarray) -> "Mesh":
        v = np.ascontiguousarray(verts, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        return Mesh(np.ascontiguousarray(v[:, 0]), np.ascontiguousarray(v[:, 1]),
                    np.ascontiguousarray(v[:, 2]), np.ascontiguousarray(t[:, 0]),
                    np.ascontiguousarray(t[:, 1]), np.ascontiguousarray(t[:, 2]))

    def verts(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def tris(self) -> np.ndarray:
        return np.stack([self.t0, self.t1, self.t2], axis=1)


# --------------------------------------------------------------------------
# sphere triangulations
# --------------------------------------------------------------------------

def _orient_outward(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Flip triangles of a star-shaped (about the origin) surface so that they
    are counter-clockwise seen from outside."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    out = tris.copy()
    flip = s < 0
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    """The regular icosahedron with vertices (0, +-1, +-phi) and cyclic
    permutations, scaled to the unit sphere; faces found as the 20 triples of
    mutually adjacent vertices and oriented outward."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * phi))
            v.append((s1, s2 * phi, 0.0))
            v.append((s2 * phi, 0.0, s1))
    v = np.array(v, dtype=np.float64)
    d2 = ((v[:, None, :] - v[None, :, :]) ** 2).sum(-1)
    adj = np.abs(d2 - 4.0) < 1e-9  # edge length 2 before scaling
    faces = []
    n = len(v)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, _orient_outward(v, np.array(faces, dtype=np.int64))


def icosphere(subdivisions: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: recursive 1->4 midpoint split of the icosahedron, every
    new vertex projected to the unit sphere at each level.  Vertex order: the
    12 icosahedron vertices, then midpoints in creation order.  Gives
    10*4^L + 2 vertices and 20*4^L triangles."""
    verts, tris = icosahedron()
    vl = [tuple(p) for p in verts]
    for _ in range(subdivisions):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            m = cache.get(key)
            if m is None:
                p = np.add(vl[a], vl[b]) * 0.5
                p = p / np.linalg.norm(p)
                m = len(vl)
                vl.append(tuple(p))
                cache[key] = m
            return m

        new = []
        for a, b, c in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = np.array(new, dtype=np.int64)
    return np.array(vl, dtype=np.float64), tris


def geodesic_sphere(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Class-I geodesic sphere of frequency ``freq``: every icosahedron face is
    split into freq^2 triangles on a barycentric lattice and the lattice
    points are projected to the unit sphere.  10*f^2+2 vertices, 20*f^2
    triangles.  Vertex order: icosahedron vertices, then edge points (edge in
    order of first appearance), then face-interior points."""
    if freq < 1:
        raise ValueError("freq must be >= 1")
    ico, faces = icosahedron()
    pts: list[np.ndarray] = [p for p in ico]
    edge_pts: dict[tuple[int, int], list[int]] = {}

    def edge_index(a: int, b: int, s: int) -> int:
        """Index of the point s/freq of the way from corner a to corner b."""
        if s == 0:
            return a
        if s == freq:
            return b
        key = (a, b) if a < b else (b, a)
        lst = edge_pts.get(key)
        if lst is None:
            lo, hi = key
            lst = []
            for t in range(1, freq):
                p = ico[lo] * (freq - t) + ico[hi] * t
                lst.append(len(pts))
                pts.append(p / np.linalg.norm(p))
            edge_pts[key] = lst
        return lst[s - 1] if a < b else lst[freq - s - 1]

    out = []
    for a, b, c in faces:
        # lattice point (i, j): a + i/f (b - a) + j/f (c - a), i + j <= f
        idx = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                if j == 0:
                    idx[i, j] = edge_index(a, b, i)
                elif i == 0:
                    idx[i, j] = edge_index(a, c, j)
                elif i + j == freq:
                    idx[i, j] = edge_index(b, c, j)
                else:
                    p = (ico[a] * (freq - i - j) + ico[b] * i + ico[c] * j)
                    idx[i, j] = len(pts)
                    pts.append(p / np.linalg.norm(p))
        for i in range(freq):
            for j in range(freq - i):
                out.append((idx[i, j], idx[i + 1, j], idx[i, j + 1]))
                if i + j + 1 < freq:
                    out.append((idx[i + 1, j], idx[i + 1, j + 1], idx[i, j + 1]))
    verts = np.array(pts, dtype=np.float64)
    tris = _orient_outward(verts, np.array(out, dtype=np.int64))
    return verts, tris


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def sphere_workload(n: int, radius: float, subdivisions: int, seed: int,
                    noise_over_h: float = 0.0, domain: float = 1.0):
    """A sphere of ``radius`` on an n^3 grid over [0, domain]^3.

    The centre is ``domain/2 + U(-h, h)^3`` (three draws of
    ``numpy.random.default_rng(seed)``), the surface is the icosphere with
    ``subdivisions`` levels, and, if ``noise_over_h > 0``, each vertex is then
    moved along its unit radial direction by ``N(0, (noise_over_h*h)^2)``
    (nv further draws of the same generator)."""
    h = domain / n
    rng = np.random.default_rng(seed)
    centre = domain / 2.0 + rng.uniform(-h, h, size=3)
    unit, tris = icosphere(subdivisions)
    r = np.full(len(unit), radius)
    if noise_over_h > 0.0:
        r = r + rng.normal(0.0, noise_over_h * h, size=len(unit))
    verts = centre[None, :] + unit * r[:, None]
    grid = Grid(n, n, n, 0.0, 0.0, 0.0, h)
    return grid, Mesh.from_arrays(verts, tris), centre


def polar_revolution_workload(n: int, radius: float, freq: int, seed: int,
                              domain: float = 1.0):
    """Skirted-bubble-like closed surface of revolution about z: the unit
    geodesic sphere of frequency ``freq`` mapped radially by
    rho(theta) = R (1 - 0.3 cos^2 theta + 0.2 cos^4 theta), centred at
    ``domain/2 + U(-h, h)^3``."""
    h = domain / n
    rng = np.random.default_rng(seed)
    centre = domain / 2.0 + rng.uniform(-h, h, size=3)
    unit, tris = geodesic_sphere(freq)
    c = unit[:, 2]
    rho = radius * (1.0 - 0.3 * c * c + 0.2 * c ** 4)
    verts = centre[None, :] + unit * rho[:, None]
    grid = Grid(n, n, n, 0.0, 0.0, 0.0, h)
    return grid, Mesh.from_arrays(verts, tris), centre


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation matrix from a uniform unit quaternion
    (Shoemake, "Uniform random rotations", Graphics Gems III, 1992): three
    draws u1, u2, u3 of U[0, 1)."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, size=3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoids_workload(n: int, count: int, seed: int, axis_lo: float = 2.0, axis_hi: float = 12.0,
                        max_aspect: float = 1.5, gap_over_h: float = 4.0, edge_over_h: float = 0.5,
                        domain: float = 1.0):
    """``count`` disjoint ellipsoidal droplets in one mesh on an n^3 grid.

    For each droplet in turn, with ``numpy.random.default_rng(seed)``:
    semi-axes drawn U[axis_lo h, axis_hi h]^3 until max/min <= max_aspect;
    an orientation from ``random_rotation``; a centre drawn
    U[lo, hi]^3 (lo = largest semi-axis + 3h from the domain walls) until
    its bounding sphere keeps ``gap_over_h`` cells from every earlier one.
    The surface is the unit geodesic sphere of frequency
    ceil(1.21 (abc)^(1/3) / (edge_over_h h)) (mean edge near edge_over_h h
    on the equivalent sphere) mapped by the semi-axes and the rotation, so
    triangle sizes vary within and between droplets.  Returns the grid, the
    mesh (droplet after droplet) and a (count, 7) array of centre, semi-axes
    and frequency per droplet."""
    h = domain / n
    rng = np.random.default_rng(seed)
    cache: dict[int, tuple[np.ndarray, np.ndarray]] = {}
    verts, tris, info = [], [], []
    placed: list[tuple[np.ndarray, float]] = []
    nv = 0
    for _ in range(count):
        while True:
            ax = rng.uniform(axis_lo * h, axis_hi * h, size=3)
            if ax.max() <= max_aspect * ax.min():
                break
        rot = random_rotation(rng)
        r = float(ax.max())
        lo, hi = r + 3 * h, domain - r - 3 * h
        for _attempt in range(100000):
            c = rng.uniform(lo, hi, size=3)
            if all(np.linalg.norm(c - c2) >= r + r2 + gap_over_h * h for c2, r2 in placed):
                break
        else:
            raise RuntimeError("could not place the droplets")
        placed.append((c, r))
        freq = int(math.ceil(1.21 * float(np.prod(ax)) ** (1.0 / 3.0) / (edge_over_h * h)))
        if freq not in cache:
            cache[freq] = geodesic_sphere(freq)
        unit, t = cache[freq]
        verts.append(c[None, :] + (unit * ax[None, :]) @ rot.T)
        tris.append(t + nv)
        nv += len(unit)
        info.append([*c, *ax, freq])
    grid = Grid(n, n, n, 0.0, 0.0, 0.0, h)
    return grid, Mesh.from_arrays(np.concatenate(verts), np.concatenate(tris)), np.array(info)


def real_sph_harm(l: int, m: int, unit: np.ndarray) -> np.ndarray:
    """Real spherical harmonic of degree l, order m at unit vectors [n, 3]:
    Y_l^0; sqrt(2) Re Y_l^m for m > 0; sqrt(2) Im Y_l^|m| for m < 0 (complex
    harmonics of scipy.special.sph_harm_y, polar angle from +z)."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(unit[:, 2], -1.0, 1.0))
    phi = np.arctan2(unit[:, 1], unit[:, 0])
    y = sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return y.real
    return math.sqrt(2.0) * (y.real if m > 0 else y.imag)


def sh_spheres_workload(n: int, count: int, seed: int, r_lo: float = 4.0, r_hi: float = 20.0,
                        degree: int = 8, amp_max: float = 0.1, edge_over_h: float = 0.5,
                        gap_over_h: float = 4.0, domain: float = 1.0, return_surfaces: bool = False):
    """``count`` disjoint spheres with spherical-harmonic perturbations in one
    mesh on an n^3 grid.

    For each droplet in turn, with ``numpy.random.default_rng(seed)``: the
    radius R ~ U[r_lo h, r_hi h]; the relative amplitude A ~ U[0, amp_max];
    coefficients c_lm ~ N(0, 1) / l^2 for 2 <= l <= degree, -l <= m <= l (in
    that order); a centre drawn U[lo, hi]^3 (lo = 1.1 R + 3h from the walls)
    until its bounding sphere keeps ``gap_over_h`` cells from every earlier
    one.  The surface is the unit geodesic sphere of frequency
    ceil(1.21 R / (edge_over_h h)) mapped radially by
    r(u) = R (1 + A f(u) / max |f|), f = sum c_lm Y_lm(u) (real harmonics,
    :func:`real_sph_harm`; the maximum over the mesh vertices), so every
    radius lies in [(1 - A) R, (1 + A) R].  Returns the grid, the mesh and a
    (count, 6) array of centre, R, A and frequency per droplet; with
    return_surfaces also a list of the droplets' exact surfaces, dicts with
    centre, R, A, coef [(l, m, c_lm)] and fmax."""
    h = domain / n
    rng = np.random.default_rng(seed)
    cache: dict[int, tuple[np.ndarray, np.ndarray]] = {}
    verts, tris, info, surfaces = [], [], [], []
    placed: list[tuple[np.ndarray, float]] = []
    nv = 0
    for _ in range(count):
        R = float(rng.uniform(r_lo * h, r_hi * h))
        A = float(rng.uniform(0.0, amp_max))
        coef = [(l, m, float(rng.normal()) / (l * l)) for l in range(2, degree + 1) for m in range(-l, l + 1)]
        rb = 1.1 * R
        lo, hi = rb + 3 * h, domain - rb - 3 * h
        for _attempt in range(100000):
            c = rng.uniform(lo, hi, size=3)
            if all(np.linalg.norm(c - c2) >= rb + r2 + gap_over_h * h for c2, r2 in placed):
                break
        else:
            raise RuntimeError("could not place the droplets")
        placed.append((c, rb))
        freq = int(math.ceil(1.21 * R / (edge_over_h * h)))
        if freq not in cache:
            cache[freq] = geodesic_sphere(freq)
        unit, t = cache[freq]
        f = np.zeros(len(unit))
        for l, m, cl in coef:
            f += cl * real_sph_harm(l, m, unit)
        fmax = float(np.abs(f).max())
        r = R * (1.0 + A * f / fmax) if fmax > 0.0 else np.full(len(unit), R)
        verts.append(c[None, :] + unit * r[:, None])
        tris.append(t + nv)
        nv += len(unit)
        info.append([*c, R, A, freq])
        surfaces.append(dict(centre=c.copy(), R=R, A=A, coef=coef, fmax=fmax))
    grid = Grid(n, n, n, 0.0, 0.0, 0.0, h)
    mesh = Mesh.from_arrays(np.concatenate(verts), np.concatenate(tris))
    if return_surfaces:
        return grid, mesh, np.array(info), surfaces
    return grid, mesh, np.array(info)


#: Named workloads: (builder, kwargs).  "sphere_32" is the small plain-FP64
#: case (R = 0.25, 4 subdivisions, 5,120 triangles, 32^3); "sphere_128" is the
#: 128^3 sphere of R = 0.3 with 6 subdivisions (81,920 triangles) and radial
#: noise of 0.01 h; "ellipsoids_256" is 64 disjoint ellipsoidal droplets on
#: 256^3 with edges near h/2; "revolution_512" is the 512^3 surface of
#: revolution with 1,997,120 triangles; "sh_spheres_128" is 8 disjoint
#: spheres with spherical-harmonic perturbations (R in [4h, 20h], degree <= 8,
#: amplitude <= 0.1 R) on 128^3, the learned-curvature workload;
#: "sh_spheres_256" is 64 of them on 256^3 (about 223k interfacial cells).
WORKLOADS = {
    "sphere_32": (sphere_workload, dict(n=32, radius=0.25, subdivisions=4, noise_over_h=0.0)),
    "sphere_128": (sphere_workload, dict(n=128, radius=0.3, subdivisions=6, noise_over_h=0.01)),
    "ellipsoids_256": (ellipsoids_workload, dict(n=256, count=64)),
    "revolution_512": (polar_revolution_workload, dict(n=512, radius=0.2, freq=316)),
    "sh_spheres_128": (sh_spheres_workload, dict(n=128, count=8)),
    "sh_spheres_256": (sh_spheres_workload, dict(n=256, count=64)),
}


def make_workload(name: str, seed: int = 0):
    fn, kw = WORKLOADS[name]
    return fn(seed=seed, **kw)


# --------------------------------------------------------------------------
# simple closed shapes for closed-form checks
# --------------------------------------------------------------------------

def box_mesh(lo, hi) -> Mesh:
    """Axis-aligned box [lo, hi] as 12 outward triangles."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    v = np.array([[lo[0] if (c & 1) == 0 else hi[0],
                   lo[1] if (c & 2) == 0 else hi[1],
                   lo[2] if (c & 4) == 0 else hi[2]] for c in range(8)])
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    tris = np.array(t, dtype=np.int64)
    centre = 0.5 * (lo + hi)
    return Mesh.from_arrays(v, _orient_outward(v - centre, tris))


def tetra_mesh(p0, p1, p2, p3) -> Mesh:
    """Tetrahedron with the given corners as 4 outward triangles."""
    v = np.array([p0, p1, p2, p3], dtype=np.float64)
    tris = np.array([(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)], dtype=np.int64)
    return Mesh.from_arrays(v, _orient_outward(v - v.mean(axis=0), tris))


def subdivided_cube_mesh(lo, size: float, m: int, rotation=None) -> Mesh:
    """Surface of the cube [lo, lo+size]^3 with each face split into an m x m
    lattice of squares, two triangles each; optionally rotated about the cube
    centre by the 3x3 matrix ``rotation``.  Closed, outward oriented."""
    lo = np.asarray(lo, dtype=np.float64)
    pts: dict[tuple[int, int, int], int] = {}
    vl: list[tuple[float, float, float]] = []

    def vid(a: int, b: int, c: int) -> int:
        key = (a, b, c)
        i = pts.get(key)
        if i is None:
            i = len(vl)
            pts[key] = i
            vl.append((lo[0] + size * a / m, lo[1] + size * b / m, lo[2] + size * c / m))
        return i

    tris = []
    for axis in range(3):
        for side in (0, m):
            for u in range(m):
                for w in range(m):
                    def p(du, dw):
                        q = [0, 0, 0]
                        q[axis] = side
                        q[(axis + 1) % 3] = u + du
                        q[(axis + 2) % 3] = w + dw
                        return vid(*q)
                    a, b, c, d = p(0, 0), p(1, 0), p(1, 1), p(0, 1)
                    tris += [(a, b, c), (a, c, d)]
    v = np.array(vl, dtype=np.float64)
    centre = lo + 0.5 * size
    t = _orient_outward(v - centre, np.array(tris, dtype=np.int64))
    if rotation is not None:
        v = centre + (v - centre) @ np.asarray(rotation, dtype=np.float64).T
    return Mesh.from_arrays(v, t)


def uv_sphere_mesh(centre, radius: float, n_lat: int, n_lon: int, rotation=None) -> Mesh:
    """Latitude-longitude sphere: n_lat - 1 rings of n_lon vertices between
    two poles, quads split into two triangles and a fan of n_lon triangles at
    each pole, so the poles have valence n_lon (high-valence vertices for the
    ring capacities).  Optionally rotated by the 3x3 matrix ``rotation``.
    Closed, outward oriented."""
    centre = np.asarray(centre, dtype=np.float64)
    verts = [(0.0, 0.0, 1.0)]
    for i in range(1, n_lat):
        th = math.pi * i / n_lat
        for j in range(n_lon):
            ph = 2.0 * math.pi * j / n_lon
            verts.append((math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)))
    verts.append((0.0, 0.0, -1.0))
    v = np.array(verts, dtype=np.float64)
    south = len(verts) - 1

    def ring(i, j):
        return 1 + (i - 1) * n_lon + (j % n_lon)

    t = []
    for j in range(n_lon):
        t.append((0, ring(1, j), ring(1, j + 1)))
        t.append((south, ring(n_lat - 1, j + 1), ring(n_lat - 1, j)))
        for i in range(1, n_lat - 1):
            a, b, c, d = ring(i, j), ring(i + 1, j), ring(i + 1, j + 1), ring(i, j + 1)
            t += [(a, b, c), (a, c, d)]
    tris = _orient_outward(v, np.array(t, dtype=np.int64))
    if rotation is not None:
        v = v @ np.asarray(rotation, dtype=np.float64).T
    return Mesh.from_arrays(centre + radius * v, tris)


# --------------------------------------------------------------------------
# staggered face velocities
# --------------------------------------------------------------------------

def _face_coords(grid: Grid):
    xf = grid.x0 + grid.h * np.arange(grid.nx + 1)
    yf = grid.y0 + grid.h * np.arange(grid.ny + 1)
    zf = grid.z0 + grid.h * np.arange(grid.nz + 1)
    xc = grid.x0 + grid.h * (np.arange(grid.nx) + 0.5)
    yc = grid.y0 + grid.h * (np.arange(grid.ny) + 0.5)
    zc = grid.z0 + grid.h * (np.arange(grid.nz) + 0.5)
    return xf, yf, zf, xc, yc, zc


def psi_face_velocity(grid: Grid):
    """Face-averaged normal velocities of u = (sin pi x cos pi y,
    -cos pi x sin pi y, 0), built from the stream function
    psi = sin(pi x) sin(pi y) / pi as flux differences, so that the staggered
    field is discretely divergence free to rounding."""
    xf, yf, _, _, _, _ = _face_coords(grid)
    h = grid.h

    def psi(x, y):
        return np.sin(np.pi * x) * np.sin(np.pi * y) / np.pi

    # U at x-face i, cell row j: (psi(x_i, y_{j+1}) - psi(x_i, y_j)) / h
    U2 = (psi(xf[None, :], yf[1:, None]) - psi(xf[None, :], yf[:-1, None])) / h  # (ny, nx+1)
    V2 = -(psi(xf[None, 1:], yf[:, None]) - psi(xf[None, :-1], yf[:, None])) / h  # (ny+1, nx)
    U = np.ascontiguousarray(np.broadcast_to(U2, (grid.nz, grid.ny, grid.nx + 1)))
    V = np.ascontiguousarray(np.broadcast_to(V2, (grid.nz, grid.ny + 1, grid.nx)))
    W = np.zeros((grid.nz + 1, grid.ny, grid.nx))
    return U, V, W


def psi_velocity_exact(x, y, z):
    """The continuous field behind :func:`psi_face_velocity`."""
    return (np.sin(np.pi * x) * np.cos(np.pi * y),
            -np.cos(np.pi * x) * np.sin(np.pi * y),
            np.zeros_like(np.asarray(z, dtype=np.float64)))


def uniform_face_velocity(grid: Grid, u):
    U = np.full((grid.nz, grid.ny, grid.nx + 1), float(u[0]))
    V = np.full((grid.nz, grid.ny + 1, grid.nx), float(u[1]))
    W = np.full((grid.nz + 1, grid.ny, grid.nx), float(u[2]))
    return U, V, W


def affine_face_velocity(grid: Grid, c, B):
    """Normal velocities of u(x) = c + B x sampled at the face centres (the
    face average of an affine field)."""
    c = np.asarray(c, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    xf, yf, zf, xc, yc, zc = _face_coords(grid)
    X, Y, Z = np.meshgrid(xf, yc, zc, indexing="ij")
    U = (c[0] + B[0, 0] * X + B[0, 1] * Y + B[0, 2] * Z).transpose(2, 1, 0)
    X, Y, Z = np.meshgrid(xc, yf, zc, indexing="ij")
    V = (c[1] + B[1, 0] * X + B[1, 1] * Y + B[1, 2] * Z).transpose(2, 1, 0)
    X, Y, Z = np.meshgrid(xc, yc, zf, indexing="ij")
    W = (c[2] + B[2, 0] * X + B[2, 1] * Y + B[2, 2] * Z).transpose(2, 1, 0)
    return (np.ascontiguousarray(U), np.ascontiguousarray(V), np.ascontiguousarray(W))


# --------------------------------------------------------------------------
# mesh validity (host-side input check)
# --------------------------------------------------------------------------

def mesh_edges_ok(mesh: Mesh) -> bool:
    """True iff every directed edge appears exactly once and its reverse also
    appears exactly once (closed, consistently oriented 2-manifold edges)."""
    t = mesh.tris().astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    key = e[:, 0] * (mesh.nv + 1) + e[:, 1]
    rkey = e[:, 1] * (mesh.nv + 1) + e[:, 0]
    u, cnt = np.unique(key, return_counts=True)
    if np.any(cnt != 1):
        return False
    return bool(np.all(np.isin(rkey, u)))
