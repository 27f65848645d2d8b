"""Seeded input generators: closed, outward, counted as stated."""
import numpy as np
import pytest

from paper_2505_06932_amd import inputs as I
from tests.pins import polyhedron_volume


@pytest.mark.parametrize("L,nv,nt", [(0, 12, 20), (4, 2562, 5120), (6, 40962, 81920)])
def test_icosphere_counts_closed(L, nv, nt):
    v, t = I.icosphere(L)
    m = I.Mesh.from_arrays(v, t)
    assert (m.nv, m.nt) == (nv, nt)
    assert I.mesh_edges_ok(m)
    assert m.nv - 3 * m.nt // 2 + m.nt == 2  # Euler characteristic of a sphere
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    assert polyhedron_volume(v, t) > 0


@pytest.mark.parametrize("f", [1, 2, 5, 16])
def test_geodesic_counts_closed(f):
    v, t = I.geodesic_sphere(f)
    m = I.Mesh.from_arrays(v, t)
    assert (m.nv, m.nt) == (10 * f * f + 2, 20 * f * f)
    assert I.mesh_edges_ok(m)
    assert polyhedron_volume(v, t) > 0


def test_workloads_deterministic_and_sized():
    g1, m1, c1 = I.make_workload("sphere_32", seed=3)
    g2, m2, c2 = I.make_workload("sphere_32", seed=3)
    assert np.array_equal(m1.x, m2.x) and np.array_equal(c1, c2)
    assert (g1.nx, m1.nt) == (32, 5120)
    assert np.all(np.abs(c1 - 0.5) <= g1.h)
    g, m, c = I.make_workload("sphere_128", seed=0)
    assert (g.nx, m.nt) == (128, 81920)
    r = np.linalg.norm(m.verts() - c, axis=1)
    assert abs(r.std() - 0.01 * g.h) < 0.1 * 0.01 * g.h  # radial noise of 0.01 h


def test_simple_shapes_closed():
    assert I.mesh_edges_ok(I.box_mesh([0.1, 0.2, 0.3], [0.4, 0.5, 0.9]))
    assert I.mesh_edges_ok(I.tetra_mesh([0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]))
    cm = I.subdivided_cube_mesh([0.2, 0.2, 0.2], 0.5, 3)
    assert I.mesh_edges_ok(cm)
    assert abs(polyhedron_volume(cm.verts(), cm.tris()) - 0.125) < 1e-15


def test_psi_field_discretely_divergence_free():
    g = I.Grid(16, 16, 8, 0.0, 0.0, 0.0, 1.0 / 16)
    U, V, W = I.psi_face_velocity(g)
    div = (U[:, :, 1:] - U[:, :, :-1] + V[:, 1:, :] - V[:, :-1, :] + W[1:] - W[:-1]) / g.h
    assert np.abs(div).max() < 1e-12


def test_ellipsoid_droplets_as_drawn():
    g, m, info = I.make_workload("ellipsoids_256", seed=0)
    g2, m2, info2 = I.make_workload("ellipsoids_256", seed=0)
    assert np.array_equal(m.x, m2.x) and np.array_equal(info, info2)
    assert g.nx == 256 and len(info) == 64
    c, ax, f = info[:, :3], info[:, 3:6], info[:, 6].astype(int)
    assert np.all(ax >= 2 * g.h) and np.all(ax <= 12 * g.h)
    assert np.all(ax.max(1) <= 1.5 * ax.min(1))
    r = ax.max(1)
    d = np.linalg.norm(c[:, None] - c[None], axis=2) - r[:, None] - r[None]
    np.fill_diagonal(d, np.inf)
    assert d.min() >= 4 * g.h  # bounding spheres keep 4 cells apart
    assert np.all(c - r[:, None] >= 3 * g.h) and np.all(c + r[:, None] <= 1 - 3 * g.h)
    assert m.nt == int((20 * f * f).sum()) and m.nv == int((10 * f * f + 2).sum())
    assert I.mesh_edges_ok(m)
    # every droplet is its affinely mapped geodesic sphere: vertices on the
    # ellipsoid surface, outward orientation
    v, t, s = m.verts(), m.tris(), 0
    for k in range(64):
        nvk = 10 * f[k] ** 2 + 2
        ntk = 20 * f[k] ** 2
        assert polyhedron_volume(v, t[s:s + ntk], origin=c[k]) > 0
        s += ntk
    # mean edge near h/2 overall
    e = np.linalg.norm(v[t[:, 0]] - v[t[:, 1]], axis=1)
    assert 0.35 * g.h < e.mean() < 0.65 * g.h


def test_random_rotation_is_proper_orthogonal():
    rng = np.random.default_rng(5)
    for _ in range(20):
        R = I.random_rotation(rng)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14


def test_real_sph_harm_orthonormal():
    """Gauss-Legendre quadrature in cos(theta) times the trapezoid rule in
    phi (exact for these degrees): the real harmonics of degree <= 8 are
    orthonormal on the unit sphere."""
    x, w = np.polynomial.legendre.leggauss(12)
    phi = 2 * np.pi * np.arange(24) / 24
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct * ct)
    unit = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wq = np.repeat(w, 24) * (2 * np.pi / 24)
    Y = np.stack([I.real_sph_harm(l, m, unit) for l in range(9) for m in range(-l, l + 1)])
    G = (Y * wq) @ Y.T
    assert np.abs(G - np.eye(len(Y))).max() < 1e-12


def test_sh_spheres_workload():
    grid, mesh, info = I.sh_spheres_workload(64, 3, seed=1, r_lo=4.0, r_hi=10.0)
    assert I.mesh_edges_ok(mesh)
    h = grid.h
    v = mesh.verts()
    start = 0
    for c, R, A, freq in zip(info[:, :3], info[:, 3], info[:, 4], info[:, 5]):
        n = 10 * int(freq) ** 2 + 2
        r = np.linalg.norm(v[start:start + n] - c, axis=1)
        assert 4 * h <= R <= 10 * h and 0 <= A <= 0.1
        assert r.min() >= (1 - A) * R * (1 - 1e-12) and r.max() <= (1 + A) * R * (1 + 1e-12)
        assert abs(max(r.max() / R - 1, 1 - r.min() / R) - A) < 1e-12  # the amplitude is attained
        start += n
    assert start == mesh.nv
