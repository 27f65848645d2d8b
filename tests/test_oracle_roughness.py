"""Pins of the roughness oracle (oracle/roughness.py, paper section 3.4)
against what geometry fixes: the geometric Laplacian of a regular fan, the
dihedral roughness against the sphere's curvature (appendix A of the paper),
invariances, the simultaneous Laplacian equations, exact volume
conservation of the edge smoothing, and the schedule's independence."""
import numpy as np
import pytest

from oracle import roughness as RG
from paper_2505_06932_amd import inputs as I


def _bipyramid(n=7, top=0.3, bottom=0.8):
    ang = 2 * np.pi * np.arange(n) / n
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], 1)
    X = np.vstack([ring, [[0, 0, top], [0, 0, -bottom]]])
    T = []
    for k in range(n):
        T.append([k, (k + 1) % n, n])        # upper fan, outward
        T.append([(k + 1) % n, k, n + 1])    # lower fan, outward
    return X, np.array(T)


def test_geometric_laplacian_regular_fan():
    X, T = _bipyramid(7, top=0.3)
    topo = RG.Topology(T, len(X))
    GL = RG.geometric_laplacian(X, topo)
    # the apex sees a regular polygon centred below it: GL is its height
    assert np.allclose(GL[7], [0, 0, 0.3], rtol=0, atol=1e-15)
    assert np.allclose(GL[8], [0, 0, -0.8], rtol=0, atol=1e-15)
    # a ring vertex: weights 1/|x_i - x_j| by hand
    i = 0
    nb = topo.ring[i]
    assert sorted(nb) == [1, 6, 7, 8]
    w = np.array([1 / np.linalg.norm(X[i] - X[j]) for j in nb])
    assert np.allclose(GL[i], X[i] - (w[:, None] * X[nb]).sum(0) / w.sum(), rtol=0, atol=1e-15)


def test_geometric_laplacian_scales_and_moves_with_the_mesh():
    rng = np.random.default_rng(1)
    unit, T = I.icosphere(2)
    X = unit * (1 + 0.02 * rng.normal(size=len(unit)))[:, None]
    topo = RG.Topology(T, len(X))
    GL = RG.geometric_laplacian(X, topo)
    Q = I.random_rotation(rng)
    GL2 = RG.geometric_laplacian(2.5 * X @ Q.T + [1, 2, 3], topo)
    assert np.allclose(GL2, 2.5 * GL @ Q.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mesh", ["ico3", "ico4", "geo10"])
def test_dihedral_roughness_measures_sphere_curvature(mesh):
    """Appendix A: arccos(1 - R_e) / d estimates the curvature 1/R (d the
    distance between the two triangle centres); averaged over the edges of a
    sphere the estimate is within 1% of 1/R."""
    unit, T = {"ico3": lambda: I.icosphere(3), "ico4": lambda: I.icosphere(4),
               "geo10": lambda: I.geodesic_sphere(10)}[mesh]()
    R = 0.7
    X = R * unit / np.linalg.norm(unit, axis=1)[:, None]
    topo = RG.Topology(T, len(X))
    _, parts = RG.roughness(X, topo)
    cen = X[T].mean(1)
    est = []
    for (a, b), re in parts["Re"].items():
        t1, _ = topo.half[(a, b)]
        t2, _ = topo.half[(b, a)]
        d = np.linalg.norm(cen[t1] - cen[t2])
        est.append(np.arccos(1 - re) / d)
    assert abs(np.mean(est) * R - 1) < 0.01


def test_flat_regions_have_no_roughness():
    mesh = I.subdivided_cube_mesh(np.zeros(3), 1.0, 6)
    X, T = mesh.verts(), mesh.tris()
    topo = RG.Topology(T, len(X))
    R, parts = RG.roughness(X, topo)
    # the face centres: their whole two-ring lies inside one face, where every R_e is 0
    face_centre = [i for i in range(len(X)) if np.sum((np.abs(X[i] - 0.5) < 1e-12)) == 2]
    assert face_centre
    for i in face_centre:
        assert R[i] == 0.0
    # an edge along a cube edge separates perpendicular faces: R_e = 1
    on_edge = [(a, b) for (a, b) in parts["Re"] if np.sum(np.isin(X[a], [0.0, 1.0]) & np.isin(X[b], [0.0, 1.0])
                                                          & np.isclose(X[a], X[b])) == 2]
    assert on_edge and all(abs(parts["Re"][e] - 1.0) < 1e-12 for e in on_edge)


def test_triangle_statistic_special_cases():
    # equal variances: the plain mean of the G_i; zero variances: also the mean
    X, T = _bipyramid(6, top=1.0, bottom=1.0)  # the regular octahedron-like bipyramid
    topo = RG.Topology(T, len(X))
    _, p = RG.roughness(X, topo)
    for t, c in enumerate(T):
        v = p["V"][c]
        if np.allclose(v, v[0]):
            assert p["Rt"][t] == pytest.approx(p["G"][c].mean(), abs=1e-15)


def test_roughness_invariances():
    rng = np.random.default_rng(2)
    unit, T = I.icosphere(2)
    X = unit * (1 + 0.05 * rng.normal(size=len(unit)))[:, None]
    topo = RG.Topology(T, len(X))
    R, p = RG.roughness(X, topo)
    Q = I.random_rotation(rng)
    R2, p2 = RG.roughness(3.0 * X @ Q.T + [0.5, -1, 2], topo)
    assert np.allclose(p2["Rt"], p["Rt"], rtol=0, atol=1e-12)  # dihedral statistics are scale-free
    assert np.allclose(R2, 9.0 * R, rtol=1e-10, atol=0)          # R^l carries the triangle areas


def test_laplacian_pair_solves_the_simultaneous_equations():
    rng = np.random.default_rng(3)
    unit, T = I.icosphere(2)
    X = unit * (1 + 0.05 * rng.normal(size=len(unit)))[:, None]
    topo = RG.Topology(T, len(X))
    for eid, a, b in topo.edges[::37]:
        x1s, x2s = RG.laplacian_pair(X, topo, a, b)
        r1, r2 = topo.ring[a], topo.ring[b]
        m1 = (x2s + sum(X[j] for j in r1 if j != b)) / len(r1)
        m2 = (x1s + sum(X[j] for j in r2 if j != a)) / len(r2)
        assert np.allclose(x1s, m1, rtol=0, atol=1e-14) and np.allclose(x2s, m2, rtol=0, atol=1e-14)


def test_edge_smoothing_conserves_volume_exactly():
    rng = np.random.default_rng(4)
    unit, T = I.icosphere(3)
    X = unit * (1 + 0.03 * rng.normal(size=len(unit)))[:, None] + [0.2, -0.1, 0.3]
    topo = RG.Topology(T, len(X))
    v0 = RG.enclosed_volume(X, T)
    moved = 0
    for eid, a, b in topo.edges[::11]:
        r = RG.smooth_edge(X, topo, a, b)
        if r is None:
            continue
        X[a], X[b] = r
        moved += 1
        assert abs(RG.enclosed_volume(X, T) - v0) < 1e-14 * v0
    assert moved > 50
    # smoothing lowers the roughness it acts on
    X0 = unit * (1 + 0.03 * rng.normal(size=len(unit)))[:, None]
    gl0 = np.linalg.norm(RG.geometric_laplacian(X0, topo), axis=1)
    Xs, n, _ = RG.smooth(X0, T, 0.0, -1.0)
    gl1 = np.linalg.norm(RG.geometric_laplacian(Xs, topo), axis=1)
    assert n > 0 and gl1.mean() < 0.7 * gl0.mean()
    assert abs(RG.enclosed_volume(Xs, T) / RG.enclosed_volume(X0, T) - 1) < 1e-13


def test_smoothing_leaves_a_regular_plane_alone():
    mesh = I.subdivided_cube_mesh(np.zeros(3), 1.0, 6)
    X, T = mesh.verts(), mesh.tris()
    topo = RG.Topology(T, len(X))
    for eid, a, b in topo.edges:
        # both ends strictly inside one face, with their whole one-rings
        if all(np.sum(np.abs(X[v] - 0.5) < 1.5 / 6 + 1e-12) == 2 for v in (a, b)):
            r = RG.smooth_edge(X, topo, a, b)
            assert r is not None
            assert np.allclose(r[0], X[a], rtol=0, atol=1e-15) and np.allclose(r[1], X[b], rtol=0, atol=1e-15)


def test_fmix32_reference_values():
    """MurmurHash3's finalizer: 0 maps to 0, and it is a bijection on a sample."""
    assert RG.fmix32(0) == 0
    vals = {RG.fmix32(i) for i in range(1, 20000)}
    assert len(vals) == 19999 and 0 not in vals
    assert RG.fmix32(1) == 0x514E28B7


def test_schedule_rounds_are_independent_and_complete():
    rng = np.random.default_rng(5)
    unit, T = I.icosphere(2)
    X = unit * (1 + 0.05 * rng.normal(size=len(unit)))[:, None]
    topo = RG.Topology(T, len(X))
    edges = topo.edges[::3]
    rounds = RG.schedule(topo, edges)
    seen = [e[0] for rnd in rounds for e in rnd]
    assert sorted(seen) == sorted(e[0] for e in edges)
    first = min(edges, key=lambda e: RG.priority(e[0]))
    assert first in rounds[0]
    # an edge is taken exactly when no pending edge within one ring comes before it
    pending = list(edges)
    for rnd in rounds:
        taken = {e[0] for e in rnd}
        for e in pending:
            near = {e[1], e[2], *topo.ring[e[1]], *topo.ring[e[2]]}
            blocked = any(RG.priority(f[0]) < RG.priority(e[0]) and (f[1] in near or f[2] in near) for f in pending)
            assert (e[0] in taken) == (not blocked), e
        pending = [e for e in pending if e[0] not in taken]
    for rnd in rounds:
        for e in rnd:
            near = {e[1], e[2], *topo.ring[e[1]], *topo.ring[e[2]]}
            for f in rnd:
                if f is not e:
                    assert f[1] not in near and f[2] not in near
