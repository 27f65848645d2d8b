"""Pins of the exact-curvature reference (oracle/surfaces.py): a sphere's
2/R, and the linearised mean curvature of a perturbed sphere,
kappa = 2/R + (eps/R)(l - 1)(l + 2) Y_lm + O(eps^2) for r = R (1 + eps Y_lm)
(Y_lm an eigenfunction of the sphere's Laplacian with eigenvalue
-l(l + 1))."""
import numpy as np
import pytest

from oracle import surfaces as SF
from paper_2505_06932_amd import inputs as I


def _points(n, seed):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    return u / np.linalg.norm(u, axis=1)[:, None]


def test_sphere():
    s = dict(centre=np.array([0.3, -0.2, 0.5]), R=0.37, A=0.0, coef=[(2, 0, 1.0)], fmax=1.0)
    x = s["centre"] + 0.37 * _points(200, 1)
    assert np.allclose(SF.mean_curvature(s, x), 2 / 0.37, rtol=1e-7, atol=0)


@pytest.mark.parametrize("l,m", [(2, 0), (3, -2), (5, 4), (8, 1)])
def test_linearised_perturbation(l, m):
    eps, R = 1e-4, 0.25
    s = dict(centre=np.zeros(3), R=R, A=eps, coef=[(l, m, 1.0)], fmax=1.0)
    u = _points(300, l + 10 * m + 50)
    x = SF.project(s, u)
    Y = I.real_sph_harm(l, m, u)
    want = 2 / R + (eps / R) * (l - 1) * (l + 2) * Y
    # second-order remainder: a few eps^2 l^4 / R
    assert np.abs(SF.mean_curvature(s, x) - want).max() < 20 * eps ** 2 * l ** 4 / R + 1e-6 / R


def test_workload_surfaces_match_the_mesh():
    grid, mesh, info, surfs = I.sh_spheres_workload(64, 2, seed=3, r_lo=4.0, r_hi=8.0, return_surfaces=True)
    g2, m2, info2 = I.sh_spheres_workload(64, 2, seed=3, r_lo=4.0, r_hi=8.0)
    assert np.array_equal(mesh.verts(), m2.verts())  # the same draws with or without the surfaces
    v = mesh.verts()
    k = SF.nearest_surface(surfs, v)
    for i, s in enumerate(surfs):
        assert np.abs(SF.level(s, v[k == i])).max() < 1e-12 * s["R"]
