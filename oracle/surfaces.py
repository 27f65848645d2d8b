"""Exact mean curvature of the spherical-harmonic perturbed spheres (test
infrastructure only): the reference that the PPIC fit and the learned
surrogate are both measured against.

A droplet's surface is r(u) = R (1 + A f(u) / fmax), f = sum c_lm Y_lm(u),
around its centre c (paper_2505_06932_amd.inputs.sh_spheres_workload).  It is
the zero set of F(x) = |x - c| - r((x - c) / |x - c|); with the outward
normal n = grad F / |grad F|, the curvature is kappa = div n =
(|g|^2 tr H - g.H.g) / |g|^3 (g, H the gradient and Hessian of F), 2/R on a
sphere.  g and H come from central differences of F in double precision
with step 1e-4 R (truncation and rounding both near 1e-8 relative)."""
from __future__ import annotations

import numpy as np


def _f(surface, u):
    from paper_2505_06932_amd.inputs import real_sph_harm
    out = np.zeros(len(u))
    for l, m, c in surface["coef"]:
        out += c * real_sph_harm(l, m, u)
    return out


def radius(surface, u) -> np.ndarray:
    """r(u) for unit vectors u [n, 3]."""
    A, fm = surface["A"], surface["fmax"]
    return surface["R"] * (1.0 + (A * _f(surface, u) / fm if fm > 0.0 else 0.0))


def level(surface, x) -> np.ndarray:
    d = np.asarray(x, dtype=np.float64) - surface["centre"]
    rho = np.linalg.norm(d, axis=1)
    return rho - radius(surface, d / rho[:, None])


def project(surface, x) -> np.ndarray:
    """Radial projection of points onto the surface."""
    d = np.asarray(x, dtype=np.float64) - surface["centre"]
    u = d / np.linalg.norm(d, axis=1)[:, None]
    return surface["centre"] + u * radius(surface, u)[:, None]


def mean_curvature(surface, x) -> np.ndarray:
    """kappa = div(grad F / |grad F|) at points x [n, 3] (on the surface)."""
    x = np.asarray(x, dtype=np.float64)
    d = 1e-4 * surface["R"]
    E = np.eye(3) * d
    F0 = level(surface, x)
    g = np.empty((len(x), 3))
    H = np.empty((len(x), 3, 3))
    Fp = [level(surface, x + E[a]) for a in range(3)]
    Fm = [level(surface, x - E[a]) for a in range(3)]
    for a in range(3):
        g[:, a] = (Fp[a] - Fm[a]) / (2 * d)
        H[:, a, a] = (Fp[a] - 2 * F0 + Fm[a]) / (d * d)
    for a in range(3):
        for b in range(a + 1, 3):
            v = (level(surface, x + E[a] + E[b]) - level(surface, x + E[a] - E[b])
                 - level(surface, x - E[a] + E[b]) + level(surface, x - E[a] - E[b])) / (4 * d * d)
            H[:, a, b] = H[:, b, a] = v
    gg = np.einsum("ia,ia->i", g, g)
    tr = np.trace(H, axis1=1, axis2=2)
    gHg = np.einsum("ia,iab,ib->i", g, H, g)
    return (gg * tr - gHg) / gg ** 1.5


def nearest_surface(surfaces, x) -> np.ndarray:
    """Index of the droplet whose centre is closest to each point."""
    C = np.array([s["centre"] for s in surfaces])
    return np.argmin(((np.asarray(x)[:, None, :] - C[None]) ** 2).sum(-1), axis=1)
