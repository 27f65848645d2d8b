"""Fixtures under tests/golden: values fixed by the paper's text or by a hand
derivation, each file citing its source."""
import os
from fractions import Fraction

import numpy as np

from paper_2505_06932_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = v
    return out


def test_default_fit_parameters_follow_the_paper(oracle):
    g = _read("ppic_parameters.txt")
    p = oracle.PPICParams()
    assert p.delta_over_h == float(g["delta_over_h"][0])
    assert p.rings == int(g["rings"][0])
    assert int(g["n_min_weighted_lower"][0]) <= p.n_min <= int(g["n_min_weighted_upper"][0])


def test_golden_sphere_kappa(oracle):
    g = _read("ppic_parameters.txt")
    r = 0.41
    k = oracle.kappa_of([0, 0, 0, -1 / (2 * r), 0, -1 / (2 * r)])
    assert abs(k * r - float(g["sphere_kappa_times_r"][0])) < 1e-14


def test_golden_tet_corner(oracle):
    g = _read("tet_corner.txt")
    nx, ny, nz = (int(v) for v in g["grid"][:3])
    x0, y0, z0, h = (float(v) for v in g["grid"][3:])
    grid = I.Grid(nx, ny, nz, x0, y0, z0, h)
    c = np.array([float(v) for v in g["corner"]])
    s = float(g["leg"][0])
    m = I.tetra_mesh(c, c + [s, 0, 0], c + [0, s, 0], c + [0, 0, s])
    alpha, isif = oracle.volume_fraction(grid, m)
    i, j, k = (int(v) for v in g["cell"])
    want = Fraction(int(g["alpha_num"][0]), int(g["alpha_den"][0]))
    assert abs(alpha[k, j, i] - float(want)) <= 1e-15
    assert isif.sum() == 1
