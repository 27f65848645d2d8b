"""Pins for the oracle's RK4 vertex advection (paper sec. 3.1: the front
vertices move with the interpolated velocity, classical fourth-order
Runge-Kutta, the face velocities held fixed over the step)."""
import numpy as np
import pytest

from paper_2505_06932_amd import inputs as I

GRID = I.Grid(16, 14, 12, -0.2, 0.1, 0.05, 0.0625)


def _interior_points(g, n, rng, margin=3.0):
    lo = np.array([g.x0, g.y0, g.z0]) + margin * g.h
    hi = np.array([g.x0 + g.nx * g.h, g.y0 + g.ny * g.h, g.z0 + g.nz * g.h]) - margin * g.h
    return lo + rng.uniform(size=(n, 3)) * (hi - lo)


def test_uniform_field_translates(oracle):
    u0 = np.array([0.3, -1.1, 0.45])
    U, V, W = I.uniform_face_velocity(GRID, u0)
    p = _interior_points(GRID, 300, np.random.default_rng(0))
    out = oracle.advect_rk4(GRID, p[:, 0], p[:, 1], p[:, 2], U, V, W, 0.02)
    assert np.abs(out - (p + 0.02 * u0)).max() <= 4e-16 * (np.abs(p).max() + 1)


@pytest.mark.parametrize("seed", range(3))
def test_affine_field_gives_the_rk4_polynomial(oracle, seed):
    """The interpolant reproduces affine fields u = c + B x, and for the
    linear system dx/dt = B x + c one RK4 step is
    x + h (I + hB/2 + (hB)^2/6 + (hB)^3/24) (B x + c)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=3)
    B = rng.normal(size=(3, 3))
    U, V, W = I.affine_face_velocity(GRID, c, B)
    p = _interior_points(GRID, 300, rng, margin=4.0)
    h = 0.01
    out = oracle.advect_rk4(GRID, p[:, 0], p[:, 1], p[:, 2], U, V, W, h)
    M = h * B
    P = np.eye(3) + M / 2 + M @ M / 6 + M @ M @ M / 24
    ref = p + h * (p @ B.T + c) @ P.T
    assert np.abs(out - ref).max() <= 1e-13


def test_fourth_order_within_a_cell(oracle):
    """Inside one cell the interpolant is a fixed polynomial, so the step's
    error against a finely sub-stepped solution falls 16-fold when dt
    halves (global fourth order: local error order five, 32-fold per step,
    here compared over a fixed time with 1, 2, 4 steps)."""
    g = I.Grid(16, 16, 16, 0.0, 0.0, 0.0, 1.0 / 16)
    U, V, W = I.psi_face_velocity(g)
    p0 = np.array([[5.5, 6.5, 7.5]]) * g.h  # a cell centre

    def run(n, T):
        p = p0.copy()
        for _ in range(n):
            p = oracle.advect_rk4(g, p[:, 0], p[:, 1], p[:, 2], U, V, W, T / n)
        return p[0]

    T = 0.02  # |u| <= 1: the point moves less than a third of a cell
    ref = run(512, T)
    e = [np.linalg.norm(run(n, T) - ref) for n in (1, 2, 4)]
    assert 12.0 < e[0] / e[1] < 20.0 and 12.0 < e[1] / e[2] < 20.0


def test_leaving_the_grid_is_reported(oracle):
    u0 = np.array([1.0, 0.0, 0.0])
    U, V, W = I.uniform_face_velocity(GRID, u0)
    x_edge = GRID.x0 + (GRID.nx - 1) * GRID.h - 1e-3  # in cell nx - 2, the last admissible one
    out = oracle.advect_rk4(GRID, np.array([x_edge, 0.5]), np.array([0.5, 0.5]), np.array([0.4, 0.4]), U, V, W,
                            0.05, check=False)
    assert np.all(np.isnan(out[0])) and np.all(np.isfinite(out[1]))
    with pytest.raises(Exception):
        oracle.advect_rk4(GRID, np.array([x_edge]), np.array([0.5]), np.array([0.4]), U, V, W, 0.05)
