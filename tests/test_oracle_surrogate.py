"""Pins of the learned-curvature oracle (oracle/surrogate.py) against what the
mathematics fixes: the cube group, the stencil of a rotated front computed by
the volume-fraction oracle, the exact gradient by central differences, the
closed form of Adam's first step, bfloat16 rounding by torch's conversion, and
predictions of networks whose symmetry is known."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import surrogate as S
from paper_2505_06932_amd import inputs as I


def test_cube_group():
    mats = [S.cube_matrix(s) for s in range(48)]
    keys = {m.tobytes() for m in mats}
    assert len(keys) == 48
    for m in mats:
        assert np.array_equal(m @ m.T, np.eye(3, dtype=np.int64))
        assert abs(round(np.linalg.det(m))) == 1
    # closed under products
    for a in mats[::5]:
        for b in mats[::7]:
            assert (a @ b).tobytes() in keys
    # the error set: identity, quarter turn about z, cyclic exchange, point reflection
    x = np.array([1, 2, 3])
    got = [tuple(S.cube_matrix(s) @ x) for s in S.ERROR_SET]
    assert got == [(1, 2, 3), (-2, 1, 3), (2, 3, 1), (-1, -2, -3)]


def test_offsets_order():
    off = S.offsets()
    assert off.shape == (27, 3)
    assert tuple(off[13]) == (0, 0, 0)
    assert tuple(off[14]) == (1, 0, 0) and tuple(off[16]) == (0, 1, 0) and tuple(off[22]) == (0, 0, 1)


def test_transform_matches_rotated_function():
    """Stencil of f sampled at cell centres around c, mapped by P, equals the
    stencil of f(c + P^T (x - c)); the normal maps to P n."""
    rng = np.random.default_rng(3)
    coef = rng.normal(size=10)

    def f(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return (coef[0] + coef[1] * x + coef[2] * y * y + coef[3] * z ** 3 + coef[4] * x * y
                + coef[5] * y * z * z + coef[6] * np.sin(x + 2 * z) + coef[7] * x * y * z)

    c = rng.normal(size=3)
    h = 0.37
    off = S.offsets().astype(np.float64)
    F = np.concatenate([f(c + h * off), [0.6, -0.48, 0.64]])[None, :]
    for s in range(48):
        P = S.cube_matrix(s).astype(np.float64)
        want = np.concatenate([f(c + h * (off @ P)), P @ F[0, 27:]])  # rows of off @ P are P^T d
        assert np.allclose(S.transform(F, s)[0], want, rtol=0, atol=1e-13)


def test_transform_composes():
    rng = np.random.default_rng(4)
    F = rng.normal(size=(5, 30))
    for a in (3, 17, 24, 40):
        for b in (7, 11, 30):
            ab = [s for s in range(48) if np.array_equal(S.cube_matrix(s), S.cube_matrix(b) @ S.cube_matrix(a))][0]
            assert np.array_equal(S.transform(S.transform(F, a), b), S.transform(F, ab))


def _mapped_mesh(mesh, P, c0):
    v = (mesh.verts() - c0) @ P.T.astype(np.float64) + c0
    t = mesh.tris()
    if round(np.linalg.det(P)) < 0:
        t = t[:, [0, 2, 1]]
    return I.Mesh.from_arrays(v, t)


@pytest.mark.parametrize("sym", [17, 24, 7, 45])
def test_stencil_of_mapped_front(sym):
    """Features of the front mapped by a cube symmetry about a cell centre,
    computed from scratch by the volume-fraction and frame-normal oracles,
    equal the mapped features of the original front."""
    grid, mesh, _ = I.sphere_workload(24, 0.27, 3, seed=5, noise_over_h=0.05)
    h = grid.h
    c0 = np.array([11.5, 12.5, 11.5]) * h  # a cell centre: the map permutes the cells
    P = S.cube_matrix(sym)
    mesh2 = _mapped_mesh(mesh, P, c0)
    alpha, _ = oracle.volume_fraction(grid, mesh)
    alpha2, _ = oracle.volume_fraction(grid, mesh2)
    cells, _, _ = oracle.cell_lists(grid, mesh)
    F, final = S.features(grid, mesh, alpha, cells)
    ijk = np.stack([cells % grid.nx, (cells // grid.nx) % grid.ny, cells // (grid.nx * grid.ny)], 1)
    cen = (ijk + 0.5) * h
    ijk2 = np.rint((cen - c0) @ P.T.astype(np.float64) / h + c0 / h - 0.5).astype(np.int64)
    inside = np.all((ijk2 >= 1) & (ijk2 < grid.nx - 1), axis=1) & np.all((ijk >= 1) & (ijk < grid.nx - 1), axis=1)
    cells2 = ijk2[:, 0] + grid.nx * (ijk2[:, 1] + grid.ny * ijk2[:, 2])
    F2, final2 = S.features(grid, mesh2, alpha2, cells2)
    assert inside.sum() > 100
    assert np.array_equal(final[inside], final2[inside])
    G = S.transform(F[inside], sym)
    assert np.abs(G[:, :27] - F2[inside, :27]).max() < 1e-12
    assert np.abs(G[:, 27:] - F2[inside, 27:]).max() < 1e-12


def test_frame_normal_icosahedron_radial():
    """Every vertex normal of a regular icosahedron points along the radius."""
    unit, tris = I.icosahedron()
    unit = unit / np.linalg.norm(unit, axis=1)[:, None]
    c = np.array([0.5, 0.5, 0.5])
    mesh = I.Mesh.from_arrays(c + 0.3 * unit, tris)
    grid = I.Grid(16, 16, 16, 0.0, 0.0, 0.0, 1.0 / 16)
    cells, _, _ = oracle.cell_lists(grid, mesh)
    vs, d2, n = oracle.frame_normal(grid, mesh, cells)
    assert np.abs(n - unit[vs]).max() < 1e-15
    # closest vertex by brute force on the host
    ijk = np.stack([cells % 16, (cells // 16) % 16, cells // 256], 1)
    cen = (ijk + 0.5) / 16
    dd = ((cen[:, None, :] - mesh.verts()[None]) ** 2).sum(-1)
    assert np.array_equal(vs, dd.argmin(1)) and np.allclose(d2, dd.min(1), rtol=0, atol=1e-15)


def test_bf16_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, size=5000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, -(1.0 + 3 * 2 ** -8)]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), want)
    assert S.bf16([1.0 + 2 ** -8])[0] == 1.0  # a tie goes to the even neighbour
    assert S.bf16([1.0 + 2 ** -8 + 2 ** -20])[0] == 1.0 + 2 ** -7


def _theta(rng, scale=0.3):
    th = rng.normal(size=S.NP) * scale
    return th


def test_gradient_central_differences():
    rng = np.random.default_rng(7)
    th = _theta(rng)
    F = rng.uniform(0, 1, size=(9, 30))
    t = rng.normal(size=9)
    _, g = S.loss_grad(th, F, t, quant=False)
    eps = 1e-6
    idx = np.concatenate([rng.choice(S.NP, 60, replace=False), [S.OFF_B1 + 3, S.OFF_W2 + 70, S.OFF_W3 + 5, S.OFF_B3]])
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (S.loss_grad(tp, F, t, quant=False)[0] - S.loss_grad(tm, F, t, quant=False)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), k


def test_quantised_network_close_to_exact():
    """Rounding at the product's points changes outputs and gradients by a
    few bfloat16 units only."""
    rng = np.random.default_rng(8)
    th = _theta(rng, 0.2).astype(np.float32).astype(np.float64)
    F = rng.uniform(0, 1, size=(256, 30))
    t = rng.normal(size=256)
    yq, y = S.forward(th, F, True), S.forward(th, F, False)
    assert np.abs(yq - y).max() < 0.05 * np.abs(y).max()
    _, gq = S.loss_grad(th, F, t, True)
    _, g = S.loss_grad(th, F, t, False)
    assert np.linalg.norm(gq - g) < 0.03 * np.linalg.norm(g)


def test_quantised_forward_hand_case():
    """A network whose every weight, bias and input is a bfloat16 value and
    whose hidden layers see exact values: one hidden unit per layer active."""
    th = np.zeros(S.NP)
    W1 = th[S.OFF_W1:S.OFF_B1].reshape(64, 30)
    W1[0, 13] = 0.5        # h1[0] = tanh(0.5 alpha_centre)
    W2 = th[S.OFF_W2:S.OFF_B2].reshape(64, 64)
    W2[5, 0] = 2.0         # h2[5] = tanh(2 h1[0] + b2[5])
    th[S.OFF_B2 + 5] = 0.25
    th[S.OFF_W3 + 5] = -1.5
    th[S.OFF_B3] = 0.125
    F = np.zeros((1, 30))
    F[0, 13] = 0.75
    h1 = S.bf16(math.tanh(0.375))[0]
    h2 = S.bf16(math.tanh(2 * h1 + 0.25))[0]
    assert S.forward(th, F)[0] == pytest.approx(-1.5 * h2 + 0.125, abs=1e-15)
    # the low part carries the bits bfloat16 drops: alpha = 1/3
    F[0, 13] = np.float32(1 / 3)
    x = np.float64(np.float32(1 / 3))
    xh = S.bf16(x)[0]
    xl = S.bf16(x - xh)[0]
    assert abs(xh + xl - x) < 2 ** -16 * x
    h1 = S.bf16(math.tanh(0.5 * xh + 0.5 * xl))[0]
    h2 = S.bf16(math.tanh(2 * h1 + 0.25))[0]
    assert S.forward(th, F)[0] == pytest.approx(-1.5 * h2 + 0.125, abs=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(9)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = S.adam(th, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    assert np.allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_quadratic():
    th = np.array([3.0, -2.0, 0.5])
    m = v = np.zeros(3)
    for k in range(1, 3001):
        th, m, v = S.adam(th, m, v, 2 * th, k, 0.01)
    assert np.abs(th).max() < 1e-2


def test_training_reduces_loss_on_a_smooth_target():
    """Plain gradient steps on the quantised network lower the loss on a
    target that depends smoothly on the stencil."""
    rng = np.random.default_rng(10)
    th = _theta(rng, 0.1)
    th[S.OFF_W3:S.OFF_B3] *= 0.1
    F = rng.uniform(0, 1, size=(512, 30))
    t = 0.3 * (F[:, 14] - F[:, 12]) + 0.2 * F[:, 29]
    l0, _ = S.loss_grad(th, F, t)
    m = v = np.zeros(S.NP)
    for k in range(1, 201):
        _, g = S.loss_grad(th, F, t)
        th, m, v = S.adam(th, m, v, g, k, 3e-3)
    l1, _ = S.loss_grad(th, F, t)
    assert l1 < 0.2 * l0


def test_predict_symmetric_networks():
    rng = np.random.default_rng(11)
    F = rng.uniform(0, 1, size=(40, 30))
    F[:, 27:] /= np.linalg.norm(F[:, 27:], axis=1)[:, None]
    # output = b3 only: no spread
    th = np.zeros(S.NP)
    th[S.OFF_B3] = 0.375
    mean, spread = S.predict(th, F)
    assert np.all(mean == 0.375) and np.all(spread == 0.0)
    # reads the centre volume fraction only: invariant under every symmetry
    th = np.zeros(S.NP)
    th[S.OFF_W1 + 13] = 1.0
    th[S.OFF_W2 + 0] = 1.0
    th[S.OFF_W3 + 0] = 1.0
    mean, spread = S.predict(th, F)
    assert np.all(spread == 0.0)
    # reads n_z: the four symmetries see n_z, n_z, n_x, -n_z
    th = np.zeros(S.NP)
    th[S.OFF_W1 + 29] = 0.5
    th[S.OFF_W2 + 0] = 1.0
    th[S.OFF_W3 + 0] = 1.0
    _, spread = S.predict(th, F, quant=False)
    y = lambda nz: np.tanh(np.tanh(0.5 * nz))
    Y = np.stack([y(F[:, 29]), y(F[:, 29]), y(F[:, 27]), y(-F[:, 29])])
    assert np.allclose(spread, Y.max(0) - Y.min(0), rtol=0, atol=1e-15)


def test_learned_curvature_fallback_rule():
    grid, mesh, _ = I.sphere_workload(24, 0.3, 3, seed=2, noise_over_h=0.0)
    alpha, _ = oracle.volume_fraction(grid, mesh)
    cells, _, _ = oracle.cell_lists(grid, mesh)
    ppic = oracle.ppic(grid, mesh, cells)["kappa"]
    th = np.zeros(S.NP)
    th[S.OFF_W1 + 27] = 1.0  # spread grows with |n_x - n_y| and the like
    th[S.OFF_W2] = 1.0
    th[S.OFF_W3] = 0.1
    th[S.OFF_B3] = 0.2
    k, fb, spread = S.learned_curvature(grid, mesh, alpha, cells, th, 0.05, ppic)
    assert 0 < fb.sum() < len(cells)
    assert np.array_equal(fb, spread > 0.05)
    assert np.array_equal(k[fb], ppic[fb])
    mean, _ = S.predict(th, S.features(grid, mesh, alpha, cells)[0])
    assert np.array_equal(k[~fb], mean[~fb] / grid.h)


def test_committed_parameters_predict_sphere_curvature():
    """The trained parameters shipped with the package, evaluated by the
    oracle's network on the R = 8h sphere (inside the training range): the
    trusted cells' kappa agrees with the exact 2/R to a few percent."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2505_06932_amd",
                        "surrogate_theta.npy")
    th = np.load(path, allow_pickle=False)
    assert th.shape == (S.NP,) and th.dtype == np.float32 and np.all(np.isfinite(th))
    grid, mesh, _ = I.make_workload("sphere_32", 0)
    alpha, _ = oracle.volume_fraction(grid, mesh)
    cells, _, _ = oracle.cell_lists(grid, mesh)
    F, final = S.features(grid, mesh, alpha, cells)
    mean, spread = S.predict(th.astype(np.float64), F)
    trusted = final & (spread <= 0.01)
    assert trusted.mean() > 0.5
    rel = np.abs(mean[trusted] / grid.h / (2.0 / 0.25) - 1.0)
    assert np.median(rel) < 0.05
