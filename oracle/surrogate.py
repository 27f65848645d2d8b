"""Learned curvature surrogate: the plain CPU definitions its GPU kernels are
checked against.  Test infrastructure only: nothing in the product imports it.

The surrogate replaces the PPIC volume fit (paper sec. 3.2) where it is
trusted.  Its input is what the fit sees around an interfacial cell, in a
form a small network can take: the 27 volume fractions of the 3x3x3 block of
cells centred on the cell (the exact polyhedral fractions of sec. 3.1) and
the frame normal of the fit (the area-weighted normal of the front vertex
closest to the cell centre, sec. 3.2 step 2).  Its output is kappa h.

Network: 30 -> 64 -> 64 -> 1, tanh hidden units, a linear output.  The
product evaluates it with bfloat16 operands and single-precision sums; the
forward and backward passes here have a flag, `quant`, that rounds to
bfloat16 at exactly the points where the product does, so that the two agree
to single-precision rounding.  With quant=False they are the exact
double-precision network and its exact gradient.

  * features: x_hi = bf16(x), x_lo = bf16(x - x_hi) for each of the 30 single
    precision inputs (the pair keeps 16 significant bits of every volume
    fraction); the first layer sees both through the same weights;
  * weights W1, W2, w3 rounded to bf16; biases kept in single precision;
  * activations h1, h2 rounded to bf16 after tanh;
  * backward: the loss gradient dy = 2 (y - t) / B (mean squared error over a
    batch of B samples); dz2 = bf16(dy w3 (1 - h2^2)) and dz1 =
    bf16((W2^T dz2) (1 - h1^2)), the derivative of tanh taken from the stored
    (rounded) activation; every weight gradient is a sum over samples of a
    rounded dz times a rounded activation (x_hi + x_lo for the first layer);
    bias gradients sum the rounded dz.

Error estimate: the network is not equivariant, but kappa is invariant under
the 48 symmetries of the cube applied to the stencil and the normal
together.  The estimate is the spread (max - min) of the predictions over a
fixed set of four of them; the prediction is their mean, ((y0 + y1) + (y2 +
y3)) / 4.  A cell falls back to the PPIC fit when the spread exceeds a stated
bound, or when the closest vertex is not within 1.5 h of the cell centre (the
cell-list build then has no final closest vertex for it).

Parameter vector theta (single precision, 6209 values): W1 [64][30] row-major
(row = hidden unit), b1 [64], W2 [64][64] row-major (row = output unit), b2
[64], w3 [64], b3 [1].
"""
from __future__ import annotations

import itertools

import numpy as np

N_IN, N_HID = 30, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_HID * N_IN
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID
NP = OFF_B3 + 1

# the six permutations of the axes in lexicographic order
_PERMS = list(itertools.permutations(range(3)))
# the four symmetries of the error estimate: identity, a quarter turn about
# z, the cyclic exchange of the axes, the point reflection
ERROR_SET = (0, 17, 24, 7)


def cube_matrix(sym: int) -> np.ndarray:
    """Symmetry sym in [0, 48) of the cube as a signed permutation matrix:
    permutation sym // 8 of the axes (lexicographic order), axis a negated
    where bit a of sym % 8 is set; (P x)_a = s_a x_perm[a]."""
    perm, signs = _PERMS[sym // 8], sym % 8
    P = np.zeros((3, 3), dtype=np.int64)
    for a in range(3):
        P[a, perm[a]] = -1 if (signs >> a) & 1 else 1
    return P


def offsets() -> np.ndarray:
    """The 27 stencil offsets (di, dj, dk), entry q = 9 (dk+1) + 3 (dj+1) + (di+1)."""
    return np.array([(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)],
                    dtype=np.int64)


def stencil(grid, alpha, cell_ids) -> np.ndarray:
    """Volume fractions of the 3x3x3 block around each listed cell, [n, 27]
    (alpha is the dense field [nz, ny, nx]); cells outside the grid read 0."""
    ids = np.asarray(cell_ids, dtype=np.int64)
    i, j, k = ids % grid.nx, (ids // grid.nx) % grid.ny, ids // (grid.nx * grid.ny)
    out = np.zeros((len(ids), 27))
    for q, (di, dj, dk) in enumerate(offsets()):
        ii, jj, kk = i + di, j + dj, k + dk
        inside = (ii >= 0) & (ii < grid.nx) & (jj >= 0) & (jj < grid.ny) & (kk >= 0) & (kk < grid.nz)
        out[inside, q] = alpha[kk[inside], jj[inside], ii[inside]]
    return out


def features(grid, mesh, alpha, cell_ids):
    """Network inputs [n, 30] (27 volume fractions, frame normal) and whether
    each cell has a final closest vertex (within 1.5 h of its centre)."""
    import oracle
    _, d2, nrm = oracle.frame_normal(grid, mesh, cell_ids)
    reach2 = (1.5 * grid.h) ** 2 * (1.0 - 1e-12)
    return np.concatenate([stencil(grid, alpha, cell_ids), nrm], axis=1), d2 < reach2


def transform(F, sym: int) -> np.ndarray:
    """Features of the configuration mapped by symmetry sym: the field
    alpha'(x) = alpha(P^T x) has stencil entry alpha'(d) = alpha(P^T d); the
    normal maps to P n."""
    P = cube_matrix(sym)
    F = np.asarray(F, dtype=np.float64)
    out = np.empty_like(F)
    off = offsets()
    for q, d in enumerate(off):
        e = P.T @ d
        qe = 9 * (e[2] + 1) + 3 * (e[1] + 1) + (e[0] + 1)
        out[:, q] = F[:, qe]
    out[:, 27:30] = F[:, 27:30] @ P.T.astype(np.float64)
    return out


def bf16(x) -> np.ndarray:
    """Nearest bfloat16 (ties to even) of the single-precision value of x."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    assert t.shape == (NP,)
    return dict(W1=t[OFF_W1:OFF_B1].reshape(N_HID, N_IN), b1=t[OFF_B1:OFF_W2],
                W2=t[OFF_W2:OFF_B2].reshape(N_HID, N_HID), b2=t[OFF_B2:OFF_W3], w3=t[OFF_W3:OFF_B3],
                b3=float(t[OFF_B3]))


def _forward(theta, F, quant):
    p = unpack(np.asarray(theta, dtype=np.float32) if quant else theta)
    F = np.asarray(F, dtype=np.float64)
    if quant:
        x = F.astype(np.float32).astype(np.float64)
        xh = bf16(x)
        xl = bf16(x - xh)
        W1, W2, w3 = bf16(p["W1"]), bf16(p["W2"]), bf16(p["w3"])
        z1 = xh @ W1.T + xl @ W1.T + p["b1"]
        h1 = bf16(np.tanh(z1))
        z2 = h1 @ W2.T + p["b2"]
        h2 = bf16(np.tanh(z2))
        xs = xh + xl
    else:
        W1, W2, w3 = p["W1"], p["W2"], p["w3"]
        z1 = F @ W1.T + p["b1"]
        h1 = np.tanh(z1)
        z2 = h1 @ W2.T + p["b2"]
        h2 = np.tanh(z2)
        xs = F
    y = h2 @ w3 + p["b3"]
    return y, dict(xs=xs, h1=h1, h2=h2, W2=W2, w3=w3)


def forward(theta, F, quant: bool = True) -> np.ndarray:
    """Network output (kappa h) for every row of F [n, 30]."""
    return _forward(theta, F, quant)[0]


def loss_grad(theta, F, t, quant: bool = True):
    """Mean squared error over the batch and its gradient [NP] (for quant=True,
    the gradient of the rounded network as the product forms it)."""
    y, c = _forward(theta, F, quant)
    t = np.asarray(t, dtype=np.float64)
    B = len(t)
    r = y - t
    loss = float(np.sum(r * r) / B)
    dy = 2.0 * r / B
    q = bf16 if quant else (lambda a: a)
    h1, h2 = c["h1"], c["h2"]
    dz2 = q(dy[:, None] * c["w3"][None, :] * (1.0 - h2 * h2))
    dz1 = q((dz2 @ c["W2"]) * (1.0 - h1 * h1))
    g = np.zeros(NP)
    g[OFF_W1:OFF_B1] = (dz1.T @ c["xs"]).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(0)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(0)
    g[OFF_W3:OFF_B3] = dy @ h2
    g[OFF_B3] = dy.sum()
    return loss, g


def adam(theta, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, ICLR 2015) with bias correction; step
    counts from 1.  Returns (theta, m, v)."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(theta, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(theta, F, quant: bool = True):
    """Predictions over the error set: (mean kappa h, spread) per row of F."""
    Y = np.stack([forward(theta, transform(F, s), quant) for s in ERROR_SET])
    mean = ((Y[0] + Y[1]) + (Y[2] + Y[3])) / 4.0
    return mean, Y.max(0) - Y.min(0)


def learned_curvature(grid, mesh, alpha, cell_ids, theta, bound: float, ppic_kappa):
    """Curvature of every listed cell: the surrogate's mean prediction / h
    where its spread is at most `bound` (in units of kappa h) and the cell has
    a final closest vertex, the PPIC curvature (given) elsewhere.  Returns
    (kappa, fallback mask, spread)."""
    F, final = features(grid, mesh, alpha, cell_ids)
    mean, spread = predict(theta, F)
    fb = ~final | ~(spread <= bound)
    kappa = np.where(fb, ppic_kappa, mean / grid.h)
    return kappa, fb, spread
