"""Local roughness detection and volume-conserving edge smoothing of the front
(paper section 3.4): plain CPU definitions the GPU kernels are checked
against.  Test infrastructure only.

Topology of a closed, consistently oriented triangle mesh:
  * the one-ring N1(i) of vertex i: the vertices sharing an edge with it;
  * an undirected edge {a, b} is identified by its half-edge a -> b with
    a < b, i.e. by 3 t + k for the triangle t whose corners k, k+1 (mod 3)
    are a, b in that order; this id orders the edges;
  * the triangles T1(i) incident to i, and T2(i) the triangles with a
    corner in {i} plus N1(i) (the two-ring of triangles).

Metrics (sec. 3.4):
  * geometric Laplacian GL_i = x_i - sum_j w_ij x_j / sum_j w_ij over
    N1(i), w_ij = 1 / |x_i - x_j|; its length is the first metric;
  * edge roughness R_e = 1 - n_1 . n_2 (unit normals of the two triangles
    at the edge);
  * per vertex G_i, V_i: mean and variance (population, divided by the
    number of edges) of R_e over the edges at i;
  * per triangle R_t = sum G_i V_i / sum V_i over its corners (the plain
    mean of the G_i when every V_i is 0);
  * per vertex R^l_i = sum over T_l(i) of A_t R_t, divided by |T_l(i)|,
    l = 1, 2, and R_i = max(R^1_i, R^2_i), the second metric.

Smoothing (sec. 3.4, after Kuprat et al., J. Comput. Phys. 2001, their
algorithm 4): a vertex is rough when |GL_i| and R_i both exceed their
thresholds; an edge is smoothed when both its vertices are rough.  For edge
(v1, v2), with n_i = |N1(v_i)| and S_1, S_2 the sums of the one-ring
positions of v1 without v2 and of v2 without v1, the simultaneous Laplacian
positions are x1s = (S_2 + n_2 S_1) / (n_1 n_2 - 1), x2s = (x1s + S_2) / n_2.
With d_i = x_is - x_i, the vertices move to x_i + d_i + h n: the enclosed
volume V = (1/6) sum_t x_t0 . (x_t1 x x_t2) then changes by exactly
(c + h n . g) / 6, with
    g = A_1 + A_2 + y x (d_1 - d_2),  c = d_1 . A_1 + d_2 . A_2 + d_1 . (d_2 x y),
A_i = sum over the triangles (v_i, a, b) at v_i (corners in cyclic order
from v_i) of (a - x_i) x (b - x_i), and y = y_a - y_b, the far corners of
the triangle holding the half-edge v1 -> v2 and of the one holding v2 -> v1.
The displacement of least length that conserves the volume is along g:
n = g / |g| and h = -c / |g|.  (The text prints the last term of the
numerator of h as d_1 . (y x d_1), which vanishes identically; the term the
volume requires is d_1 . (d_2 x y).)  An edge with g = 0 is left alone.

Schedule: the flagged edges are smoothed in rounds; in each round an edge is
taken when no other edge still pending lies within one ring of it (an end of
one is an end or a one-ring vertex of an end of the other) and comes before
it in the priority order: edges by (fmix32(id), id), fmix32 the 32-bit
finalizer of MurmurHash3 (Appleby), which scatters neighbouring ids so that
the rounds stay few.  Edges of one round move disjoint vertices and read no
vertex another one moves, so each round is the same as smoothing its edges
one by one.
"""
from __future__ import annotations

import numpy as np


class Topology:
    def __init__(self, tris: np.ndarray, nv: int):
        self.tris = np.asarray(tris, dtype=np.int64)
        self.nv = nv
        nt = len(self.tris)
        self.inc = [[] for _ in range(nv)]  # incident triangles, ascending
        for t in range(nt):
            for k in range(3):
                self.inc[self.tris[t, k]].append(t)
        self.ring = []  # N1(i), in the order of the incident triangles (the corner after i)
        for i in range(nv):
            r = []
            for t in self.inc[i]:
                k = int(np.nonzero(self.tris[t] == i)[0][0])
                r.append(int(self.tris[t, (k + 1) % 3]))
            self.ring.append(r)
        # half-edge -> triangle holding it
        self.half = {}
        for t in range(nt):
            for k in range(3):
                a, b = int(self.tris[t, k]), int(self.tris[t, (k + 1) % 3])
                self.half[(a, b)] = (t, k)
        self.edges = []  # (id, a, b) with a < b, ascending id
        for t in range(nt):
            for k in range(3):
                a, b = int(self.tris[t, k]), int(self.tris[t, (k + 1) % 3])
                if a < b:
                    self.edges.append((3 * t + k, a, b))

    def far_corner(self, a, b):
        t, k = self.half[(a, b)]
        return int(self.tris[t, (k + 2) % 3])

    def two_ring_tris(self, i):
        vs = {i, *self.ring[i]}
        out = set()
        for u in vs:
            out.update(self.inc[u])
        return out


def _unit_normals(X, tris):
    a, b, c = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    n = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(n, axis=1)
    return n / np.linalg.norm(n, axis=1)[:, None], area


def geometric_laplacian(X, topo: Topology) -> np.ndarray:
    """GL_i for every vertex [nv, 3]."""
    out = np.empty_like(X)
    for i in range(topo.nv):
        num = np.zeros(3)
        den = 0.0
        for j in topo.ring[i]:
            w = 1.0 / np.linalg.norm(X[i] - X[j])
            num += w * X[j]
            den += w
        out[i] = X[i] - num / den
    return out


def roughness(X, topo: Topology):
    """(R_i [nv], and the intermediates: R_e per edge id, G, V, R_t, R^1, R^2)."""
    n, area = _unit_normals(X, topo.tris)
    Re = {}
    for eid, a, b in topo.edges:
        t1, _ = topo.half[(a, b)]
        t2, _ = topo.half[(b, a)]
        Re[(a, b)] = 1.0 - float(n[t1] @ n[t2])
    G = np.empty(topo.nv)
    V = np.empty(topo.nv)
    for i in range(topo.nv):
        vals = np.array([Re[(min(i, j), max(i, j))] for j in topo.ring[i]])
        G[i] = vals.mean()
        V[i] = ((vals - G[i]) ** 2).mean()
    nt = len(topo.tris)
    Rt = np.empty(nt)
    for t in range(nt):
        c = topo.tris[t]
        sv = V[c].sum()
        Rt[t] = (G[c] * V[c]).sum() / sv if sv > 0.0 else G[c].mean()
    R1 = np.empty(topo.nv)
    R2 = np.empty(topo.nv)
    for i in range(topo.nv):
        t1 = topo.inc[i]
        R1[i] = sum(area[t] * Rt[t] for t in t1) / len(t1)
        t2 = topo.two_ring_tris(i)
        R2[i] = sum(area[t] * Rt[t] for t in t2) / len(t2)
    return np.maximum(R1, R2), dict(Re=Re, G=G, V=V, Rt=Rt, R1=R1, R2=R2, area=area)


def enclosed_volume(X, tris) -> float:
    """(1/6) sum x0 . (x1 x x2) over the triangles."""
    a, b, c = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    return float(np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0)


def _area_gradient(X, topo: Topology, i):
    """A_i = sum over the triangles (i, a, b) at i of (a - x_i) x (b - x_i)."""
    A = np.zeros(3)
    for t in topo.inc[i]:
        k = int(np.nonzero(topo.tris[t] == i)[0][0])
        a, b = topo.tris[t, (k + 1) % 3], topo.tris[t, (k + 2) % 3]
        A += np.cross(X[a] - X[i], X[b] - X[i])
    return A


def laplacian_pair(X, topo: Topology, v1: int, v2: int):
    """Simultaneous Laplacian positions (x1s, x2s) of the ends of an edge:
    each the mean of its one-ring with the other end at its new position."""
    r1, r2 = topo.ring[v1], topo.ring[v2]
    n1, n2 = len(r1), len(r2)
    S1 = sum((X[j] for j in r1 if j != v2), np.zeros(3))
    S2 = sum((X[j] for j in r2 if j != v1), np.zeros(3))
    x1s = (S2 + n2 * S1) / (n1 * n2 - 1)
    x2s = (x1s + S2) / n2
    return x1s, x2s


def smooth_edge(X, topo: Topology, v1: int, v2: int):
    """New positions (x1, x2) of the ends of edge (v1, v2), or None if g = 0."""
    x1s, x2s = laplacian_pair(X, topo, v1, v2)
    d1, d2 = x1s - X[v1], x2s - X[v2]
    A1, A2 = _area_gradient(X, topo, v1), _area_gradient(X, topo, v2)
    y = X[topo.far_corner(v1, v2)] - X[topo.far_corner(v2, v1)]
    g = A1 + A2 + np.cross(y, d1 - d2)
    gg = float(g @ g)
    if gg == 0.0:
        return None
    c = float(d1 @ A1 + d2 @ A2 + d1 @ np.cross(d2, y))
    step = -c / gg * g  # h n with n = g / |g|, h = -c / |g|
    return x1s + step, x2s + step


def flagged_edges(topo: Topology, gl_mag, rough, gl_threshold, rough_threshold):
    rough_v = (np.asarray(gl_mag) > gl_threshold) & (np.asarray(rough) > rough_threshold)
    return [(eid, a, b) for eid, a, b in topo.edges if rough_v[a] and rough_v[b]], rough_v


def fmix32(x: int) -> int:
    """The 32-bit finalizer of MurmurHash3."""
    x &= 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x85EBCA6B) & 0xFFFFFFFF
    x ^= x >> 13
    x = (x * 0xC2B2AE35) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def priority(eid: int):
    return (fmix32(eid), eid)


def schedule(topo: Topology, edges):
    """Rounds of the flagged edges (lists of (id, a, b))."""
    pending = list(edges)
    rounds = []
    while pending:
        at = {}
        for e in pending:
            at.setdefault(e[1], []).append(e)
            at.setdefault(e[2], []).append(e)
        take = []
        for e in pending:
            eid, a, b = e
            pe = priority(eid)
            near = {a, b, *topo.ring[a], *topo.ring[b]}
            if not any(priority(f[0]) < pe for u in near for f in at.get(u, ())):
                take.append(e)
        rounds.append(take)
        ids = {e[0] for e in take}
        pending = [e for e in pending if e[0] not in ids]
    return rounds


def smooth(X, tris, gl_threshold, rough_threshold, gl_mag=None, rough=None):
    """Detection and smoothing of one front: (new positions, number of edges
    moved, rounds).  The metrics are those of X unless given."""
    X = np.array(X, dtype=np.float64)
    topo = Topology(tris, len(X))
    if gl_mag is None:
        gl_mag = np.linalg.norm(geometric_laplacian(X, topo), axis=1)
    if rough is None:
        rough, _ = roughness(X, topo)
    edges, _ = flagged_edges(topo, gl_mag, rough, gl_threshold, rough_threshold)
    rounds = schedule(topo, edges)
    moved = 0
    for rnd in rounds:
        new = []
        for eid, a, b in rnd:
            r = smooth_edge(X, topo, a, b)
            if r is not None:
                new.append((a, b, r))
        for a, b, (p, q) in new:
            X[a], X[b] = p, q
            moved += 1
    return X, moved, rounds
