// ftc_device.hpp -- device-side geometry shared by the library's kernels.
//
// Every decision that selects a discrete result (which cell holds a point,
// whether a triangle has a positive-area piece in a cell, which vertex is
// nearest, whether a triangle centre lies inside the support) is evaluated
// with the operation order spelled out below and no contraction into fused
// multiply-adds (the library is compiled with -ffp-contract=off), so the
// decisions are reproducible on any IEEE-754 binary64 implementation that
// follows the same order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ftc.h"

namespace ftc {

// Device error latch bits (combined with atomicOr).
enum : int32_t { ERR_DOMAIN = 1, ERR_MESH = 2, ERR_CAPACITY = 4 };

struct Grid {
  int32_t nx, ny, nz;
  double x0, y0, z0, h;
};

struct Mesh {
  int32_t nv, nt;
  const double *x, *y, *z;
  const int32_t *t0, *t1, *t2;
};

__host__ __device__ inline double dim_org(const Grid& g, int d) {
  return d == 0 ? g.x0 : (d == 1 ? g.y0 : g.z0);
}
__host__ __device__ inline int32_t dim_n(const Grid& g, int d) {
  return d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
}

// Grid plane i along an axis: origin + i * h (one product, one sum).
__device__ inline double grid_plane(double org, int64_t i, double h) { return org + (double)i * h; }

// Half-open cell index of coordinate x: plane(i) <= x < plane(i+1), exact
// with respect to grid_plane.
__device__ inline int64_t cell_index(double x, double org, double h) {
  int64_t i = (int64_t)floor((x - org) / h);
  while (grid_plane(org, i, h) > x) --i;
  while (grid_plane(org, i + 1, h) <= x) ++i;
  return i;
}

// A vertex is admissible if it lies in [plane(2), plane(n-2)) on every axis.
__device__ inline bool in_margin(const Grid& g, double x, double y, double z) {
  const double p[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double lo = grid_plane(dim_org(g, d), 2, g.h);
    double hi = grid_plane(dim_org(g, d), dim_n(g, d) - 2, g.h);
    if (!(p[d] >= lo && p[d] < hi)) return false;
  }
  return true;
}

// All three corner indices of triangle t lie in [0, nv).
__device__ inline bool tri_ok(const Mesh& m, int32_t t) {
  const int32_t a = m.t0[t], b = m.t1[t], c = m.t2[t];
  return a >= 0 && b >= 0 && c >= 0 && a < m.nv && b < m.nv && c < m.nv;
}

struct Tri {
  double v[3][3];
};

__device__ inline Tri load_tri(const Mesh& m, int32_t t) {
  Tri T;
  const int32_t c[3] = {m.t0[t], m.t1[t], m.t2[t]};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    T.v[r][0] = m.x[c[r]];
    T.v[r][1] = m.y[c[r]];
    T.v[r][2] = m.z[c[r]];
  }
  return T;
}

// Cell-index range of the triangle's bounding box.
__device__ inline void tri_range(const Grid& g, const Tri& T, int64_t lo[3], int64_t hi[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double mn = fmin(fmin(T.v[0][d], T.v[1][d]), T.v[2][d]);
    double mx = fmax(fmax(T.v[0][d], T.v[1][d]), T.v[2][d]);
    lo[d] = cell_index(mn, dim_org(g, d), g.h);
    hi[d] = cell_index(mx, dim_org(g, d), g.h);
  }
}

// ---------------------------------------------------------------------------
// Triangle / cell clipping.
//
// Polygon clipped successively by x >= xlo, x <= xhi, y >= ylo, y <= yhi,
// z >= zlo, z <= zhi (closed).  For an edge p -> q (polygon order) with one
// end in and one strictly out, the cut point is computed from the endpoint a
// with the smaller coordinate d towards the other endpoint b:
//   t = (c - a_d) / (b_d - a_d),  r_e = a_e + t * (b_e - a_e),  r_d = c.
// Emission per edge: in->in: q; in->out: cut (skipped when p_d == c);
// out->in: cut (skipped when q_d == c), then q.  The piece counts when
// (1) no coordinate of all three triangle corners equals the cell's upper
// plane on that axis (a triangle in a grid plane belongs to the cell above),
// (2) at least three corners remain, and (3) the fan-summed vector area
// sum_j (q_j - q_0) x (q_{j+1} - q_0) is not the zero vector.
// ---------------------------------------------------------------------------

constexpr int kMaxPoly = 12;

struct Poly {
  int n;
  double x[kMaxPoly], y[kMaxPoly], z[kMaxPoly];
};

__device__ inline double poly_coord(const Poly& P, int i, int d) {
  return d == 0 ? P.x[i] : (d == 1 ? P.y[i] : P.z[i]);
}

// A convex polygon cut by one plane gains at most one corner, so after six
// planes a triangle has at most nine; the bound check only guards memory.
__device__ inline void poly_push(Poly& P, double x, double y, double z) {
  if (P.n >= kMaxPoly) return;
  P.x[P.n] = x;
  P.y[P.n] = y;
  P.z[P.n] = z;
  ++P.n;
}

__device__ inline void poly_push_cut(Poly& out, const Poly& in, int ip, int iq, int d, double c) {
  double pd = poly_coord(in, ip, d), qd = poly_coord(in, iq, d);
  int ia = pd < qd ? ip : iq;
  int ib = pd < qd ? iq : ip;
  double ad = poly_coord(in, ia, d), bd = poly_coord(in, ib, d);
  double t = (c - ad) / (bd - ad);
  double rx = d == 0 ? c : in.x[ia] + t * (in.x[ib] - in.x[ia]);
  double ry = d == 1 ? c : in.y[ia] + t * (in.y[ib] - in.y[ia]);
  double rz = d == 2 ? c : in.z[ia] + t * (in.z[ib] - in.z[ia]);
  poly_push(out, rx, ry, rz);
}

__device__ inline void clip_plane(const Poly& in, Poly& out, int d, double c, bool upper) {
  out.n = 0;
  for (int e = 0; e < in.n; ++e) {
    int iq = (e + 1 == in.n) ? 0 : e + 1;
    double pd = poly_coord(in, e, d), qd = poly_coord(in, iq, d);
    bool pin = upper ? (pd <= c) : (pd >= c);
    bool qin = upper ? (qd <= c) : (qd >= c);
    if (pin && qin) {
      poly_push(out, in.x[iq], in.y[iq], in.z[iq]);
    } else if (pin) {
      if (pd != c) poly_push_cut(out, in, e, iq, d, c);
    } else if (qin) {
      if (qd != c) poly_push_cut(out, in, e, iq, d, c);
      poly_push(out, in.x[iq], in.y[iq], in.z[iq]);
    }
  }
}

// Clip T to cell (i, j, k); true if the piece counts.  On return `P` holds
// the clipped polygon.
__device__ inline bool clip_cell(const Grid& g, const Tri& T, int64_t i, int64_t j, int64_t k, Poly& P) {
  const int64_t ijk[3] = {i, j, k};
  double lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = grid_plane(dim_org(g, d), ijk[d], g.h);
    hi[d] = grid_plane(dim_org(g, d), ijk[d] + 1, g.h);
    if (T.v[0][d] == hi[d] && T.v[1][d] == hi[d] && T.v[2][d] == hi[d]) return false;
  }
  Poly A;
  A.n = 3;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    A.x[r] = T.v[r][0];
    A.y[r] = T.v[r][1];
    A.z[r] = T.v[r][2];
  }
  clip_plane(A, P, 0, lo[0], false);
  if (P.n == 0) return false;
  clip_plane(P, A, 0, hi[0], true);
  if (A.n == 0) return false;
  clip_plane(A, P, 1, lo[1], false);
  if (P.n == 0) return false;
  clip_plane(P, A, 1, hi[1], true);
  if (A.n == 0) return false;
  clip_plane(A, P, 2, lo[2], false);
  if (P.n == 0) return false;
  clip_plane(P, A, 2, hi[2], true);
  if (A.n < 3) return false;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int j2 = 1; j2 + 1 < A.n; ++j2) {
    double ux = A.x[j2] - A.x[0], uy = A.y[j2] - A.y[0], uz = A.z[j2] - A.z[0];
    double vx = A.x[j2 + 1] - A.x[0], vy = A.y[j2 + 1] - A.y[0], vz = A.z[j2 + 1] - A.z[0];
    sx += uy * vz - uz * vy;
    sy += uz * vx - ux * vz;
    sz += ux * vy - uy * vx;
  }
  if (sx == 0.0 && sy == 0.0 && sz == 0.0) return false;
  P = A;
  return true;
}

// z-column integrals of a piece: flux = integral of n_z dA (signed projected
// area, fan from corner 0), vol = integral of (z - zlo) n_z dA (z is linear on
// the piece, so each fan triangle contributes its area times its corner mean).
__device__ inline void piece_z_integrals(const Poly& P, double zlo, double& flux, double& vol) {
  double f = 0.0, v = 0.0;
  for (int j = 1; j + 1 < P.n; ++j) {
    double A = 0.5 * ((P.x[j] - P.x[0]) * (P.y[j + 1] - P.y[0]) - (P.x[j + 1] - P.x[0]) * (P.y[j] - P.y[0]));
    f += A;
    v += A * ((P.z[0] + P.z[j] + P.z[j + 1]) / 3.0 - zlo);
  }
  flux = f;
  vol = v;
}

}  // namespace ftc
