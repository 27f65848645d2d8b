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

// Division by a fixed divisor d < 2^31 through a multiply-high (Granlund &
// Montgomery, PLDI 1994, round-up variant): for 0 <= n < 2^31,
// n / d == (umulhi(m, n) + n) >> l with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1; the sum cannot overflow 32 bits.
struct FastDiv {
  uint32_t d, m, l;
  __host__ __device__ FastDiv() : d(1), m(1), l(0) {}
  __host__ explicit FastDiv(uint32_t div) : d(div), m(1), l(0) {
    while ((1ull << l) < d) ++l;
    m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  }
  __device__ uint32_t div(uint32_t n) const { return (__umulhi(m, n) + n) >> l; }
};

struct Grid {
  int32_t nx, ny, nz;
  double x0, y0, z0, h;
  FastDiv dnx, dny, dncol;  // divisions by nx, ny and nx*ny
};

// (i, j, k) of a linear cell id (lin < 2^31).
struct Cell3 {
  int32_t i, j, k;
};
__device__ inline Cell3 unpack_cell(const Grid& g, int32_t lin) {
  const uint32_t u = (uint32_t)lin;
  const uint32_t k = g.dncol.div(u);
  const uint32_t r = u - k * g.dncol.d;
  const uint32_t j = g.dnx.div(r);
  return Cell3{(int32_t)(r - j * g.dnx.d), (int32_t)j, (int32_t)k};
}

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
__host__ __device__ inline double grid_plane(double org, int64_t i, double h) { return org + (double)i * h; }

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

// Triangle from the packed records: corners (t0, t1, t2, 0) as one int4,
// coordinates (x, y, z, 0) as two double2 per vertex.
__device__ inline Tri load_tri_packed(const int4* tri4, const double2* vtx4, int32_t t) {
  Tri T;
  const int4 c = tri4[t];
  const int32_t cr[3] = {c.x, c.y, c.z};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double2 a = vtx4[2 * (int64_t)cr[r]], b = vtx4[2 * (int64_t)cr[r] + 1];
    T.v[r][0] = a.x;
    T.v[r][1] = a.y;
    T.v[r][2] = b.x;
  }
  return T;
}

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
//
// A stage whose plane leaves every corner inside emits each corner once, in
// the same cyclic order shifted by one.  A convex polygon gains at most one
// corner per plane (nine after six planes; the bound checks only guard
// memory).
// ---------------------------------------------------------------------------

constexpr int kMaxPoly = 9;

struct Piece {
  bool keep;
  double flux;  // integral of n_z dA over the piece
  double vol;   // integral of (z - zlo) n_z dA over the piece
  bool over_cap;  // a clip with fewer than kMaxPoly corner slots outgrew them: no result, clip again with kMaxPoly
};

// Planes of cell (i, j, k); false if the half-open rule gives the triangle to
// the next cell (all three corners on an upper plane).
__host__ __device__ inline bool cell_planes(const Grid& g, const Tri& T, int64_t i, int64_t j, int64_t k, double lo[3],
                                   double hi[3]) {
  const int64_t ijk[3] = {i, j, k};
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = grid_plane(dim_org(g, d), ijk[d], g.h);
    hi[d] = grid_plane(dim_org(g, d), ijk[d] + 1, g.h);
    if (T.v[0][d] == hi[d] && T.v[1][d] == hi[d] && T.v[2][d] == hi[d]) ok = false;
  }
  return ok;
}

// Words of the face-neighbour band of the occupancy bitmap I: bit q of word
// w is set for cell c = 32 w + q when c is not in I and one of c -+ 1,
// c -+ sy, c -+ sz is.  Every set cell of I lies at least two cells inside
// the grid, so these linear shifts reach exactly its face neighbours (a
// shift that wraps a row or slice lands on a boundary cell, never set).
struct BandWords {
  const uint32_t* I;
  int64_t nwords, ncell, sy, sz;
  // the 32 bits of I from cell `start` on (zero outside the grid)
  __device__ uint32_t bits_at(int64_t start) const {
    const int64_t w = start >= 0 ? start >> 5 : -((-start + 31) >> 5);
    const int off = (int)(start - 32 * w);
    const uint32_t lo = (w >= 0 && w < nwords) ? I[w] : 0u;
    const uint32_t hi = (w + 1 >= 0 && w + 1 < nwords) ? I[w + 1] : 0u;
    return off == 0 ? lo : ((lo >> off) | (hi << (32 - off)));
  }
  __device__ uint32_t word(int64_t w) const {
    const int64_t b = 32 * w;
    const uint32_t nb = bits_at(b - 1) | bits_at(b + 1) | bits_at(b - sy) | bits_at(b + sy) | bits_at(b - sz) |
                        bits_at(b + sz);
    uint32_t band = nb & ~I[w];
    const int64_t rest = ncell - b;  // cells of this word inside the grid
    if (rest < 32) band &= rest > 0 ? ((1u << rest) - 1u) : 0u;
    return band;
  }
};

// Compact index of grid cell `lin` among the interfacial cells (its rank in
// the occupancy bitmap, from the popcount prefix sums), -1 if it holds no
// piece.
__device__ inline int32_t cell_rank(const uint32_t* bitmap, const int32_t* word_off, int64_t lin) {
  const uint32_t w = bitmap[lin >> 5];
  if (!((w >> (lin & 31)) & 1u)) return -1;
  const uint32_t below = (lin & 31) ? (w & ((1u << (lin & 31)) - 1u)) : 0u;
  return word_off[lin >> 5] + __popc(below);
}

__device__ inline double cell_centre(double org, int32_t i, double h) { return org + ((double)i + 0.5) * h; }

struct P3 {
  double x, y, z;
};

// Vertex coordinates from the packed (x, y, z, 0) record.
__device__ inline P3 vtx(const double2* vtx4, int32_t v) {
  const double2 a = vtx4[2 * (int64_t)v], b = vtx4[2 * (int64_t)v + 1];
  return P3{a.x, a.y, b.x};
}

// (squared distance, vertex) ordered lexicographically: the closest vertex,
// lowest index on ties.
__device__ inline bool lex_less(double d, int32_t v, double bd, int32_t bv) {
  return d < bd || (d == bd && v < bv);
}

// d^2 = dx dx + dy dy + dz dz (in that order) of vertex v to xc, kept when
// it beats (bd, bv).
__device__ inline void consider(const double2* vtx4, int32_t v, const double xc[3], double& bd, int32_t& bv) {
  const P3 p = vtx(vtx4, v);
  const double dx = p.x - xc[0], dy = p.y - xc[1], dz = p.z - xc[2];
  const double d2 = dx * dx + dy * dy + dz * dz;
  if (lex_less(d2, v, bd, bv)) {
    bd = d2;
    bv = v;
  }
}

// Candidate classes decided from the corners alone, taking exactly the
// decisions the clipping would take: stages are visited in order while the
// polygon is still the (rotated) triangle; 0 = no piece (half-open rule, or
// a stage with every corner strictly outside), 1 = the piece is the whole
// triangle (no stage cuts), 2 = some stage cuts, so the candidate must be
// clipped.
__host__ __device__ inline int classify_candidate(const Grid& g, const Tri& T, int64_t i, int64_t j, int64_t k) {
  double lo[3], hi[3];
  if (!cell_planes(g, T, i, j, k, lo, hi)) return 0;
#pragma unroll
  for (int stage = 0; stage < 6; ++stage) {
    const int d = stage >> 1;
    const bool upper = stage & 1;
    const double c = upper ? hi[d] : lo[d];
    const double a = T.v[0][d], b = T.v[1][d], e = T.v[2][d];
    const bool ia = upper ? a <= c : a >= c, ib = upper ? b <= c : b >= c, ie = upper ? e <= c : e >= c;
    if (!ia && !ib && !ie) return 0;
    if (!(ia && ib && ie)) return 2;
  }
  return 1;
}

// Stages whose plane has triangle corners on both sides (the closed
// inside test of the clipping): bit s for stage s.  Candidates with equal
// masks take the same branches through most of the clipping.
__host__ __device__ inline uint32_t crossing_mask(const Grid& g, const Tri& T, int64_t i, int64_t j, int64_t k) {
  const int64_t ijk[3] = {i, j, k};
  uint32_t mask = 0u;
#pragma unroll
  for (int stage = 0; stage < 6; ++stage) {
    const int d = stage >> 1;
    const bool upper = stage & 1;
    const double c = grid_plane(dim_org(g, d), ijk[d] + (upper ? 1 : 0), g.h);
    const double a = T.v[0][d], b = T.v[1][d], e = T.v[2][d];
    const bool ia = upper ? a <= c : a >= c, ib = upper ? b <= c : b >= c, ie = upper ? e <= c : e >= c;
    if ((ia || ib || ie) && !(ia && ib && ie)) mask |= 1u << stage;
  }
  return mask;
}

// Stages that certainly cut nothing: every triangle corner lies inside the
// stage's plane by more than 1e-12 (1 + X), X the largest corner coordinate
// magnitude.  Every point the clipping emits is a rounded interpolation
// between points it emitted before, within a few units in the last place of
// X of the triangle's convex hull, so it lies inside such a plane as well:
// the stage leaves the polygon whole (and only rotates it).
__host__ __device__ inline uint32_t inside_mask(const Grid& g, const Tri& T, int64_t i, int64_t j, int64_t k) {
  const int64_t ijk[3] = {i, j, k};
  double X = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int d = 0; d < 3; ++d) X = fmax(X, fabs(T.v[r][d]));
  const double tol = 1e-12 * (1.0 + X);
  uint32_t mask = 0u;
#pragma unroll
  for (int stage = 0; stage < 6; ++stage) {
    const int d = stage >> 1;
    const bool upper = stage & 1;
    const double c = grid_plane(dim_org(g, d), ijk[d] + (upper ? 1 : 0), g.h);
    const double mn = fmin(fmin(T.v[0][d], T.v[1][d]), T.v[2][d]);
    const double mx = fmax(fmax(T.v[0][d], T.v[1][d]), T.v[2][d]);
    if (upper ? (mx < c - tol) : (mn > c + tol)) mask |= 1u << stage;
  }
  return mask;
}

// Fan integrals of a polygon given by corner accessors (corner 0 is the fan
// apex): membership by the vector area, flux and vol by the z-column rule.
// CAP bounds n; the sums do not depend on it.
template <int CAP = kMaxPoly, class CX>
__host__ __device__ inline Piece fan_piece(int n, double zlo, CX cx) {
  Piece out{false, 0.0, 0.0};
  if (n < 3) return out;
  const double x0 = cx(0, 0), y0 = cx(0, 1), z0 = cx(0, 2);
  double sx = 0.0, sy = 0.0, sz = 0.0, f = 0.0, v = 0.0;
#pragma unroll
  for (int jj = 1; jj + 1 < CAP; ++jj) {
    if (jj + 1 < n) {
      const double x1 = cx(jj, 0), y1 = cx(jj, 1), z1 = cx(jj, 2);
      const double x2 = cx(jj + 1, 0), y2 = cx(jj + 1, 1), z2 = cx(jj + 1, 2);
      const double ux = x1 - x0, uy = y1 - y0, uz = z1 - z0;
      const double vx = x2 - x0, vy = y2 - y0, vz = z2 - z0;
      sx += uy * vz - uz * vy;
      sy += uz * vx - ux * vz;
      sz += ux * vy - uy * vx;
      // the fan triangle's signed area projected on the xy plane, and that
      // area times the mean of (z - zlo) over its corners
      const double A = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
      f += A;
      v += A * ((z0 + z1 + z2) / 3.0 - zlo);
    }
  }
  if (sx == 0.0 && sy == 0.0 && sz == 0.0) return out;
  out.keep = true;
  out.flux = f;
  out.vol = v;
  return out;
}

// Piece of a candidate of class 1: the triangle itself (after six stages
// that cut nothing the corner order is back to t0, t1, t2).
__host__ __device__ inline Piece whole_piece(const Tri& T, double zlo) {
  return fan_piece(3, zlo, [&](int q, int d) { return q == 0 ? T.v[0][d] : (q == 1 ? T.v[1][d] : T.v[2][d]); });
}

// Per-lane compaction buffer in LDS: [coordinate][corner][lane], CAP corners.
template <int LANES, int CAP = kMaxPoly>
struct PolyLDS {
  double v[3][CAP][LANES];
};

// One of three values by a run-time index, without indexing registers.
__host__ __device__ inline double sel3(int d, double a, double b, double c) { return d == 0 ? a : (d == 1 ? b : c); }

// Full clipping of a candidate.  The polygon lives in registers (static
// physical slots) with a copy in the lane's LDS buffer for reads at dynamic
// positions.  Logical corner i (polygon order) is physical slot
// (i + rot) mod n, so a stage that cuts nothing only advances rot.  A stage
// that cuts takes one of two routes with identical results:
//  * the inside corners form one cyclic run (the case of a convex polygon):
//    exactly two edges cross the plane; their cut points are computed from
//    endpoints read from LDS, and each output corner is written to its
//    position in the emission order, counted with bit masks over the edges;
//  * otherwise (possible only through rounding): the corners are brought
//    into logical order and every edge is processed in turn.
// Either way the output is the stage's emission sequence (first kMaxPoly
// corners), stored to LDS at positions 0.. and reloaded with rot = 0.
// `skip`: stages known to cut nothing (a subset of inside_mask), which then
// only rotate the polygon.
// CAP < kMaxPoly builds the same clip with CAP corner slots (fewer
// registers and LDS): while every stage emits at most CAP corners it does
// exactly what the kMaxPoly build does; a stage that would emit more returns
// over_cap instead, and the caller clips that candidate again with
// kMaxPoly slots.  A triangle that cuts at most one plane of each axis never
// exceeds six corners.
template <int LANES, int CAP>
__host__ __device__ inline Piece clip_piece(const Grid& g, const Tri& T, int64_t i, int64_t j, int64_t k,
                                            PolyLDS<LANES, CAP>& L, int lane, uint32_t skip = 0u) {
  static_assert(CAP >= 3 && CAP <= kMaxPoly, "polygon capacity");
  Piece none{false, 0.0, 0.0, false};
  const Piece grown{false, 0.0, 0.0, true};
  double lo[3], hi[3];
  if (!cell_planes(g, T, i, j, k, lo, hi)) return none;
  double P[3][CAP];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int q = 0; q < CAP; ++q) {
      P[d][q] = q < 3 ? T.v[q][d] : 0.0;
      if (q < 3) L.v[d][q][lane] = T.v[q][d];
    }
  int n = 3, rot = 0;
  // unrolled: the axis and side of every stage are constants, so the
  // coordinate selects fold away
#pragma unroll
  for (int stage = 0; stage < 6; ++stage) {
    const int d = stage >> 1;
    const bool upper = stage & 1;
    if ((skip >> stage) & 1u) {
      rot = rot + 1 == n ? 0 : rot + 1;
      continue;
    }
    const double c = upper ? sel3(d, hi[0], hi[1], hi[2]) : sel3(d, lo[0], lo[1], lo[2]);
    uint32_t mp = 0;  // inside corners by physical slot
#pragma unroll
    for (int q = 0; q < CAP; ++q) {
      const double x = sel3(d, P[0][q], P[1][q], P[2][q]);
      if (q < n && (upper ? (x <= c) : (x >= c))) mp |= 1u << q;
    }
    const uint32_t full = (1u << n) - 1u;
    if (mp == 0u) return none;
    if (mp == full) {
      rot = rot + 1 == n ? 0 : rot + 1;
      continue;
    }
    // by logical corner: m (corner e inside), Qm (corner e + 1 inside)
    const uint32_t m = rot ? (((mp >> rot) | (mp << (n - rot))) & full) : mp;
    const uint32_t Qm = ((m >> 1) | (m << (n - 1))) & full;
    if (__builtin_popcount(m ^ Qm) == 2) {
      const int e_out = __builtin_ctz(m & ~Qm);  // inside -> outside
      const int e_in = __builtin_ctz(~m & Qm);   // outside -> inside
      double X[2][3];
      bool emit[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int e = s ? e_in : e_out;
        int ps = e + rot;
        if (ps >= n) ps -= n;
        const int qs = ps + 1 == n ? 0 : ps + 1;
        double pp[3], qq[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          pp[f] = L.v[f][ps][lane];
          qq[f] = L.v[f][qs][lane];
        }
        const double pd = sel3(d, pp[0], pp[1], pp[2]), qd = sel3(d, qq[0], qq[1], qq[2]);
        // no cut point where the inside end lies on the plane
        emit[s] = s ? qd != c : pd != c;
        const bool pa = pd < qd;
        const double ad = pa ? pd : qd, bd = pa ? qd : pd;
        const double t = (c - ad) / (bd - ad);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const double af = pa ? pp[f] : qq[f], bf = pa ? qq[f] : pp[f];
          X[s][f] = (f == d) ? c : af + t * (bf - af);
        }
      }
      const uint32_t C = ((uint32_t)emit[0] << e_out) | ((uint32_t)emit[1] << e_in);
      const int n_out = __builtin_popcount(m) + __builtin_popcount(C);
      if (CAP < kMaxPoly && n_out > CAP) return grown;
      // corner i = e + 1 of edge e follows the cut point of edge e
#pragma unroll
      for (int q = 0; q < CAP; ++q) {
        if (q < n && ((mp >> q) & 1u)) {
          int li = q - rot;
          if (li < 0) li += n;
          const int e = li == 0 ? n - 1 : li - 1;
          const int pos = __builtin_popcount(C & ((2u << e) - 1u)) + __builtin_popcount(Qm & ((1u << e) - 1u));
          if (pos < CAP) {
#pragma unroll
            for (int f = 0; f < 3; ++f) L.v[f][pos][lane] = P[f][q];
          }
        }
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int e = s ? e_in : e_out;
        const int pos = __builtin_popcount(C & ((1u << e) - 1u)) + __builtin_popcount(Qm & ((1u << e) - 1u));
        if (emit[s] && pos < CAP) {
#pragma unroll
          for (int f = 0; f < 3; ++f) L.v[f][pos][lane] = X[s][f];
        }
      }
      n = n_out > CAP ? CAP : n_out;
    } else {
      // logical order in registers, then every edge in turn
      if (rot) {
#pragma unroll
        for (int q = 0; q < CAP; ++q) {
          int ps = q + rot;
          if (ps >= n) ps -= n;
          if (q < n) {
#pragma unroll
            for (int f = 0; f < 3; ++f) P[f][q] = L.v[f][ps][lane];
          }
        }
      }
      int o = 0;  // corners emitted, also those beyond the CAP slots
#pragma unroll
      for (int e = 0; e < CAP; ++e) {
        if (e < n) {
          double q0 = P[0][0], q1 = P[1][0], q2 = P[2][0];
          if (e + 1 < CAP && e + 1 < n) {
            q0 = P[0][e + 1];
            q1 = P[1][e + 1];
            q2 = P[2][e + 1];
          }
          const double pp[3] = {P[0][e], P[1][e], P[2][e]};
          const double qq[3] = {q0, q1, q2};
          const double pd = sel3(d, pp[0], pp[1], pp[2]), qd = sel3(d, qq[0], qq[1], qq[2]);
          const bool pin = upper ? (pd <= c) : (pd >= c);
          const bool qin = upper ? (qd <= c) : (qd >= c);
          const bool cut = pin != qin && (pin ? pd != c : qd != c);
          if (cut) {
            if (o < CAP) {
              const bool pa = pd < qd;
              const double ad = pa ? pd : qd, bd = pa ? qd : pd;
              const double t = (c - ad) / (bd - ad);
#pragma unroll
              for (int f = 0; f < 3; ++f) {
                const double af = pa ? pp[f] : qq[f], bf = pa ? qq[f] : pp[f];
                L.v[f][o][lane] = (f == d) ? c : af + t * (bf - af);
              }
            }
            ++o;
          }
          if (qin) {
            if (o < CAP) {
              L.v[0][o][lane] = q0;
              L.v[1][o][lane] = q1;
              L.v[2][o][lane] = q2;
            }
            ++o;
          }
        }
      }
      if (CAP < kMaxPoly && o > CAP) return grown;
      n = o > CAP ? CAP : o;
      if (n == 0) return none;
    }
    rot = 0;
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int q = 0; q < CAP; ++q) P[f][q] = L.v[f][q][lane];
  }
  if (rot) {
#pragma unroll
    for (int q = 0; q < CAP; ++q) {
      int ps = q + rot;
      if (ps >= n) ps -= n;
      if (q < n) {
#pragma unroll
        for (int f = 0; f < 3; ++f) P[f][q] = L.v[f][ps][lane];
      }
    }
  }
  return fan_piece<CAP>(n, lo[2], [&](int q, int d) { return P[d][q]; });
}

}  // namespace ftc
