// ppic.hip -- PPIC curvature by the volume fit (paper section 3.2).
//
// The cell-list build prepares what this needs from the front: each
// vertex's incident triangles (ascending), the triangles' corners packed as
// (t0, t1, t2, 0) and the vertex coordinates as (x, y, z, 0), and the
// closest vertex of every interfacial cell among the vertices of the 3x3x3
// block of cells around it (lowest index on ties).  A vertex outside the
// block is at least 1.5 h from the cell centre, so a best squared distance
// below (1.5 h)^2 is final; any other cell searches all vertices here.
//
// The ring of a cell is T_R, with T_1 the triangles at the closest vertex v*
// and T_{r+1} the triangles sharing a vertex with T_r.  Writing V_r for the
// corners of T_r (V_0 = {v*}), T_r is the set of triangles with a corner in
// V_{r-1}, and V_r is V_{r-1} plus the corners of the triangles at the
// vertices new in V_{r-1}.
//
// Fast shape (k_ppic_fast), G lanes per interfacial cell, one pass:
//   1. V_0 = {v*}; the triangles at v* give the frame normal (their cross
//      products summed in ascending triangle order) and, for R >= 2, their
//      corners join V (a key-only hash set in LDS, insertion order kept);
//   2. levels 2 .. R-1: each lane takes one vertex new in the previous level
//      and adds the corners of its triangles to V;
//   3. the ring T_R: each lane takes vertices u of V_{R-1} and keeps a
//      triangle at u exactly when u is its first corner (t0, t1, t2 order)
//      that lies in V_{R-1}, so every triangle is kept once;
//   4. one pass over the ring: triangle-centre distances, Wendland weights
//      with delta = delta_over_h h, the triangle's projection into the frame
//      (coordinates divided by h for conditioning), its six moments by the
//      edge-midpoint rule (exact for quadratics) and the integral of its
//      plane, accumulated into the weighted normal equations M a = b;
//      all-reduce over the cell's lanes;
//   5. when delta needs no adjustment (at least n_min triangles inside it,
//      or all of them, or no adjustment allowed): Cholesky factorisation of
//      M with one step of iterative refinement, curvature kappa = 2H at the
//      frame origin and the interface normal.
// A cell whose vertex set or ring exceeds the fast capacities, or whose
// support must grow, is queued for the wide shape.
//
// Wide shape (k_ppic_wide; k_ppic_wide_sel for the learned curvature's
// fallback cells): 64 lanes per cell, one cell per workgroup at a time,
// rings of up to 256 vertices and 512 triangles kept with their ring level
// in an open-addressing hash, the support grown as the parameters allow,
// the fit and the solve in the same workgroup.
//
// Every loop bound that encloses a cross-lane operation is uniform over the
// wavefront (maxima over its cells), so LDS phases are separated by plain
// workgroup barriers.
#include <float.h>

#include <algorithm>

#include "ftc_ws.hpp"
#include "dpp.hpp"
#include "xcd.hpp"

namespace ftc {
namespace {

constexpr int kWideBlocks = 64;  // persistent workgroups of the wide shape

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Capacities of the wide shape.
template <int G_, int HS_, int VC_, int TC_, int CR_>
struct Cfg {
  static constexpr int G = G_;        // lanes per cell
  static constexpr int NG = 64 / G_;  // cells per wavefront
  static constexpr int HS = HS_;      // hash slots (power of two)
  static constexpr int VC = VC_;      // ring-vertex capacity (owner table holds bytes: <= 256)
  static constexpr int TC = TC_;      // ring-triangle capacity
  static constexpr int CR = CR_;      // candidates per lane per batch
  static constexpr int Batch = CR_ * G_;
  static constexpr int FW = (3 * TC_ + 31) / 32;  // words of the first-occurrence bitmap
  static_assert((HS_ & (HS_ - 1)) == 0 && HS_ >= 2 * VC_, "hash size");
  static_assert(VC_ <= 256, "owner table holds bytes");
};
using Wide = Cfg<64, 512, 256, 512, 4>;

struct PPICArgs {
  Grid g;
  int32_t nv;
  PPICParams prm;
  const int4* tri4;
  const double2* vtx4;
  const int32_t* cell_ids;
  const int32_t* vt_off;
  const int32_t* vt_ids;
  const double* best_d2;
  const int32_t* best_v;
  const int2* best_inc;  // (offset, count) of best_v's incident triangles
  int32_t* counters;
  int32_t* ovf_cells;
  double* frame_n;  // [3][cell_cap] frame normal of each cell (the paraboloid cell integrals read it)
  int32_t cell_cap;
  double *kappa, *nx, *ny, *nz, *coeff;
  int32_t *status, *diag;
  int32_t queue_chunk;  // fast shape: 0 a static split of the cell groups, else the work queue's chunk
  const int32_t* sel;  // null: every interfacial cell; else the cells sel[0, counters[C_NSEL])
  int32_t* n_sel_out;  // receives the selection's count (may be null)
};

template <int HS>
__device__ inline int hslot(int32_t key) {
  return (int)(((uint32_t)key * 2654435761u) >> (32 - ilog2(HS)));
}

// Ballot of this lane's group, in the group's low bits.
template <int G>
__device__ inline uint64_t gballot(bool p, int grp) {
  const uint64_t b = __ballot(p);
  if constexpr (G == 64)
    return b;
  else
    return (b >> (G * grp)) & ((1ull << G) - 1ull);
}

// Sum over each aligned group of G lanes, the same bits in every lane: each
// step adds a value from a partner lane that adds this lane's value back.
// Called with all 64 lanes active.
template <int G>
__device__ inline double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_d<kDppSwap1>(v);
  if constexpr (G >= 4) v += dpp_d<kDppSwap2>(v);
  if constexpr (G >= 8) v += dpp_d<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_d<kDppMirror>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// group_sum in single precision
template <int G>
__device__ inline float group_sum_f(float v) {
  if constexpr (G >= 2) v += dpp_f<kDppSwap1>(v);
  if constexpr (G >= 4) v += dpp_f<kDppSwap2>(v);
  if constexpr (G >= 8) v += dpp_f<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_f<kDppMirror>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Integer sum over each aligned group of G lanes (the steps of group_sum).
template <int G>
__device__ inline int group_sum_i(int v) {
  if constexpr (G >= 2) v += dpp_i<kDppSwap1>(v);
  if constexpr (G >= 4) v += dpp_i<kDppSwap2>(v);
  if constexpr (G >= 8) v += dpp_i<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_i<kDppMirror>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Exclusive prefix sum over the lanes of each aligned group of G lanes (gl
// the lane's index in its group), and the group's total in *total.
// Groups of up to 16 lanes shift within rows of 16 lanes (DPP row_shr);
// a lane takes a shifted value only from its own group.  Called with every
// lane of the wavefront active.
template <int G>
__device__ inline int group_excl_scan(int v, int gl, int* total) {
  int inc = v;
  if constexpr (G <= 16) {
    if constexpr (G >= 2) { const int t = dpp_i<kDppShr + 1>(inc); if (gl >= 1) inc += t; }
    if constexpr (G >= 4) { const int t = dpp_i<kDppShr + 2>(inc); if (gl >= 2) inc += t; }
    if constexpr (G >= 8) { const int t = dpp_i<kDppShr + 4>(inc); if (gl >= 4) inc += t; }
    if constexpr (G >= 16) { const int t = dpp_i<kDppShr + 8>(inc); if (gl >= 8) inc += t; }
    *total = group_sum_i<G>(v);
  } else {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int t = __shfl_up(inc, o, G);
      if (gl >= o) inc += t;
    }
    *total = __shfl(inc, G - 1, G);
  }
  return inc - v;
}

// x / 3 correctly rounded: a product with the rounded reciprocal, corrected
// once with the exact remainder (Markstein, IBM J. Res. Dev. 34, 1990).
__device__ inline double div3(double x) {
  constexpr double kThird = 1.0 / 3.0;
  const double q = x * kThird;
  return fma(fma(-q, 3.0, x), kThird, q);
}

// packed index of entry (a, b), a <= b, of a symmetric 6x6 matrix
__host__ __device__ constexpr int P6(int a, int b) { return a * 6 - a * (a - 1) / 2 + (b - a); }

// Lower Cholesky factor of a packed symmetric 6x6 matrix, in place
// (m[P6(j, i)] becomes L(i, j) for i >= j) with the reciprocal diagonal in
// invd; false if a pivot is not above tol times the trace (the matrix is
// then rank deficient for the purpose of the fit).
template <class T>
__device__ inline bool chol6(T* m, T* invd, T tol) {
  const T trace = m[P6(0, 0)] + m[P6(1, 1)] + m[P6(2, 2)] + m[P6(3, 3)] + m[P6(4, 4)] + m[P6(5, 5)];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T d = m[P6(j, j)];
#pragma unroll
    for (int p = 0; p < j; ++p) d -= m[P6(p, j)] * m[P6(p, j)];
    if (!(d > tol * trace)) ok = false;
    const T ljj = sqrt(d > T(0) ? d : T(1e-30));
    m[P6(j, j)] = ljj;
    const T inv = T(1) / ljj;
    invd[j] = inv;
#pragma unroll
    for (int i2 = j + 1; i2 < 6; ++i2) {
      T s2 = m[P6(j, i2)];
#pragma unroll
      for (int p = 0; p < j; ++p) s2 -= m[P6(p, i2)] * m[P6(p, j)];
      m[P6(j, i2)] = s2 * inv;
    }
  }
  return ok;
}

// x = (L L^T)^-1 rhs in double arithmetic, L from chol6 (of either type);
// rhs and x may alias.
template <class T>
__device__ inline void chol6_solve(const T* L, const T* invd, const double* rhs, double* x) {
  double y[6];
#pragma unroll
  for (int i2 = 0; i2 < 6; ++i2) {
    double s2 = rhs[i2];
#pragma unroll
    for (int p = 0; p < i2; ++p) s2 -= (double)L[P6(p, i2)] * y[p];
    y[i2] = s2 * (double)invd[i2];
  }
#pragma unroll
  for (int i2 = 5; i2 >= 0; --i2) {
    double s2 = y[i2];
#pragma unroll
    for (int p = i2 + 1; p < 6; ++p) s2 -= (double)L[P6(i2, p)] * x[p];
    x[i2] = s2 * (double)invd[i2];
  }
}

// The local frame of a cell: origin xc (the cell centre), tangents t1, t2
// completing the frame normal n to a right-handed orthonormal basis (Duff
// et al., JCGT 2017), and 1/h.
struct Frame {
  double xc[3];
  double t1[3], t2[3], n[3];
  double inv_h;
};

__device__ inline void duff_tangents(double n0, double n1, double n2, double t1[3], double t2[3]) {
  const double sg = copysign(1.0, n2);
  const double fa = -1.0 / (sg + n2);
  const double fb = n0 * n1 * fa;
  t1[0] = 1.0 + sg * n0 * n0 * fa;
  t1[1] = sg * fb;
  t1[2] = -sg * n0;
  t2[0] = fb;
  t2[1] = sg + n1 * n1 * fa;
  t2[2] = -n1;
}

// Moments of one triangle (corners a, b, e) in the h-scaled frame, in type
// T: mom = integrals over its projection of (1, xi, eta, xi^2, xi eta,
// eta^2) by the edge-midpoint rule, vt = the integral of its plane.  The
// differences to the frame origin are taken in double precision.
template <class T>
__device__ inline void tri_moments(const Frame& F, const P3& a, const P3& b, const P3& e, T mom[6], T& vt) {
  const P3 p[3] = {a, b, e};
  T xi[3], eta[3], zeta[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T dx = (T)(p[c].x - F.xc[0]), dy = (T)(p[c].y - F.xc[1]), dz = (T)(p[c].z - F.xc[2]);
    xi[c] = fma(dz, (T)F.t1[2], fma(dy, (T)F.t1[1], dx * (T)F.t1[0])) * (T)F.inv_h;
    eta[c] = fma(dz, (T)F.t2[2], fma(dy, (T)F.t2[1], dx * (T)F.t2[0])) * (T)F.inv_h;
    zeta[c] = fma(dz, (T)F.n[2], fma(dy, (T)F.n[1], dx * (T)F.n[0])) * (T)F.inv_h;
  }
  const T area = T(0.5) * fma(xi[1] - xi[0], eta[2] - eta[0], -((xi[2] - xi[0]) * (eta[1] - eta[0])));
  T sm[6] = {T(3), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T mx = T(0.5) * (xi[c] + xi[(c + 1) % 3]);
    const T my = T(0.5) * (eta[c] + eta[(c + 1) % 3]);
    sm[1] += mx;
    sm[2] += my;
    sm[3] = fma(mx, mx, sm[3]);
    sm[4] = fma(mx, my, sm[4]);
    sm[5] = fma(my, my, sm[5]);
  }
  const T a3 = area * (T(1) / T(3));
#pragma unroll
  for (int q = 0; q < 6; ++q) mom[q] = a3 * sm[q];
  vt = a3 * (zeta[0] + zeta[1] + zeta[2]);
}

// Weight w of the triangle whose centre lies at squared distance dd, inside
// the support of squared radius lim: Wendland's C2 function of q = d/delta.
__device__ inline double wendland(double dd, double inv_delta) {
  const double qq = sqrt(dd) * inv_delta;
  const double om = 1.0 - qq;
  return (1.0 + 4.0 * qq) * (om * om) * (om * om);
}

// Squared distance of the centre of triangle (a, b, e) to xc, each centre
// coordinate (c0 + c1 + c2) / 3 in corner order: the support decision.
__device__ inline double centre_d2(const P3& a, const P3& b, const P3& e, const double xc[3]) {
  const double cx = div3(a.x + b.x + e.x);
  const double cy = div3(a.y + b.y + e.y);
  const double cz = div3(a.z + b.z + e.z);
  const double dx = cx - xc[0], dy = cy - xc[1], dz = cz - xc[2];
  return dx * dx + dy * dy + dz * dz;
}

// Accumulate w m m^T (upper triangle, packed) and w vt m.
template <class T>
__device__ inline void accumulate(T* acc, T w, const T mom[6], T vt) {
  const T wv = w * vt;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const T wa = w * mom[a];
#pragma unroll
    for (int b = a; b < 6; ++b) acc[P6(a, b)] = fma(wa, mom[b], acc[P6(a, b)]);
    acc[21 + a] = fma(wv, mom[a], acc[21 + a]);
  }
}

// One cell, by one thread: the paraboloid coefficients in the h-scaled
// frame, scaled back, kappa = 2H at the frame origin and the interface
// normal.  F holds the fit slots at a stride of fs: the frame normal in 27-29
// and the weighted count in 30 (-1: ring beyond every capacity, -2: no
// closest vertex), and either (solved = false) the 27 sums of the normal
// equations in 0-26, factored here by Cholesky with one step of iterative
// refinement against the unfactored sums, or (solved = true) the
// coefficients in 0-5 and 1 or 0 (full rank or not) in 6.
__device__ inline void solve_cell(const PPICArgs& A, int32_t c, const double* F, int64_t fs, bool solved) {
  const int64_t cs = A.cell_cap;
  const double h = A.g.h, inv_h = 1.0 / h;
  const double wcnt = F[30 * fs];
  const double n0 = F[27 * fs], n1 = F[28 * fs], n2 = F[29 * fs];
  double co[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
  double kap = NAN, ni0 = NAN, ni1 = NAN, ni2 = NAN;
  uint32_t st = wcnt == -1.0 ? FTC_CELL_OVERFLOW : 0u;
  if (wcnt >= 0.0) {
    double ah[6];
    bool have = false;
    if (solved) {
      have = F[6 * fs] > 0.0;
#pragma unroll
      for (int i2 = 0; i2 < 6; ++i2) ah[i2] = F[i2 * fs];
    } else {
      double acc[27];
#pragma unroll
      for (int qa = 0; qa < 27; ++qa) acc[qa] = F[qa * fs];
      double invd[6];
      have = chol6(acc, invd, 1e-14) && wcnt >= 6.0;
      if (have) {
        chol6_solve(acc, invd, acc + 21, ah);
        // residual with the unfactorised matrix, read again (the compiler
        // barriers keep the reads of a row next to their use: the solve then
        // holds few registers beyond the factor)
        asm volatile("" ::: "memory");
        double r6[6];
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) {
          double s2 = acc[21 + i2];
#pragma unroll
          for (int p = 0; p < 6; ++p) s2 -= F[(i2 <= p ? P6(i2, p) : P6(p, i2)) * fs] * ah[p];
          r6[i2] = s2;
          asm volatile("" ::: "memory");
        }
        chol6_solve(acc, invd, r6, r6);
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) ah[i2] += r6[i2];
      }
    }
    if (!have) {
      st |= FTC_CELL_RANK;
    } else {
      co[0] = h * ah[0];
      co[1] = ah[1];
      co[2] = ah[2];
      co[3] = ah[3] * inv_h;
      co[4] = ah[4] * inv_h;
      co[5] = ah[5] * inv_h;
      const double gx = co[1], gy = co[2];
      const double num = 2.0 * co[3] * (1.0 + gy * gy) - 2.0 * gx * gy * co[4] + 2.0 * co[5] * (1.0 + gx * gx);
      const double sq = 1.0 + gx * gx + gy * gy;
      kap = -num / (sq * sqrt(sq));
      double t1[3], t2[3];
      duff_tangents(n0, n1, n2, t1, t2);
      ni0 = n0 - co[1] * t1[0] - co[2] * t2[0];
      ni1 = n1 - co[1] * t1[1] - co[2] * t2[1];
      ni2 = n2 - co[1] * t1[2] - co[2] * t2[2];
      const double il = 1.0 / sqrt(ni0 * ni0 + ni1 * ni1 + ni2 * ni2);
      ni0 *= il;
      ni1 *= il;
      ni2 *= il;
    }
  }
  A.kappa[c] = kap;
  A.nx[c] = ni0;
  A.ny[c] = ni1;
  A.nz[c] = ni2;
  A.frame_n[c] = n0;
  A.frame_n[cs + c] = n1;
  A.frame_n[2 * cs + c] = n2;
  if (A.coeff)
    for (int qa = 0; qa < 6; ++qa) A.coeff[qa * cs + c] = st ? NAN : co[qa];
  if (A.status) A.status[c] = (int32_t)st;
}

__device__ inline void write_diag(const PPICArgs& A, int32_t c, int32_t vs, int32_t nT, int32_t cnt, int32_t it) {
  if (!A.diag) return;
  const int64_t cs = A.cell_cap;
  A.diag[c] = vs;
  A.diag[cs + c] = nT;
  A.diag[2 * cs + c] = cnt;
  A.diag[3 * cs + c] = it;
}

// Closest vertex of the cell with centre xc: the pre-pass result when it
// is final, else (need) a search over all vertices by the G lanes of the
// cell.  Called by all 64 lanes.
// searched: whether the search ran for this cell; inc: the pre-pass's
// incident-triangle range (offset, count) of its vertex, valid otherwise.
template <int G>
__device__ inline int32_t closest_vertex(const PPICArgs& A, int32_t c, bool act, const double xc[3], int gl,
                                         bool& searched, int2& inc) {
  const double reach = 1.5 * A.g.h;
  const double reach2 = reach * reach * (1.0 - 1e-12);
  int32_t vs = act ? A.best_v[c] : 0;
  inc = act ? A.best_inc[c] : make_int2(0, 0);
  const bool need = act && !(vs != INT_MAX && A.best_d2[c] < reach2);
  searched = need;
  if (__any(need)) {
    double bd = DBL_MAX;
    int32_t bv = INT_MAX;
    if (need)
      for (int32_t v = gl; v < A.nv; v += G) consider(A.vtx4, v, xc, bd, bv);
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) {
      const double od = __shfl_xor(bd, o, 64);
      const int32_t ov = __shfl_xor(bv, o, 64);
      if (lex_less(od, ov, bd, bv)) {
        bd = od;
        bv = ov;
      }
    }
    if (need) vs = bv;
  }
  return vs;
}

template <int G>
__device__ inline int32_t closest_vertex(const PPICArgs& A, int32_t c, bool act, const double xc[3], int gl) {
  bool searched;
  int2 inc;
  return closest_vertex<G>(A, c, act, xc, gl, searched, inc);
}

// Cell groups of the fast shape for workgroup `bid` of `nblk`.  The groups
// are split into kXCD contiguous ranges, one per XCD (workgroups are dealt
// to the XCDs in turn, so each L2 holds one part of the front).
//   chunk = 0: a static split, workgroup bid taking groups bid / kXCD,
//     bid / kXCD + nblk / kXCD, ... of its XCD's range;
//   chunk > 0: a work queue, the workgroups of an XCD taking `chunk` groups
//     at a time from their range through its counter qctr[x * kQStride],
//     then from the other XCDs' ranges in turn once theirs is empty (a
//     plain read first skips the ranges already taken).  The counters start
//     at zero; the wide shape's kernel, next in the same stream, clears them.
template <class Body>
__device__ inline void for_cell_groups(int32_t ngroups, int32_t bid, int32_t nblk, int32_t chunk, int32_t* qctr,
                                       Body body) {
  const int32_t per = (ngroups + kXCD - 1) / kXCD;
  if (chunk <= 0) {
    const int32_t xcd = bid % kXCD, nj = nblk / kXCD;
    for (int32_t q = bid / kXCD; q < per; q += nj) {
      const int32_t gi = xcd * per + q;
      if (gi >= ngroups) break;
      body(gi);
    }
    return;
  }
  const int32_t x0 = bid % kXCD;
  for (int32_t d = 0; d < kXCD; ++d) {
    const int32_t x = (x0 + d) % kXCD;
    const int32_t lo = x * per, hi = min(lo + per, ngroups);
    int32_t* ctr = qctr + x * kQStride;
    if (d > 0) {
      int32_t seen = 0;
      if (threadIdx.x == 0) seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (lo + __shfl(seen, 0, 64) >= hi) continue;
    }
    for (;;) {
      int32_t q0 = 0;
      if (threadIdx.x == 0) q0 = atomicAdd(ctr, chunk);
      q0 = __shfl(q0, 0, 64);
      if (lo + q0 >= hi) break;
      const int32_t g1 = min(lo + q0 + chunk, hi);
      for (int32_t gi = lo + q0; gi < g1; ++gi) body(gi);
    }
  }
}

// ------------------------------------------------------------ wide shape
// Ring-building state, dead once the rings are complete.
template <class C>
struct RingMem {
  int32_t hkey[C::HS];    // hash set of vertices: -1 empty, v new in this ring, v | kPlaced in V
  int32_t hval[C::HS];    // new vertex: first occurrence (3 x position + corner); placed: its ring
  int32_t V[C::VC];       // ring vertices
  int32_t Vo[C::VC];      // offset of their incident-triangle lists
  int32_t Vs[C::VC + 1];  // prefix sums of their degrees
  uint32_t fbits[C::FW];  // first occurrences of the new vertices of the current ring
  uint8_t own[C::Batch];  // ring vertex of each candidate of the current batch
};
// Fit state, alive after the rings.
template <class C>
struct FitMem {
  double W[C::TC];   // weights of the triangles inside the support
  int32_t S[C::TC];  // those triangles
};
template <class C>
struct __align__(8) CellMem {
  union {
    RingMem<C> r;
    FitMem<C> f;
  } u;
  int32_t T[C::TC];  // ring triangles
};

constexpr int32_t kPlaced = INT32_MIN;  // vertex ids are below 2^31 - 1, so key | kPlaced != -1

// Insert a key that is not placed (if absent, as a new vertex) and return
// its slot; -1 if the table is full.
template <class C>
__device__ inline int hinsert(RingMem<C>& M, int32_t key) {
  int s = hslot<C::HS>(key);
#pragma unroll 1
  for (int p = 0; p < C::HS; ++p) {
    const int32_t prev = atomicCAS(&M.hkey[s], -1, key);
    if (prev == -1 || prev == key) return s;
    s = (s + 1) & (C::HS - 1);
  }
  return -1;
}

// Ring of the vertex key if it is placed in V (0 for v*), else -1.  home is
// the table entry at the key's home slot, read beforehand.
template <class C>
__device__ inline int ring_of(const RingMem<C>& M, int32_t key, int32_t home) {
  const int32_t placed = key | kPlaced;
  int s = hslot<C::HS>(key);
  if (home == placed) return M.hval[s];
  if (home == -1 || home == key) return -1;
#pragma unroll 1
  for (int p = 0; p < C::HS; ++p) {
    s = (s + 1) & (C::HS - 1);
    const int32_t k = M.hkey[s];
    if (k == placed) return M.hval[s];
    if (k == -1 || k == key) return -1;
  }
  return -1;
}

// The queued cells (ovf_cells[0, counters[C_NOVF])) or, with kSel, the
// cells of the surrogate's selection, one at a time per workgroup `bid` of
// `nblk` (64 lanes): rings built level by level (the candidates of ring r
// are the incident triangles of the vertices new in V_{r-1}, spread over
// the lanes through prefix sums of their degrees; a candidate is kept from
// the first of its corners that is new in V_{r-1}, and only if none of its
// corners lies in V_{r-2}; corners of kept triangles not yet placed enter
// the table marked with their first occurrence and are placed in V_r in
// that order), the support grown by `grow` until `n_min` triangles fall
// inside it (or the ring is exhausted, or `max_iter` adjustments), the fit
// and the solve.
template <class C, bool kSel>
__device__ inline void ppic_wide_cells(const PPICArgs& A, int32_t bid, int32_t nblk) {
  constexpr int G = C::G;
  static_assert(G == 64, "one cell per wavefront");
  __shared__ CellMem<C> CM;
  RingMem<C>& RM = CM.u.r;
  FitMem<C>& FM = CM.u.f;
  const Grid& g = A.g;
  const int gl = threadIdx.x;
  const int32_t nitems = kSel ? min(A.counters[C_NSEL], A.cell_cap) : min(A.counters[C_NOVF], A.cell_cap);
  const double h = g.h;
  const int R = A.prm.rings;
  const uint64_t below_me = (1ull << gl) - 1ull;

  for (int32_t item = bid; item < nitems; item += nblk) {
    const int32_t c = kSel ? A.sel[item] : A.ovf_cells[item];
    const Cell3 cc3 = unpack_cell(g, A.cell_ids[c]);
    const double xc[3] = {cell_centre(g.x0, cc3.i, h), cell_centre(g.y0, cc3.j, h), cell_centre(g.z0, cc3.k, h)};
    const int32_t vs = closest_vertex<G>(A, c, true, xc, gl);
    bool ok = vs >= 0 && vs < A.nv;

    // ---- ring neighbourhood
    for (int s = gl; s < C::HS; s += G) {
      RM.hkey[s] = -1;
      RM.hval[s] = INT_MAX;
    }
    __syncthreads();
    if (ok && gl == 0) {
      RM.hkey[hslot<C::HS>(vs)] = vs | kPlaced;  // empty table
      RM.hval[hslot<C::HS>(vs)] = 0;
      const int32_t o0 = A.vt_off[vs];
      RM.V[0] = vs;
      RM.Vo[0] = o0;
      RM.Vs[0] = 0;
      RM.Vs[1] = A.vt_off[vs + 1] - o0;
    }
    __syncthreads();
    int32_t nV = 1, nT = 0;
    bool ovf = false;
    double n0 = 0.0, n1 = 0.0, n2 = 1.0;
    int32_t nVprev = 0;  // V_{r-2} is V[0, nVprev); the vertices new in V_{r-1} are V[nVprev, nV)
    for (int r = 1; r <= R; ++r) {
      for (int w = gl; w < C::FW; w += G) RM.fbits[w] = 0u;
      // T_r = T_{r-1} plus the triangles at the vertices new in V_{r-1} with
      // no corner in V_{r-2}; their candidates f in [flo, fhi), in batches
      const int nVc = min(nV, C::VC);
      const bool go_r = ok && !ovf;
      const int flo = go_r ? RM.Vs[nVprev] : 0, fhi = go_r ? RM.Vs[nVc] : 0;
      const int tot = fhi - flo;
      const int nb = (tot + C::Batch - 1) / C::Batch;
      const int prounds = tot > 0 ? (nVc - nVprev + G - 1) / G : 0;
      bool full = false;
      for (int b = 0; b < nb; ++b) {
        const int b0 = flo + b * C::Batch;
        // owners of the candidates [b0, b0 + Batch)
        for (int k = 0; k < prounds; ++k) {
          const int p = nVprev + k * G + gl;
          if (p < nVc) {
            const int lo = max(RM.Vs[p], b0), hi = min(RM.Vs[p + 1], b0 + C::Batch);
            for (int f = lo; f < hi; ++f) RM.own[f - b0] = (uint8_t)p;
          }
        }
        __syncthreads();
        const int kact = min(C::CR, max(0, (fhi - b0 + G - 1) / G));
        int32_t ct[C::CR], cu[C::CR];
#pragma unroll
        for (int k = 0; k < C::CR; ++k) {
          ct[k] = -1;
          cu[k] = -1;
          if (k < kact) {
            const int f = b0 + k * G + gl;
            if (f < fhi) {
              const int p = RM.own[f - b0];
              cu[k] = RM.V[p];
              ct[k] = A.vt_ids[RM.Vo[p] + (f - RM.Vs[p])];
            }
          }
        }
        int4 cc[C::CR];
#pragma unroll
        for (int k = 0; k < C::CR; ++k)
          if (k < kact) cc[k] = A.tri4[ct[k] >= 0 ? ct[k] : 0];
        // kept from the first of its corners that is new in V_{r-1}: corners
        // before the owner lie outside V_{r-1}, corners after it outside
        // V_{r-2}
        int32_t hk0[C::CR], hk1[C::CR], hk2[C::CR];
#pragma unroll
        for (int k = 0; k < C::CR; ++k)
          if (k < kact) {
            hk0[k] = RM.hkey[hslot<C::HS>(cc[k].x)];
            hk1[k] = RM.hkey[hslot<C::HS>(cc[k].y)];
            hk2[k] = RM.hkey[hslot<C::HS>(cc[k].z)];
          }
#pragma unroll
        for (int k = 0; k < C::CR; ++k)
          if (k < kact) {
            bool keep = ct[k] >= 0;
            int l0 = -1, l1 = -1, l2 = -1;  // rings of the corners, -1 outside V_{r-1}
            if (keep) {
              const int eu = cc[k].x == cu[k] ? 0 : (cc[k].y == cu[k] ? 1 : 2);
              l0 = eu == 0 ? r - 1 : ring_of<C>(RM, cc[k].x, hk0[k]);
              l1 = eu == 1 ? r - 1 : ring_of<C>(RM, cc[k].y, hk1[k]);
              l2 = eu == 2 ? r - 1 : ring_of<C>(RM, cc[k].z, hk2[k]);
              if (eu >= 1 && l0 >= 0) keep = false;
              if (eu >= 2 && l1 >= 0) keep = false;
              if (eu < 1 && l1 >= 0 && l1 < r - 1) keep = false;
              if (eu < 2 && l2 >= 0 && l2 < r - 1) keep = false;
            }
            const uint64_t bal = gballot<G>(keep, 0);
            if (keep) {
              const int pos = nT + __popcll(bal & below_me);
              if (pos < C::TC) {
                CM.T[pos] = ct[k];
                if (r < R) {
                  // corners outside V_{r-1} enter the table, marked with
                  // their first occurrence
                  const int32_t cr[3] = {cc[k].x, cc[k].y, cc[k].z};
                  const int lv[3] = {l0, l1, l2};
#pragma unroll
                  for (int e = 0; e < 3; ++e) {
                    if (lv[e] >= 0) continue;
                    const int s = hinsert<C>(RM, cr[e]);
                    if (s >= 0)
                      atomicMin(&RM.hval[s], 3 * pos + e);
                    else
                      full = true;
                  }
                }
              }
            }
            nT += __popcll(bal);
          }
        __syncthreads();
      }
      if (nT > C::TC || __any(full)) ovf = true;

      if (r == 1) {
        // normal of v*: T_1 is v*'s incident list, ascending; the cross
        // products are summed serially in that order
        const int n1c = (ok && !ovf) ? nT : 0;
        const int nr = (n1c + G - 1) / G;
        const int qn = min(n1c, G);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < nr; ++k) {
          const int i = k * G + gl;
          const int4 t4 = A.tri4[i < n1c ? CM.T[i] : 0];
          const P3 a = vtx(A.vtx4, t4.x), bb = vtx(A.vtx4, t4.y), e = vtx(A.vtx4, t4.z);
          const double ux = bb.x - a.x, uy = bb.y - a.y, uz = bb.z - a.z;
          const double wx = e.x - a.x, wy = e.y - a.y, wz = e.z - a.z;
          const double cx = uy * wz - uz * wy;
          const double cy = uz * wx - ux * wz;
          const double cz = ux * wy - uy * wx;
          for (int qq = 0; qq < qn; ++qq) {
            const double x = __shfl(cx, qq, G), y = __shfl(cy, qq, G), z = __shfl(cz, qq, G);
            if (k * G + qq < n1c) {
              s0 += x;
              s1 += y;
              s2 += z;
            }
          }
        }
        if (ok && !ovf) {
          const double nl = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
          n0 = s0 / nl;
          n1 = s1 / nl;
          n2 = s2 / nl;
        }
      }
      if (r == R) break;

      // V_r: the new corners of T_r in order of first occurrence
      const bool go = ok && !ovf;
      for (int s = gl; s < C::HS; s += G) {
        const int32_t f = RM.hval[s];
        if (go && RM.hkey[s] >= 0 && f < 3 * C::TC) atomicOr(&RM.fbits[f >> 5], 1u << (f & 31));
      }
      __syncthreads();
      int nnew = 0;
#pragma unroll
      for (int w = 0; w < C::FW; ++w) nnew += __popc(RM.fbits[w]);
      for (int s = gl; s < C::HS; s += G) {
        const int32_t f = RM.hval[s], key = RM.hkey[s];
        if (go && key >= 0 && f < 3 * C::TC) {
          int rank = __popc(RM.fbits[f >> 5] & ((1u << (f & 31)) - 1u));
          for (int w = 0; w < (f >> 5); ++w) rank += __popc(RM.fbits[w]);
          const int pos = nV + rank;
          if (pos < C::VC) {
            const int32_t o0 = A.vt_off[key];
            RM.V[pos] = key;
            RM.Vo[pos] = o0;
            RM.Vs[pos + 1] = A.vt_off[key + 1] - o0;  // degree, turned into a prefix sum below
          }
          RM.hkey[s] = key | kPlaced;
          RM.hval[s] = r;
        }
      }
      const int nV0 = nV;
      if (go) nV += nnew;
      nVprev = nV0;
      if (nV > C::VC) ovf = true;
      __syncthreads();
      // prefix sums of the new degrees, in place
      const int pend = (ok && !ovf) ? nV : nV0;
      const int vrounds = (pend - nV0 + G - 1) / G;
      int32_t run = (ok && !ovf) ? RM.Vs[nV0] : 0;
      for (int k = 0; k < vrounds; ++k) {
        const int p = nV0 + k * G + gl;
        int32_t inc = p < pend ? RM.Vs[p + 1] : 0;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
          const int32_t t = __shfl_up(inc, o, G);
          if (gl >= o) inc += t;
        }
        if (p < pend) RM.Vs[p + 1] = run + inc;
        run += __shfl(inc, G - 1, G);
      }
      __syncthreads();
    }

    if (ovf) ok = false;
    const int nTc = ok ? min(nT, C::TC) : 0;
    Frame F;
    F.xc[0] = xc[0];
    F.xc[1] = xc[1];
    F.xc[2] = xc[2];
    F.n[0] = n0;
    F.n[1] = n1;
    F.n[2] = n2;
    duff_tangents(n0, n1, n2, F.t1, F.t2);
    F.inv_h = 1.0 / h;

    // ---- centre distances (kept in the weight list's storage), support
    // radius, weights
    const int drounds = (nTc + G - 1) / G;
    for (int k = 0; k < drounds; ++k) {
      const int i = k * G + gl;
      if (i < nTc) {
        const int4 c4 = A.tri4[CM.T[i]];
        FM.W[i] = centre_d2(vtx(A.vtx4, c4.x), vtx(A.vtx4, c4.y), vtx(A.vtx4, c4.z), xc);
      }
    }
    __syncthreads();
    double delta = A.prm.delta_over_h * h;
    int32_t it = 0, cnt = 0;
    if (ok) {
      for (;;) {
        const double lim = delta * delta;
        int mine = 0;
        for (int i = gl; i < nTc; i += G) mine += FM.W[i] < lim ? 1 : 0;
        cnt = group_sum_i<G>(mine);
        if (cnt >= A.prm.n_min || cnt == nTc || it == A.prm.max_iter) break;
        delta = delta * A.prm.grow;
        ++it;
      }
    }
    {
      const double lim = delta * delta;
      const double inv_delta = 1.0 / delta;
      // compaction in place: an entry moves to a position not after its own,
      // and every lane reads its round's entries before any lane writes
      int nw = 0;
      for (int k = 0; k < drounds; ++k) {
        const int i = k * G + gl;
        const double dd = i < nTc ? FM.W[i] : DBL_MAX;
        const int32_t ti = i < nTc ? CM.T[i] : 0;
        const bool keep = i < nTc && dd < lim;
        const uint64_t bal = gballot<G>(keep, 0);
        __syncthreads();
        if (keep) {
          const int pos = nw + __popcll(bal & below_me);
          FM.W[pos] = wendland(dd, inv_delta);
          FM.S[pos] = ti;
        }
        nw += __popcll(bal);
        __syncthreads();
      }
    }
    __syncthreads();

    // ---- weighted moments and normal equations
    double acc[27];
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = 0.0;
    const int wrounds = ok ? (cnt + G - 1) / G : 0;
    for (int k = 0; k < wrounds; ++k) {
      const int j = k * G + gl;
      if (j < cnt) {
        const int4 t4 = A.tri4[FM.S[j]];
        double mom[6], vt;
        tri_moments(F, vtx(A.vtx4, t4.x), vtx(A.vtx4, t4.y), vtx(A.vtx4, t4.z), mom, vt);
        accumulate(acc, FM.W[j], mom, vt);
      }
    }
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = group_sum<G>(acc[qa]);

    // ---- the normal equations, solved by one lane
    __syncthreads();
    if (gl == 0) {
#pragma unroll
      for (int qa = 0; qa < 27; ++qa) FM.W[qa] = acc[qa];
      FM.W[27] = n0;
      FM.W[28] = n1;
      FM.W[29] = n2;
      FM.W[30] = ok ? (double)cnt : (ovf ? -1.0 : -2.0);
    }
    __syncthreads();
    if (gl == 0) {
      solve_cell(A, c, FM.W, 1, false);
      write_diag(A, c, vs, nT, cnt, it);
    }
    __syncthreads();
  }
}

// The cells the fast shape queued.  The queue's count is read by every
// workgroup before the last one to finish clears it for the next call; the
// fast shape's work-queue counters are cleared on the way.
__global__ __launch_bounds__(64) void k_ppic_wide(PPICArgs A) {
  // the fast shape's work-queue counters, for the next call
  if (blockIdx.x == 0 && threadIdx.x < kXCD) A.counters[C_QUEUE0 + threadIdx.x * kQStride] = 0;
  ppic_wide_cells<Wide, false>(A, blockIdx.x, gridDim.x);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&A.counters[C_WIDE_DONE], 1) == (int32_t)gridDim.x - 1) {
      __threadfence();
      A.counters[C_NOVF] = 0;
      A.counters[C_WIDE_DONE] = 0;
    }
  }
}

// The cells the learned curvature hands over, sel[0, counters[C_NSEL]), with
// the wide shape: a selection is a small part of the cells, and the wide
// shape's per-cell latency is the lower.
__global__ __launch_bounds__(64) void k_ppic_wide_sel(PPICArgs A) { ppic_wide_cells<Wide, true>(A, blockIdx.x, gridDim.x); }

// After it: report the selection's count and clear it for the next call (a
// kernel of its own: a completion count over the selection kernel's
// workgroups, one same-address atomic each, cost about 40 us).
__global__ void k_sel_done(int32_t* counters, int32_t* n_sel_out) {
  if (n_sel_out) *n_sel_out = counters[C_NSEL];
  counters[C_NSEL] = 0;
}

// ------------------------------------------------------------ fast shape
template <int G_>
struct FastCfg {
  static constexpr int G = G_;        // lanes per cell
  static constexpr int NG = 64 / G_;  // cells per wavefront
  static constexpr int HV = 64;       // slots of the vertex set (power of two)
  static constexpr int VC = 32;       // vertices of V_{R-1}
  static constexpr int TC = 64;       // ring triangles
  static constexpr int IB = 8;        // incident triangles of one vertex loaded together
  static_assert(IB * 3 <= 32, "new-corner mask");
};

// Per cell: the vertex set and the ring, then (after the fit) the sums.
union FastMem {
  struct {
    int32_t hv[64];    // V as an open-addressing hash set, -1 empty
    int32_t V[32];     // V in insertion order
    int32_t T[3][64];  // corners of the ring triangles
  } r;
  double S[32];  // the 27 sums, the frame normal, the weighted count
};

// The vertex set is an open-addressing hash in LDS (-1 empty, linear
// probing from the key's home slot).  Callers take the first probe of a
// batch of keys together: an insert as one compare-and-swap at the home
// slot, whose previous content tells a new key (empty), a present one (the
// key) and a collision (another key); a lookup as one read.  Only a
// collision continues here with the probes after slot s: insert (true when
// this lane added the key; full is set if the sequence wraps) ...
template <int HS>
__device__ inline bool vset_insert_after(int32_t* hv, int32_t key, int s, bool& full) {
#pragma unroll 1
  for (int p = 1; p < HS; ++p) {
    s = (s + 1) & (HS - 1);
    const int32_t prev = atomicCAS(&hv[s], -1, key);
    if (prev == -1) return true;
    if (prev == key) return false;
  }
  full = true;
  return false;
}

// ... and lookup.
template <int HS>
__device__ inline bool vset_has_after(const int32_t* hv, int32_t key, int s) {
#pragma unroll 1
  for (int p = 1; p < HS; ++p) {
    s = (s + 1) & (HS - 1);
    const int32_t cur = hv[s];
    if (cur == key) return true;
    if (cur == -1) return false;
  }
  return false;
}

// Corners of the triangles at vertex u (incident list [off, off + deg))
// join the vertex set; the ones this lane adds are appended to V in lane
// order.  The wavefront loops to the largest degree, IB incidences at a
// time with their loads issued together.
template <class C>
__device__ inline void expand_vertex(const PPICArgs& A, FastMem& M, int32_t u, int32_t off, int deg, int gl,
                                     int& nV, bool& full) {
  constexpr int G = C::G, IB = C::IB;
  const int md = wave_max_dpp(deg);
  for (int j0 = 0; j0 < md; j0 += IB) {
    int32_t tt[IB];
#pragma unroll
    for (int j = 0; j < IB; ++j) tt[j] = j0 + j < deg ? A.vt_ids[off + j0 + j] : -1;
    int4 cc[IB];
#pragma unroll
    for (int j = 0; j < IB; ++j) cc[j] = tt[j] >= 0 ? A.tri4[tt[j]] : make_int4(-1, -1, -1, -1);
    // the first probes of all corners issued together (a lane's LDS
    // operations complete in order, so a key repeated in the batch is added
    // by its first occurrence), then the probe sequences of the collisions
    // in corner order: the lanes that add each key are those of one insert
    // after the other
    int32_t pv[IB][3];
    uint32_t want = 0u;
#pragma unroll
    for (int j = 0; j < IB; ++j) {
      const int32_t cr[3] = {cc[j].x, cc[j].y, cc[j].z};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const bool w = cr[e] >= 0 && cr[e] != u;
        pv[j][e] = w ? atomicCAS(&M.r.hv[hslot<C::HV>(cr[e])], -1, cr[e]) : cr[e];
        if (w) want |= 1u << (3 * j + e);
      }
    }
    uint32_t added = 0u;
#pragma unroll
    for (int j = 0; j < IB; ++j) {
      const int32_t cr[3] = {cc[j].x, cc[j].y, cc[j].z};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const uint32_t bit = 1u << (3 * j + e);
        if (!(want & bit) || pv[j][e] == cr[e]) continue;
        if (pv[j][e] == -1 || vset_insert_after<C::HV>(M.r.hv, cr[e], hslot<C::HV>(cr[e]), full)) added |= bit;
      }
    }
    int total;
    int pos = nV + group_excl_scan<G>(__popc(added), gl, &total);
#pragma unroll
    for (int j = 0; j < IB; ++j) {
      const int32_t cr[3] = {cc[j].x, cc[j].y, cc[j].z};
#pragma unroll
      for (int e = 0; e < 3; ++e)
        if ((added >> (3 * j + e)) & 1u) {
          if (pos < C::VC) M.r.V[pos] = cr[e];
          ++pos;
        }
    }
    nV += total;
  }
}

// The triangles at vertex u of V_{R-1} that have u as their first corner in
// V_{R-1} are appended to the ring in lane order.
template <class C>
__device__ inline void ring_vertex(const PPICArgs& A, FastMem& M, int32_t u, int32_t off, int deg, int gl, int& nT) {
  constexpr int G = C::G, IB = C::IB;
  const int md = wave_max_dpp(deg);
  for (int j0 = 0; j0 < md; j0 += IB) {
    int32_t tt[IB];
#pragma unroll
    for (int j = 0; j < IB; ++j) tt[j] = j0 + j < deg ? A.vt_ids[off + j0 + j] : -1;
    int4 cc[IB];
#pragma unroll
    for (int j = 0; j < IB; ++j) cc[j] = tt[j] >= 0 ? A.tri4[tt[j]] : make_int4(-1, -1, -1, -1);
    // u is t1 or t2: the triangle is kept unless an earlier corner is in
    // the set; the home slots of those corners are read together first
    int32_t hx[IB], hy[IB];
#pragma unroll
    for (int j = 0; j < IB; ++j) {
      const bool nx = tt[j] >= 0 && cc[j].x != u, ny = nx && cc[j].y != u;
      hx[j] = nx ? M.r.hv[hslot<C::HV>(cc[j].x)] : -1;
      hy[j] = ny ? M.r.hv[hslot<C::HV>(cc[j].y)] : -1;
    }
    uint32_t kept = 0u;
#pragma unroll
    for (int j = 0; j < IB; ++j) {
      bool keep = tt[j] >= 0;
      if (keep && cc[j].x != u) {
        const int32_t x = cc[j].x, y = cc[j].y;
        const bool inx = hx[j] == x || (hx[j] != -1 && vset_has_after<C::HV>(M.r.hv, x, hslot<C::HV>(x)));
        keep = !inx && (y == u || !(hy[j] == y || (hy[j] != -1 && vset_has_after<C::HV>(M.r.hv, y, hslot<C::HV>(y)))));
      }
      if (keep) kept |= 1u << j;
    }
    int total;
    int pos = nT + group_excl_scan<G>(__popc(kept), gl, &total);
#pragma unroll
    for (int j = 0; j < IB; ++j)
      if ((kept >> j) & 1u) {
        if (pos < C::TC) {
          M.r.T[0][pos] = cc[j].x;
          M.r.T[1][pos] = cc[j].y;
          M.r.T[2][pos] = cc[j].z;
        }
        ++pos;
      }
    nT += total;
  }
}

// The fast shape over every interfacial cell, G lanes per cell; kMixed:
// the normal equations formed and factored in single precision, refined
// twice with double-precision residuals g = sum_t w_t (V_t - m_t . a) m_t
// = b - M a of the same triangles (moments again in double precision),
// solved with the single-precision factor; each step shrinks the error by
// about cond(M) times the single-precision unit roundoff.  A
// single-precision pivot at or below 1e-6 of the trace marks the cell rank
// deficient.
template <int G, bool kMixed, bool kPrefetch = true>
__device__ inline void ppic_fast(const PPICArgs& A, int32_t bid, int32_t nblk) {
  using C = FastCfg<G>;
  constexpr int NG = C::NG;
  __shared__ FastMem SM[NG];
  const Grid& g = A.g;
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  FastMem& M = SM[grp];
  const int32_t nitems = min(A.counters[C_NIF], A.cell_cap);
  const double h = g.h;
  const int R = A.prm.rings;
  const int32_t ngroups = (nitems + NG - 1) / NG;

  for_cell_groups(ngroups, bid, nblk, A.queue_chunk, A.counters + C_QUEUE0, [&](int32_t gi) {
    const int32_t c = gi * NG + grp;
    const bool act = c < nitems;
    int32_t vs;
    bool searched;
    int2 inc;
    {
      const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
      const double xc[3] = {cell_centre(g.x0, cc3.i, h), cell_centre(g.y0, cc3.j, h), cell_centre(g.z0, cc3.k, h)};
      vs = closest_vertex<G>(A, c, act, xc, gl, searched, inc);
    }
    const bool ok = act && vs >= 0 && vs < A.nv;

    // ---- V_0 = {v*}
    for (int s = gl; s < C::HV; s += G) M.r.hv[s] = -1;
    __syncthreads();
    if (ok && gl == 0) {
      M.r.hv[hslot<C::HV>(vs)] = vs;
      M.r.V[0] = vs;
    }
    __syncthreads();
    int nV = 1;
    bool full = false;
    double n0 = 0.0, n1 = 0.0, n2 = 1.0;

    // ---- the triangles at v*: frame normal (cross products summed in
    // ascending triangle order) and, for R >= 2, V_1
    {
      int32_t o0 = inc.x;
      int deg0 = inc.y;
      if (searched && ok) {
        o0 = A.vt_off[vs];
        deg0 = A.vt_off[vs + 1] - o0;
      }
      if (!ok) deg0 = 0;
      const int nr = wave_max_dpp((deg0 + G - 1) / G);
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int k = 0; k < nr; ++k) {
        const int i = k * G + gl;
        const bool have = i < deg0;
        const int4 t4 = A.tri4[have ? A.vt_ids[o0 + i] : 0];
        const P3 a = vtx(A.vtx4, t4.x), b = vtx(A.vtx4, t4.y), e = vtx(A.vtx4, t4.z);
        if (R >= 2) {
          // the corners join V while the vertex records are in flight; first
          // probes together, then the collisions in corner order
          const int32_t cr[3] = {t4.x, t4.y, t4.z};
          int32_t pv[3];
#pragma unroll
          for (int e2 = 0; e2 < 3; ++e2)
            pv[e2] = have && cr[e2] != vs ? atomicCAS(&M.r.hv[hslot<C::HV>(cr[e2])], -1, cr[e2]) : cr[e2];
          uint32_t added = 0u;
#pragma unroll
          for (int e2 = 0; e2 < 3; ++e2) {
            if (!have || cr[e2] == vs || pv[e2] == cr[e2]) continue;
            if (pv[e2] == -1 || vset_insert_after<C::HV>(M.r.hv, cr[e2], hslot<C::HV>(cr[e2]), full))
              added |= 1u << e2;
          }
          int total;
          int pos = nV + group_excl_scan<G>(__popc(added), gl, &total);
#pragma unroll
          for (int e2 = 0; e2 < 3; ++e2)
            if ((added >> e2) & 1u) {
              if (pos < C::VC) M.r.V[pos] = cr[e2];
              ++pos;
            }
          nV += total;
        }
        const double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
        const double wx = e.x - a.x, wy = e.y - a.y, wz = e.z - a.z;
        const double cx = uy * wz - uz * wy;
        const double cy = uz * wx - ux * wz;
        const double cz = ux * wy - uy * wx;
        const int qn = wave_max_dpp(min(max(deg0 - k * G, 0), G));  // lanes holding a triangle, at most
#pragma unroll 4
        for (int qq = 0; qq < qn; ++qq) {
          const double x = __shfl(cx, qq, G), y = __shfl(cy, qq, G), z = __shfl(cz, qq, G);
          if (k * G + qq < deg0) {
            s0 += x;
            s1 += y;
            s2 += z;
          }
        }
      }
      const double nl = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
      n0 = s0 / nl;
      n1 = s1 / nl;
      n2 = s2 / nl;
    }
    bool ovf = nV > C::VC || gballot<G>(full, grp) != 0;
    __syncthreads();

    // ---- V_2 .. V_{R-1}: corners of the triangles at the vertices new in
    // the previous level
    int nVprev = 1;
    for (int r = 2; r <= R - 1; ++r) {
      const int lo = nVprev, hi = nV;
      nVprev = nV;
      const bool go = ok && !ovf;
      const int rounds = wave_max_dpp(go ? (hi - lo + G - 1) / G : 0);
      for (int k = 0; k < rounds; ++k) {
        const int p = lo + k * G + gl;
        const bool have = go && p < hi;
        const int32_t u = have ? M.r.V[p] : 0;
        const int32_t off = have ? A.vt_off[u] : 0;
        const int deg = have ? A.vt_off[u + 1] - off : 0;
        expand_vertex<C>(A, M, u, off, deg, gl, nV, full);
      }
      if (nV > C::VC || gballot<G>(full, grp) != 0) ovf = true;
      __syncthreads();
    }

    // ---- the ring T_R
    int nT = 0;
    {
      const bool go = ok && !ovf;
      const int nVc = go ? nV : 0;
      const int rounds = wave_max_dpp((nVc + G - 1) / G);
      for (int k = 0; k < rounds; ++k) {
        const int p = k * G + gl;
        const bool have = p < nVc;
        const int32_t u = have ? M.r.V[p] : 0;
        const int32_t off = have ? A.vt_off[u] : 0;
        const int deg = have ? A.vt_off[u + 1] - off : 0;
        ring_vertex<C>(A, M, u, off, deg, gl, nT);
      }
      if (nT > C::TC) ovf = true;
    }
    __syncthreads();

    // ---- one pass over the ring at the first support radius
    Frame F;
    {
      const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
      F.xc[0] = cell_centre(g.x0, cc3.i, h);
      F.xc[1] = cell_centre(g.y0, cc3.j, h);
      F.xc[2] = cell_centre(g.z0, cc3.k, h);
    }
    F.n[0] = n0;
    F.n[1] = n1;
    F.n[2] = n2;
    duff_tangents(n0, n1, n2, F.t1, F.t2);
    F.inv_h = 1.0 / h;
    const bool fit = ok && !ovf;
    const int nTc = fit ? nT : 0;
    const double delta = A.prm.delta_over_h * h;
    const double lim = delta * delta, inv_delta = 1.0 / delta;
    const int frounds = wave_max_dpp((nTc + G - 1) / G);
    int mine = 0;
    using AccT = typename std::conditional<kMixed, float, double>::type;
    AccT acc[27];
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = AccT(0);
    // kPrefetch: each round's vertex records are loaded during the round
    // before (the registers they take make a build held to 128 VGPRs spill)
    auto ring_tri = [&](int k, bool& valid, P3& a, P3& b, P3& e) {
      const int i = k * G + gl;
      valid = i < nTc;
      const int32_t c0 = valid ? M.r.T[0][i] : 0, c1 = valid ? M.r.T[1][i] : 0, c2 = valid ? M.r.T[2][i] : 0;
      a = vtx(A.vtx4, c0);
      b = vtx(A.vtx4, c1);
      e = vtx(A.vtx4, c2);
    };
    bool valid;
    P3 a, b, e;
    if constexpr (kPrefetch) ring_tri(0, valid, a, b, e);
    for (int k = 0; k < frounds; ++k) {
      bool valid1;
      P3 a1, b1, e1;
      if constexpr (kPrefetch)
        ring_tri(k + 1, valid1, a1, b1, e1);
      else
        ring_tri(k, valid, a, b, e);
      const double dd = centre_d2(a, b, e, F.xc);
      const bool in = valid && dd < lim;
      mine += in ? 1 : 0;
      const double w = in ? wendland(dd, inv_delta) : 0.0;
      AccT mom[6], vt;
      tri_moments(F, a, b, e, mom, vt);
      accumulate(acc, (AccT)w, mom, vt);
      if constexpr (kPrefetch) {
        valid = valid1;
        a = a1;
        b = b1;
        e = e1;
      }
    }
    const int cnt = group_sum_i<G>(mine);
    // the support needs adjusting: the wide shape takes the cell
    const bool grow = fit && !(cnt >= A.prm.n_min || cnt == nTc || A.prm.max_iter == 0);
    const bool queue = ok && (ovf || grow);
    if (queue && gl == 0) A.ovf_cells[atomicAdd(&A.counters[C_NOVF], 1)] = c;

    double ah[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool full_rank = false;
    if constexpr (kMixed) {
#pragma unroll
      for (int qa = 0; qa < 27; ++qa) acc[qa] = group_sum_f<G>(acc[qa]);
      float invf[6];
      full_rank = chol6(acc, invf, 1e-6f) && cnt >= 6;
      double rhs[6];
#pragma unroll
      for (int qa = 0; qa < 6; ++qa) rhs[qa] = (double)acc[21 + qa];
      chol6_solve(acc, invf, rhs, ah);
      for (int pass = 0; pass < 2; ++pass) {
        double gr[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < frounds; ++k) {
          const int i = k * G + gl;
          const bool valid = i < nTc;
          const int32_t c0 = valid ? M.r.T[0][i] : 0, c1 = valid ? M.r.T[1][i] : 0, c2 = valid ? M.r.T[2][i] : 0;
          const P3 a = vtx(A.vtx4, c0), b = vtx(A.vtx4, c1), e = vtx(A.vtx4, c2);
          const double dd = centre_d2(a, b, e, F.xc);
          const double w = valid && dd < lim ? wendland(dd, inv_delta) : 0.0;
          double mom[6], vt;
          tri_moments(F, a, b, e, mom, vt);
          double rr = vt;
#pragma unroll
          for (int q2 = 0; q2 < 6; ++q2) rr -= mom[q2] * ah[q2];
          const double wr = w * rr;
#pragma unroll
          for (int q2 = 0; q2 < 6; ++q2) gr[q2] = fma(wr, mom[q2], gr[q2]);
        }
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) gr[q2] = group_sum<G>(gr[q2]);
        chol6_solve(acc, invf, gr, gr);
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) ah[q2] += gr[q2];
      }
    } else {
#pragma unroll
      for (int qa = 0; qa < 27; ++qa) acc[qa] = group_sum<G>(acc[qa]);
    }

    // ---- solve (one lane per cell) and outputs
    __syncthreads();
    if (gl == 0) {
      if constexpr (kMixed) {
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) M.S[q2] = ah[q2];
        M.S[6] = full_rank ? 1.0 : 0.0;
      } else {
#pragma unroll
        for (int qa = 0; qa < 27; ++qa) M.S[qa] = acc[qa];
      }
      M.S[27] = F.n[0];
      M.S[28] = F.n[1];
      M.S[29] = F.n[2];
      M.S[30] = ok ? (double)cnt : -2.0;
    }
    __syncthreads();
    if (act && !queue && gl == 0) {
      solve_cell(A, c, M.S, 1, kMixed);
      write_diag(A, c, vs, nT, cnt, 0);
    }
    __syncthreads();
  });
}

__global__ __launch_bounds__(64) void k_ppic_fast4(PPICArgs A) { ppic_fast<4, false>(A, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_ppic_fast8(PPICArgs A) { ppic_fast<8, false>(A, blockIdx.x, gridDim.x); }
// The same held to four wavefronts per SIMD (128 VGPRs, some spilled, the
// fit without its round-ahead loads): on a front whose cell groups fill the
// chip at most three times at that occupancy, the fewer rounds of
// wavefronts pay for the spills.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_ppic_fast8_w4(PPICArgs A) { ppic_fast<8, false, false>(A, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64) void k_ppic_fast16(PPICArgs A) { ppic_fast<16, false>(A, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64) void k_ppic_fast32(PPICArgs A) { ppic_fast<32, false>(A, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64) void k_ppic_fast64(PPICArgs A) { ppic_fast<64, false>(A, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64) void k_ppic_fast8_mixed(PPICArgs A) { ppic_fast<8, true>(A, blockIdx.x, gridDim.x); }

inline int32_t round_up(int64_t n, int64_t m) { return (int32_t)((n + m - 1) / m * m); }

}  // namespace

hipError_t launch_ppic(const ftc_cells* ws, const Mesh& m, const PPICParams& p, double* kappa, double* nx,
                       double* ny, double* nz, double* coeff, int32_t* cell_status, int32_t* diag, hipStream_t s) {
  return launch_ppic_cells(ws, m, p, kappa, nx, ny, nz, coeff, cell_status, diag, nullptr, nullptr, s);
}

hipError_t launch_ppic_cells(const ftc_cells* ws, const Mesh& m, const PPICParams& p, double* kappa, double* nx,
                             double* ny, double* nz, double* coeff, int32_t* cell_status, int32_t* diag,
                             const int32_t* sel, int32_t* n_sel_out, hipStream_t s) {
  const Grid& g = ws->grid;
  PPICArgs A;
  A.g = g;
  A.nv = m.nv;
  A.prm = p;
  A.tri4 = reinterpret_cast<int4*>(ws->tri4);
  A.vtx4 = reinterpret_cast<double2*>(ws->vtx4);
  A.cell_ids = ws->cell_ids;
  A.vt_off = ws->vt_off;
  A.vt_ids = ws->vt_ids;
  A.best_d2 = ws->best_d2;
  A.best_v = ws->best_v;
  A.best_inc = reinterpret_cast<const int2*>(ws->best_inc);
  A.counters = ws->counters;
  A.ovf_cells = ws->ovf_cells;
  A.frame_n = ws->frame_n;
  A.cell_cap = ws->cell_cap;
  A.kappa = kappa;
  A.nx = nx;
  A.ny = ny;
  A.nz = nz;
  A.coeff = coeff;
  A.status = cell_status;
  A.diag = diag;
  A.queue_chunk = ws->tune.queue_chunk;
  A.sel = sel;
  A.n_sel_out = n_sel_out;
  time_start(ws, FTC_KERNEL_PPIC, s);
  if (sel) {
    hipLaunchKernelGGL(k_ppic_wide_sel, dim3(round_up(std::min<int64_t>(std::max<int64_t>(ws->cell_cap, 1), 2048), kXCD)),
                       dim3(64), 0, s, A);
    hipLaunchKernelGGL(k_sel_done, dim3(1), dim3(1), 0, s, ws->counters, n_sel_out);
  } else {
    const int lanes = p.mixed ? 8 : ws->tune.ring_lanes;
    const int64_t groups = ((int64_t)ws->cell_cap * lanes + 63) / 64;
    // a work queue without a grid of its own: the wavefronts the chip holds
    // at the fast shape's occupancy (three per SIMD, four SIMDs per CU)
    const int64_t grid_cap = ws->tune.ring_blocks > 0 ? ws->tune.ring_blocks
                             : (ws->tune.queue_chunk > 0 ? 12 * (int64_t)ws->cu_count : 65536);
    const dim3 grid(round_up(std::min<int64_t>(std::max<int64_t>(groups, 1), grid_cap), kXCD));
    if (p.mixed)
      hipLaunchKernelGGL(k_ppic_fast8_mixed, grid, dim3(64), 0, s, A);
    else if (lanes == 4)
      hipLaunchKernelGGL(k_ppic_fast4, grid, dim3(64), 0, s, A);
    else if (lanes == 16)
      hipLaunchKernelGGL(k_ppic_fast16, grid, dim3(64), 0, s, A);
    else if (lanes == 32)
      hipLaunchKernelGGL(k_ppic_fast32, grid, dim3(64), 0, s, A);
    else if (lanes == 64)
      hipLaunchKernelGGL(k_ppic_fast64, grid, dim3(64), 0, s, A);
    else if (groups <= 3 * 16 * (int64_t)ws->cu_count)  // up to three rounds at four wavefronts per SIMD
      hipLaunchKernelGGL(k_ppic_fast8_w4, grid, dim3(64), 0, s, A);
    else
      hipLaunchKernelGGL(k_ppic_fast8, grid, dim3(64), 0, s, A);
    hipLaunchKernelGGL(k_ppic_wide, dim3(kWideBlocks), dim3(64), 0, s, A);
  }
  time_stop(ws, FTC_KERNEL_PPIC, s);
  return hipGetLastError();
}

}  // namespace ftc
