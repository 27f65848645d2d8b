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
// Ring pass (k_ppic_rings; ppic_cells, one template for two shapes): the
// fast shape gives 8 lanes to each interfacial cell (8 cells per wavefront)
// and holds rings of up to 32 vertices and 64 triangles in LDS; cells whose
// ring is larger are queued for the wide shape (64 lanes per cell, rings of
// 256 vertices and 512 triangles), which runs in the solve launch.  Cells are assigned so that each XCD
// processes a contiguous range, which keeps each L2 on one part of the front.
//   1. ring neighbourhood: V_0 = {v*}; T_r = triangles with a corner in
//      V_{r-1}; V_r = V_{r-1} plus the corners of T_r.  Built incrementally:
//      a triangle with a corner in V_{r-2} is already in T_{r-1}, so the
//      candidates of ring r are the incident triangles of the vertices new
//      in V_{r-1}, spread over the lanes through prefix sums of their
//      degrees.  A candidate is kept from the first of its corners (t0, t1,
//      t2 order) that is new in V_{r-1}, and only if none of its corners lies
//      in V_{r-2}; the ring level of every placed vertex is stored with it in
//      an open-addressing hash table in LDS.  Corners of kept triangles that
//      are not yet placed enter the table at once, marked with their first
//      occurrence (3 x position + corner), and are then placed in V_r in that
//      order;
//   2. normal of v* (area-weighted, summed in ascending triangle order: T_1
//      is v*'s incident list) and a right-handed tangent frame (Duff et al.,
//      JCGT 2017);
//   3. triangle-centre distances, the support radius grown by `grow` until
//      `n_min` triangles fall inside (or the ring is exhausted, or
//      `max_iter` adjustments), Wendland weights of the triangles inside.
//      The fast shape writes the weighted triangles (id and weight, 12
//      bytes each) to a per-cell list in HBM, with the frame normal and the
//      count; the wide shape goes on with steps 4 and 5 itself.
// Fit pass (k_ppic_fit), the cells of the fast shape, 8 lanes per cell:
//   4. per lane: each listed triangle's corners (from the packed corner
//      array, which stays in L2), its projection into the frame
//      (coordinates divided by h for conditioning), its six moments by the
//      edge-midpoint rule (exact for quadratics) and the integral of its
//      plane, and the weighted normal equations M a = b accumulated in
//      registers; all-reduce over the cell's lanes with row permutations;
//      the 27 sums are stored per cell.
// Solve pass (k_ppic_wide_solve), one thread per cell:
//   5. Cholesky factorisation of the packed M with one step of iterative
//      refinement, curvature kappa = 2H at the frame origin and the
//      interface normal.
// Every loop bound is uniform over the wavefront (maxima over its cells), so
// LDS phases are separated by plain workgroup barriers.
#include <float.h>

#include <algorithm>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kXCD = 8;          // accelerator complex dies; workgroups are dealt to them in turn
constexpr int kWideBlocks = 64;  // persistent workgroups of the wide shape

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <int G_, int HS_, int VC_, int TC_, int CR_>
struct Cfg {
  static constexpr int G = G_;        // lanes per cell
  static constexpr int NG = 64 / G_;  // cells per wavefront
  static constexpr int HS = HS_;      // hash slots (power of two)
  static constexpr int VC = VC_;      // ring-vertex capacity (owner table holds bytes: <= 256)
  static constexpr int TC = TC_;      // ring-triangle capacity
  static constexpr int CR = CR_;      // candidates per lane per batch
  static constexpr int Batch = CR_ * G_;
  static constexpr int TR = (TC_ + G_ - 1) / G_;
  static constexpr int FW = (3 * TC_ + 31) / 32;  // words of the first-occurrence bitmap
  static_assert((HS_ & (HS_ - 1)) == 0 && HS_ >= 2 * VC_, "hash size");
  static_assert(VC_ <= 256, "owner table holds bytes");
};
using Fast = Cfg<8, 64, 32, 64, 6>;
// the same capacities with 16 lanes per cell (4 cells per wavefront): the
// queue to the wide shape, and so every result, is the same as Fast's
using Fast16 = Cfg<16, 64, 32, 64, 3>;
using Wide = Cfg<64, 512, 256, 512, 4>;

// ----------------------------------------------------------------- main kernel
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
  int32_t* counters;
  int32_t* ovf_cells;
  double* fit;
  int32_t* wl_tri;  // per cell: the triangles of its fit (ids; the fit pass reads their corners)
  double* wl_w;
  int32_t cell_cap;
  double *kappa, *nx, *ny, *nz, *coeff;
  int32_t *status, *diag;
  const int32_t* sel;  // null: every interfacial cell; else the cells sel[0, counters[C_NSEL])
  int32_t* n_sel_out;  // receives the selection's count (may be null)
};



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

template <int HS>
__device__ inline int hslot(int32_t key) {
  return (int)(((uint32_t)key * 2654435761u) >> (32 - ilog2(HS)));
}

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

// Ballot of this lane's group, in the group's low bits.
template <int G>
__device__ inline uint64_t gballot(bool p, int grp) {
  const uint64_t b = __ballot(p);
  if constexpr (G == 64)
    return b;
  else
    return (b >> (G * grp)) & ((1ull << G) - 1ull);
}

__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Lane permutations within rows of 16 lanes (data-parallel primitives):
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}

// Sum over each aligned group of G lanes, the same bits in every lane: each
// step adds a value from a partner lane that adds this lane's value back.
// Called with all 64 lanes active.
template <int G>
__device__ inline double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_d<0xB1>(v);
  if constexpr (G >= 4) v += dpp_d<0x4E>(v);
  if constexpr (G >= 8) v += dpp_d<0x141>(v);
  if constexpr (G >= 16) v += dpp_d<0x140>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
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

// One cell, by one thread: the paraboloid coefficients in the h-scaled
// frame, scaled back, kappa = 2H at the frame origin and the interface
// normal.  F holds the fit slots at a stride of fs: the frame normal in 27-29
// and the weighted count in 30, and either (solved = false) the 27 sums of
// the normal equations in 0-26, factored here by Cholesky with one step of
// iterative refinement against the unfactored sums, or (solved = true) the
// coefficients in 0-5 and 1 or 0 (full rank or not) in 6.
__device__ inline void solve_cell(const PPICArgs& A, int32_t c, const double* F, int64_t fs, bool solved) {
  const int64_t cs = A.cell_cap;
  const double h = A.g.h, inv_h = 1.0 / h;
  {
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
          // residual with the unfactorised matrix, read again
          double r6[6];
#pragma unroll
          for (int i2 = 0; i2 < 6; ++i2) {
            double s2 = acc[21 + i2];
#pragma unroll
            for (int p = 0; p < 6; ++p) s2 -= F[(i2 <= p ? P6(i2, p) : P6(p, i2)) * fs] * ah[p];
            r6[i2] = s2;
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
        // the tangents of the frame again (Duff et al.)
        const double sg = copysign(1.0, n2);
        const double fa = -1.0 / (sg + n2);
        const double fb = n0 * n1 * fa;
        const double t1x = 1.0 + sg * n0 * n0 * fa, t1y = sg * fb, t1z = -sg * n0;
        const double t2x = fb, t2y = sg + n1 * n1 * fa, t2z = -n1;
        ni0 = n0 - co[1] * t1x - co[2] * t2x;
        ni1 = n1 - co[1] * t1y - co[2] * t2y;
        ni2 = n2 - co[1] * t1z - co[2] * t2z;
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
    if (A.coeff)
      for (int qa = 0; qa < 6; ++qa) A.coeff[qa * cs + c] = st ? NAN : co[qa];
    if (A.status) A.status[c] = (int32_t)st;
  }
}

// The cells of one shape, processed by workgroup `bid` of `nblk` (64 lanes).
// kQueue = false: every interfacial cell, overflowing cells queued.
// kQueue = true: the queued cells.
// kSel: the cells of the surrogate's selection (with the wide shape).
template <class C, bool kQueue, bool kSel = false>
__device__ inline void ppic_cells(const PPICArgs& A, int32_t bid, int32_t nblk) {
  constexpr int G = C::G, NG = C::NG;
  __shared__ CellMem<C> SM[NG];
  const Grid& g = A.g;
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  CellMem<C>& CM = SM[grp];
  RingMem<C>& RM = CM.u.r;
  FitMem<C>& FM = CM.u.f;
  const int32_t nitems = kSel ? min(A.counters[C_NSEL], A.cell_cap)
                              : (kQueue ? min(A.counters[C_NQUEUED], A.cell_cap) : min(A.counters[C_NIF], A.cell_cap));
  const double h = g.h;
  const int R = A.prm.rings;
  const double reach = 1.5 * h;
  const double reach2 = reach * reach * (1.0 - 1e-12);
  const uint64_t below_me = (1ull << gl) - 1ull;

  // each XCD takes a contiguous range of cell groups
  const int32_t ngroups = (nitems + NG - 1) / NG;
  const int32_t per = (ngroups + kXCD - 1) / kXCD;
  const int32_t xcd = bid % kXCD, nj = nblk / kXCD;
  for (int32_t q = bid / kXCD; q < per; q += nj) {
    const int32_t gi = xcd * per + q;
    if (gi >= ngroups) break;
    const int32_t item = gi * NG + grp;
    const bool act = item < nitems;
    const int32_t c = act ? (kSel ? A.sel[item] : (kQueue ? A.ovf_cells[item] : item)) : 0;
    const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
    const double xc[3] = {cell_centre(g.x0, cc3.i, h), cell_centre(g.y0, cc3.j, h), cell_centre(g.z0, cc3.k, h)};

    // ---- closest vertex: pre-pass result, else a search over all vertices
    int32_t vs = act ? A.best_v[c] : 0;
    const bool need = act && !(vs != INT_MAX && A.best_d2[c] < reach2);
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
    bool ok = act && vs >= 0 && vs < A.nv;

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
      const int nb = wave_max_i((tot + C::Batch - 1) / C::Batch);
      const int prounds = wave_max_i(tot > 0 ? (nVc - nVprev + G - 1) / G : 0);
      bool full = false;
      for (int b = 0; b < nb; ++b) {
        const int b0 = flo + b * C::Batch;
        // owners of the candidates [b0, b0 + Batch)
        for (int k = 0; k < prounds; ++k) {
          const int p = nVprev + k * G + gl;
          if (tot > 0 && p < nVc) {
            const int lo = max(RM.Vs[p], b0), hi = min(RM.Vs[p + 1], b0 + C::Batch);
            for (int f = lo; f < hi; ++f) RM.own[f - b0] = (uint8_t)p;
          }
        }
        __syncthreads();
        const int kact = wave_max_i(min(C::CR, max(0, (fhi - b0 + G - 1) / G)));
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
            const uint64_t bal = gballot<G>(keep, grp);
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
      if (nT > C::TC || gballot<G>(full, grp)) ovf = true;

      if (r == 1) {
        // normal of v*: T_1 is v*'s incident list, ascending; the cross
        // products are summed serially in that order
        const int n1c = (ok && !ovf) ? nT : 0;
        const int nr = wave_max_i((n1c + G - 1) / G);
        const int qn = wave_max_i(min(n1c, G));
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
      const int vrounds = wave_max_i((pend - nV0 + G - 1) / G);
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

    if (!kQueue && ovf && ok) {
      // a ring beyond this shape's capacities: the wide shape takes the cell
      if (gl == 0) A.ovf_cells[atomicAdd(&A.counters[C_NOVF], 1)] = c;
    }
    const bool emit = act && !(!kQueue && ovf && ok);
    if (ovf) ok = false;
    const int nTc = ok ? min(nT, C::TC) : 0;

    const double sg = copysign(1.0, n2);
    const double fa = -1.0 / (sg + n2);
    const double fb = n0 * n1 * fa;
    const double t1x = 1.0 + sg * n0 * n0 * fa, t1y = sg * fb, t1z = -sg * n0;
    const double t2x = fb, t2y = sg + n1 * n1 * fa, t2z = -n1;

    // ---- centre distances (kept in the weight list's storage), support
    // radius, weights
    const int drounds = wave_max_i((nTc + G - 1) / G);
    {
      int4 cn = A.tri4[gl < nTc ? CM.T[gl] : 0];
      for (int k = 0; k < drounds; ++k) {
        const int i = k * G + gl;
        const int4 c4 = cn;
        cn = A.tri4[i + G < nTc ? CM.T[i + G] : 0];
        const P3 a = vtx(A.vtx4, c4.x), b = vtx(A.vtx4, c4.y), e = vtx(A.vtx4, c4.z);
        const double cx = div3(a.x + b.x + e.x);
        const double cy = div3(a.y + b.y + e.y);
        const double cz = div3(a.z + b.z + e.z);
        const double dx = cx - xc[0], dy = cy - xc[1], dz = cz - xc[2];
        if (i < nTc) FM.W[i] = dx * dx + dy * dy + dz * dz;
      }
    }
    double delta = A.prm.delta_over_h * h;
    int32_t it = 0, cnt = 0;
    bool done = !ok;
    for (;;) {
      const double lim = delta * delta;
      int mine = 0;
      for (int i = gl; i < nTc; i += G) mine += FM.W[i] < lim ? 1 : 0;
#pragma unroll
      for (int o = G / 2; o >= 1; o >>= 1) mine += __shfl_xor(mine, o, 64);
      if (!done) {
        cnt = mine;
        if (cnt >= A.prm.n_min || cnt == nTc || it == A.prm.max_iter) {
          done = true;
        } else {
          delta = delta * A.prm.grow;
          ++it;
        }
      }
      if (!__any(!done)) break;
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
        const uint64_t bal = gballot<G>(keep, grp);
        if (keep) {
          const int pos = nw + __popcll(bal & below_me);
          const double qq = sqrt(dd) * inv_delta;
          const double om = 1.0 - qq;
          const double wt = (1.0 + 4.0 * qq) * (om * om) * (om * om);
          if constexpr (kQueue) {
            FM.W[pos] = wt;
            FM.S[pos] = ti;
          } else {
            A.wl_w[(int64_t)c * kFitList + pos] = wt;
            A.wl_tri[(int64_t)c * kFitList + pos] = ti;
          }
        }
        nw += __popcll(bal);
      }
    }
    __syncthreads();

    if constexpr (!kQueue) {
      // the fit pass takes the list; a queued cell is marked for it to skip
      if (act && gl == 0) {
        const int64_t cs = A.cell_cap;
        A.fit[27 * cs + c] = n0;
        A.fit[28 * cs + c] = n1;
        A.fit[29 * cs + c] = n2;
        A.fit[30 * cs + c] = !emit ? -3.0 : (ok ? (double)cnt : (ovf ? -1.0 : -2.0));
        if (A.diag && emit) {
          A.diag[c] = vs;
          A.diag[cs + c] = nT;
          A.diag[2 * cs + c] = cnt;
          A.diag[3 * cs + c] = it;
        }
      }
      __syncthreads();
      continue;
    }

    // ---- weighted moments and normal equations
    const double inv_h = 1.0 / h;
    double acc[27];
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = 0.0;
    const int wrounds = wave_max_i(ok ? (cnt + G - 1) / G : 0);
    int4 tn = A.tri4[(ok && gl < cnt) ? FM.S[gl] : 0];
    for (int k = 0; k < wrounds; ++k) {
      const int j = k * G + gl;
      const bool valid = ok && j < cnt;
      const double w = valid ? FM.W[j] : 0.0;
      const int4 t4 = tn;
      {
        const int jn = j + G;
        tn = A.tri4[(ok && jn < cnt) ? FM.S[jn] : 0];
      }
      const int32_t cr[3] = {t4.x, t4.y, t4.z};
      double xi[3], eta[3], zeta[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const P3 p = vtx(A.vtx4, cr[e]);
        const double dx = p.x - xc[0], dy = p.y - xc[1], dz = p.z - xc[2];
        xi[e] = fma(dz, t1z, fma(dy, t1y, dx * t1x)) * inv_h;
        eta[e] = fma(dz, t2z, fma(dy, t2y, dx * t2x)) * inv_h;
        zeta[e] = fma(dz, n2, fma(dy, n1, dx * n0)) * inv_h;
      }
      const double area = 0.5 * fma(xi[1] - xi[0], eta[2] - eta[0], -((xi[2] - xi[0]) * (eta[1] - eta[0])));
      double sm[6] = {3.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double mx = 0.5 * (xi[e] + xi[(e + 1) % 3]);
        const double my = 0.5 * (eta[e] + eta[(e + 1) % 3]);
        sm[1] += mx;
        sm[2] += my;
        sm[3] = fma(mx, mx, sm[3]);
        sm[4] = fma(mx, my, sm[4]);
        sm[5] = fma(my, my, sm[5]);
      }
      const double a3 = area * (1.0 / 3.0);
      double mom[6];
#pragma unroll
      for (int qa = 0; qa < 6; ++qa) mom[qa] = a3 * sm[qa];
      const double wv = w * (a3 * (zeta[0] + zeta[1] + zeta[2]));
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double wa = w * mom[a];
#pragma unroll
        for (int b = a; b < 6; ++b) acc[P6(a, b)] = fma(wa, mom[b], acc[P6(a, b)]);
        acc[21 + a] = fma(wv, mom[a], acc[21 + a]);
      }
    }
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = group_sum<G>(acc[qa]);

    // ---- the normal equations (weighted count -1: ring beyond the
    // capacities, -2: no closest vertex), solved by one lane per cell
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
    if (emit && gl == 0) {
      const int64_t cs = A.cell_cap;
      solve_cell(A, c, FM.W, 1, false);
      if (A.diag) {
        A.diag[c] = vs;
        A.diag[cs + c] = nT;
        A.diag[2 * cs + c] = cnt;
        A.diag[3 * cs + c] = it;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_ppic_rings(PPICArgs A) { ppic_cells<Fast, false>(A, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64) void k_ppic_rings16(PPICArgs A) {
  ppic_cells<Fast16, false>(A, blockIdx.x, gridDim.x);
}
// The cells the learned curvature hands over, sel[0, counters[C_NSEL]), with
// the wide shape (rings, fit and solve in the workgroup, one cell at a
// time): a selection is a small part of the cells, and the wide shape's
// per-cell latency is the lower.
__global__ __launch_bounds__(64) void k_ppic_wide_sel(PPICArgs A) { ppic_cells<Wide, true, true>(A, blockIdx.x, gridDim.x); }

// After it: report the selection's count and clear it for the next call (a
// kernel of its own: a completion count over the selection kernel's
// workgroups, one same-address atomic each, cost about 40 us).
__global__ void k_sel_done(int32_t* counters, int32_t* n_sel_out) {
  if (n_sel_out) *n_sel_out = counters[C_NSEL];
  counters[C_NSEL] = 0;
}

// Weighted moments and normal equations of the cells whose ring fitted the
// fast shape: 8 lanes per cell (8 cells per wavefront) over the cell's
// weighted-triangle list; sums reduced over the lanes and stored for the
// solve pass.
constexpr int kFitG = 8;
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_ppic_fit(PPICArgs A) {
  constexpr int G = kFitG, NG = 64 / kFitG;
  __shared__ double stage[NG][28];
  const Grid& g = A.g;
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  const int32_t nitems = min(A.counters[C_NIF], A.cell_cap);
  const int64_t cs = A.cell_cap;
  const double h = g.h, inv_h = 1.0 / h;
  // the ring pass has finished queueing: hand the count to the wide shape
  // and start the next call's queue empty
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.counters[C_NQUEUED] = A.counters[C_NOVF];
    A.counters[C_NOVF] = 0;
  }
  const int32_t ngroups = (nitems + NG - 1) / NG;
  const int32_t per = (ngroups + kXCD - 1) / kXCD;
  const int32_t xcd = blockIdx.x % kXCD, nj = gridDim.x / kXCD;
  for (int32_t q = blockIdx.x / kXCD; q < per; q += nj) {
    const int32_t gi = xcd * per + q;
    if (gi >= ngroups) break;
    const int32_t c = gi * NG + grp;
    const bool act = c < nitems;
    const double wc = act ? A.fit[30 * cs + c] : -2.0;
    const int cnt = wc > 0.0 ? (int)wc : 0;
    const double n0 = act ? A.fit[27 * cs + c] : 0.0, n1 = act ? A.fit[28 * cs + c] : 0.0,
                 n2 = act ? A.fit[29 * cs + c] : 1.0;
    const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
    const double xc[3] = {cell_centre(g.x0, cc3.i, h), cell_centre(g.y0, cc3.j, h), cell_centre(g.z0, cc3.k, h)};
    const double sg = copysign(1.0, n2);
    const double fa = -1.0 / (sg + n2);
    const double fb = n0 * n1 * fa;
    const double t1x = 1.0 + sg * n0 * n0 * fa, t1y = sg * fb, t1z = -sg * n0;
    const double t2x = fb, t2y = sg + n1 * n1 * fa, t2z = -n1;
    double acc[27];
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = 0.0;
    const int wrounds = wave_max_i((cnt + G - 1) / G);
    const int32_t* lt = A.wl_tri + (int64_t)(act ? c : 0) * kFitList;
    const double* lw = A.wl_w + (int64_t)(act ? c : 0) * kFitList;
    // entries of the next round (triangle ids, then their corners) are loaded
    // while this round is computed; a lane past the list (or a cell with an
    // empty list, whose entries were never written) takes vertex 0 with weight 0
    const int4 kNone = make_int4(0, 0, 0, 0);
    int4 tn = gl < cnt ? A.tri4[lt[gl]] : kNone;
    double wn = gl < cnt ? lw[gl] : 0.0;
    for (int k = 0; k < wrounds; ++k) {
      const int j = k * G + gl;
      const int4 t4 = tn;
      const double w = wn;
      if (k + 1 < wrounds) {
        const int jn = j + G;
        tn = jn < cnt ? A.tri4[lt[jn]] : kNone;
        wn = jn < cnt ? lw[jn] : 0.0;
      }
      const int32_t cr[3] = {t4.x, t4.y, t4.z};
      double xi[3], eta[3], zeta[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const P3 p = vtx(A.vtx4, cr[e]);
        const double dx = p.x - xc[0], dy = p.y - xc[1], dz = p.z - xc[2];
        xi[e] = fma(dz, t1z, fma(dy, t1y, dx * t1x)) * inv_h;
        eta[e] = fma(dz, t2z, fma(dy, t2y, dx * t2x)) * inv_h;
        zeta[e] = fma(dz, n2, fma(dy, n1, dx * n0)) * inv_h;
      }
      const double area = 0.5 * fma(xi[1] - xi[0], eta[2] - eta[0], -((xi[2] - xi[0]) * (eta[1] - eta[0])));
      double sm[6] = {3.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double mx = 0.5 * (xi[e] + xi[(e + 1) % 3]);
        const double my = 0.5 * (eta[e] + eta[(e + 1) % 3]);
        sm[1] += mx;
        sm[2] += my;
        sm[3] = fma(mx, mx, sm[3]);
        sm[4] = fma(mx, my, sm[4]);
        sm[5] = fma(my, my, sm[5]);
      }
      const double a3 = area * (1.0 / 3.0);
      double mom[6];
#pragma unroll
      for (int qa = 0; qa < 6; ++qa) mom[qa] = a3 * sm[qa];
      const double wv = w * (a3 * (zeta[0] + zeta[1] + zeta[2]));
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double wa = w * mom[a];
#pragma unroll
        for (int b = a; b < 6; ++b) acc[P6(a, b)] = fma(wa, mom[b], acc[P6(a, b)]);
        acc[21 + a] = fma(wv, mom[a], acc[21 + a]);
      }
    }
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) acc[qa] = group_sum<G>(acc[qa]);
    // staged through LDS so that each lane stores a few of the 27 sums
    if (gl == 0) {
#pragma unroll
      for (int qa = 0; qa < 27; ++qa) stage[grp][qa] = acc[qa];
    }
    __syncthreads();
    if (act && wc >= 0.0)
      for (int qa = gl; qa < 27; qa += G) A.fit[qa * cs + c] = stage[grp][qa];
    __syncthreads();
  }
}

template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// group_sum in single precision
template <int G>
__device__ inline float group_sum_f(float v) {
  if constexpr (G >= 2) v += dpp_f<0xB1>(v);
  if constexpr (G >= 4) v += dpp_f<0x4E>(v);
  if constexpr (G >= 8) v += dpp_f<0x141>(v);
  if constexpr (G >= 16) v += dpp_f<0x140>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Mixed precision variant of the fit pass: the weighted normal equations
// are formed and factored in single precision; the solution is then
// improved twice by iterative refinement with residuals evaluated in double
// precision triangle by triangle, g = sum_t w_t (V_t - m_t . a) m_t = b - M a
// (the double-precision moments of the same weighted triangles), solved with
// the single-precision factor.  Each step shrinks the error by about
// cond(M) times the single-precision unit roundoff.  A single-precision
// pivot at or below 1e-6 of the trace marks the cell rank deficient.  The
// coefficients (h-scaled frame) and the rank flag go to the fit slots for
// the solve pass.
__global__ __launch_bounds__(64) void k_ppic_fit_mixed(PPICArgs A) {
  constexpr int G = kFitG, NG = 64 / kFitG;
  const Grid& g = A.g;
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  const int32_t nitems = min(A.counters[C_NIF], A.cell_cap);
  const int64_t cs = A.cell_cap;
  const double h = g.h, inv_h = 1.0 / h;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.counters[C_NQUEUED] = A.counters[C_NOVF];
    A.counters[C_NOVF] = 0;
  }
  const int32_t ngroups = (nitems + NG - 1) / NG;
  const int32_t per = (ngroups + kXCD - 1) / kXCD;
  const int32_t xcd = blockIdx.x % kXCD, nj = gridDim.x / kXCD;
  for (int32_t q = blockIdx.x / kXCD; q < per; q += nj) {
    const int32_t gi = xcd * per + q;
    if (gi >= ngroups) break;
    const int32_t c = gi * NG + grp;
    const bool act = c < nitems;
    const double wc = act ? A.fit[30 * cs + c] : -2.0;
    const int cnt = wc > 0.0 ? (int)wc : 0;
    const double n0 = act ? A.fit[27 * cs + c] : 0.0, n1 = act ? A.fit[28 * cs + c] : 0.0,
                 n2 = act ? A.fit[29 * cs + c] : 1.0;
    const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
    const double xc[3] = {cell_centre(g.x0, cc3.i, h), cell_centre(g.y0, cc3.j, h), cell_centre(g.z0, cc3.k, h)};
    const double sg = copysign(1.0, n2);
    const double fa = -1.0 / (sg + n2);
    const double fb = n0 * n1 * fa;
    const double t1x = 1.0 + sg * n0 * n0 * fa, t1y = sg * fb, t1z = -sg * n0;
    const double t2x = fb, t2y = sg + n1 * n1 * fa, t2z = -n1;
    const int wrounds = wave_max_i((cnt + G - 1) / G);
    const int32_t* lt = A.wl_tri + (int64_t)(act ? c : 0) * kFitList;
    const double* lw = A.wl_w + (int64_t)(act ? c : 0) * kFitList;
    const int4 kNone = make_int4(0, 0, 0, 0);

    // moments of one listed triangle in the h-scaled frame (type T)
    auto moments = [&](const int4 t4, auto zero, auto* mom, auto& vt) {
      using T = decltype(zero);
      const int32_t cr[3] = {t4.x, t4.y, t4.z};
      T xi[3], eta[3], zeta[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const P3 p = vtx(A.vtx4, cr[e]);
        const T dx = (T)(p.x - xc[0]), dy = (T)(p.y - xc[1]), dz = (T)(p.z - xc[2]);
        xi[e] = fma(dz, (T)t1z, fma(dy, (T)t1y, dx * (T)t1x)) * (T)inv_h;
        eta[e] = fma(dz, (T)t2z, fma(dy, (T)t2y, dx * (T)t2x)) * (T)inv_h;
        zeta[e] = fma(dz, (T)n2, fma(dy, (T)n1, dx * (T)n0)) * (T)inv_h;
      }
      const T area = T(0.5) * fma(xi[1] - xi[0], eta[2] - eta[0], -((xi[2] - xi[0]) * (eta[1] - eta[0])));
      T sm[6] = {T(3), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const T mx = T(0.5) * (xi[e] + xi[(e + 1) % 3]);
        const T my = T(0.5) * (eta[e] + eta[(e + 1) % 3]);
        sm[1] += mx;
        sm[2] += my;
        sm[3] = fma(mx, mx, sm[3]);
        sm[4] = fma(mx, my, sm[4]);
        sm[5] = fma(my, my, sm[5]);
      }
      const T a3 = area * (T(1) / T(3));
#pragma unroll
      for (int qa = 0; qa < 6; ++qa) mom[qa] = a3 * sm[qa];
      vt = a3 * (zeta[0] + zeta[1] + zeta[2]);
    };

    // ---- single precision: normal equations, factor, first solution
    float accf[27];
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) accf[qa] = 0.0f;
    for (int k = 0; k < wrounds; ++k) {
      const int j = k * G + gl;
      const int4 t4 = j < cnt ? A.tri4[lt[j]] : kNone;
      const float w = j < cnt ? (float)lw[j] : 0.0f;
      float mom[6], vt;
      moments(t4, 0.0f, mom, vt);
      const float wv = w * vt;
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const float wa = w * mom[a];
#pragma unroll
        for (int b = a; b < 6; ++b) accf[P6(a, b)] = fmaf(wa, mom[b], accf[P6(a, b)]);
        accf[21 + a] = fmaf(wv, mom[a], accf[21 + a]);
      }
    }
#pragma unroll
    for (int qa = 0; qa < 27; ++qa) accf[qa] = group_sum_f<G>(accf[qa]);
    float invf[6];
    const bool full = chol6(accf, invf, 1e-6f) && cnt >= 6;
    double ah[6], rhs[6];
#pragma unroll
    for (int qa = 0; qa < 6; ++qa) rhs[qa] = (double)accf[21 + qa];
    chol6_solve(accf, invf, rhs, ah);

    // ---- two refinement steps with double-precision residuals
    for (int it = 0; it < 2; ++it) {
      double gr[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < wrounds; ++k) {
        const int j = k * G + gl;
        const int4 t4 = j < cnt ? A.tri4[lt[j]] : kNone;
        const double w = j < cnt ? lw[j] : 0.0;
        double mom[6], vt;
        moments(t4, 0.0, mom, vt);
        double r = vt;
#pragma unroll
        for (int a = 0; a < 6; ++a) r -= mom[a] * ah[a];
        const double wr = w * r;
#pragma unroll
        for (int a = 0; a < 6; ++a) gr[a] = fma(wr, mom[a], gr[a]);
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) gr[a] = group_sum<G>(gr[a]);
      chol6_solve(accf, invf, gr, gr);
#pragma unroll
      for (int a = 0; a < 6; ++a) ah[a] += gr[a];
    }
    if (act && wc >= 0.0 && gl < 7) A.fit[gl * cs + c] = gl < 6 ? ah[gl] : (full ? 1.0 : 0.0);
  }
}

// Blocks [0, kWideBlocks): the cells queued for the wide shape, each solved
// in its block; the other blocks: one thread per remaining cell.
__global__ __launch_bounds__(64) void k_ppic_wide_solve(PPICArgs A) {
  if ((int32_t)blockIdx.x < kWideBlocks) {
    ppic_cells<Wide, true>(A, blockIdx.x, kWideBlocks);
    return;
  }
  const int32_t nitems = min(A.counters[C_NIF], A.cell_cap);
  const int64_t cs = A.cell_cap;
  const int32_t nb = gridDim.x - kWideBlocks;
  for (int32_t c = (blockIdx.x - kWideBlocks) * 64 + threadIdx.x; c < nitems; c += nb * 64) {
    const double* F = A.fit + c;
    if (F[30 * cs] == -3.0) continue;  // queued: solved by the wide shape
    solve_cell(A, c, F, cs, A.prm.mixed != 0);
  }
}

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
  int4* tri4 = reinterpret_cast<int4*>(ws->tri4);
  double2* vtx4 = reinterpret_cast<double2*>(ws->vtx4);
  PPICArgs A;
  A.g = g;
  A.nv = m.nv;
  A.prm = p;
  A.tri4 = tri4;
  A.vtx4 = vtx4;
  A.cell_ids = ws->cell_ids;
  A.vt_off = ws->vt_off;
  A.vt_ids = ws->vt_ids;
  A.best_d2 = ws->best_d2;
  A.best_v = ws->best_v;
  A.counters = ws->counters;
  A.ovf_cells = ws->ovf_cells;
  A.fit = ws->fit;
  A.wl_tri = ws->wl_tri;
  A.wl_w = ws->wl_w;
  A.cell_cap = ws->cell_cap;
  A.kappa = kappa;
  A.nx = nx;
  A.ny = ny;
  A.nz = nz;
  A.coeff = coeff;
  A.status = cell_status;
  A.diag = diag;
  A.sel = sel;
  A.n_sel_out = n_sel_out;
  const bool lanes16 = ws->tune.ring_lanes == 16;
  const int64_t groups = ((int64_t)ws->cell_cap + (lanes16 ? Fast16::NG : Fast::NG) - 1) / (lanes16 ? Fast16::NG : Fast::NG);
  const int64_t grid_cap = ws->tune.ring_blocks > 0 ? ws->tune.ring_blocks : 65536;
  const int32_t blocks = round_up(std::min<int64_t>(std::max<int64_t>(groups, 1), grid_cap), kXCD);
  time_start(ws, FTC_KERNEL_PPIC, s);
  if (sel) {
    hipLaunchKernelGGL(k_ppic_wide_sel, dim3(round_up(std::min<int64_t>(std::max<int64_t>(ws->cell_cap, 1), 2048), kXCD)),
                       dim3(64), 0, s, A);
    hipLaunchKernelGGL(k_sel_done, dim3(1), dim3(1), 0, s, ws->counters, n_sel_out);
  } else {
    if (lanes16)
      hipLaunchKernelGGL(k_ppic_rings16, dim3(blocks), dim3(64), 0, s, A);
    else
      hipLaunchKernelGGL(k_ppic_rings, dim3(blocks), dim3(64), 0, s, A);
    const dim3 fit_grid(round_up(std::min<int64_t>(std::max<int64_t>(((int64_t)ws->cell_cap + 7) / 8, 1), 65536), kXCD));
    if (p.mixed)
      hipLaunchKernelGGL(k_ppic_fit_mixed, fit_grid, dim3(64), 0, s, A);
    else
      hipLaunchKernelGGL(k_ppic_fit, fit_grid, dim3(64), 0, s, A);
    hipLaunchKernelGGL(k_ppic_wide_solve, dim3(kWideBlocks + grid_blocks(ws->cell_cap, 64)), dim3(64), 0, s, A);
  }
  time_stop(ws, FTC_KERNEL_PPIC, s);
  return hipGetLastError();
}

}  // namespace ftc
