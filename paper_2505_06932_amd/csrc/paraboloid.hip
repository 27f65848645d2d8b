// paraboloid.hip -- volume fraction under the fitted paraboloid (paper
// section 3.2: alpha is the volume of the cell below the local paraboloid
// over the cell volume).
//
// Per interfacial cell, in cell units (the cube [-1/2, 1/2]^3 around the
// cell centre) and in the PPIC frame (t1, t2, n): the paraboloid is the graph
// zeta = P(xi, eta), and the cube is, for every (xi, eta), the chord
// zeta_lo(xi, eta) <= zeta <= zeta_hi(xi, eta) cut out by its three slabs.
//   alpha = integral over xi of G(xi),
//   G(xi) = integral over eta of clamp(P - zeta_lo, 0, zeta_hi - zeta_lo).
// For fixed xi the integrand is piecewise polynomial in eta between the
// crossings of the slab planes and the roots of P = plane, so G is exact
// (up to rounding).  G is analytic in xi between the events where that
// structure changes: the projected cube corners, the xi at which a conic
// P = plane has a tangent along eta, and the xi at which such a conic meets
// a projected cube edge.  Between consecutive events the xi integral is a
// Gauss-Legendre rule in theta with xi = u0 + (u1 - u0)(1 - cos theta)/2,
// which absorbs the square-root behaviour of G at tangencies: 16 nodes for
// the volume, 24 for the surface integrals (whose normal integral needs
// them for 1e-10 on patches of kappa h near 0.07).
// The surface integrals (area, curvature, normal over the part of the
// paraboloid inside the cell) share the same xi rule: at each node the eta
// intervals where the surface lies in the cube are those between the same
// breakpoints, the normal integral is polynomial (exact) and the area and
// curvature take an 8-node Gauss rule per interval.
// One wavefront per cell: its lanes compute the events, rank-sort them in
// LDS and share the quadrature nodes.
#include <math.h>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 64;       // one wavefront per workgroup and per cell
constexpr int kQV = 16;      // Gauss nodes per xi interval, volume
constexpr int kQS = 24;      // Gauss nodes per xi interval, surface integrals
constexpr int kEvents = 26;  // 8 corners + 12 edges + 6 face tangencies
constexpr int kSlots = 56;   // 2 values per event, the two ends, padding
constexpr int kEta = 24;     // eta breakpoints per G evaluation

constexpr int kS = 8;        // Gauss nodes per eta interval of the surface integrals

// The quadrature tables, one device array (read through the cache, indexed
// per lane): the xi rules, tau[kQV], omega[kQV] then tau[kQS], omega[kQS]
// (xi = u0 + (u1 - u0) tau, weight (u1 - u0) omega), then sx[kS], sw[kS]
// (plain Gauss-Legendre on [0, 1]).  A kernel's view selects its xi rule.
constexpr int kEtaOff = 2 * kQV + 2 * kQS;
struct Nodes {
  const double* p;
  int q;  // nodes of the xi rule
  __device__ int xi_off() const { return q == kQV ? 0 : 2 * kQV; }
  __device__ double tau(int k) const { return p[xi_off() + k]; }
  __device__ double omega(int k) const { return p[xi_off() + q + k]; }
  __device__ double sx(int k) const { return p[kEtaOff + k]; }
  __device__ double sw(int k) const { return p[kEtaOff + kS + k]; }
};
static_assert(kEtaOff + 2 * kS == kQuadNodes, "quadrature table size");

// The cell's paraboloid and cube in its local frame, cell units.  The two
// faces x_k = -+1/2 of axis k (n_k != 0) are the planes
// zeta = c0 + cx xi + ce eta with the same cx, ce: lo the one below the other
// along n, hi the one above.
struct Local {
  double b[6];  // zeta = b0 + b1 xi + b2 eta + b3 xi^2 + b4 xi eta + b5 eta^2
  double lo[3], hi[3], cx[3], ce[3];
  double t1[3], t2[3], n[3];
  double inv_dce[3];  // 1 / (ce_j - ce_k) for the axis pairs (0,1), (0,2), (1,2); 0 if parallel
  int has;            // bit k: n_k != 0
};

__device__ inline bool has_axis(const Local& L, int k) { return (L.has >> k) & 1; }

__device__ inline Local make_local(const double n[3], const double a[6], double h) {
  Local L;
  const double sg = copysign(1.0, n[2]);
  const double fa = -1.0 / (sg + n[2]);
  const double fb = n[0] * n[1] * fa;
  L.t1[0] = 1.0 + sg * n[0] * n[0] * fa;
  L.t1[1] = sg * fb;
  L.t1[2] = -sg * n[0];
  L.t2[0] = fb;
  L.t2[1] = sg + n[1] * n[1] * fa;
  L.t2[2] = -n[1];
  L.b[0] = a[0] / h;
  L.b[1] = a[1];
  L.b[2] = a[2];
  L.b[3] = a[3] * h;
  L.b[4] = a[4] * h;
  L.b[5] = a[5] * h;
  L.has = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L.n[k] = n[k];
    // face x_k = w: xi t1_k + eta t2_k + zeta n_k = w
    const bool hk = n[k] != 0.0;
    L.has |= hk ? 1 << k : 0;
    const double inv = hk ? 1.0 / n[k] : 0.0;
    L.cx[k] = -L.t1[k] * inv;
    L.ce[k] = -L.t2[k] * inv;
    L.lo[k] = -0.5 * fabs(inv);
    L.hi[k] = 0.5 * fabs(inv);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = j + 1; k < 3; ++k) {
      const double d = L.ce[j] - L.ce[k];
      L.inv_dce[j + k - 1] = (has_axis(L, j) && has_axis(L, k) && d != 0.0) ? 1.0 / d : 0.0;
    }
  return L;
}

// The same value in every lane, moved to scalar registers: the per-cell
// state is computed by every lane of the wavefront alike.
__device__ inline double uniform(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ inline Local uniform(const Local& L) {
  Local U;
#pragma unroll
  for (int k = 0; k < 6; ++k) U.b[k] = uniform(L.b[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    U.lo[k] = uniform(L.lo[k]);
    U.hi[k] = uniform(L.hi[k]);
    U.cx[k] = uniform(L.cx[k]);
    U.ce[k] = uniform(L.ce[k]);
    U.t1[k] = uniform(L.t1[k]);
    U.t2[k] = uniform(L.t2[k]);
    U.n[k] = uniform(L.n[k]);
    U.inv_dce[k] = uniform(L.inv_dce[k]);
  }
  U.has = __builtin_amdgcn_readfirstlane(L.has);
  return U;
}

// Real roots of qa t^2 + qb t + qc (linear when qa == 0); absent roots NaN.
__device__ inline void roots2(double qa, double qb, double qc, double& r0, double& r1) {
  r0 = NAN;
  r1 = NAN;
  if (qa == 0.0) {
    if (qb != 0.0) r0 = -qc / qb;
    return;
  }
  const double d = qb * qb - 4.0 * qa * qc;
  if (d < 0.0) return;
  const double q = -0.5 * (qb + copysign(sqrt(d), qb));
  r0 = q / qa;
  if (q != 0.0) r1 = qc / q;
}

__device__ inline void cswap(double& a, double& b) {
  const double lo = fmin(a, b), hi = fmax(a, b);
  a = lo;
  b = hi;
}

// The eta integrals at one xi: out[0] = G(xi), the exact integral of
// clamp(P - zeta_lo, 0, zeta_hi - zeta_lo); with kSurf, over the eta where
// the surface point lies in the cube, out[1] = int W, out[2] = int kappa W
// (Gauss, smooth between the breakpoints) and out[3..5] = int (-P_xi, -P_eta,
// 1) (exact), W = sqrt(1 + P_xi^2 + P_eta^2) and kappa = 2H.
template <bool kSurf>
__device__ void eta_integrals(const Local& L, const Nodes& N, double xi, double out[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) out[q] = 0.0;
  double emin = -1.0, emax = 1.0;  // |eta| <= sqrt(3)/2 inside the cube
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (has_axis(L, k)) continue;
    // n_k == 0: the slab -1/2 <= t1_k xi + t2_k eta <= 1/2 bounds eta (or xi)
    if (L.t2[k] == 0.0) {
      if (fabs(L.t1[k] * xi) > 0.5) return;
    } else {
      const double r0 = (-0.5 - L.t1[k] * xi) / L.t2[k], r1 = (0.5 - L.t1[k] * xi) / L.t2[k];
      emin = fmax(emin, fmin(r0, r1));
      emax = fmin(emax, fmax(r0, r1));
    }
  }
  if (!(emax > emin)) return;
  // the face planes at this xi: zeta = a + ce eta
  double la[3], ha[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double base = L.cx[k] * xi;
    la[k] = L.lo[k] + base;
    ha[k] = L.hi[k] + base;
  }
  const double q2 = L.b[5], q1 = L.b[2] + L.b[4] * xi, q0 = L.b[0] + (L.b[1] + L.b[3] * xi) * xi;
  // breakpoints, each clamped into [emin, emax]; absent ones (NaN) go to emax
  double s[kEta];
  auto clampe = [&](double v) { return (v >= emin && v <= emax) ? v : (v < emin ? emin : emax); };
  // slots 0..11: where the faces of two different axes cross
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = j + 1; k < 3; ++k) {
      const double inv = L.inv_dce[j + k - 1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double aj = (u & 1) ? ha[j] : la[j], ak = (u & 2) ? ha[k] : la[k];
        s[4 * (j + k - 1) + u] = clampe(inv != 0.0 ? (ak - aj) * inv : NAN);
      }
    }
  // slots 12..23: where the paraboloid meets a face
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      double r0 = NAN, r1 = NAN;
      if (has_axis(L, k)) roots2(q2, q1 - L.ce[k], q0 - (u ? ha[k] : la[k]), r0, r1);
      s[12 + 4 * k + 2 * u] = clampe(r0);
      s[13 + 4 * k + 2 * u] = clampe(r1);
    }
  // Batcher's odd-even merge sort network, ascending
#pragma unroll
  for (int p = 1; p < kEta; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < kEta; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i)
          if (i + j + k < kEta && (i + j) / (2 * p) == (i + j + k) / (2 * p)) cswap(s[i + j], s[i + j + k]);
  // runs of adjacent eta intervals where the surface lies in the cube.  There
  // are at most four: for convex P, {P < zeta_hi} is one interval and
  // {P > zeta_lo} leaves out at most three (one per lower face); for concave
  // P the same with the roles exchanged.
  constexpr int kRuns = 4;
  double ra[kRuns], rc[kRuns], rlast = 0.0;
  int nrun = 0;
#pragma unroll
  for (int k = 0; k < kRuns; ++k) {
    ra[k] = 0.0;
    rc[k] = -1.0;
  }
#pragma unroll
  for (int i = 0; i <= kEta; ++i) {
    const double a = i == 0 ? emin : s[i - 1], c = i == kEta ? emax : s[i];
    if (!(c > a)) continue;
    const double m = 0.5 * (a + c), r = 0.5 * (c - a);
    // the active lower and upper faces are the highest and lowest at the
    // midpoint; on [a, c] the same ones stay active and P stays on one side
    double zl = -INFINITY, zh = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (!has_axis(L, k)) continue;
      zl = fmax(zl, la[k] + L.ce[k] * m);
      zh = fmin(zh, ha[k] + L.ce[k] * m);
    }
    if (!(zl < zh)) continue;
    const double pm = (q2 * m + q1) * m + q0;
    if (!(pm > zl)) continue;
    // over [m - r, m + r]: the integral of a polynomial f is 2r (f(m) + f2 r^2 / 3)
    if (pm >= zh) {
      out[0] += 2.0 * r * (zh - zl);
      continue;
    }
    out[0] += 2.0 * r * ((pm - zl) + q2 * r * r * (1.0 / 3.0));
    if (kSurf) {
      // the surface lies inside the cube on [a, c]: the normal integral is
      // exact here; the interval joins the current run of such intervals
      const double pxm = L.b[1] + 2.0 * L.b[3] * xi + L.b[4] * m;
      const double pem = L.b[2] + L.b[4] * xi + 2.0 * L.b[5] * m;
      out[3] -= 2.0 * r * pxm;
      out[4] -= 2.0 * r * pem;
      out[5] += 2.0 * r;
      const bool extend = nrun > 0 && rlast == a;
      if (!extend && nrun == kRuns) {
        // a fifth run (not possible in exact arithmetic): reported, not
        // folded into a neighbouring run -- the cell's curvature and normal
        // become NaN
        out[1] = NAN;
        out[5] = NAN;
      }
      const int slot = extend ? nrun - 1 : min(nrun, kRuns - 1);
#pragma unroll
      for (int k = 0; k < kRuns; ++k) {
        if (k != slot) continue;
        if (!extend && nrun < kRuns) ra[k] = a;
        rc[k] = c;
      }
      if (!extend) nrun = min(nrun + 1, kRuns);
      rlast = c;
    }
  }
  if (kSurf) {
    // area and curvature over each run: the integrand (W, kappa W) does not
    // depend on the faces, so it is smooth across the breakpoints inside a run
#pragma unroll
    for (int run = 0; run < kRuns; ++run) {
      const double a = ra[run], c = rc[run];
      if (!(c > a)) continue;
      double sa = 0.0, sk = 0.0;
#pragma unroll
      for (int q = 0; q < kS; ++q) {
        const double eta = a + (c - a) * N.sx(q);
        const double px = L.b[1] + 2.0 * L.b[3] * xi + L.b[4] * eta;
        const double pe = L.b[2] + L.b[4] * xi + 2.0 * L.b[5] * eta;
        const double w2 = 1.0 + px * px + pe * pe;
        sa += N.sw(q) * sqrt(w2);
        sk -= N.sw(q) * ((1.0 + pe * pe) * 2.0 * L.b[3] - 2.0 * px * pe * L.b[4] + (1.0 + px * px) * 2.0 * L.b[5]) / w2;
      }
      out[1] += (c - a) * sa;
      out[2] += (c - a) * sk;
    }
  }
}

// xi of the points where the curve P = zeta_face of face plane (c0, cx, ce)
// meets the line eta = al + be xi.
__device__ inline void conic_line(const Local& L, double c0, double cx, double ce, double al, double be, double& r0,
                                  double& r1) {
  const double A = L.b[3], B = L.b[4], C = L.b[5];
  const double D = L.b[1] - cx, E = L.b[2] - ce, F = L.b[0] - c0;
  roots2(A + B * be + C * be * be, B * al + 2.0 * C * al * be + D + E * be, C * al * al + E * al + F, r0, r1);
}

// a[k] for a per-lane k, as selects (indexing the per-cell arrays with a
// lane-dependent index would move them to scratch memory)
__device__ inline double pick3(double a0, double a1, double a2, int k) { return k == 0 ? a0 : (k == 1 ? a1 : a2); }
#define PICK3(arr, k) pick3((arr)[0], (arr)[1], (arr)[2], (k))

// Coordinate w of face lo (hi) of axis k: the face the lower (upper) plane lies in.
__device__ inline double face_w(const Local& L, int k, bool upper) {
  return (PICK3(L.n, k) > 0.0) == upper ? 0.5 : -0.5;
}

// Event e of the xi breakpoints, at most two values (NaN when absent):
//   e < 8: projected corner e;
//   8 <= e < 20: edge (j, k, u) (axis pair j < k, u selects the faces): where
//     the paraboloid crosses that cube edge, kept only on the edge segment;
//   20 <= e < 26: face plane (k, upper) = (e - 20) % 3, (e - 20) / 3: where the
//     curve P = plane has a tangent along eta, kept only inside that face.
__device__ inline void xi_event(const Local& L, int e, double& v0, double& v1) {
  v0 = NAN;
  v1 = NAN;
  if (e < 8) {
    const double x = (e & 1) ? 0.5 : -0.5, y = (e & 2) ? 0.5 : -0.5, z = (e & 4) ? 0.5 : -0.5;
    v0 = L.t1[0] * x + L.t1[1] * y + L.t1[2] * z;
    return;
  }
  if (e < 20) {
    const int q = e - 8, pair = q / 4, u = q % 4;
    const int j = pair == 2 ? 1 : 0, k = pair == 0 ? 1 : 2, i = 3 - j - k;
    const bool uj = u & 1, uk = (u & 2) != 0;
    const double wj = face_w(L, j, uj), wk = face_w(L, k, uk);
    const bool hj = has_axis(L, j), hk = has_axis(L, k);
    if (hj && hk) {
      const double inv = PICK3(L.inv_dce, pair);
      if (inv == 0.0) return;  // the edge projects onto xi = const: its ends are corners
      const double cj = uj ? PICK3(L.hi, j) : PICK3(L.lo, j), ck = uk ? PICK3(L.hi, k) : PICK3(L.lo, k);
      // the edge line: c_j + cx_j xi + ce_j eta = c_k + cx_k xi + ce_k eta
      const double al = (ck - cj) * inv, be = (PICK3(L.cx, k) - PICK3(L.cx, j)) * inv;
      // the crossing lies on both faces' curves; the face of the axis with
      // the larger |n| has the well-conditioned one (a face almost parallel
      // to n has coefficients of order 1/n_k)
      if (fabs(PICK3(L.n, j)) >= fabs(PICK3(L.n, k)))
        conic_line(L, cj, PICK3(L.cx, j), PICK3(L.ce, j), al, be, v0, v1);
      else
        conic_line(L, ck, PICK3(L.cx, k), PICK3(L.ce, k), al, be, v0, v1);
    } else if (hj || hk) {
      // one face is a slab boundary t1_m xi + t2_m eta = w_m of an axis with n_m == 0
      const int f = hj ? j : k, m = hj ? k : j;
      const double wm = hj ? wk : wj;
      if (PICK3(L.t2, m) == 0.0) return;  // a line xi = const: its ends are corners
      const double cf = (hj ? uj : uk) ? PICK3(L.hi, f) : PICK3(L.lo, f);
      conic_line(L, cf, PICK3(L.cx, f), PICK3(L.ce, f), wm / PICK3(L.t2, m), -PICK3(L.t1, m) / PICK3(L.t2, m), v0, v1);
    } else {
      return;  // an edge along n: a point in projection, a corner
    }
    // keep the crossings on the edge segment x_j = wj, x_k = wk, |x_i| <= 1/2
    const double c = PICK3(L.t1, j) * wj + PICK3(L.t1, k) * wk, d = 0.5 * fabs(PICK3(L.t1, i));
    if (!(v0 >= c - d && v0 <= c + d)) v0 = NAN;
    if (!(v1 >= c - d && v1 <= c + d)) v1 = NAN;
    return;
  }
  const int f = (e - 20) % 3;
  const bool up = (e - 20) >= 3;
  if (!has_axis(L, f)) return;
  const double c0 = up ? PICK3(L.hi, f) : PICK3(L.lo, f);
  const double A = L.b[3], B = L.b[4], C = L.b[5];
  const double D = L.b[1] - PICK3(L.cx, f), E = L.b[2] - PICK3(L.ce, f), F = L.b[0] - c0;
  roots2(B * B - 4.0 * C * A, 2.0 * B * E - 4.0 * C * D, E * E - 4.0 * C * F, v0, v1);
  if (C == 0.0) return;  // no tangent along eta: keep the candidates as they are
  // keep a tangency only inside its face: the other two coordinates within 1/2
  auto inside = [&](double xi) {
    const double eta = -(B * xi + E) / (2.0 * C);
    const double zeta = c0 + PICK3(L.cx, f) * xi + PICK3(L.ce, f) * eta;
    bool in = true;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m == f) continue;
      const double x = PICK3(L.t1, m) * xi + PICK3(L.t2, m) * eta + PICK3(L.n, m) * zeta;
      in = in && fabs(x) <= 0.5 + 1e-12;
    }
    return in;
  };
  if (!isnan(v0) && !inside(v0)) v0 = NAN;
  if (!isnan(v1) && !inside(v1)) v1 = NAN;
}

template <bool kSurf>
__device__ void paraboloid_cells(const double* frame_n, const double* coeff, double h, const int32_t* counters,
                                 int32_t cell_cap, Nodes N, double* alpha_out, double* kappa_out, double* normal_out) {
  __shared__ double ev[kSlots];
  __shared__ double xs[kSlots];
  const int lane = threadIdx.x;
  const int32_t nif = min(counters[C_NIF], cell_cap);
  const int64_t cs = cell_cap;
  for (int32_t c = blockIdx.x; c < nif; c += gridDim.x) {
    const double n[3] = {frame_n[c], frame_n[cs + c], frame_n[2 * cs + c]};
    double a[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) a[r] = coeff[r * cs + c];
    bool finite = isfinite(n[0]) && isfinite(n[1]) && isfinite(n[2]);
#pragma unroll
    for (int r = 0; r < 6; ++r) finite = finite && isfinite(a[r]);
    if (!finite) {  // a failed fit: nothing to integrate (the same for every lane)
      if (lane == 0) {
        alpha_out[c] = NAN;
        if (kSurf && kappa_out) kappa_out[c] = NAN;
        if (kSurf && normal_out)
          for (int d = 0; d < 3; ++d) normal_out[d * cs + c] = NAN;
      }
      continue;
    }
    const Local L = uniform(make_local(n, a, h));
    double xa = INFINITY, xb = -INFINITY;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      double v, w;
      xi_event(L, e, v, w);
      xa = fmin(xa, v);
      xb = fmax(xb, v);
    }
    if (lane < kEvents) {
      double v0, v1;
      xi_event(L, lane, v0, v1);
      ev[2 * lane] = (v0 > xa && v0 < xb) ? v0 : INFINITY;
      ev[2 * lane + 1] = (v1 > xa && v1 < xb) ? v1 : INFINITY;
    } else if (lane < kEvents + 2) {
      ev[2 * kEvents + (lane - kEvents)] = lane == kEvents ? xa : xb;
    } else if (2 * kEvents + (lane - kEvents) < kSlots) {
      ev[2 * kEvents + (lane - kEvents)] = INFINITY;
    }
    __syncthreads();
    // rank sort of the finite entries (ties by slot)
    int nf = 0;
    if (lane < kSlots) {
      const double v = ev[lane];
      int r = 0;
      for (int j = 0; j < kSlots; ++j) {
        const double u = ev[j];
        r += (u < v || (u == v && j < lane)) ? 1 : 0;
      }
      if (v < INFINITY) xs[r] = v;
    }
    for (int j = 0; j < kSlots; ++j) nf += ev[j] < INFINITY ? 1 : 0;
    __syncthreads();
    constexpr int kOut = kSurf ? 6 : 1;
    double acc[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) acc[q] = 0.0;
    constexpr int kQ = kSurf ? kQS : kQV;
    const int nodes = (nf - 1) * kQ;
    for (int q = lane; q < nodes; q += kT) {
      const int i = q / kQ, k = q % kQ;
      const double u0 = xs[i], u1 = xs[i + 1];
      if (!(u1 > u0)) continue;
      double g[6];
      eta_integrals<kSurf>(L, N, u0 + (u1 - u0) * N.tau(k), g);
      const double wq = (u1 - u0) * N.omega(k);
#pragma unroll
      for (int o = 0; o < kOut; ++o) acc[o] += wq * g[o];
    }
#pragma unroll
    for (int o = 0; o < kOut; ++o)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[o] += __shfl_xor(acc[o], off, kT);
    if (lane == 0) {
      alpha_out[c] = acc[0];
      if (kSurf) {
        // area acc[1], int kappa W acc[2] (cell units: kappa h), normal integral acc[3..5] in the frame
        if (kappa_out) kappa_out[c] = acc[1] > 0.0 ? acc[2] / acc[1] / h : NAN;
        if (normal_out) {
          double w[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) w[d] = acc[3] * L.t1[d] + acc[4] * L.t2[d] + acc[5] * L.n[d];
          const double nl = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
#pragma unroll
          for (int d = 0; d < 3; ++d) normal_out[d * cs + c] = nl > 0.0 ? w[d] / nl : NAN;
        }
      }
    }
    __syncthreads();
  }
}

// The volume alone fits three wavefronts per SIMD (168 registers, a few
// spilled: 412 -> 373 us on the 128^3 sphere); with the surface integrals
// the spills cost more than the occupancy gains, so that kernel keeps two.
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(3))) void k_paraboloid_alpha(
    const double* frame_n, const double* coeff, double h, const int32_t* counters, int32_t cell_cap, Nodes N,
    double* alpha_out) {
  paraboloid_cells<false>(frame_n, coeff, h, counters, cell_cap, N, alpha_out, nullptr, nullptr);
}

__global__ __launch_bounds__(kT) void k_paraboloid_surface(const double* frame_n, const double* coeff, double h,
                                                           const int32_t* counters, int32_t cell_cap, Nodes N,
                                                           double* alpha_out, double* kappa_out, double* normal_out) {
  paraboloid_cells<true>(frame_n, coeff, h, counters, cell_cap, N, alpha_out, kappa_out, normal_out);
}

// n-point Gauss-Legendre rule on [-1, 1] by Newton's method on the Legendre
// recurrence, mapped through theta = (x + 1) pi / 2, u = (1 - cos theta) / 2:
// tau[n], omega[n].
void xi_rule(int n, double* tau, double* omega) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double x = cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    const double w = 2.0 / ((1.0 - x * x) * dp * dp);
    const double th = (x + 1.0) * pi / 2.0;
    tau[i] = 0.5 * (1.0 - cos(th));
    omega[i] = w * (pi / 2.0) * sin(th) * 0.5;
  }
}

// The node table: both xi rules, then the eta rule (kS-point Gauss-Legendre
// on [0, 1]).
void make_nodes(double* out) {
  xi_rule(kQV, out, out + kQV);
  xi_rule(kQS, out + 2 * kQV, out + 2 * kQV + kQS);
  double* sx = out + kEtaOff;
  double* sw = out + kEtaOff + kS;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < kS; ++i) {
    double x = cos(pi * (i + 0.75) / (kS + 0.5)), dp = 1.0, p0 = 1.0, p1 = x;
    for (int it = 0; it < 100; ++it) {
      p0 = 1.0;
      p1 = x;
      for (int k = 2; k <= kS; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = kS * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    p0 = 1.0;
    p1 = x;
    for (int k = 2; k <= kS; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = kS * (x * p1 - p0) / (x * x - 1.0);
    sx[i] = 0.5 * (x + 1.0);
    sw[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // half the weight on [-1, 1]
  }
}

}  // namespace

void paraboloid_nodes(double* out) { make_nodes(out); }

hipError_t launch_paraboloid_cell(const ftc_cells* ws, const double* coeff, double* alpha_out, double* kappa_out,
                                  double* normal_out, hipStream_t s) {
  const Nodes NV{ws->quad_nodes, kQV}, NS{ws->quad_nodes, kQS};
  const dim3 grid(grid_blocks(ws->cell_cap, 1, 65535));
  if (kappa_out || normal_out)
    hipLaunchKernelGGL(k_paraboloid_surface, grid, dim3(kT), 0, s, ws->frame_n, coeff, ws->grid.h, ws->counters,
                       ws->cell_cap, NS, alpha_out, kappa_out, normal_out);
  else
    hipLaunchKernelGGL(k_paraboloid_alpha, grid, dim3(kT), 0, s, ws->frame_n, coeff, ws->grid.h, ws->counters,
                       ws->cell_cap, NV, alpha_out);
  return hipGetLastError();
}

}  // namespace ftc
