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
// 16-node Gauss-Legendre rule in theta with xi = u0 + (u1 - u0)(1 - cos
// theta)/2, which absorbs the square-root behaviour of G at tangencies.
// One wavefront per cell: its lanes compute the events, rank-sort them in
// LDS and share the quadrature nodes.
#include <math.h>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 64;         // one wavefront per workgroup and per cell
constexpr int kQ = 16;         // Gauss nodes per xi interval
constexpr int kEvents = 38;    // 8 corners + 6 planes x (1 tangency + 4 edges)
constexpr int kSlots = 80;     // 2 values per event, the two ends, padding
constexpr int kEta = 32;       // eta breakpoints per G evaluation (26 used)

struct Nodes {
  double tau[kQ], omega[kQ];  // xi = u0 + (u1 - u0) tau, weight (u1 - u0) omega
};

// zeta = c0 + cx xi + ce eta: one face plane of the cube in the local frame
struct Line {
  double c0, cx, ce;
};

// The cell's paraboloid and cube in its local frame, cell units.
struct Local {
  double b[6];        // zeta = b0 + b1 xi + b2 eta + b3 xi^2 + b4 xi eta + b5 eta^2
  Line lo[3], hi[3];  // lower / upper face plane of axis k (where n_k != 0)
  bool has[3];        // n_k != 0
  double s1[3], s2[3];  // axis k with n_k == 0: the slab -1/2 <= s1 xi + s2 eta <= 1/2
  double t1[3];
};

__device__ inline Local make_local(const double n[3], const double a[6], double h) {
  Local L;
  const double sg = copysign(1.0, n[2]);
  const double fa = -1.0 / (sg + n[2]);
  const double fb = n[0] * n[1] * fa;
  const double t1[3] = {1.0 + sg * n[0] * n[0] * fa, sg * fb, -sg * n[0]};
  const double t2[3] = {fb, sg + n[1] * n[1] * fa, -n[1]};
  L.b[0] = a[0] / h;
  L.b[1] = a[1];
  L.b[2] = a[2];
  L.b[3] = a[3] * h;
  L.b[4] = a[4] * h;
  L.b[5] = a[5] * h;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L.t1[k] = t1[k];
    L.has[k] = n[k] != 0.0;
    L.s1[k] = t1[k];
    L.s2[k] = t2[k];
    // face x_k = -+1/2: xi t1_k + eta t2_k + zeta n_k = w
    const double inv = L.has[k] ? 1.0 / n[k] : 0.0;
    const Line m = {-0.5 * inv, -t1[k] * inv, -t2[k] * inv};
    const Line p = {0.5 * inv, -t1[k] * inv, -t2[k] * inv};
    L.lo[k] = n[k] > 0.0 ? m : p;
    L.hi[k] = n[k] > 0.0 ? p : m;
  }
  return L;
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

// G(xi): the exact eta integral of clamp(P - zeta_lo, 0, zeta_hi - zeta_lo).
__device__ double eta_integral(const Local& L, double xi) {
  double emin = -1.0, emax = 1.0;  // |eta| <= sqrt(3)/2 inside the cube
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (L.has[k]) continue;
    if (L.s2[k] == 0.0) {
      if (fabs(L.s1[k] * xi) > 0.5) return 0.0;
    } else {
      const double r0 = (-0.5 - L.s1[k] * xi) / L.s2[k], r1 = (0.5 - L.s1[k] * xi) / L.s2[k];
      emin = fmax(emin, fmin(r0, r1));
      emax = fmin(emax, fmax(r0, r1));
    }
  }
  if (!(emax > emin)) return 0.0;
  double la[3], le[3], ha[3], he[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    la[k] = L.lo[k].c0 + L.lo[k].cx * xi;
    le[k] = L.lo[k].ce;
    ha[k] = L.hi[k].c0 + L.hi[k].cx * xi;
    he[k] = L.hi[k].ce;
  }
  const double q2 = L.b[5], q1 = L.b[2] + L.b[4] * xi, q0 = L.b[0] + (L.b[1] + L.b[3] * xi) * xi;
  // candidate breakpoints, each clamped into [emin, emax]; absent ones (NaN)
  // go to emax, where they bound empty intervals
  double s[kEta];
  auto clampe = [&](double v) { return (v >= emin && v <= emax) ? v : (v < emin ? emin : emax); };
#pragma unroll
  for (int i = 0; i < kEta; ++i) s[i] = emax;
  // slots 0..11: crossings of the planes of two different axes
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = j + 1; k < 3; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double aj = (u & 1) ? ha[j] : la[j], ej = (u & 1) ? he[j] : le[j];
        const double ak = (u & 2) ? ha[k] : la[k], ek = (u & 2) ? he[k] : le[k];
        const double v = (L.has[j] && L.has[k] && ej != ek) ? (ak - aj) / (ej - ek) : NAN;
        s[4 * (j + k - 1) + u] = clampe(v);
      }
  // slots 12..23: roots of P = plane; slot 24: emin
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      double r0 = NAN, r1 = NAN;
      if (L.has[k]) roots2(q2, q1 - (u ? he[k] : le[k]), q0 - (u ? ha[k] : la[k]), r0, r1);
      s[12 + 4 * k + 2 * u] = clampe(r0);
      s[13 + 4 * k + 2 * u] = clampe(r1);
    }
  s[24] = emin;
  // bitonic sort of the 32 values, ascending
#pragma unroll
  for (int size = 2; size <= kEta; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
      for (int i = 0; i < kEta; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          if ((i & size) == 0)
            cswap(s[i], s[j]);
          else
            cswap(s[j], s[i]);
        }
      }
  double g = 0.0;
#pragma unroll
  for (int i = 0; i + 1 < kEta; ++i) {
    const double a = s[i], c = s[i + 1];
    if (!(c > a)) continue;
    const double m = 0.5 * (a + c), r = 0.5 * (c - a);
    // the active lower and upper faces are the highest and lowest at the
    // midpoint; on [a, c] the same ones stay active and P stays on one side
    double zl = -INFINITY, zh = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (!L.has[k]) continue;
      zl = fmax(zl, la[k] + le[k] * m);
      zh = fmin(zh, ha[k] + he[k] * m);
    }
    if (!(zl < zh)) continue;
    const double pm = (q2 * m + q1) * m + q0;
    if (!(pm > zl)) continue;
    // over [m - r, m + r]: the integral of a polynomial f is 2r (f(m) + f2 r^2 / 3)
    if (pm >= zh)
      g += 2.0 * r * (zh - zl);
    else
      g += 2.0 * r * ((pm - zl) + q2 * r * r * (1.0 / 3.0));
  }
  return g;
}

// The conic P = plane p meets the line eta = al + be xi: its xi.
__device__ inline void conic_line(const Local& L, const Line& p, double al, double be, double& r0, double& r1) {
  const double A = L.b[3], B = L.b[4], C = L.b[5];
  const double D = L.b[1] - p.cx, E = L.b[2] - p.ce, F = L.b[0] - p.c0;
  roots2(A + B * be + C * be * be, B * al + 2.0 * C * al * be + D + E * be, C * al * al + E * al + F, r0, r1);
}

// Event `e` of the xi breakpoints: e < 8 a projected corner; otherwise plane
// p = (e - 8) / 5 (lo_0, lo_1, lo_2, hi_0, hi_1, hi_2) and kind (e - 8) % 5:
// 0 the tangency of its conic along eta, 1..4 its conic against the four
// face lines of the two other axes (their planes' edge lines, or the slab
// boundaries where n_k == 0).
__device__ inline void xi_event(const Local& L, int e, double& v0, double& v1) {
  v0 = NAN;
  v1 = NAN;
  if (e < 8) {
    const double x = (e & 1) ? 0.5 : -0.5, y = (e & 2) ? 0.5 : -0.5, z = (e & 4) ? 0.5 : -0.5;
    v0 = L.t1[0] * x + L.t1[1] * y + L.t1[2] * z;
    return;
  }
  const int q = e - 8, pi = q / 5, kind = q % 5, kp = pi % 3;
  if (!L.has[kp]) return;
  const Line p = pi < 3 ? L.lo[kp] : L.hi[kp];
  if (kind == 0) {
    const double A = L.b[3], B = L.b[4], C = L.b[5];
    const double D = L.b[1] - p.cx, E = L.b[2] - p.ce, F = L.b[0] - p.c0;
    roots2(B * B - 4.0 * C * A, 2.0 * B * E - 4.0 * C * D, E * E - 4.0 * C * F, v0, v1);
    return;
  }
  const int ko = (kp + 1 + (kind - 1) / 2) % 3, side = (kind - 1) & 1;
  if (L.has[ko]) {
    const Line o = side ? L.hi[ko] : L.lo[ko];
    const double dce = p.ce - o.ce;
    if (dce == 0.0) return;  // the edge line is xi = const: its ends are corners
    conic_line(L, p, -(p.c0 - o.c0) / dce, -(p.cx - o.cx) / dce, v0, v1);
  } else {
    if (L.s2[ko] == 0.0) return;  // the slab bounds xi alone: corners
    const double w = side ? 0.5 : -0.5;
    conic_line(L, p, w / L.s2[ko], -L.s1[ko] / L.s2[ko], v0, v1);
  }
}

__global__ __launch_bounds__(kT) void k_paraboloid_alpha(const double* fit, const double* coeff, double h,
                                                         const int32_t* counters, int32_t cell_cap, Nodes N,
                                                         double* alpha_out) {
  __shared__ double ev[kSlots];
  __shared__ double xs[kSlots];
  const int lane = threadIdx.x;
  const int32_t nif = min(counters[C_NIF], cell_cap);
  const int64_t cs = cell_cap;
  for (int32_t c = blockIdx.x; c < nif; c += gridDim.x) {
    const double n[3] = {fit[27 * cs + c], fit[28 * cs + c], fit[29 * cs + c]};
    double a[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) a[r] = coeff[r * cs + c];
    const Local L = make_local(n, a, h);
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
    } else if (lane < kEvents + 4) {
      ev[2 * kEvents + (lane - kEvents)] = INFINITY;
    }
    __syncthreads();
    // rank sort of the finite entries (ties by slot)
    int nf = 0;
    for (int i = lane; i < kSlots; i += kT) {
      const double v = ev[i];
      int r = 0;
      for (int j = 0; j < kSlots; ++j) {
        const double u = ev[j];
        r += (u < v || (u == v && j < i)) ? 1 : 0;
      }
      if (v < INFINITY) xs[r] = v;
    }
    for (int j = 0; j < kSlots; ++j) nf += ev[j] < INFINITY ? 1 : 0;
    __syncthreads();
    double acc = 0.0;
    const int nodes = (nf - 1) * kQ;
    for (int q = lane; q < nodes; q += kT) {
      const int i = q / kQ, k = q % kQ;
      const double u0 = xs[i], u1 = xs[i + 1];
      if (u1 > u0) acc += (u1 - u0) * N.omega[k] * eta_integral(L, u0 + (u1 - u0) * N.tau[k]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kT);
    if (lane == 0) alpha_out[c] = acc;
    __syncthreads();
  }
}

// 16-point Gauss-Legendre rule on [-1, 1] by Newton's method on the Legendre
// recurrence, mapped through theta = (x + 1) pi / 2, u = (1 - cos theta) / 2.
Nodes make_nodes() {
  Nodes N;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < kQ; ++i) {
    double x = cos(pi * (i + 0.75) / (kQ + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= kQ; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = kQ * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= kQ; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = kQ * (x * p1 - p0) / (x * x - 1.0);
    const double w = 2.0 / ((1.0 - x * x) * dp * dp);
    const double th = (x + 1.0) * pi / 2.0;
    N.tau[i] = 0.5 * (1.0 - cos(th));
    N.omega[i] = w * (pi / 2.0) * sin(th) * 0.5;
  }
  return N;
}

}  // namespace

hipError_t launch_paraboloid_alpha(const ftc_cells* ws, const double* coeff, double* alpha_out, hipStream_t s) {
  static const Nodes N = make_nodes();
  hipLaunchKernelGGL(k_paraboloid_alpha, dim3(grid_blocks(ws->cell_cap, 1, 65535)), dim3(kT), 0, s, ws->fit, coeff,
                     ws->grid.h, ws->counters, ws->cell_cap, N, alpha_out);
  return hipGetLastError();
}

}  // namespace ftc
