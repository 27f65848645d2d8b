// ppic.hip -- PPIC curvature by the volume fit (paper section 3.2).
//
// Pre-passes:
//   * vertex -> incident triangles (CSR, ascending triangle id);
//   * closest vertex of every interfacial cell, vertex-centric: every vertex
//     offers its squared distance to the centres of the 27 cells around its
//     own cell (64-bit atomicMin on the IEEE bits, which order like the
//     values for non-negative doubles), then the vertices that attain the
//     minimum offer their index (atomicMin: lowest index on ties).  A cell
//     whose best distance is not below 1.5 h (the distance to any cell
//     outside the 27) falls back to a search over all vertices.
//
// Main kernel: 16 lanes per interfacial cell, 4 cells per 64-lane wavefront
// (one wavefront per workgroup), per-cell state in LDS.
//   1. normal of the closest vertex (area-weighted, summed in ascending
//      triangle order) and a right-handed tangent frame (Duff et al., JCGT
//      2017);
//   2. ring neighbourhood: V_0 = {v*}; T_r = triangles with a corner in
//      V_{r-1}, each taken once, from the first of its corners (t0, t1, t2
//      order) that lies in V_{r-1}; V_r = V_{r-1} plus the new corners of
//      T_r in first-occurrence order.  Membership and first occurrence use an
//      open-addressing hash table per cell in LDS;
//   3. triangle-centre distances, the support radius grown by `grow` until
//      `n_min` triangles fall inside (or the ring is exhausted, or
//      `max_iter` adjustments), Wendland weights;
//   4. per lane: the triangles' projection into the frame (coordinates
//      divided by h for conditioning), the six moments by the edge-midpoint
//      rule (exact for quadratics), the integral of each triangle's plane,
//      and the weighted normal equations M a = b accumulated in registers;
//      butterfly reduction over the 16 lanes;
//   5. packed in-register Cholesky factorisation with one step of iterative
//      refinement, curvature kappa = 2H at the frame origin, interface normal.
// Every loop bound is uniform over the wavefront (maxima over its 4 cells),
// so LDS phases are separated by plain workgroup barriers.
#include <float.h>

#include <algorithm>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 4096;

constexpr int G = 16;        // lanes per cell
constexpr int NG = 64 / G;   // cells per wavefront
constexpr int kHS = 256;     // hash slots per cell
constexpr int kVC = 128;     // ring-vertex capacity
constexpr int kTC = 128;     // ring-triangle capacity
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

// ----------------------------------------------------------------- pre-passes
__global__ void k_clear_ppic(int32_t* vt_off, int64_t n1, int32_t* vt_cursor, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = g0; i < n1; i += stride) vt_off[i] = 0;
  for (int64_t i = g0; i < n2; i += stride) vt_cursor[i] = 0;
}

__global__ void k_vt_count(Mesh m, int32_t* vt_cnt) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nt || !tri_ok(m, t)) return;
  atomicAdd(&vt_cnt[m.t0[t]], 1);
  atomicAdd(&vt_cnt[m.t1[t]], 1);
  atomicAdd(&vt_cnt[m.t2[t]], 1);
}

__global__ void k_vt_scatter(Mesh m, const int32_t* vt_off, int32_t* vt_cursor, int32_t* vt_ids) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nt || !tri_ok(m, t)) return;
  const int32_t c[3] = {m.t0[t], m.t1[t], m.t2[t]};
#pragma unroll
  for (int r = 0; r < 3; ++r) vt_ids[vt_off[c[r]] + atomicAdd(&vt_cursor[c[r]], 1)] = t;
}

__global__ void k_vt_sort(int32_t nv, const int32_t* vt_off, int32_t* vt_ids) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int32_t s = vt_off[v], e = vt_off[v + 1];
  for (int32_t a = s + 1; a < e; ++a) {
    const int32_t x = vt_ids[a];
    int32_t b = a - 1;
    while (b >= s && vt_ids[b] > x) {
      vt_ids[b + 1] = vt_ids[b];
      --b;
    }
    vt_ids[b + 1] = x;
  }
}

__device__ inline int32_t cell_rank(const uint32_t* bitmap, const int32_t* word_off, int64_t lin) {
  const uint32_t w = bitmap[lin >> 5];
  if (!((w >> (lin & 31)) & 1u)) return -1;
  const uint32_t below = (lin & 31) ? (w & ((1u << (lin & 31)) - 1u)) : 0u;
  return word_off[lin >> 5] + __popc(below);
}

// Squared distance from (x, y, z) to the centre of cell (i, j, k).
__device__ inline double centre_d2(const Grid& g, int64_t i, int64_t j, int64_t k, double x, double y, double z) {
  const double dx = x - (g.x0 + ((double)i + 0.5) * g.h);
  const double dy = y - (g.y0 + ((double)j + 0.5) * g.h);
  const double dz = z - (g.z0 + ((double)k + 0.5) * g.h);
  return dx * dx + dy * dy + dz * dz;
}

__global__ void k_vstar_init(unsigned long long* best_d2, int32_t* best_v, int32_t cell_cap,
                             const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nif; c += gridDim.x * blockDim.x) {
    best_d2[c] = kInfBits;
    best_v[c] = INT_MAX;
  }
}

// PASS 0: minimum squared distance per cell; PASS 1: lowest vertex attaining it.
template <int PASS>
__global__ __launch_bounds__(kT) void k_vstar(Grid g, Mesh m, const uint32_t* bitmap, const int32_t* word_off,
                                              unsigned long long* best_d2, int32_t* best_v, int32_t cell_cap) {
  const int32_t v = blockIdx.x * kT + threadIdx.x;
  if (v >= m.nv) return;
  const double x = m.x[v], y = m.y[v], z = m.z[v];
  if (!in_margin(g, x, y, z)) return;  // latched as a domain error by the cell-list build
  const int64_t i = cell_index(x, g.x0, g.h), j = cell_index(y, g.y0, g.h), k = cell_index(z, g.z0, g.h);
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int64_t ii = i + di, jj = j + dj, kk = k + dk;  // inside the grid: the vertex is 2 cells in
        const int32_t ci = cell_rank(bitmap, word_off, ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk));
        if (ci < 0 || ci >= cell_cap) continue;
        const unsigned long long bits =
            (unsigned long long)__double_as_longlong(centre_d2(g, ii, jj, kk, x, y, z));
        if (PASS == 0) {
          atomicMin(&best_d2[ci], bits);
        } else if (bits == best_d2[ci]) {
          atomicMin(&best_v[ci], v);
        }
      }
}

// ----------------------------------------------------------------- main kernel
struct PPICArgs {
  Grid g;
  Mesh m;
  PPICParams prm;
  const int32_t* cell_ids;
  const int32_t* vt_off;
  const int32_t* vt_ids;
  const unsigned long long* best_d2;
  const int32_t* best_v;
  const int32_t* counters;
  int32_t cell_cap;
  double *kappa, *nx, *ny, *nz, *coeff;
  int32_t *status, *diag;
};

struct __align__(8) CellMem {
  double d2[kTC];
  int32_t hkey[kHS];
  int32_t hval[kHS];
  int32_t V[kVC];
  int32_t T[kTC];
};

__device__ inline int hslot(int32_t key) { return (int)(((uint32_t)key * 2654435761u) >> 24); }  // 256 slots

// Insert key (if absent) and return its slot.  The table never fills: it
// holds at most kVC + 1 < kHS keys.
__device__ inline int hinsert(CellMem& M, int32_t key) {
  int s = hslot(key);
  for (int p = 0; p < kHS; ++p) {
    const int32_t prev = atomicCAS(&M.hkey[s], -1, key);
    if (prev == -1 || prev == key) return s;
    s = (s + 1) & (kHS - 1);
  }
  return -1;
}

__device__ inline int hfind(CellMem& M, int32_t key) {
  int s = hslot(key);
  for (int p = 0; p < kHS; ++p) {
    const int32_t k = M.hkey[s];
    if (k == key) return s;
    if (k == -1) return -1;
    s = (s + 1) & (kHS - 1);
  }
  return -1;
}

// 16-bit ballot of this lane's group.
__device__ inline uint32_t gballot(bool p, int grp) { return (uint32_t)((__ballot(p) >> (G * grp)) & 0xFFFFull); }

__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline bool lex_less(double d, int32_t v, double bd, int32_t bv) {
  return d < bd || (d == bd && v < bv);
}

// packed index of entry (a, b), a <= b, of a symmetric 6x6 matrix
__host__ __device__ constexpr int P6(int a, int b) { return a * 6 - a * (a - 1) / 2 + (b - a); }

__global__ __launch_bounds__(64) void k_ppic(PPICArgs A) {
  __shared__ CellMem SM[NG];
  const Grid& g = A.g;
  const Mesh& m = A.m;
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  CellMem& M = SM[grp];
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  const double h = g.h;
  const int R = A.prm.rings;
  const double reach = 1.5 * h;
  const double reach2 = reach * reach * (1.0 - 1e-12);
  const unsigned long long reach_bits = (unsigned long long)__double_as_longlong(reach2);

  for (int32_t base = blockIdx.x * NG; base < nif; base += gridDim.x * NG) {
    const int32_t c = base + grp;
    const bool act = c < nif;
    const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
    const int32_t ci = cc3.i, cj = cc3.j, ck = cc3.k;
    const double xc[3] = {g.x0 + ((double)ci + 0.5) * h, g.y0 + ((double)cj + 0.5) * h,
                          g.z0 + ((double)ck + 0.5) * h};

    // ---- closest vertex: pre-pass result, else a search over all vertices
    int32_t vs = act ? A.best_v[c] : 0;
    const bool need = act && !(vs != INT_MAX && A.best_d2[c] < reach_bits);
    if (__any(need)) {
      double bd = DBL_MAX;
      int32_t bv = INT_MAX;
      if (need)
        for (int32_t v = gl; v < m.nv; v += G) {
          const double dx = m.x[v] - xc[0], dy = m.y[v] - xc[1], dz = m.z[v] - xc[2];
          const double d2 = dx * dx + dy * dy + dz * dz;
          if (lex_less(d2, v, bd, bv)) {
            bd = d2;
            bv = v;
          }
        }
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
    bool ok = act && vs >= 0 && vs < m.nv;

    // ---- vertex normal (every lane of the group, ascending triangle order) and frame
    double n0 = 0.0, n1 = 0.0, n2 = 1.0;
    int32_t deg0 = 0, vt0 = 0;
    if (ok) {
      n2 = 0.0;
      vt0 = A.vt_off[vs];
      deg0 = A.vt_off[vs + 1] - vt0;
      for (int32_t q = 0; q < deg0; ++q) {
        const Tri T = load_tri(m, A.vt_ids[vt0 + q]);
        const double ux = T.v[1][0] - T.v[0][0], uy = T.v[1][1] - T.v[0][1], uz = T.v[1][2] - T.v[0][2];
        const double wx = T.v[2][0] - T.v[0][0], wy = T.v[2][1] - T.v[0][1], wz = T.v[2][2] - T.v[0][2];
        n0 += uy * wz - uz * wy;
        n1 += uz * wx - ux * wz;
        n2 += ux * wy - uy * wx;
      }
      const double nl = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
      n0 /= nl;
      n1 /= nl;
      n2 /= nl;
    }
    const double sg = copysign(1.0, n2);
    const double fa = -1.0 / (sg + n2);
    const double fb = n0 * n1 * fa;
    const double t1x = 1.0 + sg * n0 * n0 * fa, t1y = sg * fb, t1z = -sg * n0;
    const double t2x = fb, t2y = sg + n1 * n1 * fa, t2z = -n1;

    // ---- ring neighbourhood
    for (int s = gl; s < kHS; s += G) {
      M.hkey[s] = -1;
      M.hval[s] = INT_MAX;
    }
    __syncthreads();
    if (ok && gl == 0) {
      const int s = hinsert(M, vs);
      M.hval[s] = -1;  // ring position 0, already in the ring
      M.V[0] = vs;
    }
    __syncthreads();
    int32_t nV = 1, nT = 0;
    bool overflow = false;
    for (int r = 1; r <= R; ++r) {
      // T_r
      nT = 0;
      if (r == 1) {
        const int rounds = wave_max_i(ok ? (deg0 + G - 1) / G : 0);
        for (int k = 0; k < rounds; ++k) {
          const int e = k * G + gl;
          const bool has = ok && e < deg0;
          const uint32_t bal = gballot(has, grp);
          if (has) {
            const int pos = nT + __popc(bal & ((1u << gl) - 1u));
            if (pos < kTC) M.T[pos] = A.vt_ids[vt0 + e];
          }
          nT += __popc(bal);
        }
      } else {
        const int nVc = min(nV, kVC);
        const int vrounds = wave_max_i(ok ? (nVc + G - 1) / G : 0);
        for (int k = 0; k < vrounds; ++k) {
          const int p = k * G + gl;
          const bool pv = ok && p < nVc;
          const int32_t u = pv ? M.V[p] : 0;
          const int32_t s0 = pv ? A.vt_off[u] : 0;
          const int32_t du = pv ? A.vt_off[u + 1] - s0 : 0;
          const int erounds = wave_max_i(du);
          for (int e = 0; e < erounds; ++e) {
            bool keep = false;
            int32_t t = 0;
            if (e < du) {
              t = A.vt_ids[s0 + e];
              const int32_t cc[3] = {m.t0[t], m.t1[t], m.t2[t]};
              int32_t first = -1;
#pragma unroll
              for (int q = 0; q < 3; ++q)
                if (first < 0 && hfind(M, cc[q]) >= 0) first = cc[q];
              keep = first == u;
            }
            const uint32_t bal = gballot(keep, grp);
            if (keep) {
              const int pos = nT + __popc(bal & ((1u << gl) - 1u));
              if (pos < kTC) M.T[pos] = t;
            }
            nT += __popc(bal);
          }
        }
      }
      if (nT > kTC) overflow = true;
      __syncthreads();
      if (r == R) break;
      // V_r: new corners of T_r, first occurrence in (triangle, corner) order
      const int nf = (ok && !overflow) ? 3 * nT : 0;
      const int frounds = wave_max_i((nf + G - 1) / G);
      for (int k = 0; k < frounds; ++k) {
        const int f = k * G + gl;
        if (f < nf) {
          const int32_t t = M.T[f / 3];
          const int q = f % 3;
          const int32_t cv = q == 0 ? m.t0[t] : (q == 1 ? m.t1[t] : m.t2[t]);
          const int s = hinsert(M, cv);
          if (s >= 0) atomicMin(&M.hval[s], f);
        }
      }
      __syncthreads();
      for (int k = 0; k < frounds; ++k) {
        const int f = k * G + gl;
        bool fresh = false;
        int s = -1;
        int32_t cv = 0;
        if (f < nf) {
          const int32_t t = M.T[f / 3];
          const int q = f % 3;
          cv = q == 0 ? m.t0[t] : (q == 1 ? m.t1[t] : m.t2[t]);
          s = hfind(M, cv);
          fresh = s >= 0 && M.hval[s] == f;
        }
        const uint32_t bal = gballot(fresh, grp);
        if (fresh) {
          const int pos = nV + __popc(bal & ((1u << gl) - 1u));
          if (pos < kVC) M.V[pos] = cv;
          M.hval[s] = -1 - pos;
        }
        nV += __popc(bal);
      }
      if (nV > kVC) overflow = true;
      __syncthreads();
    }
    if (overflow) ok = false;
    const int nTc = min(nT, kTC);

    // ---- centre distances and support radius
    const int trounds = wave_max_i(ok ? (nTc + G - 1) / G : 0);
    for (int k = 0; k < trounds; ++k) {
      const int i = k * G + gl;
      if (ok && i < nTc) {
        const Tri T = load_tri(m, M.T[i]);
        const double cx = (T.v[0][0] + T.v[1][0] + T.v[2][0]) / 3.0;
        const double cy = (T.v[0][1] + T.v[1][1] + T.v[2][1]) / 3.0;
        const double cz = (T.v[0][2] + T.v[1][2] + T.v[2][2]) / 3.0;
        const double dx = cx - xc[0], dy = cy - xc[1], dz = cz - xc[2];
        M.d2[i] = dx * dx + dy * dy + dz * dz;
      }
    }
    __syncthreads();
    double delta = A.prm.delta_over_h * h;
    int32_t it = 0, cnt = 0;
    bool done = !ok;
    for (;;) {
      const double lim = delta * delta;
      int mine = 0;
      if (!done)
        for (int i = gl; i < nTc; i += G) mine += M.d2[i] < lim ? 1 : 0;
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

    // ---- weighted moments and normal equations
    const double lim = delta * delta;
    const double inv_h = 1.0 / h;
    double acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = 0.0;
    for (int k = 0; k < trounds; ++k) {
      const int i = k * G + gl;
      if (!(ok && i < nTc)) continue;
      const double dd = M.d2[i];
      if (!(dd < lim)) continue;
      const double qq = sqrt(dd) / delta;
      const double om = 1.0 - qq;
      const double w = (1.0 + 4.0 * qq) * (om * om) * (om * om);
      const Tri T = load_tri(m, M.T[i]);
      double xi[3], eta[3], zeta[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double dx = T.v[r][0] - xc[0], dy = T.v[r][1] - xc[1], dz = T.v[r][2] - xc[2];
        xi[r] = fma(dz, t1z, fma(dy, t1y, dx * t1x)) * inv_h;
        eta[r] = fma(dz, t2z, fma(dy, t2y, dx * t2x)) * inv_h;
        zeta[r] = fma(dz, n2, fma(dy, n1, dx * n0)) * inv_h;
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
      for (int q = 0; q < 6; ++q) mom[q] = a3 * sm[q];
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
    for (int q = 0; q < 27; ++q) {
#pragma unroll
      for (int o = G / 2; o >= 1; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
    }

    // ---- solve (every lane of the group holds M and b).  M is kept in LDS
    // (the distance array is no longer needed) for the refinement residual,
    // and factorised in place in the accumulator registers.
    __syncthreads();
    if (gl == 0) {
#pragma unroll
      for (int q = 0; q < 21; ++q) M.d2[q] = acc[q];
    }
    __syncthreads();
    double co[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
    double kap = NAN, ni0 = NAN, ni1 = NAN, ni2 = NAN;
    uint32_t st = overflow ? FTC_CELL_OVERFLOW : 0u;
    if (ok) {
      const double trace =
          acc[P6(0, 0)] + acc[P6(1, 1)] + acc[P6(2, 2)] + acc[P6(3, 3)] + acc[P6(4, 4)] + acc[P6(5, 5)];
      // in place: acc[P6(j, i)] becomes L(i, j) for i >= j
      bool rank_ok = cnt >= 6;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double d = acc[P6(j, j)];
#pragma unroll
        for (int p = 0; p < j; ++p) d -= acc[P6(p, j)] * acc[P6(p, j)];
        if (!(d > 1e-14 * trace)) rank_ok = false;
        const double ljj = sqrt(fmax(d, DBL_MIN));
        acc[P6(j, j)] = ljj;
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i2 = j + 1; i2 < 6; ++i2) {
          double s2 = acc[P6(j, i2)];
#pragma unroll
          for (int p = 0; p < j; ++p) s2 -= acc[P6(p, i2)] * acc[P6(p, j)];
          acc[P6(j, i2)] = s2 * inv;
        }
      }
      if (!rank_ok) {
        st |= FTC_CELL_RANK;
      } else {
        double ah[6], y[6], r6[6];
        auto solve = [&](const double* rhs, double* x) {
#pragma unroll
          for (int i2 = 0; i2 < 6; ++i2) {
            double s2 = rhs[i2];
#pragma unroll
            for (int p = 0; p < i2; ++p) s2 -= acc[P6(p, i2)] * y[p];
            y[i2] = s2 / acc[P6(i2, i2)];
          }
#pragma unroll
          for (int i2 = 5; i2 >= 0; --i2) {
            double s2 = y[i2];
#pragma unroll
            for (int p = i2 + 1; p < 6; ++p) s2 -= acc[P6(i2, p)] * x[p];
            x[i2] = s2 / acc[P6(i2, i2)];
          }
        };
        solve(acc + 21, ah);
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) {
          double s2 = acc[21 + i2];
#pragma unroll
          for (int p = 0; p < 6; ++p) s2 -= M.d2[i2 <= p ? P6(i2, p) : P6(p, i2)] * ah[p];
          r6[i2] = s2;
        }
        solve(r6, r6);
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) ah[i2] += r6[i2];
        co[0] = h * ah[0];
        co[1] = ah[1];
        co[2] = ah[2];
        co[3] = ah[3] / h;
        co[4] = ah[4] / h;
        co[5] = ah[5] / h;
        const double gx = co[1], gy = co[2];
        const double num = 2.0 * co[3] * (1.0 + gy * gy) - 2.0 * gx * gy * co[4] + 2.0 * co[5] * (1.0 + gx * gx);
        const double sq = 1.0 + gx * gx + gy * gy;
        kap = -num / (sq * sqrt(sq));
        ni0 = n0 - co[1] * t1x - co[2] * t2x;
        ni1 = n1 - co[1] * t1y - co[2] * t2y;
        ni2 = n2 - co[1] * t1z - co[2] * t2z;
        const double il = 1.0 / sqrt(ni0 * ni0 + ni1 * ni1 + ni2 * ni2);
        ni0 *= il;
        ni1 *= il;
        ni2 *= il;
      }
    }
    if (act && gl == 0) {
      A.kappa[c] = kap;
      A.nx[c] = ni0;
      A.ny[c] = ni1;
      A.nz[c] = ni2;
      if (A.coeff)
        for (int q = 0; q < 6; ++q) A.coeff[(int64_t)q * A.cell_cap + c] = st ? NAN : co[q];
      if (A.status) A.status[c] = (int32_t)st;
      if (A.diag) {
        A.diag[c] = vs;
        A.diag[(int64_t)A.cell_cap + c] = nT;
        A.diag[2 * (int64_t)A.cell_cap + c] = cnt;
        A.diag[3 * (int64_t)A.cell_cap + c] = it;
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_ppic(const ftc_cells* ws, const Mesh& m, const PPICParams& p, double* kappa, double* nx,
                       double* ny, double* nz, double* coeff, int32_t* cell_status, int32_t* diag, hipStream_t s) {
  const Grid& g = ws->grid;
  hipLaunchKernelGGL(k_clear_ppic, dim3(grid_blocks((int64_t)m.nv + 1, kT, kStrideBlocks)), dim3(kT), 0, s,
                     ws->vt_off, (int64_t)m.nv + 1, ws->vt_cursor, (int64_t)m.nv);
  hipLaunchKernelGGL(k_vt_count, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, m, ws->vt_off);
  hipError_t e = scan_exclusive(ws->vt_off, m.nv, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vt_scatter, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, m, ws->vt_off, ws->vt_cursor,
                     ws->vt_ids);
  hipLaunchKernelGGL(k_vt_sort, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, m.nv, ws->vt_off, ws->vt_ids);
  hipLaunchKernelGGL(k_vstar_init, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s,
                     ws->best_d2, ws->best_v, ws->cell_cap, ws->counters);
  hipLaunchKernelGGL(k_vstar<0>, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, ws->bitmap, ws->word_off,
                     ws->best_d2, ws->best_v, ws->cell_cap);
  hipLaunchKernelGGL(k_vstar<1>, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, ws->bitmap, ws->word_off,
                     ws->best_d2, ws->best_v, ws->cell_cap);
  PPICArgs A;
  A.g = g;
  A.m = m;
  A.prm = p;
  A.cell_ids = ws->cell_ids;
  A.vt_off = ws->vt_off;
  A.vt_ids = ws->vt_ids;
  A.best_d2 = ws->best_d2;
  A.best_v = ws->best_v;
  A.counters = ws->counters;
  A.cell_cap = ws->cell_cap;
  A.kappa = kappa;
  A.nx = nx;
  A.ny = ny;
  A.nz = nz;
  A.coeff = coeff;
  A.status = cell_status;
  A.diag = diag;
  const int64_t groups = ((int64_t)ws->cell_cap + NG - 1) / NG;
  const int32_t blocks = (int32_t)std::min<int64_t>(std::max<int64_t>(groups, 1), 65536);
  time_start(ws, FTC_KERNEL_PPIC, s);
  hipLaunchKernelGGL(k_ppic, dim3(blocks), dim3(64), 0, s, A);
  time_stop(ws, FTC_KERNEL_PPIC, s);
  return hipGetLastError();
}

}  // namespace ftc
