// ppic.hip -- PPIC curvature by the volume fit (paper section 3.2).
//
// Pre-passes (integer work, once per call):
//   * vertex -> incident triangles (CSR, ascending triangle id);
//   * vertices binned by the interfacial cell that holds them; vertices in
//     cells without pieces go to a short "stray" list;
//   * closest vertex of every interfacial cell: 32 lanes per cell, one per
//     cell of the 3x3x3 block around it, all of them over the strays; lowest
//     index on ties.  A vertex outside the block is at least 1.5 h from the
//     cell centre, so a best squared distance below (1.5 h)^2 is final; any
//     other cell searches all vertices in the main kernel.
//
// Main kernel: 16 lanes per interfacial cell, 4 cells per 64-lane wavefront
// (one wavefront per workgroup), per-cell state in LDS.  Each phase issues
// all of its loads before it uses them, so a cell makes few dependent trips
// to memory.
//   1. ring neighbourhood: V_0 = {v*}; T_r = triangles with a corner in
//      V_{r-1}; V_r = V_{r-1} plus the corners of T_r.  The (vertex,
//      incident triangle) candidates of a ring are spread over the 16 lanes
//      through prefix sums of the vertex degrees; a triangle is taken once,
//      from the first of its corners (t0, t1, t2 order) that lies in
//      V_{r-1}; membership and first occurrence use an open-addressing hash
//      table; the corner ids of the ring triangles stay in LDS;
//   2. normal of v* (area-weighted, summed in ascending triangle order: T_1
//      is v*'s incident list) and a right-handed tangent frame (Duff et al.,
//      JCGT 2017);
//   3. triangle-centre distances, the support radius grown by `grow` until
//      `n_min` triangles fall inside (or the ring is exhausted, or
//      `max_iter` adjustments), Wendland weights of the triangles inside,
//      which are compacted into a list;
//   4. per lane: each listed triangle's projection into the frame
//      (coordinates divided by h for conditioning), its six moments by the
//      edge-midpoint rule (exact for quadratics) and the integral of its
//      plane, and the weighted normal equations M a = b accumulated in
//      registers; butterfly reduction over the 16 lanes;
//   5. in-register Cholesky factorisation of the packed M with one step of
//      iterative refinement, curvature kappa = 2H at the frame origin and the
//      interface normal.
// Every loop bound is uniform over the wavefront (maxima over its 4 cells),
// so LDS phases are separated by plain workgroup barriers.
#include <float.h>

#include <algorithm>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 4096;

constexpr int G = 16;            // lanes per cell
constexpr int NG = 64 / G;       // cells per wavefront
constexpr int kHS = 128;         // hash slots per cell
constexpr int kVC = 64;          // ring-vertex capacity
constexpr int kTC = 96;          // ring-triangle capacity
constexpr int kCR = 8;           // candidates per lane per batch
constexpr int kBatch = kCR * G;  // candidates per batch
constexpr int kTR = kTC / G;     // ring triangles per lane

// ----------------------------------------------------------------- pre-passes
__global__ void k_clear_ppic(int32_t* vt_off, int64_t n1, int32_t* vt_cursor, int64_t n2, int32_t* vb_off,
                             int64_t n3, int32_t* vb_cursor, int64_t n4, int32_t* counters) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = g0; i < n1; i += stride) vt_off[i] = 0;
  for (int64_t i = g0; i < n2; i += stride) vt_cursor[i] = 0;
  for (int64_t i = g0; i < n3; i += stride) vb_off[i] = 0;
  for (int64_t i = g0; i < n4; i += stride) vb_cursor[i] = 0;
  if (g0 == 0) counters[C_NSTRAY] = 0;
}

// A triangle is listed once under each of its distinct corners.
__global__ void k_vt_count(Mesh m, int32_t* vt_cnt) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nt || !tri_ok(m, t)) return;
  const int32_t a = m.t0[t], b = m.t1[t], c = m.t2[t];
  atomicAdd(&vt_cnt[a], 1);
  if (b != a) atomicAdd(&vt_cnt[b], 1);
  if (c != a && c != b) atomicAdd(&vt_cnt[c], 1);
}

__global__ void k_vt_scatter(Mesh m, const int32_t* vt_off, int32_t* vt_cursor, int32_t* vt_ids) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nt || !tri_ok(m, t)) return;
  const int32_t a = m.t0[t], b = m.t1[t], c = m.t2[t];
  vt_ids[vt_off[a] + atomicAdd(&vt_cursor[a], 1)] = t;
  if (b != a) vt_ids[vt_off[b] + atomicAdd(&vt_cursor[b], 1)] = t;
  if (c != a && c != b) vt_ids[vt_off[c] + atomicAdd(&vt_cursor[c], 1)] = t;
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

// Interfacial cell of every vertex (-1: a cell without pieces, the vertex
// becomes a stray; -2: outside the margin, latched as a domain error by the
// cell-list build) and the number of vertices per interfacial cell.
__global__ void k_vb_count(Grid g, Mesh m, const uint32_t* bitmap, const int32_t* word_off, int32_t* vcell,
                           int32_t* vb_cnt, int32_t* stray, int32_t cell_cap, int32_t* counters) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.nv) return;
  const double x = m.x[v], y = m.y[v], z = m.z[v];
  int32_t ci = -2;
  if (in_margin(g, x, y, z)) {
    const int64_t i = cell_index(x, g.x0, g.h), j = cell_index(y, g.y0, g.h), k = cell_index(z, g.z0, g.h);
    ci = cell_rank(bitmap, word_off, i + (int64_t)g.nx * (j + (int64_t)g.ny * k));
    if (ci >= cell_cap) ci = -1;
    if (ci >= 0)
      atomicAdd(&vb_cnt[ci], 1);
    else
      stray[atomicAdd(&counters[C_NSTRAY], 1)] = v;
  }
  vcell[v] = ci;
}

__global__ void k_vb_scatter(int32_t nv, const int32_t* vcell, const int32_t* vb_off, int32_t* vb_cursor,
                             int32_t* vb_ids) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int32_t ci = vcell[v];
  if (ci >= 0) vb_ids[vb_off[ci] + atomicAdd(&vb_cursor[ci], 1)] = v;
}

__device__ inline bool lex_less(double d, int32_t v, double bd, int32_t bv) {
  return d < bd || (d == bd && v < bv);
}

__device__ inline void consider(const Mesh& m, int32_t v, const double xc[3], double& bd, int32_t& bv) {
  const double dx = m.x[v] - xc[0], dy = m.y[v] - xc[1], dz = m.z[v] - xc[2];
  const double d2 = dx * dx + dy * dy + dz * dz;
  if (lex_less(d2, v, bd, bv)) {
    bd = d2;
    bv = v;
  }
}

__device__ inline double cell_centre(double org, int32_t i, double h) { return org + ((double)i + 0.5) * h; }

// 32 lanes per interfacial cell: lane l < 27 scans the vertex bin of cell l
// of the 3x3x3 block around it, every lane a share of the strays.
__global__ __launch_bounds__(kT) void k_vstar(Grid g, Mesh m, const int32_t* cell_ids, const uint32_t* bitmap,
                                              const int32_t* word_off, const int32_t* vb_off, const int32_t* vb_ids,
                                              const int32_t* stray, double* best_d2, int32_t* best_v,
                                              int32_t cell_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  const int32_t nstray = counters[C_NSTRAY];
  const int64_t gid = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t c = gid >> 5;
  const int l = (int)(gid & 31);
  double bd = DBL_MAX;
  int32_t bv = INT_MAX;
  if (c < nif) {
    const Cell3 cc = unpack_cell(g, cell_ids[c]);
    const double xc[3] = {cell_centre(g.x0, cc.i, g.h), cell_centre(g.y0, cc.j, g.h), cell_centre(g.z0, cc.k, g.h)};
    if (l < 27) {
      const int32_t ii = cc.i + l % 3 - 1, jj = cc.j + (l / 3) % 3 - 1, kk = cc.k + l / 9 - 1;
      if (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz) {
        const int32_t cr = cell_rank(bitmap, word_off, ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk));
        if (cr >= 0 && cr < cell_cap)
          for (int32_t p = vb_off[cr], e = vb_off[cr + 1]; p < e; ++p) consider(m, vb_ids[p], xc, bd, bv);
      }
    }
    for (int32_t q = l; q < nstray; q += 32) consider(m, stray[q], xc, bd, bv);
  }
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) {
    const double od = __shfl_xor(bd, o, 64);
    const int32_t ov = __shfl_xor(bv, o, 64);
    if (lex_less(od, ov, bd, bv)) {
      bd = od;
      bv = ov;
    }
  }
  if (c < nif && l == 0) {
    best_d2[c] = bd;
    best_v[c] = bv;
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
  const double* best_d2;
  const int32_t* best_v;
  const int32_t* counters;
  int32_t cell_cap;
  double *kappa, *nx, *ny, *nz, *coeff;
  int32_t *status, *diag;
};

// Ring-building state, dead once the rings are complete.
struct RingMem {
  int32_t hkey[kHS];    // hash set of ring vertices (-1: empty slot)
  int32_t hval[kHS];    // first occurrence among the new corners; -1 - position once in V
  int32_t V[kVC];       // ring vertices
  int32_t Vo[kVC];      // offset of their incident-triangle list
  int32_t Vd[kVC];      // their degrees
  int32_t Vs[kVC + 1];  // prefix sums of the degrees
  uint8_t own[kBatch];  // ring vertex of each candidate of the current batch
};
// Fit state, alive after the rings.
struct FitMem {
  double Mres[21];  // normal matrix, kept for the refinement residual
  double W[kTC];    // weights of the triangles inside the support
  int32_t S[kTC];   // their positions in the ring list
};
struct __align__(8) CellMem {
  union {
    RingMem r;
    FitMem f;
  } u;
  int32_t Tc[3][kTC];  // corners of the ring triangles
};

__device__ inline int hslot(int32_t key) { return (int)(((uint32_t)key * 2654435761u) >> 25); }  // 128 slots

// Insert key (if absent) and return its slot; -1 if the table is full.
__device__ inline int hinsert(RingMem& M, int32_t key) {
  int s = hslot(key);
  for (int p = 0; p < kHS; ++p) {
    const int32_t prev = atomicCAS(&M.hkey[s], -1, key);
    if (prev == -1 || prev == key) return s;
    s = (s + 1) & (kHS - 1);
  }
  return -1;
}

__device__ inline int hfind(const RingMem& M, int32_t key) {
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

// Membership of key, given the key stored at its home slot.
__device__ inline bool member(const RingMem& M, int32_t key, int32_t home) {
  if (home == key) return true;
  if (home == -1) return false;
  return hfind(M, key) >= 0;
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

__global__ __launch_bounds__(64) void k_ppic(PPICArgs A) {
  __shared__ CellMem SM[NG];
  const Grid& g = A.g;
  const Mesh& m = A.m;
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  CellMem& C = SM[grp];
  RingMem& RM = C.u.r;
  FitMem& FM = C.u.f;
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  const double h = g.h;
  const int R = A.prm.rings;
  const double reach = 1.5 * h;
  const double reach2 = reach * reach * (1.0 - 1e-12);
  const uint32_t below_me = (1u << gl) - 1u;

  for (int32_t base = blockIdx.x * NG; base < nif; base += gridDim.x * NG) {
    const int32_t c = base + grp;
    const bool act = c < nif;
    const Cell3 cc3 = unpack_cell(g, act ? A.cell_ids[c] : 0);
    const double xc[3] = {cell_centre(g.x0, cc3.i, h), cell_centre(g.y0, cc3.j, h), cell_centre(g.z0, cc3.k, h)};

    // ---- closest vertex: pre-pass result, else a search over all vertices
    int32_t vs = act ? A.best_v[c] : 0;
    const bool need = act && !(vs != INT_MAX && A.best_d2[c] < reach2);
    if (__any(need)) {
      double bd = DBL_MAX;
      int32_t bv = INT_MAX;
      if (need)
        for (int32_t v = gl; v < m.nv; v += G) consider(m, v, xc, bd, bv);
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
    const int32_t vsafe = ok ? vs : 0;  // a valid vertex for branch-free loads

    // ---- ring neighbourhood
    for (int s = gl; s < kHS; s += G) {
      RM.hkey[s] = -1;
      RM.hval[s] = INT_MAX;
    }
    __syncthreads();
    if (ok && gl == 0) {
      const int s = hinsert(RM, vs);  // empty table: never fails
      RM.hval[s] = -1;
      const int32_t o0 = A.vt_off[vs];
      RM.V[0] = vs;
      RM.Vo[0] = o0;
      RM.Vd[0] = A.vt_off[vs + 1] - o0;
      RM.Vs[0] = 0;
      RM.Vs[1] = RM.Vd[0];
    }
    __syncthreads();
    int32_t nV = 1, nT = 0;
    bool overflow = false;
    double n0 = 0.0, n1 = 0.0, n2 = 1.0;
    for (int r = 1; r <= R; ++r) {
      // T_r from the candidates of V_{r-1}, in batches of kBatch
      const int nVc = min(nV, kVC);
      const int tot = (ok && !overflow) ? RM.Vs[nVc] : 0;
      const int nb = wave_max_i((tot + kBatch - 1) / kBatch);
      const int prounds = wave_max_i(tot > 0 ? (nVc + G - 1) / G : 0);
      nT = 0;
      for (int b = 0; b < nb; ++b) {
        const int b0 = b * kBatch;
        // owners of the candidates [b0, b0 + kBatch)
        for (int k = 0; k < prounds; ++k) {
          const int p = k * G + gl;
          if (tot > 0 && p < nVc) {
            const int lo = max(RM.Vs[p], b0), hi = min(RM.Vs[p + 1], b0 + kBatch);
            for (int f = lo; f < hi; ++f) RM.own[f - b0] = (uint8_t)p;
          }
        }
        __syncthreads();
        int32_t ct[kCR], cu[kCR], c0[kCR], c1[kCR], c2[kCR];
#pragma unroll
        for (int k = 0; k < kCR; ++k) {
          const int f = b0 + k * G + gl;
          ct[k] = -1;
          cu[k] = -1;
          if (f < tot) {
            const int p = RM.own[f - b0];
            cu[k] = RM.V[p];
            ct[k] = A.vt_ids[RM.Vo[p] + (f - RM.Vs[p])];
          }
        }
#pragma unroll
        for (int k = 0; k < kCR; ++k) {
          const int32_t t = ct[k] >= 0 ? ct[k] : 0;
          c0[k] = m.t0[t];
          c1[k] = m.t1[t];
          c2[k] = m.t2[t];
        }
        // a triangle is kept from the first of its corners in V_{r-1}; every
        // corner before the owner must lie outside V_{r-1}
        int32_t h0[kCR], h1[kCR];
#pragma unroll
        for (int k = 0; k < kCR; ++k) {
          h0[k] = RM.hkey[hslot(c0[k])];
          h1[k] = RM.hkey[hslot(c1[k])];
        }
#pragma unroll
        for (int k = 0; k < kCR; ++k) {
          bool keep = ct[k] >= 0;
          if (keep && r > 1 && c0[k] != cu[k]) {
            keep = !member(RM, c0[k], h0[k]);
            if (keep && c1[k] != cu[k]) keep = !member(RM, c1[k], h1[k]);
          }
          const uint32_t bal = gballot(keep, grp);
          if (keep) {
            const int pos = nT + __popc(bal & below_me);
            if (pos < kTC) {
              C.Tc[0][pos] = c0[k];
              C.Tc[1][pos] = c1[k];
              C.Tc[2][pos] = c2[k];
            }
          }
          nT += __popc(bal);
        }
        __syncthreads();
      }
      if (nT > kTC) overflow = true;
      __syncthreads();

      if (r == 1) {
        // normal of v*: T_1 is v*'s incident list, ascending; the cross
        // products are summed serially in that order
        const int n1c = (ok && !overflow) ? nT : 0;
        const int nr = wave_max_i((n1c + G - 1) / G);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < nr; ++k) {
          const int i = k * G + gl;
          const bool valid = i < n1c;
          const int32_t a = valid ? C.Tc[0][i] : vsafe, bb = valid ? C.Tc[1][i] : vsafe,
                        e = valid ? C.Tc[2][i] : vsafe;
          const double ax = m.x[a], ay = m.y[a], az = m.z[a];
          const double ux = m.x[bb] - ax, uy = m.y[bb] - ay, uz = m.z[bb] - az;
          const double wx = m.x[e] - ax, wy = m.y[e] - ay, wz = m.z[e] - az;
          const double cx = uy * wz - uz * wy;
          const double cy = uz * wx - ux * wz;
          const double cz = ux * wy - uy * wx;
          for (int q = 0; q < G; ++q) {
            const double x = __shfl(cx, q, G), y = __shfl(cy, q, G), z = __shfl(cz, q, G);
            if (k * G + q < n1c) {
              s0 += x;
              s1 += y;
              s2 += z;
            }
          }
        }
        if (ok && !overflow) {
          const double nl = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
          n0 = s0 / nl;
          n1 = s1 / nl;
          n2 = s2 / nl;
        }
      }
      if (r == R) break;

      // V_r: the new corners of T_r, in (triangle, corner) order of first occurrence
      const int nf = (ok && !overflow) ? 3 * nT : 0;
      const int frounds = wave_max_i((nf + G - 1) / G);
      bool full = false;
      for (int k = 0; k < frounds; ++k) {
        const int f = k * G + gl;
        if (f < nf) {
          const int s = hinsert(RM, C.Tc[f % 3][f / 3]);
          if (s >= 0)
            atomicMin(&RM.hval[s], f);
          else
            full = true;
        }
      }
      if (gballot(full, grp)) overflow = true;
      __syncthreads();
      for (int k = 0; k < frounds; ++k) {
        const int f = k * G + gl;
        bool fresh = false;
        int s = -1;
        int32_t cv = 0;
        if (f < nf) {
          cv = C.Tc[f % 3][f / 3];
          s = hfind(RM, cv);
          fresh = s >= 0 && RM.hval[s] == f;
        }
        const uint32_t bal = gballot(fresh, grp);
        if (fresh) {
          const int pos = nV + __popc(bal & below_me);
          if (pos < kVC) {
            const int32_t o0 = A.vt_off[cv];
            RM.V[pos] = cv;
            RM.Vo[pos] = o0;
            RM.Vd[pos] = A.vt_off[cv + 1] - o0;
          }
          RM.hval[s] = -1 - pos;
        }
        nV += __popc(bal);
      }
      if (nV > kVC) overflow = true;
      __syncthreads();
      // prefix sums of the degrees
      const int nVs = (ok && !overflow) ? nV : 0;
      const int vrounds = wave_max_i((nVs + G - 1) / G);
      int32_t run = 0;
      for (int k = 0; k < vrounds; ++k) {
        const int p = k * G + gl;
        int32_t inc = p < nVs ? RM.Vd[p] : 0;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
          const int32_t t = __shfl_up(inc, o, G);
          if (gl >= o) inc += t;
        }
        if (p < nVs) RM.Vs[p + 1] = run + inc;
        run += __shfl(inc, G - 1, G);
      }
      __syncthreads();
    }
    if (overflow) ok = false;
    const int nTc = ok ? min(nT, kTC) : 0;

    const double sg = copysign(1.0, n2);
    const double fa = -1.0 / (sg + n2);
    const double fb = n0 * n1 * fa;
    const double t1x = 1.0 + sg * n0 * n0 * fa, t1y = sg * fb, t1z = -sg * n0;
    const double t2x = fb, t2y = sg + n1 * n1 * fa, t2z = -n1;

    // ---- centre distances, support radius, weights
    double d2[kTR];
#pragma unroll
    for (int k = 0; k < kTR; ++k) {
      const int i = k * G + gl;
      const bool valid = i < nTc;
      const int32_t a = valid ? C.Tc[0][i] : vsafe, b = valid ? C.Tc[1][i] : vsafe,
                    e = valid ? C.Tc[2][i] : vsafe;
      const double cx = div3(m.x[a] + m.x[b] + m.x[e]);
      const double cy = div3(m.y[a] + m.y[b] + m.y[e]);
      const double cz = div3(m.z[a] + m.z[b] + m.z[e]);
      const double dx = cx - xc[0], dy = cy - xc[1], dz = cz - xc[2];
      d2[k] = valid ? dx * dx + dy * dy + dz * dz : DBL_MAX;
    }
    double delta = A.prm.delta_over_h * h;
    int32_t it = 0, cnt = 0;
    bool done = !ok;
    for (;;) {
      const double lim = delta * delta;
      int mine = 0;
#pragma unroll
      for (int k = 0; k < kTR; ++k) mine += (k * G + gl < nTc && d2[k] < lim) ? 1 : 0;
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
      int nw = 0;
#pragma unroll
      for (int k = 0; k < kTR; ++k) {
        const bool keep = k * G + gl < nTc && d2[k] < lim;
        const uint32_t bal = gballot(keep, grp);
        if (keep) {
          const int pos = nw + __popc(bal & below_me);
          const double qq = sqrt(d2[k]) * inv_delta;
          const double om = 1.0 - qq;
          FM.W[pos] = (1.0 + 4.0 * qq) * (om * om) * (om * om);
          FM.S[pos] = k * G + gl;
        }
        nw += __popc(bal);
      }
    }
    __syncthreads();

    // ---- weighted moments and normal equations
    const double inv_h = 1.0 / h;
    double acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = 0.0;
    const int wrounds = wave_max_i(ok ? (cnt + G - 1) / G : 0);
    for (int k = 0; k < wrounds; ++k) {
      const int j = k * G + gl;
      const bool valid = ok && j < cnt;
      const int i = valid ? FM.S[j] : 0;
      const double w = valid ? FM.W[j] : 0.0;
      double xi[3], eta[3], zeta[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int32_t v = valid ? C.Tc[r][i] : vsafe;
        const double dx = m.x[v] - xc[0], dy = m.y[v] - xc[1], dz = m.z[v] - xc[2];
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
    // for the refinement residual and factorised in place in registers.
    if (gl == 0) {
#pragma unroll
      for (int q = 0; q < 21; ++q) FM.Mres[q] = acc[q];
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
      double invd[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double d = acc[P6(j, j)];
#pragma unroll
        for (int p = 0; p < j; ++p) d -= acc[P6(p, j)] * acc[P6(p, j)];
        if (!(d > 1e-14 * trace)) rank_ok = false;
        const double ljj = sqrt(fmax(d, DBL_MIN));
        acc[P6(j, j)] = ljj;
        const double inv = 1.0 / ljj;
        invd[j] = inv;
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
            y[i2] = s2 * invd[i2];
          }
#pragma unroll
          for (int i2 = 5; i2 >= 0; --i2) {
            double s2 = y[i2];
#pragma unroll
            for (int p = i2 + 1; p < 6; ++p) s2 -= acc[P6(i2, p)] * x[p];
            x[i2] = s2 * invd[i2];
          }
        };
        solve(acc + 21, ah);
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) {
          double s2 = acc[21 + i2];
#pragma unroll
          for (int p = 0; p < 6; ++p) s2 -= FM.Mres[i2 <= p ? P6(i2, p) : P6(p, i2)] * ah[p];
          r6[i2] = s2;
        }
        solve(r6, r6);
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) ah[i2] += r6[i2];
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
  const int64_t nclear = std::max<int64_t>((int64_t)m.nv + 1, (int64_t)ws->cell_cap + 1);
  hipLaunchKernelGGL(k_clear_ppic, dim3(grid_blocks(nclear, kT, kStrideBlocks)), dim3(kT), 0, s, ws->vt_off,
                     (int64_t)m.nv + 1, ws->vt_cursor, (int64_t)m.nv, ws->vb_off, (int64_t)ws->cell_cap + 1,
                     ws->vb_cursor, (int64_t)ws->cell_cap, ws->counters);
  hipLaunchKernelGGL(k_vt_count, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, m, ws->vt_off);
  hipError_t e = scan_exclusive(ws->vt_off, m.nv, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vt_scatter, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, m, ws->vt_off, ws->vt_cursor,
                     ws->vt_ids);
  hipLaunchKernelGGL(k_vt_sort, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, m.nv, ws->vt_off, ws->vt_ids);
  hipLaunchKernelGGL(k_vb_count, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, ws->bitmap, ws->word_off,
                     ws->vcell, ws->vb_off, ws->stray, ws->cell_cap, ws->counters);
  e = scan_exclusive(ws->vb_off, ws->cell_cap, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vb_scatter, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, m.nv, ws->vcell, ws->vb_off,
                     ws->vb_cursor, ws->vb_ids);
  hipLaunchKernelGGL(k_vstar, dim3(grid_blocks((int64_t)ws->cell_cap * 32, kT)), dim3(kT), 0, s, g, m,
                     ws->cell_ids, ws->bitmap, ws->word_off, ws->vb_off, ws->vb_ids, ws->stray, ws->best_d2,
                     ws->best_v, ws->cell_cap, ws->counters);
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
