// ppic.hip -- PPIC curvature by the volume fit (paper section 3.2).
//
// Pre-passes (integer work): vertex -> incident-triangle lists (ascending
// triangle id) and the front vertices binned by interfacial cell (vertices
// whose cell holds no piece go to a short "stray" list that every search
// scans).
//
// Main kernel: one 64-lane wavefront (one workgroup) per interfacial cell.
//   1. closest vertex to the cell centre: lanes scan the binned vertices of
//      the (2r+1)^3 cells around the cell, r = 1, 2, 3, until the best
//      squared distance is below the distance to any unsearched cell; then
//      (rarely) all vertices.  Ties go to the lowest vertex index.
//   2. its normal (area-weighted, summed in ascending triangle order) and a
//      right-handed tangent frame (Duff et al., JCGT 2017).
//   3. the ring neighbourhood: T_1 = triangles at the vertex, T_{r+1} =
//      triangles sharing a corner with T_r; each set is built in LDS by a
//      bitonic sort of the candidate ids and a unique pass, so it comes out
//      in ascending id order.
//   4. triangle-centre distances, the support radius grown by `grow` until
//      `n_min` triangles fall inside (or the ring is exhausted, or `max_iter`
//      adjustments), Wendland weights.
//   5. per lane: the triangle's projection into the frame (coordinates
//      divided by h for conditioning), its six moments by the edge-midpoint
//      rule (exact for quadratics) and the integral of its plane; the
//      weighted normal equations M a = b accumulated per lane, then reduced
//      across the wavefront (two butterfly steps, then a fixed-order sum over
//      LDS).
//   6. Cholesky factorisation of M with one step of iterative refinement,
//      curvature kappa = 2H at the frame origin and the interface normal.
#include <float.h>

#include <algorithm>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 4096;

constexpr int kTCap = 256;   // ring triangles
constexpr int kVCap = 256;   // ring vertices
constexpr int kCCap = 1024;  // sort candidates (power of two)
constexpr int kSearchMax = 3;

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

__device__ inline int64_t vertex_cell(const Grid& g, double x, double y, double z) {
  const int64_t i = cell_index(x, g.x0, g.h), j = cell_index(y, g.y0, g.h), k = cell_index(z, g.z0, g.h);
  return i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
}

__global__ void k_vb_count(Grid g, Mesh m, const uint32_t* bitmap, const int32_t* word_off, int32_t* vb_cnt,
                           int32_t* stray, int32_t cell_cap, int32_t* counters) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.nv) return;
  const double x = m.x[v], y = m.y[v], z = m.z[v];
  if (!in_margin(g, x, y, z)) {
    atomicOr(&counters[C_ERR], ERR_DOMAIN);
    return;
  }
  const int32_t ci = cell_rank(bitmap, word_off, vertex_cell(g, x, y, z));
  if (ci >= 0 && ci < cell_cap) {
    atomicAdd(&vb_cnt[ci], 1);
  } else {
    stray[atomicAdd(&counters[C_NSTRAY], 1)] = v;
  }
}

__global__ void k_vb_scatter(Grid g, Mesh m, const uint32_t* bitmap, const int32_t* word_off, const int32_t* vb_off,
                             int32_t* vb_cursor, int32_t* vb_ids, int32_t cell_cap) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.nv) return;
  const double x = m.x[v], y = m.y[v], z = m.z[v];
  if (!in_margin(g, x, y, z)) return;
  const int32_t ci = cell_rank(bitmap, word_off, vertex_cell(g, x, y, z));
  if (ci >= 0 && ci < cell_cap) vb_ids[vb_off[ci] + atomicAdd(&vb_cursor[ci], 1)] = v;
}

// ----------------------------------------------------------------- main kernel
struct PPICArgs {
  Grid g;
  Mesh m;
  PPICParams prm;
  const int32_t* cell_ids;
  const uint32_t* bitmap;
  const int32_t* word_off;
  const int32_t* vt_off;
  const int32_t* vt_ids;
  const int32_t* vb_off;
  const int32_t* vb_ids;
  const int32_t* stray;
  const int32_t* counters;
  int32_t cell_cap;
  double *kappa, *nx, *ny, *nz, *coeff;
  int32_t *status, *diag;
};

__device__ inline bool lex_less(double d, int32_t v, double bd, int32_t bv) {
  return d < bd || (d == bd && v < bv);
}

__device__ inline void wave_argmin(double& d, int32_t& v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double od = __shfl_xor(d, o, 64);
    const int32_t ov = __shfl_xor(v, o, 64);
    if (lex_less(od, ov, d, v)) {
      d = od;
      v = ov;
    }
  }
}

__device__ inline int32_t wave_sum_i(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline void consider_vertex(const Mesh& m, int32_t v, const double xc[3], double& bd, int32_t& bv) {
  const double dx = m.x[v] - xc[0], dy = m.y[v] - xc[1], dz = m.z[v] - xc[2];
  const double d2 = dx * dx + dy * dy + dz * dz;
  if (lex_less(d2, v, bd, bv)) {
    bd = d2;
    bv = v;
  }
}

// Bitonic sort of s[0..P) ascending, P a power of two, 64 threads.
__device__ inline void block_bitonic(int32_t* s, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int idx = threadIdx.x; idx < P; idx += 64) {
        const int p = idx ^ j;
        if (p > idx) {
          const int32_t a = s[idx], b = s[p];
          const bool up = (idx & k) == 0;
          if ((a > b) == up) {
            s[idx] = b;
            s[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Sorted unique values of cand[0..n) (INT_MAX padding excluded) -> out;
// returns the count (uniform).  Requires n <= kCCap.
__device__ inline int32_t sort_unique(int32_t* cand, int32_t n, int32_t* out, int32_t out_cap) {
  int P = 1;
  while (P < n) P <<= 1;
  for (int idx = n + threadIdx.x; idx < P; idx += 64) cand[idx] = INT_MAX;
  __syncthreads();
  block_bitonic(cand, P);
  int32_t base = 0;
  for (int c0 = 0; c0 < P; c0 += 64) {
    const int idx = c0 + threadIdx.x;
    bool keep = false;
    int32_t val = INT_MAX;
    if (idx < P) {
      val = cand[idx];
      keep = val != INT_MAX && (idx == 0 || cand[idx - 1] != val);
    }
    const uint64_t bal = __ballot(keep);
    const int32_t pre = __popcll(bal & ((1ull << threadIdx.x) - 1ull));
    if (keep && base + pre < out_cap) out[base + pre] = val;
    base += __popcll(bal);
  }
  __syncthreads();
  return base;
}

// Fill cand with the incident triangles of verts[0..nverts); returns count
// or -1 if it would exceed kCCap.
__device__ inline int32_t gather_incident(const PPICArgs& A, const int32_t* verts, int32_t nverts, int32_t* start,
                                          int32_t* cand) {
  // exclusive prefix of degrees, 64 at a time
  int32_t base = 0;
  for (int c0 = 0; c0 < nverts; c0 += 64) {
    const int a = c0 + threadIdx.x;
    int32_t deg = 0;
    if (a < nverts) deg = A.vt_off[verts[a] + 1] - A.vt_off[verts[a]];
    int32_t inc = deg;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t o = __shfl_up(inc, d, 64);
      if ((int)threadIdx.x >= d) inc += o;
    }
    if (a < nverts) start[a] = base + inc - deg;
    base += __shfl(inc, 63, 64);
  }
  __syncthreads();
  if (base > kCCap) return -1;
  for (int a = threadIdx.x; a < nverts; a += 64) {
    const int32_t s = A.vt_off[verts[a]], e = A.vt_off[verts[a] + 1];
    int32_t w = start[a];
    for (int32_t q = s; q < e; ++q) cand[w++] = A.vt_ids[q];
  }
  __syncthreads();
  return base;
}

__device__ inline void sym_set(double M[6][6], int a, int b, double v) {
  M[a][b] = v;
  M[b][a] = v;
}

__global__ __launch_bounds__(64) void k_ppic(PPICArgs A) {
  __shared__ int32_t sCand[kCCap];
  __shared__ int32_t sV[kVCap];
  __shared__ int32_t sStart[kVCap];
  __shared__ int32_t sT[kTCap];
  __shared__ double sTot[28];
  double* sRed = reinterpret_cast<double*>(sCand);  // 27 x 16 doubles, used after the ring is built

  const Grid& g = A.g;
  const Mesh& m = A.m;
  const int lane = threadIdx.x;
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  const int32_t nstray = A.counters[C_NSTRAY];
  const double h = g.h;

  for (int32_t c = blockIdx.x; c < nif; c += gridDim.x) {
    const int32_t lin = A.cell_ids[c];
    const int64_t ncol = (int64_t)g.nx * g.ny;
    const int32_t ci = lin % g.nx, cj = (lin / g.nx) % g.ny, ck = (int32_t)(lin / ncol);
    const double xc[3] = {g.x0 + ((double)ci + 0.5) * h, g.y0 + ((double)cj + 0.5) * h,
                          g.z0 + ((double)ck + 0.5) * h};

    // ---- 1. closest vertex
    double bd = DBL_MAX;
    int32_t bv = INT_MAX;
    for (int q = lane; q < nstray; q += 64) consider_vertex(m, A.stray[q], xc, bd, bv);
    bool found = false;
    for (int r = 1; r <= kSearchMax && !found; ++r) {
      const int side = 2 * r + 1, ncube = side * side * side;
      for (int q = lane; q < ncube; q += 64) {
        const int di = q % side - r, dj = (q / side) % side - r, dk = q / (side * side) - r;
        if (max(max(abs(di), abs(dj)), abs(dk)) != r && r > 1) continue;  // inner cube done already
        const int ii = ci + di, jj = cj + dj, kk = ck + dk;
        if (ii < 0 || jj < 0 || kk < 0 || ii >= g.nx || jj >= g.ny || kk >= g.nz) continue;
        const int32_t cr = cell_rank(A.bitmap, A.word_off, ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk));
        if (cr < 0 || cr >= A.cell_cap) continue;
        for (int32_t p = A.vb_off[cr]; p < A.vb_off[cr + 1]; ++p) consider_vertex(m, A.vb_ids[p], xc, bd, bv);
      }
      wave_argmin(bd, bv);
      const double reach = ((double)r + 0.5) * h;
      found = bv != INT_MAX && bd < reach * reach * (1.0 - 1e-12);
    }
    if (!found) {
      for (int32_t v = lane; v < m.nv; v += 64) consider_vertex(m, v, xc, bd, bv);
      wave_argmin(bd, bv);
    }
    const int32_t vs = bv;
    if (vs == INT_MAX) {  // no finite vertex at all: nothing to fit
      if (lane == 0) {
        A.kappa[c] = A.nx[c] = A.ny[c] = A.nz[c] = NAN;
        if (A.status) A.status[c] = (int32_t)FTC_CELL_OVERFLOW;
      }
      __syncthreads();
      continue;
    }

    // ---- 2. vertex normal (serial, ascending triangle order) and frame
    double n0 = 0.0, n1 = 0.0, n2 = 0.0;
    for (int32_t q = A.vt_off[vs]; q < A.vt_off[vs + 1]; ++q) {
      const Tri T = load_tri(m, A.vt_ids[q]);
      const double ux = T.v[1][0] - T.v[0][0], uy = T.v[1][1] - T.v[0][1], uz = T.v[1][2] - T.v[0][2];
      const double wx = T.v[2][0] - T.v[0][0], wy = T.v[2][1] - T.v[0][1], wz = T.v[2][2] - T.v[0][2];
      n0 += uy * wz - uz * wy;
      n1 += uz * wx - ux * wz;
      n2 += ux * wy - uy * wx;
    }
    {
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

    // ---- 3. ring neighbourhood
    if (lane == 0) sV[0] = vs;
    __syncthreads();
    int32_t nV = 1, nT = 0;
    bool overflow = false;
    for (int r = 1; r <= A.prm.rings; ++r) {
      const int32_t nc = gather_incident(A, sV, nV, sStart, sCand);
      if (nc < 0) {
        overflow = true;
        break;
      }
      nT = sort_unique(sCand, nc, sT, kTCap);
      if (nT > kTCap) {
        overflow = true;
        break;
      }
      if (r == A.prm.rings) break;
      if (3 * nT > kCCap) {
        overflow = true;
        break;
      }
      for (int a = lane; a < nT; a += 64) {
        const int32_t t = sT[a];
        sCand[3 * a + 0] = m.t0[t];
        sCand[3 * a + 1] = m.t1[t];
        sCand[3 * a + 2] = m.t2[t];
      }
      __syncthreads();
      nV = sort_unique(sCand, 3 * nT, sV, kVCap);
      if (nV > kVCap) {
        overflow = true;
        break;
      }
    }

    int32_t cnt = 0, it = 0;
    double co[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
    double kap = NAN, ni0 = NAN, ni1 = NAN, ni2 = NAN;
    uint32_t st = 0;
    if (overflow) {
      st = FTC_CELL_OVERFLOW;
      nT = min(nT, kTCap);
    } else {
      // ---- 4. centre distances and support radius
      constexpr int kPer = kTCap / 64;
      double d2[kPer];
      int32_t tid[kPer];
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        const int a = lane + 64 * s;
        tid[s] = a < nT ? sT[a] : -1;
        d2[s] = DBL_MAX;
        if (tid[s] >= 0) {
          const Tri T = load_tri(m, tid[s]);
          const double cx = (T.v[0][0] + T.v[1][0] + T.v[2][0]) / 3.0;
          const double cy = (T.v[0][1] + T.v[1][1] + T.v[2][1]) / 3.0;
          const double cz = (T.v[0][2] + T.v[1][2] + T.v[2][2]) / 3.0;
          const double dx = cx - xc[0], dy = cy - xc[1], dz = cz - xc[2];
          d2[s] = dx * dx + dy * dy + dz * dz;
        }
      }
      double delta = A.prm.delta_over_h * h;
      for (;;) {
        const double lim = delta * delta;
        int32_t mine = 0;
#pragma unroll
        for (int s = 0; s < kPer; ++s) mine += (tid[s] >= 0 && d2[s] < lim) ? 1 : 0;
        cnt = wave_sum_i(mine);
        if (cnt >= A.prm.n_min || cnt == nT || it == A.prm.max_iter) break;
        delta = delta * A.prm.grow;
        ++it;
      }

      // ---- 5. weighted moments, per lane
      const double lim = delta * delta;
      const double inv_h = 1.0 / h;
      double acc[27];
#pragma unroll
      for (int q = 0; q < 27; ++q) acc[q] = 0.0;
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        if (tid[s] < 0 || !(d2[s] < lim)) continue;
        const double qq = sqrt(d2[s]) / delta;
        const double om = 1.0 - qq;
        const double w = (1.0 + 4.0 * qq) * (om * om) * (om * om);
        const Tri T = load_tri(m, tid[s]);
        double xi[3], eta[3], zeta[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double dx = T.v[r][0] - xc[0], dy = T.v[r][1] - xc[1], dz = T.v[r][2] - xc[2];
          xi[r] = fma(dz, t1z, fma(dy, t1y, dx * t1x)) * inv_h;
          eta[r] = fma(dz, t2z, fma(dy, t2y, dx * t2x)) * inv_h;
          zeta[r] = fma(dz, n2, fma(dy, n1, dx * n0)) * inv_h;
        }
        const double area =
            0.5 * fma(xi[1] - xi[0], eta[2] - eta[0], -((xi[2] - xi[0]) * (eta[1] - eta[0])));
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
        const double vol = a3 * (zeta[0] + zeta[1] + zeta[2]);
        int q = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const double wa = w * mom[a];
#pragma unroll
          for (int b = a; b < 6; ++b) {
            acc[q] = fma(wa, mom[b], acc[q]);
            ++q;
          }
        }
        const double wv = w * vol;
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[21 + a] = fma(wv, mom[a], acc[21 + a]);
      }

      // ---- reduce 27 partial sums: two butterfly steps, then LDS
#pragma unroll
      for (int q = 0; q < 27; ++q) {
        acc[q] += __shfl_xor(acc[q], 32, 64);
        acc[q] += __shfl_xor(acc[q], 16, 64);
      }
      __syncthreads();  // sCand (aliased by sRed) is no longer read
      if (lane < 16) {
#pragma unroll
        for (int q = 0; q < 27; ++q) sRed[q * 16 + lane] = acc[q];
      }
      __syncthreads();
      if (lane < 27) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < 16; ++p) s += sRed[lane * 16 + p];
        sTot[lane] = s;
      }
      __syncthreads();

      // ---- 6. solve (every lane redundantly; uniform)
      double M[6][6], b[6];
      {
        int q = 0;
        for (int a = 0; a < 6; ++a)
          for (int bb = a; bb < 6; ++bb) sym_set(M, a, bb, sTot[q++]);
        for (int a = 0; a < 6; ++a) b[a] = sTot[21 + a];
      }
      const double trace = M[0][0] + M[1][1] + M[2][2] + M[3][3] + M[4][4] + M[5][5];
      double L[6][6];
      bool rank_ok = cnt >= 6;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double d = M[j][j];
#pragma unroll
        for (int p = 0; p < j; ++p) d -= L[j][p] * L[j][p];
        if (!(d > 1e-14 * trace)) rank_ok = false;
        const double ljj = sqrt(fmax(d, DBL_MIN));
        L[j][j] = ljj;
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i2 = j + 1; i2 < 6; ++i2) {
          double s2 = M[i2][j];
#pragma unroll
          for (int p = 0; p < j; ++p) s2 -= L[i2][p] * L[j][p];
          L[i2][j] = s2 * inv;
        }
      }
      if (!rank_ok) {
        st = FTC_CELL_RANK;
      } else {
        double ah[6], y[6], r6[6];
        // forward / backward substitution: L L^T ah = b
        auto chol_solve = [&](const double* rhs, double* x) {
#pragma unroll
          for (int i2 = 0; i2 < 6; ++i2) {
            double s2 = rhs[i2];
#pragma unroll
            for (int p = 0; p < i2; ++p) s2 -= L[i2][p] * y[p];
            y[i2] = s2 / L[i2][i2];
          }
#pragma unroll
          for (int i2 = 5; i2 >= 0; --i2) {
            double s2 = y[i2];
#pragma unroll
            for (int p = i2 + 1; p < 6; ++p) s2 -= L[p][i2] * x[p];
            x[i2] = s2 / L[i2][i2];
          }
        };
        chol_solve(b, ah);
        // one step of iterative refinement
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) {
          double s2 = b[i2];
#pragma unroll
          for (int p = 0; p < 6; ++p) s2 -= M[i2][p] * ah[p];
          r6[i2] = s2;
        }
        double dl[6];
        chol_solve(r6, dl);
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) ah[i2] += dl[i2];
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
    if (lane == 0) {
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
  hipLaunchKernelGGL(k_clear_ppic, dim3(grid_blocks((int64_t)ws->nv_cap + 1, kT, kStrideBlocks)), dim3(kT), 0, s,
                     ws->vt_off, (int64_t)m.nv + 1, ws->vt_cursor, (int64_t)m.nv, ws->vb_off,
                     (int64_t)ws->cell_cap + 1, ws->vb_cursor, (int64_t)ws->cell_cap, ws->counters);
  hipLaunchKernelGGL(k_vt_count, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, m, ws->vt_off);
  hipError_t e = scan_exclusive(ws->vt_off, m.nv, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vt_scatter, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, m, ws->vt_off, ws->vt_cursor,
                     ws->vt_ids);
  hipLaunchKernelGGL(k_vt_sort, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, m.nv, ws->vt_off, ws->vt_ids);
  hipLaunchKernelGGL(k_vb_count, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, ws->bitmap, ws->word_off,
                     ws->vb_off, ws->stray, ws->cell_cap, ws->counters);
  e = scan_exclusive(ws->vb_off, ws->cell_cap, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vb_scatter, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, ws->bitmap, ws->word_off,
                     ws->vb_off, ws->vb_cursor, ws->vb_ids, ws->cell_cap);
  PPICArgs A;
  A.g = g;
  A.m = m;
  A.prm = p;
  A.cell_ids = ws->cell_ids;
  A.bitmap = ws->bitmap;
  A.word_off = ws->word_off;
  A.vt_off = ws->vt_off;
  A.vt_ids = ws->vt_ids;
  A.vb_off = ws->vb_off;
  A.vb_ids = ws->vb_ids;
  A.stray = ws->stray;
  A.counters = ws->counters;
  A.cell_cap = ws->cell_cap;
  A.kappa = kappa;
  A.nx = nx;
  A.ny = ny;
  A.nz = nz;
  A.coeff = coeff;
  A.status = cell_status;
  A.diag = diag;
  const int32_t blocks = (int32_t)std::min<int64_t>(ws->cell_cap, 65536);
  time_start(ws, FTC_KERNEL_PPIC, s);
  hipLaunchKernelGGL(k_ppic, dim3(blocks > 0 ? blocks : 1), dim3(64), 0, s, A);
  time_stop(ws, FTC_KERNEL_PPIC, s);
  return hipGetLastError();
}

}  // namespace ftc
