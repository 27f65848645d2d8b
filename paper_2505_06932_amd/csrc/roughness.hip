// roughness.hip -- local roughness detection and volume-conserving edge
// smoothing of the front (paper section 3.4), on the vertex adjacency that
// the cell-list build prepares (each vertex's incident triangles in
// ascending order, packed corners and coordinates).
//
// Conventions (closed, consistently oriented front): the one-ring of vertex
// i is, over its incident triangles in ascending order, the corner that
// follows i; the undirected edge {a, b} is named by its half-edge a -> b with
// a < b, id 3 t + k for triangle t with corners k, k+1 (mod 3) = a, b; the
// twin b -> a lies in a's fan as the triangle whose corner before a is b.
//
// Metrics:
//   k_tri_normals : unit normal and area of every triangle;
//   k_vertex_stats: geometric Laplacian |x_i - sum w x_j / sum w| (w the
//                   inverse distance) and the mean G_i and population
//                   variance V_i of R_e = 1 - n1 . n2 over the edges at i;
//   k_tri_rt      : R_t = sum G V / sum V over the corners (the mean of the
//                   G if every V is 0);
//   k_vertex_rough: R_i = max(R^1, R^2), R^l the mean of A_t R_t over the
//                   triangles of the l-ring (a triangle of the two-ring is
//                   counted once, at the first of its corners in the order
//                   i, then the one-ring).
// Smoothing (after Kuprat et al. 2001, algorithm 4): edges whose two ends
// have both metrics above the thresholds are listed; in rounds, an edge is
// taken when no pending edge ordered before it (by fmix32 of the id, then
// the id) has an end within one ring of it (all rounds in one workgroup),
// and its ends move to the simultaneous Laplacian positions plus the
// least displacement along g = A1 + A2 + y x (d1 - d2) that keeps the
// enclosed volume, h n = -(d1.A1 + d2.A2 + d1.(d2 x y)) g / |g|^2 (the
// volume change of moving both ends is exactly linear in h).
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int32_t E_NONE = 0, E_PENDING = 1, E_SELECTED = 2, E_DONE = 3;

struct RoughArgs {
  int32_t nv, nt;
  const int4* tri4;
  const int32_t* vt_off;
  const int32_t* vt_ids;
  const double* x;  // positions (SoA): the metrics read the mesh, the smoothing its output copy
  const double* y;
  const double* z;
  double4* tn;      // [nt] unit normal, area
  double* vG;       // [nv]
  double* vV;       // [nv]
  double* rt;       // [nt]
  int32_t* counters;
};

struct D3 {
  double x, y, z;
};
__device__ inline D3 pos(const RoughArgs& A, int32_t v) { return D3{A.x[v], A.y[v], A.z[v]}; }
__device__ inline D3 sub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 add(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 scale(D3 a, double s) { return D3{a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 cross(D3 a, D3 b) { return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

__device__ inline int corner_of(int4 t, int32_t v) { return t.x == v ? 0 : (t.y == v ? 1 : 2); }
__device__ inline int32_t corner(int4 t, int k) { return k == 0 ? t.x : (k == 1 ? t.y : t.z); }

constexpr int kFanBatch = 4;  // incidences of a fan loaded together

// The triangle of v's fan whose corner before v is w (the half-edge w -> v),
// or -1 (the first in list order); the fan read kFanBatch incidences at a
// time, their loads issued together.
__device__ inline int32_t twin_in_fan(const RoughArgs& A, int32_t v, int32_t w) {
  const int32_t e1 = A.vt_off[v + 1];
  for (int32_t b = A.vt_off[v]; b < e1; b += kFanBatch) {
    int32_t t[kFanBatch];
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j) t[j] = b + j < e1 ? A.vt_ids[b + j] : -1;
    int4 c[kFanBatch];
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j) c[j] = t[j] >= 0 ? A.tri4[t[j]] : make_int4(-1, -1, -1, -1);
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j)
      if (t[j] >= 0 && corner(c[j], (corner_of(c[j], v) + 2) % 3) == w) return t[j];
  }
  return -1;
}

__global__ void k_tri_normals(RoughArgs A) {
  for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < A.nt; t += gridDim.x * blockDim.x) {
    const int4 c = A.tri4[t];
    const D3 a = pos(A, c.x), b = pos(A, c.y), d = pos(A, c.z);
    const D3 n = cross(sub(b, a), sub(d, a));
    const double len = sqrt(dot(n, n));
    A.tn[t] = make_double4(n.x / len, n.y / len, n.z / len, 0.5 * len);
  }
}

__global__ void k_vertex_stats(RoughArgs A, double* gl_mag) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < A.nv; v += gridDim.x * blockDim.x) {
    const D3 xv = pos(A, v);
    D3 num{0.0, 0.0, 0.0};
    double den = 0.0, sre = 0.0;
    const int32_t e0 = A.vt_off[v], e1 = A.vt_off[v + 1];
    for (int32_t e = e0; e < e1; ++e) {
      const int32_t t = A.vt_ids[e];
      const int4 c = A.tri4[t];
      const int32_t w = corner(c, (corner_of(c, v) + 1) % 3);
      const D3 xw = pos(A, w);
      const D3 dv = sub(xv, xw);
      const double wt = 1.0 / sqrt(dot(dv, dv));
      num = add(num, scale(xw, wt));
      den += wt;
      const int32_t t2 = twin_in_fan(A, v, w);
      const double4 n1 = A.tn[t];
      const double4 n2 = A.tn[t2 >= 0 ? t2 : t];
      sre += 1.0 - (n1.x * n2.x + n1.y * n2.y + n1.z * n2.z);
    }
    const int32_t m = e1 - e0;
    const double G = sre / (double)m;
    double var = 0.0;
    for (int32_t e = e0; e < e1; ++e) {
      const int32_t t = A.vt_ids[e];
      const int4 c = A.tri4[t];
      const int32_t w = corner(c, (corner_of(c, v) + 1) % 3);
      const int32_t t2 = twin_in_fan(A, v, w);
      const double4 n1 = A.tn[t];
      const double4 n2 = A.tn[t2 >= 0 ? t2 : t];
      const double d = (1.0 - (n1.x * n2.x + n1.y * n2.y + n1.z * n2.z)) - G;
      var += d * d;
    }
    A.vG[v] = G;
    A.vV[v] = var / (double)m;
    const D3 gl = sub(xv, scale(num, 1.0 / den));
    if (gl_mag) gl_mag[v] = sqrt(dot(gl, gl));
  }
}

__global__ void k_tri_rt(RoughArgs A) {
  for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < A.nt; t += gridDim.x * blockDim.x) {
    const int4 c = A.tri4[t];
    const double g0 = A.vG[c.x], g1 = A.vG[c.y], g2 = A.vG[c.z];
    const double v0 = A.vV[c.x], v1 = A.vV[c.y], v2 = A.vV[c.z];
    const double sv = (v0 + v1) + v2;
    A.rt[t] = sv > 0.0 ? ((g0 * v0 + g1 * v1) + g2 * v2) / sv : ((g0 + g1) + g2) / 3.0;
  }
}

// Position of vertex c in the order (v, then v's one-ring), or INT_MAX.
__device__ inline int32_t order_in_star(const RoughArgs& A, int32_t v, int32_t c) {
  if (c == v) return 0;
  const int32_t e0 = A.vt_off[v];
  for (int32_t e = e0; e < A.vt_off[v + 1]; ++e) {
    const int4 t = A.tri4[A.vt_ids[e]];
    if (corner(t, (corner_of(t, v) + 1) % 3) == c) return 1 + (e - e0);
  }
  return INT_MAX;
}

constexpr int kRing = 16;  // one-ring sizes kept in registers; larger ones take the fan walks

__global__ void k_vertex_rough(RoughArgs A, double* rough) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < A.nv; v += gridDim.x * blockDim.x) {
    const int32_t e0 = A.vt_off[v], e1 = A.vt_off[v + 1], deg = e1 - e0;
    double s1 = 0.0;
    for (int32_t e = e0; e < e1; ++e) {
      const int32_t t = A.vt_ids[e];
      s1 += A.tn[t].w * A.rt[t];
    }
    const double r1 = s1 / (double)deg;
    // the two-ring: triangles at v or at a one-ring vertex, each at the first
    // of its corners in the order (v, one-ring)
    double s2 = 0.0;
    int32_t n2 = 0;
    if (deg <= kRing) {
      // the one-ring in fan order, in registers (static indices only)
      int32_t ring[kRing];
#pragma unroll
      for (int q = 0; q < kRing; ++q) {
        int32_t u = -1;
        if (q < deg) {
          const int4 t = A.tri4[A.vt_ids[e0 + q]];
          u = corner(t, (corner_of(t, v) + 1) % 3);
        }
        ring[q] = u;
      }
      auto order = [&](int32_t c) {
        int32_t o = c == v ? 0 : INT_MAX;
#pragma unroll
        for (int q = kRing - 1; q >= 0; --q) o = (ring[q] == c && c != v) ? 1 + q : o;
        return o;
      };
#pragma unroll
      for (int q = -1; q < kRing; ++q) {
        if (q >= deg) break;
        const int32_t u = q < 0 ? v : ring[q];
        const int32_t ou = q + 1;
        for (int32_t f = A.vt_off[u]; f < A.vt_off[u + 1]; ++f) {
          const int32_t t = A.vt_ids[f];
          const int4 c = A.tri4[t];
          if (ou > 0 && (c.x == v || c.y == v || c.z == v)) continue;  // counted at v
          if (min(order(c.x), min(order(c.y), order(c.z))) == ou) {
            s2 += A.tn[t].w * A.rt[t];
            ++n2;
          }
        }
      }
    } else {
      for (int32_t q = -1; q < deg; ++q) {
        int32_t u = v;
        if (q >= 0) {
          const int4 t = A.tri4[A.vt_ids[e0 + q]];
          u = corner(t, (corner_of(t, v) + 1) % 3);
        }
        const int32_t ou = q + 1;
        for (int32_t f = A.vt_off[u]; f < A.vt_off[u + 1]; ++f) {
          const int32_t t = A.vt_ids[f];
          const int4 c = A.tri4[t];
          const int32_t o0 = order_in_star(A, v, c.x), o1 = order_in_star(A, v, c.y), o2 = order_in_star(A, v, c.z);
          if (min(o0, min(o1, o2)) == ou) {
            s2 += A.tn[t].w * A.rt[t];
            ++n2;
          }
        }
      }
    }
    rough[v] = fmax(r1, s2 / (double)n2);
  }
}

// ---------------------------------------------------------------- smoothing
struct SmoothArgs {
  RoughArgs R;      // x, y, z: the output positions, updated round by round
  const double* gl_mag;
  const double* rough;
  double gl_thr, rough_thr;
  int32_t* vflag;   // [nv]
  int32_t* estate;  // [3 nt] per owning half-edge
  int32_t* elist;   // [3 nt] flagged edges (ids)
};

__global__ void k_smooth_begin(const double* xi, const double* yi, const double* zi, double* xo, double* yo, double* zo,
                               int32_t nv, int32_t* counters) {
  const int32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    counters[C_RFLAG] = 0;
    counters[C_RMOVED] = 0;
  }
  for (int32_t v = i0; v < nv; v += gridDim.x * blockDim.x) {
    xo[v] = xi[v];
    yo[v] = yi[v];
    zo[v] = zi[v];
  }
}

__global__ void k_vertex_flags(SmoothArgs S) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < S.R.nv; v += gridDim.x * blockDim.x)
    S.vflag[v] = (S.gl_mag[v] > S.gl_thr && S.rough[v] > S.rough_thr) ? 1 : 0;
}

__global__ void k_edge_flags(SmoothArgs S) {
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < 3 * S.R.nt; h += gridDim.x * blockDim.x) {
    const int4 c = S.R.tri4[h / 3];
    const int32_t a = corner(c, h % 3), b = corner(c, (h % 3 + 1) % 3);
    const bool f = a < b && S.vflag[a] && S.vflag[b];
    S.estate[h] = f ? E_PENDING : E_NONE;
    if (f) S.elist[atomicAdd(&S.R.counters[C_RFLAG], 1)] = h;
  }
}

// Ends of edge id h (a -> b, a < b).
__device__ inline void edge_ends(const RoughArgs& A, int32_t h, int32_t& a, int32_t& b) {
  const int4 c = A.tri4[h / 3];
  a = corner(c, h % 3);
  b = corner(c, (h % 3 + 1) % 3);
}

// The 32-bit finalizer of MurmurHash3 (Appleby): edges are ordered by
// (fmix32(id), id), which scatters neighbouring ids and keeps the rounds few.
__device__ inline uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return x;
}
__device__ inline bool before(int32_t f, uint32_t hf, int32_t h, uint32_t hh) {
  return hf < hh || (hf == hh && f < h);
}

// A pending edge ordered before h with u as an end (u is an end or a
// one-ring vertex of an end of h), or -1.
__device__ inline int32_t blocker_at(const SmoothArgs& S, int32_t u, int32_t h) {
  const uint32_t hh = fmix32((uint32_t)h);
  const RoughArgs& A = S.R;
  for (int32_t f = A.vt_off[u]; f < A.vt_off[u + 1]; ++f) {
    const int32_t t = A.vt_ids[f];
    const int4 c = A.tri4[t];
    const int k = corner_of(c, u);
    // the two half-edges of t at u: u -> next and prev -> u
    const int ks[2] = {k, (k + 2) % 3};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int32_t id = 3 * t + ks[q];
      if (id != h && corner(c, ks[q]) < corner(c, (ks[q] + 1) % 3) && S.estate[id] == E_PENDING &&
          before(id, fmix32((uint32_t)id), h, hh))
        return id;
    }
  }
  return -1;
}

// One round's selection over the flagged edges: a pair of adjacent lanes per
// edge (edge i0/2, then + stride/2, ...), the even lane testing the end a and
// its one-ring, the odd lane the end b and its one-ring; true if any edge is
// still pending.  Both lanes of a pair read the same edge and state, so they
// follow the same path up to the exchange of their results.  Each lane of
// the first kBlockMemo edges remembers the edge that blocked it (memo, in
// LDS, -1 for none): while that edge is still pending the test is settled
// by one load, and the one-ring is searched again only once it is done.
constexpr int kBlockMemo = 4096;
__device__ bool select_edges(const SmoothArgs& S, int32_t i0, int32_t stride, int32_t* memo) {
  const RoughArgs& A = S.R;
  const int32_t n = min(A.counters[C_RFLAG], 3 * A.nt);
  const int side = i0 & 1;
  bool pending = false;
  for (int32_t i = i0 >> 1; i < n; i += stride >> 1) {
    const int32_t h = S.elist[i];
    if (S.estate[h] != E_PENDING) continue;
    pending = true;
    const bool kept = i < kBlockMemo;
    int32_t bf = kept ? memo[2 * i + side] : -1;
    if (bf >= 0 && S.estate[bf] != E_PENDING) bf = -1;
    if (bf < 0) {
      int32_t a, b;
      edge_ends(A, h, a, b);
      const int32_t v = side ? b : a;
      bf = blocker_at(S, v, h);
      for (int32_t e = A.vt_off[v]; bf < 0 && e < A.vt_off[v + 1]; ++e) {
        const int4 c = A.tri4[A.vt_ids[e]];
        bf = blocker_at(S, corner(c, (corner_of(c, v) + 1) % 3), h);
      }
    }
    if (kept) memo[2 * i + side] = bf;
    bool blocked = bf >= 0;
    blocked = (__shfl_xor((int)blocked, 1, 64) != 0) || blocked;
    // the decision reads only pending states, so selections within the
    // round cannot change it; they are marked after the round's reads
    if (!blocked && side == 0) S.elist[i] = h | INT32_MIN;
  }
  return pending;
}

// Sum of the one-ring positions of v without w, the ring size, and A_v, in
// list order; the fan read kFanBatch incidences at a time, each level of
// loads (list entries, triangle records, positions) issued together.
__device__ inline void ring_sums(const RoughArgs& A, int32_t v, int32_t w, D3& s, int32_t& n, D3& Av) {
  const D3 xv = pos(A, v);
  s = D3{0.0, 0.0, 0.0};
  Av = D3{0.0, 0.0, 0.0};
  const int32_t e0 = A.vt_off[v], e1 = A.vt_off[v + 1];
  n = e1 - e0;
  for (int32_t b = e0; b < e1; b += kFanBatch) {
    int32_t t[kFanBatch];
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j) t[j] = b + j < e1 ? A.vt_ids[b + j] : -1;
    int4 c[kFanBatch];
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j) c[j] = t[j] >= 0 ? A.tri4[t[j]] : make_int4(v, v, v, 0);
    D3 xp[kFanBatch], xq[kFanBatch];
    int32_t p[kFanBatch];
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j) {
      const int k = corner_of(c[j], v);
      p[j] = corner(c[j], (k + 1) % 3);
      xp[j] = pos(A, p[j]);
      xq[j] = pos(A, corner(c[j], (k + 2) % 3));
    }
#pragma unroll
    for (int j = 0; j < kFanBatch; ++j) {
      if (t[j] < 0) continue;
      if (p[j] != w) s = add(s, xp[j]);
      Av = add(Av, cross(sub(xp[j], xv), sub(xq[j], xv)));
    }
  }
}

// One round's moves of the selected edges i0, i0 + stride, ...
// One round's moves of the selected edges, a pair of adjacent lanes per edge
// as in select_edges: the even lane sums the one-ring of a and finds the
// triangle holding b -> a, the odd lane sums the one-ring of b; they swap
// their sums, both compute the same move, and each writes its own end.
__device__ inline double swap_pair(double v) { return __shfl_xor(v, 1, 64); }

__device__ void apply_edges(const SmoothArgs& S, double* xo, double* yo, double* zo, int32_t i0, int32_t stride) {
  const RoughArgs& A = S.R;
  const int32_t n = min(A.counters[C_RFLAG], 3 * A.nt);
  const int side = i0 & 1;
  for (int32_t i = i0 >> 1; i < n; i += stride >> 1) {
    const int32_t tag = S.elist[i];
    if (tag >= 0) continue;
    const int32_t h = tag & INT32_MAX;
    int32_t a, b;
    edge_ends(A, h, a, b);
    D3 Sm, Am;
    int32_t nm;
    ring_sums(A, side ? b : a, side ? a : b, Sm, nm, Am);
    const int32_t tb_mine = side ? 0 : twin_in_fan(A, a, b);
    const D3 So{swap_pair(Sm.x), swap_pair(Sm.y), swap_pair(Sm.z)};
    const D3 Ao{swap_pair(Am.x), swap_pair(Am.y), swap_pair(Am.z)};
    const int32_t no = __shfl_xor(nm, 1, 64);
    const int32_t tb_other = __shfl_xor(tb_mine, 1, 64);  // every exchange runs on both lanes
    const int32_t tb = side ? tb_other : tb_mine;
    const D3 S1 = side ? So : Sm, A1 = side ? Ao : Am, S2 = side ? Sm : So, A2 = side ? Am : Ao;
    const int32_t n1 = side ? no : nm, n2 = side ? nm : no;
    if (side == 0) {
      S.elist[i] = h;
      S.estate[h] = E_DONE;
    }
    const D3 x1s = scale(add(S2, scale(S1, (double)n2)), 1.0 / (double)(n1 * n2 - 1));
    const D3 x2s = scale(add(x1s, S2), 1.0 / (double)n2);
    const D3 xa = pos(A, a), xb = pos(A, b);
    const D3 d1 = sub(x1s, xa), d2 = sub(x2s, xb);
    // far corners: of the triangle holding a -> b, and of the one holding b -> a
    if (tb < 0) continue;  // no twin: an open front, left alone
    const int4 ct = A.tri4[h / 3];
    const int32_t ya = corner(ct, (h % 3 + 2) % 3);
    const int4 cb = A.tri4[tb];
    const int32_t yb = corner(cb, (corner_of(cb, a) + 1) % 3);
    const D3 yv = sub(pos(A, ya), pos(A, yb));
    const D3 g = add(add(A1, A2), cross(yv, sub(d1, d2)));
    const double gg = dot(g, g);
    if (!(gg > 0.0)) continue;
    const double c = dot(d1, A1) + dot(d2, A2) + dot(d1, cross(d2, yv));
    const D3 step = scale(g, -c / gg);
    const D3 p = side ? add(x2s, step) : add(x1s, step);
    const int32_t v = side ? b : a;
    xo[v] = p.x;
    yo[v] = p.y;
    zo[v] = p.z;
    if (side == 0) atomicAdd(&A.counters[C_RMOVED], 1);
  }
}

// All rounds in one workgroup (the flagged edges are few: local roughness):
// select, barrier, move, barrier, until a round finds nothing pending or
// max_rounds is reached.  Every thread takes the same number of rounds (the
// flag is read after a barrier), so every barrier is reached by all.
constexpr int kRoundT = 1024;
__global__ __launch_bounds__(kRoundT) void k_rounds(SmoothArgs S, double* xo, double* yo, double* zo,
                                                    int32_t max_rounds) {
  __shared__ int32_t pending;
  __shared__ int32_t memo[2 * kBlockMemo];
  for (int32_t i = threadIdx.x; i < 2 * kBlockMemo; i += blockDim.x) memo[i] = -1;
  for (int32_t r = 0; r < max_rounds; ++r) {
    if (threadIdx.x == 0) pending = 0;
    __syncthreads();
    if (select_edges(S, threadIdx.x, blockDim.x, memo)) atomicOr(&pending, 1);
    __syncthreads();
    if (pending == 0) break;
    apply_edges(S, xo, yo, zo, threadIdx.x, blockDim.x);
    __syncthreads();
  }
}

// Count of edges still pending after the rounds.
__global__ void k_smooth_end(SmoothArgs S, int32_t* d_counts) {
  __shared__ int32_t part[kT];
  const RoughArgs& A = S.R;
  const int32_t n = min(A.counters[C_RFLAG], 3 * A.nt);
  int32_t left = 0;
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) left += S.estate[S.elist[i] & INT32_MAX] == E_PENDING ? 1 : 0;
  part[threadIdx.x] = left;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d_counts[0] = n;
    d_counts[1] = A.counters[C_RMOVED];
    d_counts[2] = part[0];
  }
}

RoughArgs rough_args(const ftc_cells* ws, const Mesh& m, const double* x, const double* y, const double* z) {
  RoughArgs A;
  A.nv = m.nv;
  A.nt = m.nt;
  A.tri4 = reinterpret_cast<const int4*>(ws->tri4);
  A.vt_off = ws->vt_off;
  A.vt_ids = ws->vt_ids;
  A.x = x;
  A.y = y;
  A.z = z;
  A.tn = reinterpret_cast<double4*>(ws->r_tn);
  A.vG = ws->r_vG;
  A.vV = ws->r_vV;
  A.rt = ws->r_rt;
  A.counters = ws->counters;
  return A;
}

}  // namespace

hipError_t launch_roughness(const ftc_cells* ws, const Mesh& m, double* gl_mag, double* rough, hipStream_t s) {
  RoughArgs A = rough_args(ws, m, m.x, m.y, m.z);
  hipLaunchKernelGGL(k_tri_normals, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, A);
  hipLaunchKernelGGL(k_vertex_stats, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, A, gl_mag);
  hipLaunchKernelGGL(k_tri_rt, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, A);
  hipLaunchKernelGGL(k_vertex_rough, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, A, rough);
  return hipGetLastError();
}

hipError_t launch_smooth(const ftc_cells* ws, const Mesh& m, const double* gl_mag, const double* rough, double gl_thr,
                         double rough_thr, int32_t max_rounds, double* xo, double* yo, double* zo, int32_t* d_counts,
                         hipStream_t s) {
  SmoothArgs S;
  S.R = rough_args(ws, m, xo, yo, zo);
  S.gl_mag = gl_mag;
  S.rough = rough;
  S.gl_thr = gl_thr;
  S.rough_thr = rough_thr;
  S.vflag = ws->r_vflag;
  S.estate = ws->r_estate;
  S.elist = ws->r_elist;
  hipLaunchKernelGGL(k_smooth_begin, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, m.x, m.y, m.z, xo, yo, zo, m.nv,
                     ws->counters);
  hipLaunchKernelGGL(k_vertex_flags, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, S);
  hipLaunchKernelGGL(k_edge_flags, dim3(grid_blocks(3 * (int64_t)m.nt, kT)), dim3(kT), 0, s, S);
  if (max_rounds > 0) hipLaunchKernelGGL(k_rounds, dim3(1), dim3(kRoundT), 0, s, S, xo, yo, zo, max_rounds);
  hipLaunchKernelGGL(k_smooth_end, dim3(1), dim3(kT), 0, s, S, d_counts);
  return hipGetLastError();
}

}  // namespace ftc
