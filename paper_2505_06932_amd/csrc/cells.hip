// cells.hip -- interfacial-cell lists (triangle -> cell binning) and the
// per-piece integrals the volume fraction needs.
//
// 1. per triangle (k_tri_classify): decide every cell of its bounding box
//    from the corners alone where the clipping would cut nothing (no piece,
//    or the whole triangle); queue the others; then per queued candidate
//    (k_clip_queue): full clipping.  Every piece of positive area sets its
//    cell's bit in a grid-sized occupancy bitmap and is appended, with its
//    two z-column integrals, to a pair list (one atomic allocation per
//    workgroup; queued candidates keep their queue slot);
// 2. popcount prefix sums of the bitmap, listing the interfacial cells in
//    ascending linear id on the way -> the compact index (rank) of every
//    cell;
// 3. per pair: compact cell index and a count per cell; prefix sums of the
//    counts -> CSR offsets;
// 4. scatter the pairs into their cell's segment (any order), then place
//    each at its rank by triangle id within the segment, so that the CSR
//    lists come out in ascending triangle id whatever the scheduling was.
// The same launches also prepare what the curvature fit needs from the
// front, as extra work beside the pieces: each vertex's incident triangles
// (counted while clearing, grouped in step 4, sorted ascending afterwards), the
// vertices binned by the interfacial cell holding them (counted in step 3,
// grouped in step 4) and, from those bins, the closest vertex of every
// interfacial cell.  Per-vertex and per-cell counts are zero between builds:
// the prefix sums clear them as they read them, and each counted entry keeps
// the index its count gave it, so the grouping needs no atomics.
// After step 1 everything is integer work on device-resident counts, so the
// sequence needs no host round trip and can be captured into a graph.
#include <float.h>
#include <limits.h>

#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 2048;
constexpr int kPieceLanes = 64;  // k_clip_queue: one wavefront per workgroup

// Corner r of triangle t if it is a valid vertex index distinct from the
// triangle's earlier corners, else -1 (a triangle is listed once under each
// distinct corner).
__device__ inline int32_t distinct_corner(const Mesh& m, int32_t t, int r) {
  if (!tri_ok(m, t)) return -1;
  const int32_t a = m.t0[t];
  if (r == 0) return a;
  const int32_t b = m.t1[t];
  if (r == 1) return b != a ? b : -1;
  const int32_t c = m.t2[t];
  return (c != a && c != b) ? c : -1;
}

// Clears the per-build state, packs the vertex coordinates as (x, y, z, 0)
// and counts each vertex's incident triangles (one thread per corner, which
// keeps its index within the vertex's list).
__global__ void k_clear_build(uint32_t* bitmap, int64_t nwords, int32_t* cell_cnt, int64_t ncnt, int32_t* counters,
                              Mesh m, double2* vtx4, int32_t* vt_cnt, int32_t* vt_loc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = g0; x < 3 * (int64_t)m.nt; x += stride) {
    const int32_t v = distinct_corner(m, (int32_t)(x / 3), (int)(x % 3));
    if (v >= 0) vt_loc[x] = atomicAdd(&vt_cnt[v], 1);
  }
  for (int64_t v = g0; v < m.nv; v += stride) {
    vtx4[2 * v] = make_double2(m.x[v], m.y[v]);
    vtx4[2 * v + 1] = make_double2(m.z[v], 0.0);
  }
  for (int64_t i = g0; i < nwords; i += stride) bitmap[i] = 0u;
  for (int64_t i = g0; i < ncnt; i += stride) cell_cnt[i] = 0;
  if (g0 < C_COUNT && g0 != C_ERR) counters[g0] = 0;
}

struct PairOut {
  int32_t* lin;
  int32_t* tri;
  double* flux;
  double* vol;
  int64_t cap;
};

// Block-wide exclusive prefix of `v` and one atomic allocation of the
// block's total on *counter (same-address atomics serialise across the chip,
// so there is one per workgroup); returns this thread's first index.
template <int NT>
__device__ inline int64_t block_alloc(int32_t v, int32_t* counter, int32_t* sh) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) sh[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int w = 0; w < NW; ++w) {
      const int32_t t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[NW] = run > 0 ? atomicAdd(counter, run) : 0;
  }
  __syncthreads();
  const int64_t r = (int64_t)sh[NW] + sh[wid] + incl - v;
  __syncthreads();
  return r;
}

// Per triangle: classify every candidate cell; whole-triangle pieces go
// straight to the first region of the pair list, candidates that need
// clipping to the second (the clipping queue).  Two passes over the cheap
// classification: count, allocate, write.  A workgroup's queued candidates
// are written grouped by the set of cell planes their triangle crosses, so
// that the wavefronts of the clipping mostly take the same branches.
constexpr int kClassifyT = 512;
__global__ __launch_bounds__(kClassifyT) void k_tri_classify(Grid g, Mesh m, const double2* vtx4, int4* tri4,
                                                             uint32_t* bitmap, PairOut P, int64_t q_cap,
                                                             int32_t* counters) {
  __shared__ int32_t sh[kClassifyT / 64 + 1];
  __shared__ int32_t qoff[64];  // queued candidates per crossing mask, then their offsets
  __shared__ int32_t qbase;
  if (threadIdx.x < 64) qoff[threadIdx.x] = 0;
  __syncthreads();
  const int32_t t = blockIdx.x * kClassifyT + threadIdx.x;
  bool valid = t < m.nt;
  if (valid) {
    const int32_t a = m.t0[t], b = m.t1[t], c = m.t2[t];
    if (a >= 0 && b >= 0 && c >= 0 && a < m.nv && b < m.nv && c < m.nv) {
      tri4[t] = make_int4(a, b, c, 0);
    } else {
      tri4[t] = make_int4(0, 0, 0, 0);
      atomicOr(&counters[C_ERR], ERR_MESH);
      valid = false;
    }
  }
  Tri T;
  int64_t lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
  if (valid) {
    T = load_tri_packed(tri4, vtx4, t);
    bool ok = true;
#pragma unroll
    for (int r = 0; r < 3; ++r) ok = ok && in_margin(g, T.v[r][0], T.v[r][1], T.v[r][2]);
    if (!ok) {
      atomicOr(&counters[C_ERR], ERR_DOMAIN);
    } else {
      tri_range(g, T, lo, hi);
    }
  }
  int32_t n1 = 0, n2 = 0;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i) {
        const int cls = classify_candidate(g, T, i, j, k);
        if (cls == 1) {
          if (whole_piece(T, grid_plane(g.z0, k, g.h)).keep) {
            const int64_t lin = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
            atomicOr(&bitmap[lin >> 5], 1u << (lin & 31));
            ++n1;
          }
        } else if (cls == 2) {
          atomicAdd(&qoff[crossing_mask(g, T, i, j, k)], 1);
          ++n2;
        }
      }
  int64_t p = block_alloc<kClassifyT>(n1, &counters[C_NWHOLE], sh);
  if (threadIdx.x < 64) {
    // offsets of the mask groups and one allocation for the workgroup
    const int32_t v = qoff[threadIdx.x];
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t o = __shfl_up(incl, d, 64);
      if ((int)threadIdx.x >= d) incl += o;
    }
    qoff[threadIdx.x] = incl - v;
    if (threadIdx.x == 63) qbase = incl > 0 ? atomicAdd(&counters[C_NQUEUE], incl) : 0;
  }
  __syncthreads();
  if (n1 + n2 == 0) return;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i) {
        const int cls = classify_candidate(g, T, i, j, k);
        const int64_t lin = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        if (cls == 1) {
          const Piece pc = whole_piece(T, grid_plane(g.z0, k, g.h));
          if (pc.keep) {
            if (p < P.cap) {
              P.lin[p] = (int32_t)lin;
              P.tri[p] = t;
              P.flux[p] = pc.flux;
              P.vol[p] = pc.vol;
            } else {
              atomicOr(&counters[C_ERR], ERR_CAPACITY);
            }
            ++p;
          }
        } else if (cls == 2) {
          const int64_t q = (int64_t)qbase + atomicAdd(&qoff[crossing_mask(g, T, i, j, k)], 1);
          if (q < q_cap) {
            P.lin[P.cap + q] = (int32_t)lin;
            P.tri[P.cap + q] = t;
          } else {
            atomicOr(&counters[C_ERR], ERR_CAPACITY);
          }
        }
      }
}

// Per queued candidate (second region of the pair list): full clipping; the
// result stays in the candidate's slot, with cell -1 when there is no piece.
__global__ __launch_bounds__(kPieceLanes) void k_clip_queue(Grid g, const int4* tri4, const double2* vtx4, PairOut P,
                                                            int64_t q_cap, uint32_t* bitmap, const int32_t* counters) {
  __shared__ PolyLDS<kPieceLanes> L;
  const int lane = threadIdx.x;
  const int64_t nq = min((int64_t)counters[C_NQUEUE], q_cap);
  for (int64_t base = (int64_t)blockIdx.x * kPieceLanes; base < nq; base += (int64_t)gridDim.x * kPieceLanes) {
    const int64_t q = base + lane;
    if (q < nq) {
      const int64_t slot = P.cap + q;
      const int32_t lin = P.lin[slot];
      const Cell3 c = unpack_cell(g, lin);
      const Tri T = load_tri_packed(tri4, vtx4, P.tri[slot]);
      const Piece pc = clip_piece(g, T, c.i, c.j, c.k, L, lane, inside_mask(g, T, c.i, c.j, c.k));
      if (pc.keep) {
        atomicOr(&bitmap[lin >> 5], 1u << (lin & 31));
        P.flux[slot] = pc.flux;
        P.vol[slot] = pc.vol;
      } else {
        P.lin[slot] = -1;
      }
    }
  }
}


__device__ inline int32_t rank_of(const uint32_t* bitmap, const int32_t* word_off, int64_t lin) {
  const uint32_t w = bitmap[lin >> 5];
  const uint32_t below = (lin & 31) ? (w & ((1u << (lin & 31)) - 1u)) : 0u;
  return word_off[lin >> 5] + __popc(below);
}

// The pair list has two regions: [0, n1) whole-triangle pieces and
// [cap, cap + nq) clipped candidates (cell -1 when there was no piece).
struct PairRange {
  int64_t n1, nq, cap;
  __device__ int64_t count() const { return n1 + nq; }
  __device__ int64_t slot(int64_t idx) const { return idx < n1 ? idx : cap + (idx - n1); }
};
__device__ inline PairRange pair_range(const int32_t* counters, int64_t pair_cap, int64_t queue_cap) {
  return PairRange{min((int64_t)counters[C_NWHOLE], pair_cap), min((int64_t)counters[C_NQUEUE], queue_cap),
                   pair_cap};
}

struct VertexBins {
  int32_t nv;
  const double2* vtx4;
  int32_t* vcell;   // interfacial cell of each vertex; -1: a cell without pieces (a stray), -2: outside the margin
  int32_t* vb_cnt;  // vertices per interfacial cell
  int32_t* vb_loc;  // index of each vertex within its cell's bin
  int32_t* stray;
};

// pair -> compact cell (in place of its linear id), counted per cell, its
// index within the cell kept; and vertex -> the interfacial cell holding it,
// counted per cell with its index kept (or listed as a stray)
__global__ void k_pair_count(int32_t* pair_lin, int32_t* pair_local, const uint32_t* bitmap, const int32_t* word_off,
                             int32_t* cell_cnt, int32_t cell_cap, int64_t pair_cap, int64_t queue_cap,
                             int32_t* counters, Grid g, VertexBins B) {
  const PairRange R = pair_range(counters, pair_cap, queue_cap);
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < B.nv; v += gridDim.x * blockDim.x) {
    const P3 p = vtx(B.vtx4, v);
    int32_t ci = -2;
    if (in_margin(g, p.x, p.y, p.z)) {
      const int64_t i = cell_index(p.x, g.x0, g.h), j = cell_index(p.y, g.y0, g.h), k = cell_index(p.z, g.z0, g.h);
      ci = cell_rank(bitmap, word_off, i + (int64_t)g.nx * (j + (int64_t)g.ny * k));
      if (ci >= cell_cap) ci = -1;
      if (ci >= 0)
        B.vb_loc[v] = atomicAdd(&B.vb_cnt[ci], 1);
      else
        B.stray[atomicAdd(&counters[C_NSTRAY], 1)] = v;
    }
    B.vcell[v] = ci;
  }
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < R.count(); x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = R.slot(x);
    const int32_t lin = pair_lin[p];
    if (lin < 0) continue;
    const int32_t ci = rank_of(bitmap, word_off, lin);
    if (ci < cell_cap) {
      pair_lin[p] = ci;
      pair_local[p] = atomicAdd(&cell_cnt[ci], 1);
    } else {
      pair_lin[p] = -1;  // its cell did not fit the capacity (latched while listing the cells)
    }
  }
}

struct Adjacency {
  const int32_t* vt_off;
  const int32_t* vt_loc;
  int32_t* vt_ids;
  const int32_t* vcell;
  const int32_t* vb_off;
  const int32_t* vb_loc;
  int32_t* vb_ids;
};

// Pairs into their cell's segment, triangles into each distinct corner's
// incident list and vertices into their cell's bin, each at the index the
// counting gave it (an arbitrary order, fixed afterwards where it matters).
__global__ void k_pair_scatter(const int32_t* pair_ci, const int32_t* pair_tri, const int32_t* pair_local,
                               const int32_t* offsets, int32_t* tmp_tri, int32_t* tmp_pair, int64_t pair_cap,
                               int64_t queue_cap, int32_t* counters, Mesh m, Adjacency J) {
  const PairRange R = pair_range(counters, pair_cap, queue_cap);
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < 3 * (int64_t)m.nt;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = (int32_t)(x / 3);
    const int32_t v = distinct_corner(m, t, (int)(x % 3));
    if (v >= 0) J.vt_ids[J.vt_off[v] + J.vt_loc[x]] = t;
  }
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < m.nv; v += gridDim.x * blockDim.x) {
    const int32_t ci = J.vcell[v];
    if (ci >= 0) J.vb_ids[J.vb_off[ci] + J.vb_loc[v]] = v;
  }
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < R.count(); x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = R.slot(x);
    const int32_t ci = pair_ci[p];
    if (ci < 0) continue;
    const int64_t pos = (int64_t)offsets[ci] + pair_local[p];
    if (pos < pair_cap) {
      tmp_tri[pos] = pair_tri[p];
      tmp_pair[pos] = (int32_t)p;
    } else {
      atomicOr(&counters[C_ERR], ERR_CAPACITY);
    }
  }
}

struct PlaceArgs {
  const int32_t *tmp_tri, *tmp_pair, *pair_ci;
  const double *pair_flux, *pair_vol;
  const int32_t* offsets;
  int32_t *tri_ids, *slot_cell;
  double *piece_flux, *piece_vol;
  int32_t cell_cap;
  int64_t pair_cap;
  const int32_t* counters;
};

constexpr int kSegReg = 16;  // segment entries read in one batch of loads

// Each scattered piece moves to its rank by triangle id within its cell (a
// triangle has at most one piece per cell, so the ranks are distinct): one
// thread per piece counts the smaller triangle ids of its segment, read
// kSegReg at a time with the loads of a batch issued together.
__device__ inline void rank_place(const PlaceArgs& A, int64_t bid, int64_t nblk) {
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  const int64_t nslot = min((int64_t)A.offsets[nif], A.pair_cap);
  for (int64_t q = bid * blockDim.x + threadIdx.x; q < nslot; q += nblk * blockDim.x) {
    const int32_t p = A.tmp_pair[q];
    const int32_t ci = A.pair_ci[p];
    const int32_t t = A.tmp_tri[q];
    const int64_t s = A.offsets[ci], e = min((int64_t)A.offsets[ci + 1], A.pair_cap);
    int64_t rank = 0;
    for (int64_t b = s; b < e; b += kSegReg) {
      int32_t seg[kSegReg];
#pragma unroll
      for (int u = 0; u < kSegReg; ++u) seg[u] = b + u < e ? A.tmp_tri[b + u] : INT_MAX;
#pragma unroll
      for (int u = 0; u < kSegReg; ++u) rank += seg[u] < t ? 1 : 0;
    }
    const int64_t dst = s + rank;
    A.tri_ids[dst] = t;
    A.slot_cell[dst] = ci;
    A.piece_flux[dst] = A.pair_flux[p];
    A.piece_vol[dst] = A.pair_vol[p];
  }
}

constexpr int kSortReg = 8;  // incident lists up to this length are sorted in registers

// Vertex v's incident-triangle list sorted ascending.
__device__ inline void sort_incident(const int32_t* vt_off, int32_t* vt_ids, int32_t v) {
  const int32_t s = vt_off[v], e = vt_off[v + 1];
  if (e - s <= kSortReg) {
    // in registers: odd-even transposition sort, padding at the end
    int32_t x[kSortReg];
#pragma unroll
    for (int q = 0; q < kSortReg; ++q) x[q] = s + q < e ? vt_ids[s + q] : INT_MAX;
#pragma unroll
    for (int pass = 0; pass < kSortReg; ++pass)
#pragma unroll
      for (int q = pass & 1; q + 1 < kSortReg; q += 2) {
        const int32_t lo = min(x[q], x[q + 1]), hi = max(x[q], x[q + 1]);
        x[q] = lo;
        x[q + 1] = hi;
      }
#pragma unroll
    for (int q = 0; q < kSortReg; ++q)
      if (s + q < e) vt_ids[s + q] = x[q];
    return;
  }
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

struct VstarArgs {
  const double2* vtx4;
  const int32_t* cell_ids;
  const uint32_t* bitmap;
  const int32_t* word_off;
  const int32_t *vb_off, *vb_ids, *stray;
  double* best_d2;
  int32_t* best_v;
  int32_t cell_cap;
  const int32_t* counters;
};

// Closest vertex of each interfacial cell among the vertices binned in the
// 3x3x3 block of cells around it and the strays: 32 lanes per cell, lane
// l < 27 scans the bin of cell l of the block, every lane a share of the
// strays; lowest index on ties.  A vertex outside the block is at least
// 1.5 h from the cell centre, so a best squared distance below (1.5 h)^2 is
// final (the curvature's ring pass searches all vertices for the other
// cells).
// Called with all 64 lanes of the wavefront.
__device__ inline void closest_vertex(const Grid& g, const VstarArgs& A, int64_t gid) {
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  const int32_t nstray = A.counters[C_NSTRAY];
  const int64_t c = gid >> 5;
  const int l = (int)(gid & 31);
  double bd = DBL_MAX;
  int32_t bv = INT_MAX;
  if (c < nif) {
    const Cell3 cc = unpack_cell(g, A.cell_ids[c]);
    const double xc[3] = {cell_centre(g.x0, cc.i, g.h), cell_centre(g.y0, cc.j, g.h), cell_centre(g.z0, cc.k, g.h)};
    if (l < 27) {
      const int32_t ii = cc.i + l % 3 - 1, jj = cc.j + (l / 3) % 3 - 1, kk = cc.k + l / 9 - 1;
      if (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz) {
        const int32_t cr = cell_rank(A.bitmap, A.word_off, ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk));
        if (cr >= 0 && cr < A.cell_cap) {
          // the first few of the bin in one batch of loads (the result does
          // not depend on the order)
          const int32_t p0 = A.vb_off[cr], p1 = A.vb_off[cr + 1];
          int32_t vid[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) vid[u] = p0 + u < p1 ? A.vb_ids[p0 + u] : -1;
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (vid[u] >= 0) consider(A.vtx4, vid[u], xc, bd, bv);
          for (int32_t p = p0 + 4; p < p1; ++p) consider(A.vtx4, A.vb_ids[p], xc, bd, bv);
        }
      }
    }
    for (int32_t q = l; q < nstray; q += 32) consider(A.vtx4, A.stray[q], xc, bd, bv);
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
    A.best_d2[c] = bd;
    A.best_v[c] = bv;
  }
}

// Blocks [0, nb_place): pieces to their ranks; [nb_place, nb_place +
// nb_sort): one vertex per thread, its incident list sorted; the rest:
// closest vertices.
__global__ __launch_bounds__(kT) void k_place_sort_vstar(PlaceArgs A, int32_t nb_place, int32_t nb_sort, Grid g,
                                                         int32_t nv, const int32_t* vt_off, int32_t* vt_ids,
                                                         VstarArgs V) {
  const int32_t b = blockIdx.x;
  if (b < nb_place) {
    rank_place(A, b, nb_place);
  } else if (b < nb_place + nb_sort) {
    const int32_t v = (b - nb_place) * kT + threadIdx.x;
    if (v < nv) sort_incident(vt_off, vt_ids, v);
  } else {
    closest_vertex(g, V, (int64_t)(b - nb_place - nb_sort) * kT + threadIdx.x);
  }
}

}  // namespace

hipError_t launch_cell_lists(ftc_cells* ws, const Mesh& m, hipStream_t s) {
  const Grid& g = ws->grid;
  int4* tri4 = reinterpret_cast<int4*>(ws->tri4);
  double2* vtx4 = reinterpret_cast<double2*>(ws->vtx4);
  hipLaunchKernelGGL(k_clear_build, dim3(kStrideBlocks), dim3(kT), 0, s, ws->bitmap, ws->nwords, ws->offsets,
                     (int64_t)ws->cell_cap + 1, ws->counters, m, vtx4, ws->vt_cursor, ws->vt_loc);
  PairOut P{ws->pair_cell, ws->pair_tri, ws->pair_flux, ws->pair_vol, ws->pair_cap};
  time_start(ws, FTC_KERNEL_TRI_PIECES, s);
  hipLaunchKernelGGL(k_tri_classify, dim3(grid_blocks(m.nt, kClassifyT)), dim3(kClassifyT), 0, s, g, m, vtx4, tri4,
                     ws->bitmap, P, ws->queue_cap, ws->counters);
  hipLaunchKernelGGL(k_clip_queue, dim3(grid_blocks(ws->queue_cap, kPieceLanes, 8192)), dim3(kPieceLanes), 0, s, g,
                     tri4, vtx4, P, ws->queue_cap, ws->bitmap, ws->counters);
  time_stop(ws, FTC_KERNEL_TRI_PIECES, s);
  hipError_t e = scan_popcount_emit(ws->bitmap, ws->word_off, ws->nwords, ws->scan_tmp, ws->counters + C_NIF,
                                    ws->cell_ids, ws->cell_cap, ws->counters, s);
  if (e != hipSuccess) return e;
  const int64_t npair_max = ws->pair_cap + ws->queue_cap;
  VertexBins B{m.nv, vtx4, ws->vcell, ws->vb_cursor, ws->vb_loc, ws->stray};
  hipLaunchKernelGGL(k_pair_count, dim3(grid_blocks(npair_max, kT, kStrideBlocks)), dim3(kT), 0, s, ws->pair_cell,
                     ws->pair_local, ws->bitmap, ws->word_off, ws->offsets, ws->cell_cap, ws->pair_cap,
                     ws->queue_cap, ws->counters, g, B);
  const ScanSeg segs[3] = {{ws->offsets, ws->offsets, ws->cell_cap, ws->counters + C_NPAIRS, nullptr},
                           {ws->vt_cursor, ws->vt_off, m.nv, nullptr, ws->vt_cursor},
                           {ws->vb_cursor, ws->vb_off, ws->cell_cap, nullptr, ws->vb_cursor}};
  e = scan_exclusive_multi(segs, 3, ws->scan_tmp, s);
  if (e != hipSuccess) return e;
  Adjacency J{ws->vt_off, ws->vt_loc, ws->vt_ids, ws->vcell, ws->vb_off, ws->vb_loc, ws->vb_ids};
  hipLaunchKernelGGL(k_pair_scatter, dim3(grid_blocks(npair_max, kT, kStrideBlocks)), dim3(kT), 0, s, ws->pair_cell,
                     ws->pair_tri, ws->pair_local, ws->offsets, ws->tmp_tri, ws->tmp_pair, ws->pair_cap, ws->queue_cap,
                     ws->counters, m, J);
  PlaceArgs A{ws->tmp_tri,  ws->tmp_pair,  ws->pair_cell,  ws->pair_flux, ws->pair_vol, ws->offsets,
              ws->tri_ids,  ws->slot_cell, ws->piece_flux, ws->piece_vol, ws->cell_cap, ws->pair_cap,
              ws->counters};
  VstarArgs V{vtx4,       ws->cell_ids, ws->bitmap,  ws->word_off, ws->vb_off,  ws->vb_ids,
              ws->stray,  ws->best_d2,  ws->best_v,  ws->cell_cap, ws->counters};
  const int32_t nb_place = grid_blocks(ws->pair_cap, kT, kStrideBlocks);
  const int32_t nb_sort = grid_blocks(m.nv, kT);
  const int32_t nb_vstar = grid_blocks((int64_t)ws->cell_cap * 32, kT);
  time_start(ws, FTC_KERNEL_PIECE_RANK, s);
  hipLaunchKernelGGL(k_place_sort_vstar, dim3(nb_place + nb_sort + nb_vstar), dim3(kT), 0, s, A, nb_place, nb_sort, g,
                     m.nv, ws->vt_off, ws->vt_ids, V);
  time_stop(ws, FTC_KERNEL_PIECE_RANK, s);
  e = hipGetLastError();
  if (e == hipSuccess) {
    ws->built_nv = m.nv;
    ws->built_nt = m.nt;
    ++ws->builds;
  }
  return e;
}

}  // namespace ftc
