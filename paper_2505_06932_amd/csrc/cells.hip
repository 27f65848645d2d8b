// cells.hip -- interfacial-cell lists (triangle -> cell binning) and the
// per-piece integrals the volume fraction needs.
//
// 1. per triangle (k_tri_classify): decide every cell of its bounding box
//    from the corners alone where the clipping would cut nothing (no piece,
//    or the whole triangle); queue the others; then per queued candidate
//    (k_clip_mark): full clipping.  Every piece of positive area is appended,
//    with its two z-column integrals, to a pair list (one atomic allocation
//    per workgroup; queued candidates keep their queue slot) and sets its
//    cell's bit in a grid-sized occupancy bitmap;
// 2. popcount prefix sums of the bitmap, listing the interfacial cells in
//    ascending linear id on the way -> the compact index (rank) of every
//    cell;
// 3. per pair: compact cell index and a count per cell; prefix sums of the
//    counts -> CSR offsets;
// 4. scatter the pairs into their cell's segment (any order) as 32-byte
//    records carrying everything the next step needs, then place each at
//    its rank by triangle id within the segment, so that the CSR lists come
//    out in ascending triangle id whatever the scheduling was, and sum each
//    cell's piece integrals in that order (for the volume fraction).
// Lanes of one atomic instruction that hit the same address are served one
// after another, and neighbouring pieces, corners and vertices share cells,
// words and vertices: every count and every bitmap bit is taken with one
// atomic instruction per wavefront in which each distinct counter or word
// appears once (the lanes grouped by key beforehand, in an LDS hash for
// counts, by a loop over the few distinct words for bitmap bits).  Every walk over
// triangles, pairs, vertices or cells gives each XCD a contiguous share, so
// that the mesh records, bitmap words and list segments that neighbours
// share meet in one L2.
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

#include "dpp.hpp"
#include "ftc_ws.hpp"
#include "xcd.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 8192;  // grid of the clearing and pair walks: eight wavefronts per SIMD
constexpr int kPieceLanes = 64;  // k_clip_mark: one wavefront per workgroup
// k_clip_mark's polygon buffer: six corner slots per lane, enough for any
// candidate that cuts at most one plane of each axis, which keeps the buffer
// to 9 KB per wavefront (four wavefronts per SIMD).  A lane whose polygon
// outgrows them is clipped again with kMaxPoly slots, kWideLanes lanes at a
// time over the same memory.
constexpr int kFastPoly = 6;
constexpr int kWideLanes = kPieceLanes * kFastPoly / kMaxPoly;
union ClipLDS {
  PolyLDS<kPieceLanes, kFastPoly> fast;
  PolyLDS<kWideLanes, kMaxPoly> wide;
};
static_assert(sizeof(PolyLDS<kWideLanes, kMaxPoly>) <= sizeof(PolyLDS<kPieceLanes, kFastPoly>), "wide view fits");

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
// and counts each vertex's incident triangles (one lane per corner, which
// keeps its index within the vertex's list).
__global__ __launch_bounds__(kT) void k_clear_build(uint32_t* bitmap, int64_t nwords, int32_t* cell_cnt, int64_t ncnt,
                                                   int32_t* counters, Mesh m, double2* vtx4, int32_t* vt_cnt,
                                                   int32_t* vt_loc) {
  __shared__ CountLDS cl[kT / 64];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  XcdWalk(3 * (int64_t)m.nt, blockIdx.x, gridDim.x).run([&](int64_t x, bool ok) {
    const int32_t v = ok ? distinct_corner(m, (int32_t)(x / 3), (int)(x % 3)) : -1;
    const int32_t loc = wave_count_add(vt_cnt, v, v >= 0, cl[threadIdx.x >> 6]);
    if (v >= 0) vt_loc[x] = loc;
  });
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
  const int32_t incl = wave_incl_scan_dpp(v);
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
// that the wavefronts of the clipping mostly take the same branches.  768
// triangles per workgroup make those groups larger than 512 do while two
// workgroups still fit a CU at this kernel's register count (six wavefronts
// per SIMD); 1,024 would leave one.
constexpr int kClassifyT = 768;
__global__ __launch_bounds__(kClassifyT) void k_tri_classify(Grid g, Mesh m, const double2* vtx4, int4* tri4,
                                                             PairOut P, int64_t q_cap, int32_t* counters) {
  __shared__ int32_t sh[kClassifyT / 64 + 1];
  __shared__ int32_t qoff[64];  // queued candidates per crossing mask, then their offsets
  __shared__ int32_t qbase;
  if (threadIdx.x < 64) qoff[threadIdx.x] = 0;
  __syncthreads();
  // the XCDs take contiguous ranges of triangles (the grid is a multiple of kXCD)
  const int32_t lb = (blockIdx.x % kXCD) * (gridDim.x / kXCD) + blockIdx.x / kXCD;
  const int32_t t = lb * kClassifyT + threadIdx.x;
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
  // Whether a whole-triangle piece counts does not depend on the cell (the
  // vector area of the triangle itself).  The first pass keeps the class of
  // the first 32 candidates (2 bits each) and the crossing mask of the first
  // 8 (6 bits each) for the second.
  const bool tri_keep = valid && whole_piece(T, 0.0).keep;
  uint64_t cls_bits = 0u, mask_bits = 0u;
  int32_t n1 = 0, n2 = 0, idx = 0;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i, ++idx) {
        int cls = classify_candidate(g, T, i, j, k);
        if (cls == 1 && !tri_keep) cls = 0;
        if (idx < 32) cls_bits |= (uint64_t)cls << (2 * idx);
        if (cls == 1) {
          ++n1;
        } else if (cls == 2) {
          const uint32_t mk = crossing_mask(g, T, i, j, k);
          if (idx < 8) mask_bits |= (uint64_t)mk << (6 * idx);
          atomicAdd(&qoff[mk], 1);
          ++n2;
        }
      }
  int64_t p = block_alloc<kClassifyT>(n1, &counters[C_NWHOLE], sh);
  if (threadIdx.x < 64) {
    // offsets of the mask groups and one allocation for the workgroup
    const int32_t v = qoff[threadIdx.x];
    const int32_t incl = wave_incl_scan_dpp(v);
    qoff[threadIdx.x] = incl - v;
    if (threadIdx.x == 63) qbase = incl > 0 ? atomicAdd(&counters[C_NQUEUE], incl) : 0;
  }
  __syncthreads();
  if (n1 + n2 == 0) return;
  idx = 0;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i, ++idx) {
        int cls;
        if (idx < 32) {
          cls = (int)((cls_bits >> (2 * idx)) & 3u);
        } else {
          cls = classify_candidate(g, T, i, j, k);
          if (cls == 1 && !tri_keep) cls = 0;
        }
        const int64_t lin = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        if (cls == 1) {
          const Piece pc = whole_piece(T, grid_plane(g.z0, k, g.h));
          if (p < P.cap) {
            P.lin[p] = (int32_t)lin;
            P.tri[p] = t;
            P.flux[p] = pc.flux;
            P.vol[p] = pc.vol;
          } else {
            atomicOr(&counters[C_ERR], ERR_CAPACITY);
          }
          ++p;
        } else if (cls == 2) {
          const uint32_t mk = idx < 8 ? (uint32_t)((mask_bits >> (6 * idx)) & 63u) : crossing_mask(g, T, i, j, k);
          const int64_t q = (int64_t)qbase + atomicAdd(&qoff[mk], 1);
          if (q < q_cap) {
            P.lin[P.cap + q] = (int32_t)lin;
            P.tri[P.cap + q] = t;
          } else {
            atomicOr(&counters[C_ERR], ERR_CAPACITY);
          }
        }
      }
}

// Workgroups [0, nb_clip): per queued candidate (second region of the pair
// list), full clipping; the result stays in the candidate's slot, with cell
// -1 when there is no piece.  The others: the whole-triangle pieces (first
// region).  Both set the occupancy bits of their pieces' cells.
__global__ __launch_bounds__(kPieceLanes) __attribute__((amdgpu_waves_per_eu(4))) void k_clip_mark(Grid g, const int4* tri4, const double2* vtx4, PairOut P,
                                                           int64_t q_cap, uint32_t* bitmap, const int32_t* counters,
                                                           int32_t nb_clip) {
  __shared__ ClipLDS L;
  __shared__ uint32_t acc[kPieceLanes];
  const int lane = threadIdx.x;
  if ((int32_t)blockIdx.x < nb_clip) {
    const int64_t nq = min((int64_t)counters[C_NQUEUE], q_cap);
    XcdWalk(nq, blockIdx.x, nb_clip).run([&](int64_t q, bool ok) {
      const int64_t slot = P.cap + q;
      // the candidate's clip with the given buffer view; the lanes clipped
      // again reload it rather than keep it live across the first clip
      auto clip = [&](auto& view, int idx) {
        const Cell3 c = unpack_cell(g, P.lin[slot]);
        const Tri T = load_tri_packed(tri4, vtx4, P.tri[slot]);
        return clip_piece(g, T, c.i, c.j, c.k, view, idx, inside_mask(g, T, c.i, c.j, c.k));
      };
      Piece pc{false, 0.0, 0.0, false};
      if (ok) pc = clip(L.fast, lane);
      // lanes over the six slots: again with nine, ranked among themselves
      const bool again = pc.over_cap;
      const uint64_t redo = __ballot(again);
      if (redo) {
        const int r = __popcll(redo & ((1ull << lane) - 1ull));
        const int nr = __popcll(redo);
        for (int b = 0; b < nr; b += kWideLanes)
          if (again && r >= b && r < b + kWideLanes) pc = clip(L.wide, r - b);
      }
      int32_t lin = -1;
      if (ok) {
        if (pc.keep) {
          lin = P.lin[slot];
          P.flux[slot] = pc.flux;
          P.vol[slot] = pc.vol;
        } else {
          P.lin[slot] = -1;
        }
      }
      wave_set_bits(bitmap, lin >> 5, lin & 31, lin >= 0, acc);
    });
  } else {
    const int64_t n1 = min((int64_t)counters[C_NWHOLE], P.cap);
    XcdWalk(n1, blockIdx.x - nb_clip, gridDim.x - nb_clip).run([&](int64_t p, bool ok) {
      const int32_t lin = ok ? P.lin[p] : -1;
      wave_set_bits(bitmap, lin >> 5, lin & 31, lin >= 0, acc);
    });
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
__global__ __launch_bounds__(kT) void k_pair_count(int32_t* pair_lin, int32_t* pair_local, const uint32_t* bitmap,
                                                  const int32_t* word_off, int32_t* cell_cnt, int32_t cell_cap,
                                                  int64_t pair_cap, int64_t queue_cap, int32_t* counters, Grid g,
                                                  VertexBins B) {
  __shared__ CountLDS cl[kT / 64];
  CountLDS& L = cl[threadIdx.x >> 6];
  const PairRange R = pair_range(counters, pair_cap, queue_cap);
  XcdWalk(B.nv, blockIdx.x, gridDim.x).run([&](int64_t v, bool ok) {
    int32_t ci = -2;
    if (ok) {
      const P3 p = vtx(B.vtx4, (int32_t)v);
      if (in_margin(g, p.x, p.y, p.z)) {
        const int64_t i = cell_index(p.x, g.x0, g.h), j = cell_index(p.y, g.y0, g.h), k = cell_index(p.z, g.z0, g.h);
        ci = cell_rank(bitmap, word_off, i + (int64_t)g.nx * (j + (int64_t)g.ny * k));
        if (ci >= cell_cap) ci = -1;
      }
    }
    const int32_t loc = wave_count_add(B.vb_cnt, ci, ci >= 0, L);
    if (ok) {
      if (ci >= 0)
        B.vb_loc[v] = loc;
      else if (ci == -1)
        B.stray[atomicAdd(&counters[C_NSTRAY], 1)] = (int32_t)v;
      B.vcell[v] = ci;
    }
  });
  XcdWalk(R.count(), blockIdx.x, gridDim.x).run([&](int64_t x, bool ok) {
    const int64_t p = ok ? R.slot(x) : 0;
    const int32_t lin = ok ? pair_lin[p] : -1;
    int32_t ci = -1;
    if (lin >= 0) {
      ci = rank_of(bitmap, word_off, lin);
      if (ci >= cell_cap) ci = -1;  // its cell did not fit the capacity (latched while listing the cells)
    }
    const int32_t loc = wave_count_add(cell_cnt, ci, ci >= 0, L);
    if (lin >= 0) {
      pair_lin[p] = ci;
      if (ci >= 0) pair_local[p] = loc;
    }
  });
}

struct Adjacency {
  const int32_t* vt_off;
  const int32_t* vt_loc;
  int32_t* vt_ids;
  const int32_t* vcell;
  const int32_t* vb_off;
  const int32_t* vb_loc;
  const double2* vtx4;
  double2* vb_rec;  // per binned vertex: (x, y), (z, index as the bits of a double)
};

// Pairs into their cell's segment as records, triangles into each distinct
// corner's incident list and vertices into their cell's bin, each at the
// index the counting gave it (an arbitrary order, fixed afterwards where it
// matters).
__device__ inline void put_rec(double* rec, int64_t i, int32_t tri, int32_t ci, double flux, double vol) {
  *reinterpret_cast<int4*>(rec + 4 * i) = make_int4(tri, ci, 0, 0);
  *reinterpret_cast<double2*>(rec + 4 * i + 2) = make_double2(flux, vol);
}

__global__ __launch_bounds__(kT) void k_pair_scatter(const int32_t* pair_ci, const int32_t* pair_tri,
                                                    const double* pair_flux, const double* pair_vol,
                                                    const int32_t* pair_local, const int32_t* offsets, double* rec,
                                                    int64_t pair_cap, int64_t queue_cap, int32_t* counters, Mesh m,
                                                    Adjacency J) {
  const PairRange R = pair_range(counters, pair_cap, queue_cap);
  XcdWalk(3 * (int64_t)m.nt, blockIdx.x, gridDim.x).run([&](int64_t x, bool ok) {
    if (!ok) return;
    const int32_t t = (int32_t)(x / 3);
    const int32_t v = distinct_corner(m, t, (int)(x % 3));
    if (v >= 0) J.vt_ids[J.vt_off[v] + J.vt_loc[x]] = t;
  });
  XcdWalk(m.nv, blockIdx.x, gridDim.x).run([&](int64_t v, bool ok) {
    if (!ok) return;
    const int32_t ci = J.vcell[v];
    if (ci >= 0) {
      const int64_t pos = (int64_t)J.vb_off[ci] + J.vb_loc[v];
      J.vb_rec[2 * pos] = J.vtx4[2 * v];
      J.vb_rec[2 * pos + 1] = make_double2(J.vtx4[2 * v + 1].x, __longlong_as_double((long long)v));
    }
  });
  XcdWalk(R.count(), blockIdx.x, gridDim.x).run([&](int64_t x, bool ok) {
    if (!ok) return;
    const int64_t p = R.slot(x);
    const int32_t ci = pair_ci[p];
    if (ci < 0) return;
    const int64_t pos = (int64_t)offsets[ci] + pair_local[p];
    if (pos < pair_cap)
      put_rec(rec, pos, pair_tri[p], ci, pair_flux[p], pair_vol[p]);
    else
      atomicOr(&counters[C_ERR], ERR_CAPACITY);
  });
}

struct PlaceArgs {
  const double* rec;
  const int32_t* offsets;
  int32_t* tri_ids;
  double *piece_flux, *piece_vol;
  double *cell_flux, *cell_vol;
  int32_t cell_cap;
  int64_t pair_cap;
  const int32_t* counters;
};

constexpr int kSegReg = 16;  // segment entries read in one batch of loads (long segments)
constexpr int kPlLanes = 16;  // lanes per cell
constexpr int kPlCap = 64;    // segments up to this length are staged in LDS
constexpr int kPlPer = kPlCap / kPlLanes;

__device__ inline int32_t rec_tri(const double* rec, int32_t i) { return reinterpret_cast<const int32_t*>(rec + 4 * (int64_t)i)[0]; }

// Per interfacial cell, kPlLanes lanes: the cell's scattered pieces move to
// their ranks by triangle id within its segment (a triangle has at most one
// piece per cell, so the ranks are distinct), and the cell's two integrals
// are summed over the placed pieces in a fixed order: lane l takes entries
// l, l + kPlLanes, ..., then the lanes' sums are added pairwise.  Segments
// of up to kPlCap pieces are staged in LDS and ranked there; longer ones are
// ranked from global memory, kSegReg entries per batch of loads.  Every
// slot below the pieces' total holds a record: the positions of the counted
// pieces are exactly [0, total).
__device__ inline void place_sums(const PlaceArgs& A, int64_t group, int64_t ngroup) {
  __shared__ int32_t tri_s[kT / kPlLanes][kPlCap];
  __shared__ double fv_s[kT / kPlLanes][2][kPlCap];
  const int grp = threadIdx.x / kPlLanes;
  const int32_t nif = min(A.counters[C_NIF], A.cell_cap);
  XcdWalk((int64_t)nif * kPlLanes, group, ngroup).run([&](int64_t gid, bool ok) {
    const int64_t c = gid / kPlLanes;
    const int l = (int)(gid % kPlLanes);
    ok = ok && c < nif;
    const int32_t s = ok ? A.offsets[c] : 0;
    const int32_t e = ok ? (int32_t)min((int64_t)A.offsets[c + 1], A.pair_cap) : 0;
    const int32_t len = e - s;
    double f = 0.0, v = 0.0;
    if (len <= kPlCap) {
      int32_t t[kPlPer], rank[kPlPer];
      double fl[kPlPer], vo[kPlPer];
#pragma unroll
      for (int m = 0; m < kPlPer; ++m) {
        const int32_t q = l + m * kPlLanes;
        t[m] = INT_MAX;
        fl[m] = vo[m] = 0.0;
        rank[m] = 0;
        if (q < len) {
          const int4 hd = *reinterpret_cast<const int4*>(A.rec + 4 * (int64_t)(s + q));
          const double2 fv = *reinterpret_cast<const double2*>(A.rec + 4 * (int64_t)(s + q) + 2);
          t[m] = hd.x;
          fl[m] = fv.x;
          vo[m] = fv.y;
          tri_s[grp][q] = hd.x;
        }
      }
      __builtin_amdgcn_wave_barrier();
      for (int32_t j = 0; j < len; ++j) {
        const int32_t tj = tri_s[grp][j];
#pragma unroll
        for (int m = 0; m < kPlPer; ++m) rank[m] += tj < t[m] ? 1 : 0;
      }
#pragma unroll
      for (int m = 0; m < kPlPer; ++m)
        if (l + m * kPlLanes < len) {
          const int32_t dst = s + rank[m];
          A.tri_ids[dst] = t[m];
          A.piece_flux[dst] = fl[m];
          A.piece_vol[dst] = vo[m];
          fv_s[grp][0][rank[m]] = fl[m];
          fv_s[grp][1][rank[m]] = vo[m];
        }
      __builtin_amdgcn_wave_barrier();
      for (int32_t q = l; q < len; q += kPlLanes) {
        f += fv_s[grp][0][q];
        v += fv_s[grp][1][q];
      }
    } else {
      for (int32_t q = s + l; q < e; q += kPlLanes) {
        const int32_t tq = rec_tri(A.rec, q);
        const double2 fv = *reinterpret_cast<const double2*>(A.rec + 4 * (int64_t)q + 2);
        int32_t rank = 0;
        for (int32_t b = s; b < e; b += kSegReg) {
          int32_t seg[kSegReg];
#pragma unroll
          for (int u = 0; u < kSegReg; ++u) seg[u] = b + u < e ? rec_tri(A.rec, b + u) : INT_MAX;
#pragma unroll
          for (int u = 0; u < kSegReg; ++u) rank += seg[u] < tq ? 1 : 0;
        }
        A.tri_ids[s + rank] = tq;
        A.piece_flux[s + rank] = fv.x;
        A.piece_vol[s + rank] = fv.y;
      }
      __threadfence_block();  // the placed entries, written by the cell's other lanes
      for (int32_t q = s + l; q < e; q += kPlLanes) {
        f += A.piece_flux[q];
        v += A.piece_vol[q];
      }
    }
    // the lanes' sums added pairwise: rotations by 8, 4, 2 and 1 lanes pair
    // exactly the lanes of a butterfly over the 16, since after each step a
    // lane's value equals that of the lanes the finer steps reach
    static_assert(kPlLanes == 16, "one row of 16 lanes per cell");
    f += dpp_d<kDppRor + 8>(f);
    v += dpp_d<kDppRor + 8>(v);
    f += dpp_d<kDppRor + 4>(f);
    v += dpp_d<kDppRor + 4>(v);
    f += dpp_d<kDppRor + 2>(f);
    v += dpp_d<kDppRor + 2>(v);
    f += dpp_d<kDppRor + 1>(f);
    v += dpp_d<kDppRor + 1>(v);
    if (ok && l == 0) {
      A.cell_flux[c] = f;
      A.cell_vol[c] = v;
    }
  });
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
  const int32_t* vb_off;
  const double2* vb_rec;
  const int32_t* stray;
  double* best_d2;
  int32_t* best_v;
  const int32_t* vt_off;  // the vertices' incident-triangle offsets
  int2* best_inc;         // (offset, count) of best_v's incident triangles
  int32_t nv;
  int32_t cell_cap;
  const int32_t* counters;
};

// Closest vertex of each interfacial cell among the vertices binned in the
// 3x3x3 block of cells around it and the strays: kVsLanes lanes per cell,
// each taking kVsNb cells of the block in the order below; the loads of each
// level (bitmap words and their offsets, then bin bounds) are issued
// together for all of them, then the lane's bin entries, kVsBatch records
// (position and index) at a time; every lane a share of the strays; lowest
// index on ties.  A vertex outside the block is at least 1.5 h from the
// cell centre, so a best squared distance below (1.5 h)^2 is final (the
// curvature kernel searches all vertices for the other cells).
// The cell and its six face neighbours are searched first (the first block
// cell of lanes 0-6), then the cell's lanes take their minimum; a block
// cell with m non-zero offsets lies at least m (h/2)^2 (squared) from the
// centre, so the edge and corner neighbours are searched only where that
// bound, less a relative 1e-6 that covers the rounding of the binning and
// of the centre, does not exceed the best so far (a skipped bin holds no
// vertex that could win or tie).
// Called with all 64 lanes of the wavefront.
constexpr int kVsLanes = 8;                            // lanes per cell
constexpr int kVsNb = (27 + kVsLanes - 1) / kVsLanes;  // block cells per lane
constexpr int kVsBatch = 4;                            // bin records loaded together
// block cells n = (di + 1) + 3 (dj + 1) + 9 (dk + 1) in the order searched:
// the cell, its face, edge and corner neighbours
constexpr int kVsOrder[27] = {13, 4, 10, 12, 14, 16, 22, 1, 3, 5, 7, 9, 11, 15, 17, 19, 21, 23, 25, 0, 2, 6, 8, 18, 20, 24, 26};
// entries kVsLanes u .. kVsLanes u + 7 of the order, 5 bits each (31: none),
// so that lane l's block cell of slot u is a shift of a constant
constexpr uint64_t vs_slot(int u) {
  uint64_t v = 0;
  for (int l = 0; l < kVsLanes; ++l) {
    const int p = l + kVsLanes * u;
    v |= (uint64_t)(p < 27 ? kVsOrder[p] : 31) << (5 * l);
  }
  return v;
}
static_assert(kVsLanes == 8 && kVsOrder[0] == 13, "the cell and its face neighbours fill slot 0 of lanes 0-6");

// d^2 to xc of a binned vertex record, kept when it beats (bd, bv); the
// same arithmetic as consider().
__device__ inline void consider_rec(double2 r0, double2 r1, const double xc[3], double& bd, int32_t& bv) {
  const int32_t v = (int32_t)__double_as_longlong(r1.y);
  const double dx = r0.x - xc[0], dy = r0.y - xc[1], dz = r1.x - xc[2];
  const double d2 = dx * dx + dy * dy + dz * dz;
  if (lex_less(d2, v, bd, bv)) {
    bd = d2;
    bv = v;
  }
}

// The records of the lane's bins of slots [U0, U1) as one list: entry j is
// entry j - cum[u] of bin u.
template <int U0, int U1, int B = kVsBatch>
__device__ inline void scan_bins(const VstarArgs& A, const int32_t (&p0)[kVsNb], const int32_t (&cnt)[kVsNb],
                                 const double xc[3], double& bd, int32_t& bv) {
  int32_t cum[U1 - U0 + 1];
  cum[0] = 0;
#pragma unroll
  for (int u = U0; u < U1; ++u) cum[u - U0 + 1] = cum[u - U0] + cnt[u];
  for (int32_t j0 = 0; j0 < cum[U1 - U0]; j0 += B) {
    double2 r0[B], r1[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int32_t j = j0 + q;
      int32_t p = -1;
#pragma unroll
      for (int u = U0; u < U1; ++u)
        if (j >= cum[u - U0] && j < cum[u - U0 + 1]) p = p0[u] + (j - cum[u - U0]);
      if (p >= 0) {
        r0[q] = A.vb_rec[2 * (int64_t)p];
        r1[q] = A.vb_rec[2 * (int64_t)p + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (j0 + q < cum[U1 - U0]) consider_rec(r0[q], r1[q], xc, bd, bv);
  }
}

// The minimum over a cell's 8 lanes, in all of them (exact, so any pairing
// serves).
__device__ inline void vs_min8(double& bd, int32_t& bv) {
  static_assert(kVsLanes == 8, "8 lanes per cell");
  double od = dpp_d<kDppSwap1>(bd);
  int32_t ov = dpp_i<kDppSwap1>(bv);
  if (lex_less(od, ov, bd, bv)) {
    bd = od;
    bv = ov;
  }
  od = dpp_d<kDppSwap2>(bd);
  ov = dpp_i<kDppSwap2>(bv);
  if (lex_less(od, ov, bd, bv)) {
    bd = od;
    bv = ov;
  }
  od = dpp_d<kDppHalfMirror>(bd);
  ov = dpp_i<kDppHalfMirror>(bv);
  if (lex_less(od, ov, bd, bv)) {
    bd = od;
    bv = ov;
  }
}

__device__ inline void closest_vertex(const Grid& g, const VstarArgs& A, int32_t nif, int64_t gid, bool ok) {
  const int32_t nstray = A.counters[C_NSTRAY];
  const int64_t c = gid / kVsLanes;
  const int l = (int)(gid % kVsLanes);
  double bd = DBL_MAX;
  int32_t bv = INT_MAX;
  ok = ok && c < nif;
  double xc[3] = {0.0, 0.0, 0.0};
  int32_t p0[kVsNb], cnt[kVsNb];
  if (ok) {
    const Cell3 cc = unpack_cell(g, A.cell_ids[c]);
    xc[0] = cell_centre(g.x0, cc.i, g.h);
    xc[1] = cell_centre(g.y0, cc.j, g.h);
    xc[2] = cell_centre(g.z0, cc.k, g.h);
    int64_t wd[kVsNb];
    int sh[kVsNb];
    bool in[kVsNb];
#pragma unroll
    for (int u = 0; u < kVsNb; ++u) {
      const int n = (int)((vs_slot(u) >> (5 * l)) & 31u);
      const int di = n % 3 - 1, dj = (n / 3) % 3 - 1, dk = n / 9 - 1;
      const int32_t ii = cc.i + di, jj = cc.j + dj, kk = cc.k + dk;
      in[u] = n < 27 && ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
      const int64_t lin = in[u] ? ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk) : 0;
      wd[u] = lin >> 5;
      sh[u] = (int)(lin & 31);
    }
    uint32_t bits[kVsNb];
    int32_t wo[kVsNb];
#pragma unroll
    for (int u = 0; u < kVsNb; ++u) {
      bits[u] = in[u] ? A.bitmap[wd[u]] : 0u;
      wo[u] = in[u] ? A.word_off[wd[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < kVsNb; ++u) {
      const bool set = (bits[u] >> sh[u]) & 1u;
      const int32_t cr = wo[u] + __popc(bits[u] & ((1u << sh[u]) - 1u));
      const bool has = set && cr < A.cell_cap;
      p0[u] = has ? A.vb_off[cr] : 0;
      cnt[u] = has ? A.vb_off[cr + 1] - p0[u] : 0;
    }
    scan_bins<0, 1>(A, p0, cnt, xc, bd, bv);
  }
  vs_min8(bd, bv);
  if (ok) {
    const double q2 = 0.25 * g.h * g.h * (1.0 - 1e-6);
#pragma unroll
    for (int u = 1; u < kVsNb; ++u) {
      const int n = (int)((vs_slot(u) >> (5 * l)) & 31u);
      const int nzo = (n % 3 != 1) + ((n / 3) % 3 != 1) + (n / 9 != 1);
      if (bd < (double)nzo * q2) cnt[u] = 0;
    }
    scan_bins<1, kVsNb>(A, p0, cnt, xc, bd, bv);
    for (int32_t q = l; q < nstray; q += kVsLanes) consider(A.vtx4, A.stray[q], xc, bd, bv);
  }
  vs_min8(bd, bv);
  if (ok && l == 0) {
    A.best_d2[c] = bd;
    A.best_v[c] = bv;
    // the curvature fit's first loads, one dependent level earlier
    int2 inc = make_int2(0, 0);
    if (bv >= 0 && bv < A.nv) {
      inc.x = A.vt_off[bv];
      inc.y = A.vt_off[bv + 1] - inc.x;
    }
    A.best_inc[c] = inc;
  }
}

// Workgroups [0, nb_place): pieces to their ranks and the cells' sums; the
// others: one vertex per thread, its incident list sorted.
__global__ __launch_bounds__(kT) void k_place_sort(PlaceArgs A, int32_t nb_place, int32_t nv, const int32_t* vt_off,
                                                   int32_t* vt_ids) {
  const int32_t b = blockIdx.x;
  if (b < nb_place) {
    place_sums(A, b, nb_place);
  } else {
    const int32_t v = (b - nb_place) * kT + threadIdx.x;
    if (v < nv) sort_incident(vt_off, vt_ids, v);
  }
}

// Closest vertex of every interfacial cell (its own launch: it needs about
// twice the registers of the placing).
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(7))) void k_vstar(Grid g, VstarArgs V) {
  const int32_t nif = min(V.counters[C_NIF], V.cell_cap);
  XcdWalk((int64_t)nif * kVsLanes, blockIdx.x, gridDim.x).run([&](int64_t gid, bool ok) {
    closest_vertex(g, V, nif, gid, ok);
  });
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
  hipLaunchKernelGGL(k_tri_classify, dim3(round_up_xcd(grid_blocks(m.nt, kClassifyT))), dim3(kClassifyT), 0, s, g, m,
                     vtx4, tri4, P, ws->queue_cap, ws->counters);
  // up to 16,384 one-wavefront clip workgroups, four rounds at four per SIMD:
  // shorter walks per workgroup even out the candidates' uneven cost
  // (8,192 and 4,096 were slower at 512^3)
  const int32_t nb_clip = round_up_xcd(grid_blocks(ws->queue_cap, kPieceLanes, 16384));
  const int32_t nb_mark = round_up_xcd(grid_blocks(ws->pair_cap, kPieceLanes, 4096));
  hipLaunchKernelGGL(k_clip_mark, dim3(nb_clip + nb_mark), dim3(kPieceLanes), 0, s, g, tri4, vtx4, P, ws->queue_cap,
                     ws->bitmap, ws->counters, nb_clip);
  time_stop(ws, FTC_KERNEL_TRI_PIECES, s);
  hipError_t e = scan_popcount_emit(ws->bitmap, ws->word_off, ws->nwords, ws->scan_tmp, ws->counters + C_NIF,
                                    ws->cell_ids, ws->cell_cap, ws->counters, s);
  if (e != hipSuccess) return e;
  const int64_t npair_max = ws->pair_cap + ws->queue_cap;
  const int32_t nb_pairs = round_up_xcd(grid_blocks(npair_max, kT, kStrideBlocks));
  VertexBins B{m.nv, vtx4, ws->vcell, ws->vb_cursor, ws->vb_loc, ws->stray};
  hipLaunchKernelGGL(k_pair_count, dim3(nb_pairs), dim3(kT), 0, s, ws->pair_cell, ws->pair_local, ws->bitmap,
                     ws->word_off, ws->offsets, ws->cell_cap, ws->pair_cap, ws->queue_cap, ws->counters, g, B);
  const ScanSeg segs[3] = {{ws->offsets, ws->offsets, ws->cell_cap, ws->counters + C_NPAIRS, nullptr},
                           {ws->vt_cursor, ws->vt_off, m.nv, nullptr, ws->vt_cursor},
                           {ws->vb_cursor, ws->vb_off, ws->cell_cap, nullptr, ws->vb_cursor}};
  e = scan_exclusive_multi(segs, 3, ws->scan_tmp, s);
  if (e != hipSuccess) return e;
  Adjacency J{ws->vt_off, ws->vt_loc, ws->vt_ids, ws->vcell, ws->vb_off, ws->vb_loc, vtx4,
              reinterpret_cast<double2*>(ws->vb_rec)};
  hipLaunchKernelGGL(k_pair_scatter, dim3(nb_pairs), dim3(kT), 0, s, ws->pair_cell, ws->pair_tri, ws->pair_flux,
                     ws->pair_vol, ws->pair_local, ws->offsets, ws->tmp_rec, ws->pair_cap, ws->queue_cap,
                     ws->counters, m, J);
  PlaceArgs A{ws->tmp_rec,    ws->offsets,  ws->tri_ids,  ws->piece_flux, ws->piece_vol,
              ws->cell_flux,  ws->cell_vol, ws->cell_cap, ws->pair_cap,   ws->counters};
  VstarArgs V{vtx4,       ws->cell_ids, ws->bitmap,  ws->word_off, ws->vb_off,  reinterpret_cast<const double2*>(ws->vb_rec),
              ws->stray,  ws->best_d2,  ws->best_v,  ws->vt_off,  reinterpret_cast<int2*>(ws->best_inc),
              m.nv,       ws->cell_cap, ws->counters};
  const int32_t nb_place = round_up_xcd(grid_blocks((int64_t)ws->cell_cap * kPlLanes, kT));
  const int32_t nb_sort = grid_blocks(m.nv, kT);
  const int32_t nb_vstar = round_up_xcd(grid_blocks((int64_t)ws->cell_cap * kVsLanes, kT));
  time_start(ws, FTC_KERNEL_PIECE_RANK, s);
  hipLaunchKernelGGL(k_vstar, dim3(nb_vstar), dim3(kT), 0, s, g, V);
  hipLaunchKernelGGL(k_place_sort, dim3(nb_place + nb_sort), dim3(kT), 0, s, A, nb_place, m.nv, ws->vt_off, ws->vt_ids);
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
