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
// After step 1 everything is integer work on device-resident counts, so the
// sequence needs no host round trip and can be captured into a graph.
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 2048;
constexpr int kPieceLanes = 64;  // k_clip_queue: one wavefront per workgroup

// Clears the per-build state and packs the vertex coordinates as (x, y, z, 0).
__global__ void k_clear_build(uint32_t* bitmap, int64_t nwords, int32_t* cell_cnt, int64_t ncnt, int32_t* cursor,
                              int64_t ncur, int32_t* counters, Mesh m, double2* vtx4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t v = g0; v < m.nv; v += stride) {
    vtx4[2 * v] = make_double2(m.x[v], m.y[v]);
    vtx4[2 * v + 1] = make_double2(m.z[v], 0.0);
  }
  for (int64_t i = g0; i < nwords; i += stride) bitmap[i] = 0u;
  for (int64_t i = g0; i < ncnt; i += stride) cell_cnt[i] = 0;
  for (int64_t i = g0; i < ncur; i += stride) cursor[i] = 0;
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
// classification: count, allocate, write.
constexpr int kClassifyT = 1024;
__global__ __launch_bounds__(kClassifyT) void k_tri_classify(Grid g, Mesh m, const double2* vtx4, int4* tri4,
                                                             uint32_t* bitmap, PairOut P, int64_t q_cap,
                                                             int32_t* counters) {
  __shared__ int32_t sh[kClassifyT / 64 + 1];
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
          ++n2;
        }
      }
  int64_t p = block_alloc<kClassifyT>(n1, &counters[C_NWHOLE], sh);
  int64_t q = block_alloc<kClassifyT>(n2, &counters[C_NQUEUE], sh);
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
          if (q < q_cap) {
            P.lin[P.cap + q] = (int32_t)lin;
            P.tri[P.cap + q] = t;
          } else {
            atomicOr(&counters[C_ERR], ERR_CAPACITY);
          }
          ++q;
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
      const Piece pc = clip_piece(g, T, c.i, c.j, c.k, L, lane);
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

// pair -> compact cell (in place of its linear id), counted per cell
__global__ void k_pair_count(int32_t* pair_lin, const uint32_t* bitmap, const int32_t* word_off, int32_t* cell_cnt,
                             int32_t cell_cap, int64_t pair_cap, int64_t queue_cap, const int32_t* counters) {
  const PairRange R = pair_range(counters, pair_cap, queue_cap);
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < R.count(); x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = R.slot(x);
    const int32_t lin = pair_lin[p];
    if (lin < 0) continue;
    const int32_t ci = rank_of(bitmap, word_off, lin);
    if (ci < cell_cap) {
      pair_lin[p] = ci;
      atomicAdd(&cell_cnt[ci], 1);
    } else {
      pair_lin[p] = -1;  // its cell did not fit the capacity (latched while listing the cells)
    }
  }
}

__global__ void k_pair_scatter(const int32_t* pair_ci, const int32_t* pair_tri, const int32_t* offsets,
                               int32_t* cursor, int32_t* tmp_tri, int32_t* tmp_pair, int64_t pair_cap,
                               int64_t queue_cap, int32_t* counters) {
  const PairRange R = pair_range(counters, pair_cap, queue_cap);
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < R.count(); x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = R.slot(x);
    const int32_t ci = pair_ci[p];
    if (ci < 0) continue;
    const int64_t pos = (int64_t)offsets[ci] + atomicAdd(&cursor[ci], 1);
    if (pos < pair_cap) {
      tmp_tri[pos] = pair_tri[p];
      tmp_pair[pos] = (int32_t)p;
    } else {
      atomicOr(&counters[C_ERR], ERR_CAPACITY);
    }
  }
}

// Each scattered piece moves to its rank by triangle id within its cell (a
// triangle has at most one piece per cell, so the ranks are distinct).
__global__ void k_rank_place(const int32_t* tmp_tri, const int32_t* tmp_pair, const int32_t* pair_ci,
                             const double* pair_flux, const double* pair_vol, const int32_t* offsets,
                             int32_t* tri_ids, int32_t* slot_cell, double* piece_flux, double* piece_vol,
                             int32_t cell_cap, int64_t pair_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  const int64_t nslot = min((int64_t)offsets[nif], pair_cap);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nslot; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = tmp_pair[q];
    const int32_t ci = pair_ci[p];
    const int32_t t = tmp_tri[q];
    const int64_t s = offsets[ci], e = min((int64_t)offsets[ci + 1], pair_cap);
    int64_t rank = 0;
    for (int64_t u = s; u < e; ++u) rank += tmp_tri[u] < t ? 1 : 0;
    const int64_t dst = s + rank;
    tri_ids[dst] = t;
    slot_cell[dst] = ci;
    piece_flux[dst] = pair_flux[p];
    piece_vol[dst] = pair_vol[p];
  }
}

}  // namespace

hipError_t launch_cell_lists(ftc_cells* ws, const Mesh& m, hipStream_t s) {
  const Grid& g = ws->grid;
  int4* tri4 = reinterpret_cast<int4*>(ws->tri4);
  double2* vtx4 = reinterpret_cast<double2*>(ws->vtx4);
  hipLaunchKernelGGL(k_clear_build, dim3(kStrideBlocks), dim3(kT), 0, s, ws->bitmap, ws->nwords, ws->offsets,
                     (int64_t)ws->cell_cap + 1, ws->cursor, (int64_t)ws->cell_cap, ws->counters, m, vtx4);
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
  hipLaunchKernelGGL(k_pair_count, dim3(grid_blocks(npair_max, kT, kStrideBlocks)), dim3(kT), 0, s, ws->pair_cell,
                     ws->bitmap, ws->word_off, ws->offsets, ws->cell_cap, ws->pair_cap, ws->queue_cap,
                     ws->counters);
  e = scan_exclusive(ws->offsets, ws->cell_cap, ws->scan_tmp, ws->counters + C_NPAIRS, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pair_scatter, dim3(grid_blocks(npair_max, kT, kStrideBlocks)), dim3(kT), 0, s, ws->pair_cell,
                     ws->pair_tri, ws->offsets, ws->cursor, ws->tmp_tri, ws->tmp_pair, ws->pair_cap, ws->queue_cap,
                     ws->counters);
  time_start(ws, FTC_KERNEL_PIECE_RANK, s);
  hipLaunchKernelGGL(k_rank_place, dim3(grid_blocks(ws->pair_cap, kT, kStrideBlocks)), dim3(kT), 0, s, ws->tmp_tri,
                     ws->tmp_pair, ws->pair_cell, ws->pair_flux, ws->pair_vol, ws->offsets, ws->tri_ids,
                     ws->slot_cell, ws->piece_flux, ws->piece_vol, ws->cell_cap, ws->pair_cap, ws->counters);
  time_stop(ws, FTC_KERNEL_PIECE_RANK, s);
  return hipGetLastError();
}

}  // namespace ftc
