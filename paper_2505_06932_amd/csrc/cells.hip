// cells.hip -- interfacial-cell lists (triangle -> cell binning).
//
// 1. per triangle: clip against every cell of its bounding box, count the
//    pieces, remember which of the first 32 candidates hold one, and set the
//    cell's bit in a grid-sized occupancy bitmap;
// 2. prefix sums: pieces per triangle -> piece offsets; popcount per bitmap
//    word -> compact index of every interfacial cell (rank in the bitmap);
// 3. emit the interfacial cells (ascending linear id, straight from the
//    bitmap) and every piece as (compact cell, triangle), counting pieces per
//    cell;
// 4. prefix sums of the per-cell counts -> CSR offsets; scatter the pieces;
//    sort each cell's short triangle list.
// Everything after step 1 is integer work on device-resident counts, so the
// sequence never needs the host and can be captured into a graph.
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 2048;

__global__ void k_clear_build(uint32_t* bitmap, int64_t nwords, int32_t* offsets, int64_t noff, int32_t* cursor,
                              int64_t ncur, int32_t* counters) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = g0; i < nwords; i += stride) bitmap[i] = 0u;
  for (int64_t i = g0; i < noff; i += stride) offsets[i] = 0;
  for (int64_t i = g0; i < ncur; i += stride) cursor[i] = 0;
  if (g0 < C_COUNT && g0 != C_ERR) counters[g0] = 0;
}

__global__ __launch_bounds__(kT) void k_tri_count(Grid g, Mesh m, uint32_t* bitmap, int32_t* tri_cnt,
                                                  uint32_t* tri_mask, int32_t* counters) {
  const int32_t t = blockIdx.x * kT + threadIdx.x;
  if (t >= m.nt) return;
  if (!tri_ok(m, t)) {
    atomicOr(&counters[C_ERR], ERR_MESH);
    tri_cnt[t] = 0;
    tri_mask[t] = 0u;
    return;
  }
  Tri T = load_tri(m, t);
  bool ok = true;
#pragma unroll
  for (int r = 0; r < 3; ++r) ok = ok && in_margin(g, T.v[r][0], T.v[r][1], T.v[r][2]);
  if (!ok) {
    atomicOr(&counters[C_ERR], ERR_DOMAIN);
    tri_cnt[t] = 0;
    tri_mask[t] = 0u;
    return;
  }
  int64_t lo[3], hi[3];
  tri_range(g, T, lo, hi);
  int32_t cnt = 0, idx = 0;
  uint32_t mask = 0u;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i, ++idx) {
        Poly P;
        if (!clip_cell(g, T, i, j, k, P)) continue;
        ++cnt;
        if (idx < 32) mask |= 1u << idx;
        const int64_t lin = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        atomicOr(&bitmap[lin >> 5], 1u << (lin & 31));
      }
  tri_cnt[t] = cnt;
  tri_mask[t] = mask;
}

__global__ __launch_bounds__(kT) void k_emit_cells(const uint32_t* bitmap, const int32_t* word_off, int64_t nwords,
                                                   int32_t* cell_ids, int32_t cell_cap, int32_t* counters) {
  const int64_t w = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (w >= nwords) return;
  uint32_t bits = bitmap[w];
  int32_t pos = word_off[w];
  while (bits) {
    int b = __ffs(bits) - 1;
    if (pos < cell_cap)
      cell_ids[pos] = (int32_t)(w * 32 + b);
    else
      atomicOr(&counters[C_ERR], ERR_CAPACITY);
    ++pos;
    bits &= bits - 1u;
  }
}

__device__ inline int32_t rank_of(const uint32_t* bitmap, const int32_t* word_off, int64_t lin) {
  const uint32_t w = bitmap[lin >> 5];
  const uint32_t below = (lin & 31) ? (w & ((1u << (lin & 31)) - 1u)) : 0u;
  return word_off[lin >> 5] + __popc(below);
}

__global__ __launch_bounds__(kT) void k_emit_pairs(Grid g, Mesh m, const int32_t* tri_off, const uint32_t* tri_mask,
                                                   const uint32_t* bitmap, const int32_t* word_off,
                                                   int32_t* pair_cell, int32_t* pair_tri, int64_t pair_cap,
                                                   int32_t* cell_cnt, int32_t cell_cap, int32_t* counters) {
  const int32_t t = blockIdx.x * kT + threadIdx.x;
  if (t >= m.nt) return;
  const int32_t start = tri_off[t], end = tri_off[t + 1];
  if (start == end) return;
  Tri T = load_tri(m, t);
  int64_t lo[3], hi[3];
  tri_range(g, T, lo, hi);
  const uint32_t mask = tri_mask[t];
  int32_t n = 0, idx = 0;
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i, ++idx) {
        bool kept;
        if (idx < 32) {
          kept = (mask >> idx) & 1u;
        } else {
          Poly P;
          kept = clip_cell(g, T, i, j, k, P);
        }
        if (!kept) continue;
        const int64_t lin = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        const int32_t ci = rank_of(bitmap, word_off, lin);
        const int64_t p = (int64_t)start + n;
        ++n;
        if (p < pair_cap) {
          pair_tri[p] = t;
          if (ci < cell_cap) {
            pair_cell[p] = ci;
            atomicAdd(&cell_cnt[ci], 1);
          } else {
            pair_cell[p] = -1;
            atomicOr(&counters[C_ERR], ERR_CAPACITY);
          }
        } else {
          atomicOr(&counters[C_ERR], ERR_CAPACITY);
        }
      }
}

__global__ void k_scatter(const int32_t* pair_cell, const int32_t* pair_tri, const int32_t* offsets, int32_t* cursor,
                          int32_t* tri_ids, int64_t pair_cap, const int32_t* counters) {
  const int64_t np = min((int64_t)counters[C_NPAIRS], pair_cap);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t ci = pair_cell[p];
    if (ci < 0) continue;  // its cell did not fit the capacity (error latched)
    const int64_t pos = (int64_t)offsets[ci] + atomicAdd(&cursor[ci], 1);
    if (pos < pair_cap) tri_ids[pos] = pair_tri[p];
  }
}

// Sort each cell's triangle list (ascending id) and record the owning cell of
// every CSR slot.
__global__ void k_sort_cells(const int32_t* offsets, int32_t* tri_ids, int32_t* slot_cell, int32_t cell_cap,
                             int64_t pair_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x) {
    const int64_t s = offsets[ci];
    const int64_t e = min((int64_t)offsets[ci + 1], pair_cap);
    for (int64_t a = s + 1; a < e; ++a) {
      const int32_t v = tri_ids[a];
      int64_t b = a - 1;
      while (b >= s && tri_ids[b] > v) {
        tri_ids[b + 1] = tri_ids[b];
        --b;
      }
      tri_ids[b + 1] = v;
    }
    for (int64_t a = s; a < e; ++a) slot_cell[a] = ci;
  }
}

}  // namespace

hipError_t launch_cell_lists(ftc_cells* ws, const Mesh& m, hipStream_t s) {
  const Grid& g = ws->grid;
  hipLaunchKernelGGL(k_clear_build, dim3(kStrideBlocks), dim3(kT), 0, s, ws->bitmap, ws->nwords, ws->offsets,
                     (int64_t)ws->cell_cap + 1, ws->cursor, (int64_t)ws->cell_cap, ws->counters);
  time_start(ws, FTC_KERNEL_TRI_COUNT, s);
  hipLaunchKernelGGL(k_tri_count, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, g, m, ws->bitmap, ws->tri_off,
                     ws->tri_mask, ws->counters);
  time_stop(ws, FTC_KERNEL_TRI_COUNT, s);
  hipError_t e = scan_exclusive(ws->tri_off, m.nt, ws->scan_tmp, ws->counters + C_NPAIRS, s);
  if (e != hipSuccess) return e;
  e = scan_popcount(ws->bitmap, ws->word_off, ws->nwords, ws->scan_tmp, ws->counters + C_NIF, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_emit_cells, dim3(grid_blocks(ws->nwords, kT)), dim3(kT), 0, s, ws->bitmap, ws->word_off,
                     ws->nwords, ws->cell_ids, ws->cell_cap, ws->counters);
  hipLaunchKernelGGL(k_emit_pairs, dim3(grid_blocks(m.nt, kT)), dim3(kT), 0, s, g, m, ws->tri_off, ws->tri_mask,
                     ws->bitmap, ws->word_off, ws->pair_cell, ws->pair_tri, ws->pair_cap, ws->offsets, ws->cell_cap,
                     ws->counters);
  e = scan_exclusive(ws->offsets, ws->cell_cap, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter, dim3(grid_blocks(ws->pair_cap, kT, kStrideBlocks)), dim3(kT), 0, s, ws->pair_cell,
                     ws->pair_tri, ws->offsets, ws->cursor, ws->tri_ids, ws->pair_cap, ws->counters);
  hipLaunchKernelGGL(k_sort_cells, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, ws->offsets,
                     ws->tri_ids, ws->slot_cell, ws->cell_cap, ws->pair_cap, ws->counters);
  return hipGetLastError();
}

}  // namespace ftc
