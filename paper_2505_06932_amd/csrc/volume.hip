// volume.hip -- exact volume fractions of the interfacial cells and the dense
// indicator field.
//
// With F = (0, 0, z - zlo) (divergence 1) the divergence theorem on
// Omega cap C gives |Omega cap C| = sum over the cell's pieces of the
// integral of (z - zlo) n_z dA, plus h times the wetted area W of the upper
// face (F . n vanishes on the lower and side faces).  With F = (0, 0, 1) on
// the column above the cell, W is the sum of the integrals of n_z dA over
// all pieces strictly above.  The pieces' integrals are computed and summed
// per cell while the cell lists are built (in a fixed order: lane partial
// sums over the CSR entries, then a butterfly); here
//   colsum : one bit per block of 64 columns, row and slab of 32 planes,
//            set if a cell of it holds a piece (most hold none);
//   columns: every (i, j) column walked top down over the interfacial-cell
//            bitmap, split into z chunks whose flux totals are exchanged in
//            LDS: alpha = (V + h W) / h^3 in interfacial cells, 0 or 1 in
//            the others (dense field written on the way), ERR_MESH where W
//            is not 0 or h^2 outside the front.
#include "ftc_ws.hpp"

namespace ftc {
namespace {

// Column pass.  A workgroup takes 64 consecutive columns (x) of one y row
// and splits the z range into kChunks chunks (4, 8 or 16), one wavefront
// each; lanes are columns, so bitmap reads and dense stores are coalesced
// along x.  A chunk is walked top down in segments of 32 cells:
//   1. each wavefront loads the 32 bitmap words of a segment together and
//      keeps the segment's interfacial bits; only for those cells does it
//      fetch the compact id and the flux, summed into the chunk total (the
//      bits of up to kKeepSeg segments stay in registers for step 3);
//   2. the chunk totals above give each chunk the wetted area W at its top;
//   3. each wavefront walks its chunk top down again: an interfacial cell
//      gets (V + h W) / h^3 and adds its flux to W, any other cell gets
//      round(W / h^2), which must be 0 or 1 within 1e-9 (else the front is
//      open: ERR_MESH), as must W below the lowest chunk.  Between
//      interfacial cells the walk only stores.
constexpr int kColLanes = 64;
static_assert(kColLanes == kColBlock, "a column block is one block of the column summary");
constexpr int kSeg = 32;      // cells per segment: one bit mask
constexpr int kKeepSeg = 8;   // segment masks kept between the two walks (chunks of up to 256 cells)

struct ColArgs {
  Grid g;
  const uint32_t* bitmap;
  const uint32_t* colsum;  // the column summary, or null
  const int32_t* word_off;
  const double* cell_flux;
  const double* cell_vol;
  double* alpha_if;
  double* alpha;
  int32_t cell_cap;
  int32_t* counters;
};

// Interfacial bits of cells k1, k1-1, ..., k1-31 (those >= klo) of column
// (i, j): bit q for cell k1 - q.
__device__ inline uint32_t segment_mask(const ColArgs& A, bool col_ok, int32_t i, int32_t j, int32_t k1,
                                        int32_t klo) {
  const Grid& g = A.g;
  const int64_t col = i + (int64_t)g.nx * j, sz = (int64_t)g.nx * g.ny;
  uint32_t wv[kSeg];
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    const int64_t lin = col + sz * (k1 - q);
    wv[q] = (col_ok && k1 - q >= klo) ? A.bitmap[lin >> 5] : 0u;
  }
  uint32_t m = 0u;
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    const int64_t lin = col + sz * (k1 - q);
    m |= ((wv[q] >> (lin & 31)) & 1u) << q;
  }
  return m;
}

// The column summary from the occupancy bitmap (nx a multiple of 64): one
// lane per bitmap word of a row and slab, consecutive lanes on consecutive
// words of a row (coalesced), each OR-ing its word over the slab's planes
// (loads issued together); a pair of lanes makes one block of 64 columns,
// and a ballot over the even lanes packs a wavefront's 32 bits, which are
// 32 consecutive bits of the summary.
constexpr int kSumT = 256;
__global__ __launch_bounds__(kSumT) void k_colsum(Grid g, const uint32_t* bitmap, uint32_t* colsum, int64_t nlanes) {
  const int64_t wpr = g.nx / 32;  // words per row
  const int64_t row = (int64_t)g.nx * g.ny / 32;
  for (int64_t b0 = (int64_t)blockIdx.x * kSumT + (threadIdx.x & ~63); b0 < nlanes;
       b0 += (int64_t)gridDim.x * kSumT) {
    const int64_t L = b0 + (threadIdx.x & 63);
    uint32_t any = 0u;
    if (L < nlanes) {
      const int64_t u = L % wpr, rest = L / wpr;
      const int64_t j = rest % g.ny, k0 = (rest / g.ny) * kSlab;
      const int64_t base = u + wpr * j;
      uint32_t w[kSlab];
#pragma unroll
      for (int q = 0; q < kSlab; ++q) w[q] = k0 + q < g.nz ? bitmap[base + row * (k0 + q)] : 0u;
#pragma unroll
      for (int q = 0; q < kSlab; ++q) any |= w[q];
    }
    any |= __shfl_xor(any, 1, 64);
    const uint64_t bal = __ballot(any != 0u && (threadIdx.x & 1) == 0);
    // even lane 2q holds bit q of the wavefront's 32
    uint32_t bits = 0u;
#pragma unroll
    for (int q = 0; q < 32; ++q) bits |= (uint32_t)((bal >> (2 * q)) & 1ull) << q;
    if ((threadIdx.x & 63) == 0 && b0 < nlanes) colsum[b0 >> 6] = bits;
  }
}

// Compact id of the interfacial cell lin (-2: beyond the cell capacity, a
// latched capacity error, taken with no pieces).
__device__ inline int32_t compact_id(const ColArgs& A, int64_t lin) {
  const uint32_t w = A.bitmap[lin >> 5];
  const int32_t r = A.word_off[lin >> 5] + __popc(w & ((1u << (lin & 31)) - 1u));
  return r < A.cell_cap ? r : -2;
}

template <int kChunks>
__global__ __launch_bounds__(kColLanes* kChunks) void k_columns(ColArgs A) {
  __shared__ double tot_s[kChunks][kColLanes];
  const Grid& g = A.g;
  const int lane = threadIdx.x % kColLanes, w = threadIdx.x / kColLanes;
  const int32_t i = blockIdx.x * kColLanes + lane, j = blockIdx.y;
  const bool col_ok = i < g.nx;
  const int32_t len = (g.nz + kChunks - 1) / kChunks;
  const int32_t klo = min(w * len, g.nz), khi = min(klo + len, g.nz);
  const double h = g.h, h2 = h * h, h3 = h * h * h;
  const int64_t col = i + (int64_t)g.nx * j, sz = (int64_t)g.nx * g.ny;

  // a chunk none of whose cells holds a piece (the column summary, one bit
  // per kSlab planes of this block of columns) skips the bitmap
  bool empty = false;
  if (A.colsum) {
    const int64_t nbx = g.nx / kColBlock;
    empty = true;
    for (int32_t kz = klo / kSlab; klo < khi && kz <= (khi - 1) / kSlab; ++kz) {
      const int64_t cb = ((int64_t)kz * g.ny + j) * nbx + blockIdx.x;
      if ((A.colsum[cb >> 5] >> (cb & 31)) & 1u) empty = false;
    }
  }

  // ---- 1. interfacial bits and the chunk's flux total
  uint32_t keep[kKeepSeg];
#pragma unroll
  for (int u = 0; u < kKeepSeg; ++u) keep[u] = 0u;
  double tot = 0.0;
  if (!empty) {
    int s = 0;
    for (int32_t k1 = khi - 1; k1 >= klo; k1 -= kSeg, ++s) {
      uint32_t m = segment_mask(A, col_ok, i, j, k1, klo);
#pragma unroll
      for (int u = 0; u < kKeepSeg; ++u)
        if (u == s) keep[u] = m;
      while (m) {
        const int q = __ffs(m) - 1;
        m &= m - 1u;
        const int32_t ci = compact_id(A, col + sz * (k1 - q));
        if (ci >= 0) tot += A.cell_flux[ci];
      }
    }
  }
  tot_s[w][lane] = tot;
  __syncthreads();
  double W = 0.0;
  for (int u = kChunks - 1; u > w; --u) W += tot_s[u][lane];

  // ---- 3. alpha of every cell of the chunk
  bool bad = false;
  double rr = 0.0;     // round(W / h^2) for the cells that are not interfacial
  bool fresh = false;  // rr (and its check) belongs to the current W
  int s = 0;
  for (int32_t k1 = khi - 1; k1 >= klo; k1 -= kSeg, ++s) {
    uint32_t m = 0u;
    if (s < kKeepSeg) {
#pragma unroll
      for (int u = 0; u < kKeepSeg; ++u)
        if (u == s) m = keep[u];
    } else if (!empty) {
      m = segment_mask(A, col_ok, i, j, k1, klo);
    }
    const int nq = min(kSeg, k1 - klo + 1);
    for (int q = 0; q < nq; ++q) {
      const int64_t lin = col + sz * (k1 - q);
      double a;
      if ((m >> q) & 1u) {
        const int32_t ci = compact_id(A, lin);
        const double vo = ci >= 0 ? A.cell_vol[ci] : 0.0;
        a = (vo + h * W) / h3;
        if (A.alpha_if && ci >= 0) A.alpha_if[ci] = a;
        if (ci >= 0) W += A.cell_flux[ci];
        fresh = false;
      } else {
        if (!fresh) {
          const double r = W / h2;
          rr = round(r);
          if (fabs(r - rr) > 1e-9 || (rr != 0.0 && rr != 1.0)) bad = true;
          fresh = true;
        }
        a = rr;
      }
      // the dense field is written once and read by later calls only:
      // streaming stores keep it from evicting the lists the step still uses
      if (A.alpha && col_ok) __builtin_nontemporal_store(a, &A.alpha[lin]);
    }
  }
  if (w == 0 && col_ok && fabs(W / h2) > 1e-9) bad = true;  // the column must close below the front
  if (bad) atomicOr(&A.counters[C_ERR], ERR_MESH);
}

}  // namespace

hipError_t launch_volume_fraction(const ftc_cells* ws, const Mesh& m, double* alpha_if, double* alpha_dense,
                                  hipStream_t s) {
  (void)m;  // the pieces' integrals and their per-cell sums come from the cell-list build
  const Grid& g = ws->grid;
  // the summary pays on large grids, where most chunks hold no piece (at
  // 512^3 the column pass saves 30 us for a 6 us pass over the bitmap; at
  // 256^3 and below the extra launch costs what it saves)
  const uint32_t* colsum = nullptr;
  if (g.nx % kColBlock == 0 && (int64_t)g.nx * g.ny * g.nz >= (int64_t(1) << 26)) {
    // lanes: words per row x rows x slabs; 32 summary bits per wavefront
    const int64_t nlanes = (int64_t)(g.nx / 32) * g.ny * ((g.nz + kSlab - 1) / kSlab);
    hipLaunchKernelGGL(k_colsum, dim3(grid_blocks(nlanes, kSumT, 8192)), dim3(kSumT), 0, s, g, ws->bitmap, ws->colsum,
                       nlanes);
    colsum = ws->colsum;
  }
  ColArgs A{g, ws->bitmap, colsum, ws->word_off, ws->cell_flux, ws->cell_vol, alpha_if, alpha_dense, ws->cell_cap,
            ws->counters};
  time_start(ws, FTC_KERNEL_COLUMNS, s);
  const dim3 cg((g.nx + kColLanes - 1) / kColLanes, g.ny);
  if (ws->tune.column_chunks == 4)
    hipLaunchKernelGGL(k_columns<4>, cg, dim3(kColLanes * 4), 0, s, A);
  else if (ws->tune.column_chunks == 16)
    hipLaunchKernelGGL(k_columns<16>, cg, dim3(kColLanes * 16), 0, s, A);
  else
    hipLaunchKernelGGL(k_columns<8>, cg, dim3(kColLanes * 8), 0, s, A);
  time_stop(ws, FTC_KERNEL_COLUMNS, s);
  return hipGetLastError();
}

}  // namespace ftc
