// volume.hip -- exact volume fractions of the interfacial cells and the dense
// indicator field.
//
// With F = (0, 0, z - zlo) (divergence 1) the divergence theorem on
// Omega cap C gives |Omega cap C| = sum over the cell's pieces of the
// integral of (z - zlo) n_z dA, plus h times the wetted area W of the upper
// face (F . n vanishes on the lower and side faces).  With F = (0, 0, 1) on
// the column above the cell, W is the sum of the integrals of n_z dA over
// all pieces strictly above.  Kernels:
//   sums   : one thread per interfacial cell, its pieces' integrals (computed
//            while the cell lists were built) summed in CSR order;
//   columns: every (i, j) column walked top down over the interfacial-cell
//            bitmap, split into z chunks whose flux totals are exchanged in
//            LDS: alpha = (V + h W) / h^3 in interfacial cells, 0 or 1 in
//            the others (dense field written on the way), ERR_MESH where W
//            is not 0 or h^2 outside the front.
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 4096;

// Per interfacial cell: sum of its pieces' integrals in CSR (ascending
// triangle) order.
// Pieces past the pair capacity were not stored (a latched capacity error).
__global__ void k_cell_sums(const int32_t* offsets, const double* piece_flux, const double* piece_vol,
                            double* cell_flux, double* cell_vol, int32_t cell_cap, int64_t pair_cap,
                            const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x) {
    double f = 0.0, v = 0.0;
    const int64_t e = min((int64_t)offsets[ci + 1], pair_cap);
    for (int64_t p = offsets[ci]; p < e; ++p) {
      f += piece_flux[p];
      v += piece_vol[p];
    }
    cell_flux[ci] = f;
    cell_vol[ci] = v;
  }
}

// Column pass.  A workgroup takes 64 consecutive columns (x) of one y row
// and splits the z range into kChunks chunks (4, 8 or 16), one wavefront each; lanes are
// columns, so bitmap reads and dense stores are coalesced along x.
//   1. each wavefront sums the fluxes of the interfacial cells in its chunk,
//      top down;
//   2. the chunk totals above give each chunk the wetted area W at its top;
//   3. each wavefront walks its chunk top down again: an interfacial cell
//      gets (V + h W) / h^3 and adds its flux to W, any other cell gets
//      round(W / h^2), which must be 0 or 1 within 1e-9 (else the front is
//      open: ERR_MESH), as must W below the lowest chunk.
constexpr int kColLanes = 64;
// cells of a chunk read at once: 16, or 8 with 16 chunks (whose 1024-thread
// workgroups leave 128 registers per lane)
template <int kChunks>
constexpr int sub_of() { return kChunks == 16 ? 8 : 16; }

struct ColArgs {
  Grid g;
  const uint32_t* bitmap;
  const int32_t* word_off;
  const double* cell_flux;
  const double* cell_vol;
  double* alpha_if;
  double* alpha;
  int32_t cell_cap;
  int32_t* counters;
};

// Reads kSub cells k1, k1-1, ... (those >= klo) of column (i, j): which are
// interfacial, their compact ids (-1: not interfacial; -2: interfacial but
// beyond the cell capacity, a latched capacity error, taken with no
// pieces), fluxes and (if `vol`) volume integrals.
template <bool kVol, int kSub>
__device__ inline void read_sub(const ColArgs& A, bool col_ok, int32_t i, int32_t j, int32_t k1, int32_t klo,
                                int32_t ci[kSub], double fl[kSub], double vo[kSub]) {
  const Grid& g = A.g;
  uint32_t wv[kSub], lin[kSub];  // cell ids fit in 31 bits
#pragma unroll
  for (int q = 0; q < kSub; ++q) {
    const int32_t k = k1 - q;
    lin[q] = (uint32_t)(i + (int64_t)g.nx * (j + (int64_t)g.ny * k));
    wv[q] = (col_ok && k >= klo) ? A.bitmap[lin[q] >> 5] : 0u;
  }
  int32_t wo[kSub];
#pragma unroll
  for (int q = 0; q < kSub; ++q) {
    const bool set = (wv[q] >> (lin[q] & 31)) & 1u;
    wo[q] = A.word_off[set ? (lin[q] >> 5) : 0];
    const int32_t r = wo[q] + __popc(wv[q] & ((1u << (lin[q] & 31)) - 1u));
    ci[q] = !set ? -1 : (r < A.cell_cap ? r : -2);
  }
#pragma unroll
  for (int q = 0; q < kSub; ++q) {
    const int32_t c = ci[q] >= 0 ? ci[q] : 0;
    fl[q] = ci[q] >= 0 ? A.cell_flux[c] : 0.0;
    if (kVol) vo[q] = ci[q] >= 0 ? A.cell_vol[c] : 0.0;
  }
}

template <int kChunks>
__global__ __launch_bounds__(kColLanes* kChunks) void k_columns(ColArgs A) {
  constexpr int kSub = sub_of<kChunks>();
  __shared__ double tot_s[kChunks][kColLanes];
  const Grid& g = A.g;
  const int lane = threadIdx.x % kColLanes, w = threadIdx.x / kColLanes;
  const int32_t i = blockIdx.x * kColLanes + lane, j = blockIdx.y;
  const bool col_ok = i < g.nx;
  const int32_t len = (g.nz + kChunks - 1) / kChunks;
  const int32_t klo = min(w * len, g.nz), khi = min(klo + len, g.nz);
  const double h = g.h, h2 = h * h, h3 = h * h * h;
  int32_t ci[kSub];
  double fl[kSub], vo[kSub];

  // a chunk of at most kSub cells is read once, for both walks
  const bool once = khi - klo <= kSub;
  double tot = 0.0;
  for (int32_t k1 = khi - 1; k1 >= klo; k1 -= kSub) {
    if (once)
      read_sub<true, kSub>(A, col_ok, i, j, k1, klo, ci, fl, vo);
    else
      read_sub<false, kSub>(A, col_ok, i, j, k1, klo, ci, fl, vo);
#pragma unroll
    for (int q = 0; q < kSub; ++q)
      if (ci[q] >= 0) tot += fl[q];
  }
  tot_s[w][lane] = tot;
  __syncthreads();
  double W = 0.0;
  for (int u = kChunks - 1; u > w; --u) W += tot_s[u][lane];

  bool bad = false;
  for (int32_t k1 = khi - 1; k1 >= klo; k1 -= kSub) {
    if (!once) read_sub<true, kSub>(A, col_ok, i, j, k1, klo, ci, fl, vo);
#pragma unroll
    for (int q = 0; q < kSub; ++q) {
      const int32_t k = k1 - q;
      if (!col_ok || k < klo) continue;
      double a;
      if (ci[q] != -1) {
        a = (vo[q] + h * W) / h3;
        if (A.alpha_if && ci[q] >= 0) A.alpha_if[ci[q]] = a;
        W += fl[q];
      } else {
        const double r = W / h2, rr = round(r);
        if (fabs(r - rr) > 1e-9 || (rr != 0.0 && rr != 1.0)) bad = true;
        a = rr;
      }
      if (A.alpha) A.alpha[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] = a;
    }
  }
  if (w == 0 && col_ok && fabs(W / h2) > 1e-9) bad = true;  // the column must close below the front
  if (bad) atomicOr(&A.counters[C_ERR], ERR_MESH);
}

}  // namespace

hipError_t launch_volume_fraction(const ftc_cells* ws, const Mesh& m, double* alpha_if, double* alpha_dense,
                                  hipStream_t s) {
  (void)m;  // the pieces and their integrals come from the cell-list build
  const Grid& g = ws->grid;
  hipLaunchKernelGGL(k_cell_sums, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, ws->offsets,
                     ws->piece_flux, ws->piece_vol, ws->cell_flux, ws->cell_vol, ws->cell_cap, ws->pair_cap,
                     ws->counters);
  ColArgs A{g, ws->bitmap, ws->word_off, ws->cell_flux, ws->cell_vol, alpha_if, alpha_dense, ws->cell_cap,
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
