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
//   columns: interfacial cells grouped by (i, j) column (count, scan,
//            scatter);
//   walk   : one thread per column, top to bottom, summing each cell's pieces
//            in CSR (ascending triangle) order, alpha = (V + h W) / h^3, and
//            the 0/1 value of the cells between consecutive interfacial
//            cells; a column whose W is not 0 or h^2 there latches ERR_MESH;
//   dense  : one thread per grid cell, x fastest (coalesced writes), looks
//            up its column's short list.
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 256;
constexpr int kStrideBlocks = 4096;

// Per interfacial cell: sum of its pieces' integrals in CSR (ascending
// triangle) order.
__global__ void k_cell_sums(const int32_t* offsets, const double* piece_flux, const double* piece_vol,
                            double* cell_flux, double* cell_vol, int32_t cell_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x) {
    double f = 0.0, v = 0.0;
    for (int32_t p = offsets[ci]; p < offsets[ci + 1]; ++p) {
      f += piece_flux[p];
      v += piece_vol[p];
    }
    cell_flux[ci] = f;
    cell_vol[ci] = v;
  }
}

__global__ void k_clear_cols(int32_t* col_off, int64_t n1, int32_t* col_cursor, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += stride) {
    col_off[i] = 0;
    if (i < n2) col_cursor[i] = 0;
  }
}

__global__ void k_col_count(Grid g, const int32_t* cell_ids, int32_t* col_cnt, int32_t cell_cap,
                            const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x) {
    const uint32_t lin = (uint32_t)cell_ids[ci];
    atomicAdd(&col_cnt[lin - g.dncol.div(lin) * g.dncol.d], 1);
  }
}

__global__ void k_col_scatter(Grid g, const int32_t* cell_ids, const int32_t* col_off, int32_t* col_cursor,
                              int32_t* col_cells, int32_t cell_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x) {
    const uint32_t lin = (uint32_t)cell_ids[ci];
    const uint32_t col = lin - g.dncol.div(lin) * g.dncol.d;
    col_cells[col_off[col] + atomicAdd(&col_cursor[col], 1)] = ci;
  }
}

constexpr int kColReg = 16;  // columns up to this length are handled in registers

__global__ void k_col_walk(Grid g, const int32_t* col_off, int32_t* col_cells, const int32_t* cell_ids,
                           const double* cell_flux, const double* cell_vol, int32_t* col_k, double* col_alpha,
                           double* col_below, double* alpha_if, int32_t* counters) {
  const int64_t ncol = (int64_t)g.nx * g.ny;
  const double h = g.h, h2 = h * h, h3 = h * h * h;
  for (int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; col < ncol;
       col += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = col_off[col], e = col_off[col + 1];
    if (s == e) continue;
    bool bad = false;
    double W = 0.0;
    int32_t prev_k = g.nz;
    // One step of the walk, from the top of the column down: the cells
    // between this interfacial cell and the one above have wetted area W.
    auto step = [&](int32_t q, int32_t ci, int32_t k, double f, double v) {
      if (prev_k - k > 1) {
        const double r = W / h2, rr = rint(r);
        if (fabs(r - rr) > 1e-9 || (rr != 0.0 && rr != 1.0)) bad = true;
      }
      const double alpha = (v + h * W) / h3;
      if (alpha_if) alpha_if[ci] = alpha;
      col_cells[q] = ci;
      col_k[q] = k;
      col_alpha[q] = alpha;
      W += f;
      const double rb = rint(W / h2);
      col_below[q] = rb == 1.0 ? 1.0 : 0.0;
      prev_k = k;
    };
    if (e - s <= kColReg) {
      // load, sort by compact index (== by k within a column), gather, walk
      int32_t v[kColReg];
#pragma unroll
      for (int q = 0; q < kColReg; ++q) v[q] = (s + q < e) ? col_cells[s + q] : INT_MAX;
#pragma unroll
      for (int pass = 0; pass < kColReg; ++pass)
#pragma unroll
        for (int q = (pass & 1); q + 1 < kColReg; q += 2) {
          const int32_t a = v[q], b = v[q + 1];
          v[q] = min(a, b);
          v[q + 1] = max(a, b);
        }
      int32_t kk[kColReg];
      double ff[kColReg], vv[kColReg];
#pragma unroll
      for (int q = 0; q < kColReg; ++q) {
        const bool live = s + q < e;
        kk[q] = live ? (int32_t)g.dncol.div((uint32_t)cell_ids[v[q]]) : 0;
        ff[q] = live ? cell_flux[v[q]] : 0.0;
        vv[q] = live ? cell_vol[v[q]] : 0.0;
      }
#pragma unroll
      for (int q = kColReg - 1; q >= 0; --q)
        if (s + q < e) step(s + q, v[q], kk[q], ff[q], vv[q]);
    } else {
      for (int32_t a = s + 1; a < e; ++a) {
        const int32_t x = col_cells[a];
        int32_t b = a - 1;
        while (b >= s && col_cells[b] > x) {
          col_cells[b + 1] = col_cells[b];
          --b;
        }
        col_cells[b + 1] = x;
      }
      for (int32_t q = e - 1; q >= s; --q) {
        const int32_t ci = col_cells[q];
        step(q, ci, (int32_t)g.dncol.div((uint32_t)cell_ids[ci]), cell_flux[ci], cell_vol[ci]);
      }
    }
    if (fabs(W / h2) > 1e-9) bad = true;  // the column must close below the front
    if (bad) atomicOr(&counters[C_ERR], ERR_MESH);
  }
}

// Dense field: one thread per (column, run of kDenseRun cells in z); the
// threads of a wavefront are consecutive in x, so every store instruction
// writes 64 consecutive cells.  Each thread finds its place in the column's
// short list once and walks up.
constexpr int kDenseRun = 16;
__global__ __launch_bounds__(kT) void k_dense(Grid g, const int32_t* col_off, const int32_t* col_k,
                                              const double* col_alpha, const double* col_below, double* alpha) {
  const int32_t j = blockIdx.y;
  const int32_t k0 = blockIdx.z * kDenseRun;
  const int64_t plane = (int64_t)g.nx * g.ny;
  for (int32_t i = blockIdx.x * kT + threadIdx.x; i < g.nx; i += gridDim.x * kT) {
    const int64_t col = i + (int64_t)g.nx * j;
    const int32_t s = col_off[col], e = col_off[col + 1];
    int32_t q = s;
    while (q < e && col_k[q] < k0) ++q;
    const int32_t k1 = min(k0 + kDenseRun, g.nz);
    for (int32_t k = k0; k < k1; ++k) {
      while (q < e && col_k[q] < k) ++q;
      double a = 0.0;
      if (q < e) a = (col_k[q] == k) ? col_alpha[q] : col_below[q];
      alpha[col + plane * k] = a;
    }
  }
}

}  // namespace

hipError_t launch_volume_fraction(const ftc_cells* ws, const Mesh& m, double* alpha_if, double* alpha_dense,
                                  hipStream_t s) {
  (void)m;  // the pieces and their integrals come from the cell-list build
  const Grid& g = ws->grid;
  hipLaunchKernelGGL(k_cell_sums, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, ws->offsets,
                     ws->piece_flux, ws->piece_vol, ws->cell_flux, ws->cell_vol, ws->cell_cap, ws->counters);
  hipLaunchKernelGGL(k_clear_cols, dim3(grid_blocks(ws->ncol + 1, kT, kStrideBlocks)), dim3(kT), 0, s, ws->col_off,
                     ws->ncol + 1, ws->col_cursor, ws->ncol);
  hipLaunchKernelGGL(k_col_count, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, g,
                     ws->cell_ids, ws->col_off, ws->cell_cap, ws->counters);
  hipError_t e = scan_exclusive(ws->col_off, ws->ncol, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_scatter, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, g,
                     ws->cell_ids, ws->col_off, ws->col_cursor, ws->col_cells, ws->cell_cap, ws->counters);
  time_start(ws, FTC_KERNEL_COL_WALK, s);
  hipLaunchKernelGGL(k_col_walk, dim3(grid_blocks(ws->ncol, 64, 65536)), dim3(64), 0, s, g, ws->col_off,
                     ws->col_cells, ws->cell_ids, ws->cell_flux, ws->cell_vol, ws->col_k, ws->col_alpha,
                     ws->col_below, alpha_if, ws->counters);
  time_stop(ws, FTC_KERNEL_COL_WALK, s);
  if (alpha_dense) {
    time_start(ws, FTC_KERNEL_DENSE_ALPHA, s);
    hipLaunchKernelGGL(k_dense, dim3(grid_blocks(g.nx, kT, 64), g.ny, (g.nz + kDenseRun - 1) / kDenseRun), dim3(kT),
                       0, s, g, ws->col_off, ws->col_k, ws->col_alpha, ws->col_below, alpha_dense);
    time_stop(ws, FTC_KERNEL_DENSE_ALPHA, s);
  }
  return hipGetLastError();
}

}  // namespace ftc
