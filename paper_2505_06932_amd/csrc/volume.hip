// volume.hip -- exact volume fractions of the interfacial cells and the dense
// indicator field.
//
// With F = (0, 0, z - zlo) (divergence 1) the divergence theorem on
// Omega cap C gives |Omega cap C| = sum over the cell's pieces of the
// integral of (z - zlo) n_z dA, plus h times the wetted area W of the upper
// face (F . n vanishes on the lower and side faces).  With F = (0, 0, 1) on
// the column above the cell, W is the sum of the integrals of n_z dA over
// all pieces strictly above.  Kernels:
//   pieces : one thread per (cell, triangle) piece -> its two integrals;
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

__global__ __launch_bounds__(kT) void k_vf_pieces(Grid g, Mesh m, const int32_t* slot_cell, const int32_t* tri_ids,
                                                  const int32_t* cell_ids, const int32_t* offsets,
                                                  double* piece_flux, double* piece_vol, int32_t cell_cap,
                                                  int64_t pair_cap, const int32_t* counters) {
  // only the CSR slots that were filled (fewer than the pairs on overflow)
  const int64_t np = min((int64_t)offsets[min(counters[C_NIF], cell_cap)], pair_cap);
  for (int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x; p < np; p += (int64_t)gridDim.x * kT) {
    const int32_t ci = slot_cell[p];
    const int32_t lin = cell_ids[ci];
    const int64_t i = lin % g.nx, j = (lin / g.nx) % g.ny, k = lin / ((int64_t)g.nx * g.ny);
    Tri T = load_tri(m, tri_ids[p]);
    Poly P;
    double f = 0.0, v = 0.0;
    if (clip_cell(g, T, i, j, k, P)) piece_z_integrals(P, grid_plane(g.z0, k, g.h), f, v);
    piece_flux[p] = f;
    piece_vol[p] = v;
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
  const int64_t ncol = (int64_t)g.nx * g.ny;
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x)
    atomicAdd(&col_cnt[cell_ids[ci] % ncol], 1);
}

__global__ void k_col_scatter(Grid g, const int32_t* cell_ids, const int32_t* col_off, int32_t* col_cursor,
                              int32_t* col_cells, int32_t cell_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  const int64_t ncol = (int64_t)g.nx * g.ny;
  for (int32_t ci = blockIdx.x * blockDim.x + threadIdx.x; ci < nif; ci += gridDim.x * blockDim.x) {
    const int64_t col = cell_ids[ci] % ncol;
    col_cells[col_off[col] + atomicAdd(&col_cursor[col], 1)] = ci;
  }
}

__global__ void k_col_walk(Grid g, const int32_t* col_off, int32_t* col_cells, const int32_t* cell_ids,
                           const int32_t* offsets, const double* piece_flux, const double* piece_vol,
                           int32_t* col_k, double* col_alpha, double* col_below, double* alpha_if,
                           int32_t* counters) {
  const int64_t ncol = (int64_t)g.nx * g.ny;
  const double h = g.h, h2 = h * h, h3 = h * h * h;
  for (int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; col < ncol;
       col += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = col_off[col], e = col_off[col + 1];
    if (s == e) continue;
    // ascending compact index == ascending k within one column
    for (int32_t a = s + 1; a < e; ++a) {
      const int32_t v = col_cells[a];
      int32_t b = a - 1;
      while (b >= s && col_cells[b] > v) {
        col_cells[b + 1] = col_cells[b];
        --b;
      }
      col_cells[b + 1] = v;
    }
    bool bad = false;
    double W = 0.0;
    int32_t prev_k = g.nz;
    for (int32_t q = e - 1; q >= s; --q) {
      const int32_t ci = col_cells[q];
      const int32_t k = (int32_t)(cell_ids[ci] / ncol);
      if (prev_k - k > 1) {  // non-interfacial cells between this cell and the one above
        const double r = W / h2, rr = rint(r);
        if (fabs(r - rr) > 1e-9 || (rr != 0.0 && rr != 1.0)) bad = true;
      }
      double f = 0.0, v = 0.0;
      for (int32_t p = offsets[ci]; p < offsets[ci + 1]; ++p) {
        f += piece_flux[p];
        v += piece_vol[p];
      }
      const double alpha = (v + h * W) / h3;
      if (alpha_if) alpha_if[ci] = alpha;
      col_k[q] = k;
      col_alpha[q] = alpha;
      W += f;
      const double rb = rint(W / h2);
      col_below[q] = rb == 1.0 ? 1.0 : 0.0;
      prev_k = k;
    }
    if (fabs(W / h2) > 1e-9) bad = true;  // the column must close below the front
    if (bad) atomicOr(&counters[C_ERR], ERR_MESH);
  }
}

__global__ __launch_bounds__(kT) void k_dense(Grid g, const int32_t* col_off, const int32_t* col_k,
                                              const double* col_alpha, const double* col_below, double* alpha) {
  const int64_t ncol = (int64_t)g.nx * g.ny, ncell = ncol * g.nz;
  for (int64_t lin = (int64_t)blockIdx.x * kT + threadIdx.x; lin < ncell; lin += (int64_t)gridDim.x * kT) {
    const int64_t col = lin % ncol;
    const int32_t k = (int32_t)(lin / ncol);
    const int32_t s = col_off[col], e = col_off[col + 1];
    double a = 0.0;
    for (int32_t q = s; q < e; ++q) {
      const int32_t kq = col_k[q];
      if (kq >= k) {
        a = (kq == k) ? col_alpha[q] : col_below[q];
        break;
      }
    }
    alpha[lin] = a;
  }
}

}  // namespace

hipError_t launch_volume_fraction(const ftc_cells* ws, const Mesh& m, double* alpha_if, double* alpha_dense,
                                  hipStream_t s) {
  const Grid& g = ws->grid;
  time_start(ws, FTC_KERNEL_VF_PIECES, s);
  hipLaunchKernelGGL(k_vf_pieces, dim3(grid_blocks(ws->pair_cap, kT, kStrideBlocks)), dim3(kT), 0, s, g, m,
                     ws->slot_cell, ws->tri_ids, ws->cell_ids, ws->offsets, ws->piece_flux, ws->piece_vol,
                     ws->cell_cap, ws->pair_cap, ws->counters);
  time_stop(ws, FTC_KERNEL_VF_PIECES, s);
  hipLaunchKernelGGL(k_clear_cols, dim3(grid_blocks(ws->ncol + 1, kT, kStrideBlocks)), dim3(kT), 0, s, ws->col_off,
                     ws->ncol + 1, ws->col_cursor, ws->ncol);
  hipLaunchKernelGGL(k_col_count, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, g,
                     ws->cell_ids, ws->col_off, ws->cell_cap, ws->counters);
  hipError_t e = scan_exclusive(ws->col_off, ws->ncol, ws->scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_scatter, dim3(grid_blocks(ws->cell_cap, kT, kStrideBlocks)), dim3(kT), 0, s, g,
                     ws->cell_ids, ws->col_off, ws->col_cursor, ws->col_cells, ws->cell_cap, ws->counters);
  time_start(ws, FTC_KERNEL_COL_WALK, s);
  hipLaunchKernelGGL(k_col_walk, dim3(grid_blocks(ws->ncol, kT, kStrideBlocks)), dim3(kT), 0, s, g, ws->col_off,
                     ws->col_cells, ws->cell_ids, ws->offsets, ws->piece_flux, ws->piece_vol, ws->col_k,
                     ws->col_alpha, ws->col_below, alpha_if, ws->counters);
  time_stop(ws, FTC_KERNEL_COL_WALK, s);
  if (alpha_dense) {
    time_start(ws, FTC_KERNEL_DENSE_ALPHA, s);
    hipLaunchKernelGGL(k_dense, dim3(grid_blocks(ws->ncell, kT, 16384)), dim3(kT), 0, s, g, ws->col_off, ws->col_k,
                       ws->col_alpha, ws->col_below, alpha_dense);
    time_stop(ws, FTC_KERNEL_DENSE_ALPHA, s);
  }
  return hipGetLastError();
}

}  // namespace ftc
