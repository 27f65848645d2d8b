// ftc_ws.hpp -- the workspace behind the opaque ftc_cells handle and the
// internal launchers of each kernel group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftc_device.hpp"

// Counter slots in ftc_cells::counters (device int32).
namespace ftc {
constexpr int kQuadNodes = 96;  // nodes and weights: 16 and 24 (the two xi rules) + 8 (eta rule)
enum : int {
  C_NIF = 0,      // interfacial cells of the last build
  C_NPAIRS = 1,   // (cell, triangle) pieces of the last build
  C_ERR = 2,      // latched ERR_* bits
  C_NQUEUE = 3,   // candidates queued for full clipping
  C_NWHOLE = 4,   // pieces that are whole triangles
  C_NSTRAY = 5,   // vertices in cells without pieces
  C_NOVF = 6,     // interfacial cells queued for the wide PPIC shape
  C_WIDE_DONE = 7,  // workgroups of the wide PPIC shape that have read the queue's count
  C_NSEL = 8,      // cells the learned curvature hands to PPIC (cleared after the PPIC kernel)
  C_SPARE = 9,     // unused
  C_RFLAG = 10,    // edges listed for roughness smoothing
  C_RMOVED = 11,   // edges moved by it
  C_QUEUE0 = 32,   // [8 x kQStride] next chunk of each XCD's range in the fast PPIC shape's work
                   // queue, one 128-byte line each
  C_COUNT = 32 + 8 * 32
};
constexpr int kQStride = 32;
constexpr int kColBlock = 64;  // columns along x per bit of the column summary
constexpr int kSlab = 32;      // planes along z per bit of the column summary
}  // namespace ftc

namespace ftc {
// Launch shapes chosen per workspace (ftc_set_tuning; defaults below).
struct Tuning {
  int32_t ring_lanes = 8;     // lanes per cell in the fast PPIC shape: 4, 8, 16, 32 or 64
  int32_t column_chunks = 16;  // z-chunks (wavefronts) per column block: 4, 8 or 16 (set from nz at creation)
  int32_t ring_blocks = 0;    // workgroups of the fast PPIC shape: 0 = one per cell group (or, with a work
                              // queue, the resident wavefronts), else a persistent grid of that many
  int32_t queue_chunk = 0;    // cell groups per draw from the fast PPIC shape's work queue (0: static split)
};
}  // namespace ftc

struct ftc_cells {
  int device;
  int cu_count;  // compute units of the device
  ftc::Tuning tune;
  ftc::Grid grid;
  int64_t ncell, nwords, ncol;
  int32_t nv_cap, nt_cap, cell_cap;
  int32_t built_nv, built_nt;  // front sizes of the last build (-1 before the first)
  int64_t builds;      // builds enqueued so far
  int64_t band_build;  // value of `builds` when the band was last listed (-1: never)
  int32_t band_cap;    // the band capacity of that listing
  mutable int64_t ppic_build;  // value of `builds` at the last plain PPIC call (-1: none since)
  int64_t pair_cap;
  int64_t queue_cap;  // candidates queued for full clipping (>= pair_cap)

  int32_t* counters;  // [C_COUNT]
  int32_t* scan_tmp;  // block partial sums of the device-wide scans

  // cell lists
  uint32_t* bitmap;       // [nwords] one bit per grid cell: holds a piece
  uint32_t* colsum;       // [colsum_words] one bit per (64-column block along x, row j, slab of 32
                          // planes along z): some cell of it holds a piece; written from the bitmap
                          // by the volume-fraction call when nx is a multiple of 64
  int64_t colsum_words;
  int32_t* word_off;      // [nwords+1] exclusive scan of popcount(bitmap)
  int32_t* band_off;      // [nwords+1] the same for the face-neighbour band (CSF band mode)
  // pair list: [0, pair_cap) whole-triangle pieces, [pair_cap, pair_cap +
  // queue_cap) candidates queued for clipping (cell -1 if no piece)
  int32_t* pair_cell;     // linear, then compact, cell of each piece
  int32_t* pair_tri;      // triangle of each piece
  double* pair_flux;      // integral of n_z dA
  double* pair_vol;       // integral of (z - zlo) n_z dA
  double* tmp_rec;        // [4*pair_cap] pieces scattered into their cell's segment, 32-byte records
                          // (triangle, compact cell, 0, 0 as int32; flux; volume integral)
  int32_t* cell_ids;      // [cell_cap] linear ids, ascending
  int32_t* offsets;       // [cell_cap+1] CSR offsets into tri_ids
  int32_t* pair_local;    // [pair_cap + queue_cap] index of each pair within its cell, from the counting
  int32_t* tri_ids;       // [pair_cap] CSR triangle ids, ascending per cell
  double* piece_flux;     // [pair_cap] integral of n_z dA per CSR slot
  double* piece_vol;      // [pair_cap] integral of (z - zlo) n_z dA per CSR slot

  // volume fraction
  double* cell_flux;      // [cell_cap] sum of the cell's piece fluxes
  double* cell_vol;       // [cell_cap] sum of the cell's piece volume integrals
  // PPIC
  int32_t* vt_off;        // [nv_cap+1] offsets of each vertex's incident triangles
  int32_t* vt_cursor;     // [nv_cap] triangles per vertex while counting; zero between calls
  int32_t* vt_loc;        // [3*nt_cap] index of each (triangle, corner) within the corner's list
  int32_t* vt_ids;        // [3*nt_cap] incident triangles, ascending per vertex
  int32_t* tri4;          // [4*nt_cap] corners of each triangle packed (t0, t1, t2, 0)
  double* vtx4;           // [4*nv_cap] coordinates of each vertex packed (x, y, z, 0)
  int32_t* ovf_cells;     // [cell_cap] cells queued for the wide PPIC shape
  int32_t* vcell;         // [nv_cap] interfacial cell holding each vertex (-1: none, -2: outside)
  int32_t* vb_off;        // [cell_cap+1] offsets of each interfacial cell's vertices
  int32_t* vb_cursor;     // [cell_cap] vertices per cell while counting; zero between calls
  int32_t* vb_loc;        // [nv_cap] index of each vertex within its cell's bin
  double* vb_rec;         // [4*nv_cap] vertices grouped by interfacial cell: x, y, z, index (as the bits
                          // of a double)
  int32_t* stray;         // [nv_cap] vertices in cells without pieces
  double* frame_n;        // [3 * cell_cap] frame normal of each cell's volume fit
  double* quad_nodes;     // [kQuadNodes] quadrature nodes and weights of the paraboloid cell integrals
  int32_t* sel_cells;     // [cell_cap] cells the learned curvature hands to PPIC
  // roughness detection and smoothing
  double* r_tn;           // [4 * nt_cap] unit normal and area of each triangle
  double* r_vG;           // [nv_cap] mean edge roughness at each vertex
  double* r_vV;           // [nv_cap] its variance
  double* r_rt;           // [nt_cap] triangle roughness statistic
  int32_t* r_vflag;       // [nv_cap] rough vertices
  int32_t* r_estate;      // [3 * nt_cap] state of each edge (by its owning half-edge)
  int32_t* r_elist;       // [3 * nt_cap] edges listed for smoothing
  double* best_d2;        // [cell_cap] smallest squared distance of a vertex in the 27 cells around
  int32_t* best_v;        // [cell_cap] lowest vertex attaining it
  int32_t* best_inc;      // [2 * cell_cap] (offset, count) of best_v's incident-triangle list

  // optional timing events around the dominant kernel of each call
  int timing;
  hipEvent_t ev_start[FTC_KERNEL_COUNT], ev_stop[FTC_KERNEL_COUNT];
  int ev_used[FTC_KERNEL_COUNT];
};

namespace ftc {

// Device-wide exclusive scan of n int32 values (in place: data[0..n) becomes
// the exclusive prefix sums and data[n] the total); the total is also copied
// to *total_out when non-null.  Supports n <= kScanMax.
constexpr int64_t kScanBlock = 2048;
constexpr int64_t kScanMaxBlocks = 8192;
constexpr int64_t kScanMax = kScanBlock * kScanMaxBlocks;
hipError_t scan_exclusive(int32_t* data, int64_t n, int32_t* tmp, int32_t* total_out, hipStream_t s);
// Same, with inputs popcount(words[i]) (output to out[0..n], total to out[n]).
hipError_t scan_popcount(const uint32_t* words, int32_t* out, int64_t n, int32_t* tmp, int32_t* total_out,
                         hipStream_t s);

// scan_popcount that also lists the set bits in ascending order: bit b of
// word w goes to ids[out[w] + rank of b in w] as 32 w + b; entries at or
// past `cap` are dropped and latch ERR_CAPACITY in counters[C_ERR].
hipError_t scan_popcount_emit(const uint32_t* words, int32_t* out, int64_t n, int32_t* tmp, int32_t* total_out,
                              int32_t* ids, int32_t cap, int32_t* counters, hipStream_t s);

// The same over the face-neighbour band of the occupancy bitmap (cells not
// in it with a face neighbour in it; sy = nx, sz = nx ny), computed word by
// word on the fly: out[nwords+1] offsets, ids the band cells' linear ids.
hipError_t scan_band_emit(const uint32_t* bitmap, int64_t nwords, int64_t ncell, int64_t sy, int64_t sz, int32_t* out,
                          int32_t* tmp, int32_t* total_out, int32_t* ids, int32_t cap, int32_t* counters,
                          hipStream_t s);

// Up to three independent exclusive scans in one pair of launches: segment
// q turns in[0..n) into out[0..n] (total last, and into *total when
// non-null); in place is allowed.
struct ScanSeg {
  const int32_t* in;
  int32_t* out;
  int64_t n;
  int32_t* total;
  int32_t* clear;  // NULL, or `in` again: set to zero once read (counts that must start the next call at zero)
};
constexpr int kMaxSeg = 3;
hipError_t scan_exclusive_multi(const ScanSeg* segs, int nseg, int32_t* tmp, hipStream_t s);

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

hipError_t launch_cell_lists(ftc_cells* ws, const Mesh& m, hipStream_t s);
hipError_t launch_volume_fraction(const ftc_cells* ws, const Mesh& m, double* alpha_if, double* alpha_dense,
                                  hipStream_t s);

struct PPICParams {
  double delta_over_h;
  int32_t rings, n_min;
  double grow;
  int32_t max_iter;
  int32_t mixed;  // 1: normal equations in single precision, refined in double
};
hipError_t launch_ppic(const ftc_cells* ws, const Mesh& m, const PPICParams& p, double* kappa, double* nx,
                       double* ny, double* nz, double* coeff, int32_t* cell_status, int32_t* diag,
                       hipStream_t s);
// The PPIC kernels on the cells sel[0, counters[C_NSEL]) only (sel non-null).
hipError_t launch_ppic_cells(const ftc_cells* ws, const Mesh& m, const PPICParams& p, double* kappa, double* nx,
                             double* ny, double* nz, double* coeff, int32_t* cell_status, int32_t* diag,
                             const int32_t* sel, int32_t* n_sel_out, hipStream_t s);
// Learned curvature (surrogate.hip).
hipError_t launch_features(const ftc_cells* ws, const Mesh& m, const double* alpha, float* feat, int32_t* fstat,
                           hipStream_t s);
hipError_t launch_mlp_forward(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                              const int32_t* sym, int32_t n, float* y, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                                const int32_t* sym, const float* t, int32_t n, float* grad, float* loss, float* work,
                                hipStream_t s);
// The same with the partial rows in the library's own per-device scratch
// (allocates nothing).
hipError_t launch_mlp_loss_grad_static(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                                       const int32_t* sym, const float* t, int32_t n, float* grad, float* loss,
                                       hipStream_t s);
hipError_t launch_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                           float beta2, float eps, hipStream_t s);
hipError_t launch_surrogate(const ftc_cells* ws, const Mesh& m, const double* alpha, const float* theta, float bound,
                            const PPICParams& p, double* kappa, double* nx, double* ny, double* nz, float* spread,
                            int32_t* status, int32_t* n_fallback, hipStream_t s);
// Roughness (roughness.hip).
hipError_t launch_roughness(const ftc_cells* ws, const Mesh& m, double* gl_mag, double* rough, hipStream_t s);
hipError_t launch_smooth(const ftc_cells* ws, const Mesh& m, const double* gl_mag, const double* rough, double gl_thr,
                         double rough_thr, int32_t max_rounds, double* xo, double* yo, double* zo, int32_t* d_counts,
                         hipStream_t s);
hipError_t launch_csf(const ftc_cells* ws, const double* alpha, const double* kappa, double sigma, double* fx,
                      double* fy, double* fz, hipStream_t s);
hipError_t launch_csf_band(const ftc_cells* ws, const double* alpha, const double* kappa, const double* nx,
                           const double* ny, const double* nz, double sigma, int32_t band_cap, int32_t* band_ids,
                           double* kappa_band, double* fx, double* fy, double* fz, int32_t* n_band, hipStream_t s);
// The quadrature tables of the paraboloid cell integrals, host side: out[kQuadNodes].
void paraboloid_nodes(double* out);
hipError_t launch_paraboloid_cell(const ftc_cells* ws, const double* coeff, double* alpha_out, double* kappa_out,
                                  double* normal_out, hipStream_t s);
hipError_t launch_face_flux(const ftc_cells* ws, const double* alpha, const double* kappa, int32_t band_cap,
                            const int32_t* band_ids, const double* kappa_band, const int32_t* n_band, double rho_a,
                            double rho_b, double sigma, double* flux_if, double* flux_band, hipStream_t s);
hipError_t launch_interp(const ftc_cells* ws, const Grid& g, const Mesh& m, const double* U, const double* V,
                         const double* W, double* ux, double* uy, double* uz, hipStream_t s);
hipError_t launch_advect_rk4(const ftc_cells* ws, const Grid& g, const Mesh& m, const double* U, const double* V,
                             const double* W, double dt, double* xo, double* yo, double* zo, hipStream_t s);

// Record the start / stop event of kernel `k` when timing is enabled.
inline void time_start(const ftc_cells* ws, int k, hipStream_t s) {
  if (ws->timing) (void)hipEventRecord(ws->ev_start[k], s);
}
inline void time_stop(const ftc_cells* ws, int k, hipStream_t s) {
  if (ws->timing) {
    (void)hipEventRecord(ws->ev_stop[k], s);
    const_cast<ftc_cells*>(ws)->ev_used[k] = 1;
  }
}

inline int32_t grid_blocks(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int32_t)b;
}

}  // namespace ftc
