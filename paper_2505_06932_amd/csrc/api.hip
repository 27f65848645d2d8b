// api.hip -- the C ABI declared in include/ftc.h: argument validation,
// workspace allocation and the launch sequence of each call.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "ftc_ws.hpp"

using ftc::Grid;
using ftc::Mesh;

namespace {

bool grid_valid(const ftc_grid* g) {
  return g && g->nx > 4 && g->ny > 4 && g->nz > 4 && g->h > 0.0 && isfinite(g->h) && isfinite(g->x0) &&
         isfinite(g->y0) && isfinite(g->z0);
}

bool same_grid(const Grid& a, const ftc_grid* b) {
  return a.nx == b->nx && a.ny == b->ny && a.nz == b->nz && a.x0 == b->x0 && a.y0 == b->y0 && a.z0 == b->z0 &&
         a.h == b->h;
}

Grid to_grid(const ftc_grid* g) {
  Grid r;
  r.nx = g->nx;
  r.ny = g->ny;
  r.nz = g->nz;
  r.x0 = g->x0;
  r.y0 = g->y0;
  r.z0 = g->z0;
  r.h = g->h;
  r.dnx = ftc::FastDiv((uint32_t)g->nx);
  r.dny = ftc::FastDiv((uint32_t)g->ny);
  r.dncol = ftc::FastDiv((uint32_t)((int64_t)g->nx * g->ny));
  return r;
}

bool mesh_valid(const ftc_mesh* m) {
  return m && m->nv > 0 && m->nt > 0 && m->x && m->y && m->z && m->t0 && m->t1 && m->t2;
}

Mesh to_mesh(const ftc_mesh* m) { return Mesh{m->nv, m->nt, m->x, m->y, m->z, m->t0, m->t1, m->t2}; }

bool on_device(const ftc_cells* c) {
  int dev = -1;
  return c && hipGetDevice(&dev) == hipSuccess && dev == c->device;
}

ftc_status hip_status(hipError_t e) { return e == hipSuccess ? FTC_OK : FTC_EHIP; }

constexpr int kMaxBuffers = 64;  // device buffers one workspace owns

template <class T>
hipError_t alloc(T** p, int64_t n, void** registry, int& nreg) {
  *p = nullptr;
  if (nreg >= kMaxBuffers) return hipErrorOutOfMemory;  // never writes past the registry
  void* raw = nullptr;
  hipError_t e = hipMalloc(&raw, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  registry[nreg++] = raw;
  *p = static_cast<T*>(raw);
  return hipSuccess;
}

}  // namespace

struct ftc_cells_owner {
  ftc_cells ws;
  void* buffers[kMaxBuffers];
  int nbuf;
};

extern "C" {

ftc_status ftc_cells_create(ftc_cells** out, const ftc_grid* grid, int32_t nv_capacity, int32_t nt_capacity,
                            int64_t pair_capacity, int32_t cell_capacity) {
  if (!out) return FTC_EINVAL;
  *out = nullptr;
  if (!grid_valid(grid) || nv_capacity <= 0 || nt_capacity <= 0 || pair_capacity <= 0 || cell_capacity <= 0)
    return FTC_EINVAL;
  const int64_t ncell = (int64_t)grid->nx * grid->ny * grid->nz;
  const int64_t nwords = (ncell + 31) / 32;
  const int64_t ncol = (int64_t)grid->nx * grid->ny;
  // int32 cell ids and offsets; every scanned array within the scan limit
  if (ncell >= ((int64_t)1 << 31) || 3 * pair_capacity + 1024 >= ((int64_t)1 << 31) || nwords > ftc::kScanMax ||
      ncol > ftc::kScanMax || nt_capacity > ftc::kScanMax || nv_capacity > ftc::kScanMax ||
      cell_capacity > ftc::kScanMax || (int64_t)nt_capacity * 3 >= ((int64_t)1 << 31))
    return FTC_EINVAL;

  ftc_cells_owner* o = new (std::nothrow) ftc_cells_owner();
  if (!o) return FTC_ENOMEM;
  ftc_cells& w = o->ws;
  if (hipGetDevice(&w.device) != hipSuccess ||
      hipDeviceGetAttribute(&w.cu_count, hipDeviceAttributeMultiprocessorCount, w.device) != hipSuccess) {
    delete o;
    return FTC_EHIP;
  }
  w.grid = to_grid(grid);
  // measured best column chunking: 16 chunks up to 256 cells per column, 4 above
  w.tune.column_chunks = grid->nz > 256 ? 4 : 16;
  w.ncell = ncell;
  w.nwords = nwords;
  w.ncol = ncol;
  w.nv_cap = nv_capacity;
  w.nt_cap = nt_capacity;
  w.cell_cap = cell_capacity;
  w.built_nv = -1;
  w.built_nt = -1;
  w.builds = 0;
  w.band_build = -1;
  w.band_cap = 0;
  w.ppic_build = -1;
  w.pair_cap = pair_capacity;
  const int64_t P = pair_capacity, Cc = cell_capacity, Tc = nt_capacity, Vc = nv_capacity;
  void** reg = o->buffers;
  int& n = o->nbuf;
  n = 0;
  hipError_t e = hipSuccess;
#define FTC_ALLOC(field, count) \
  if (e == hipSuccess) e = alloc(&w.field, (count), reg, n)
  FTC_ALLOC(counters, ftc::C_COUNT);
  FTC_ALLOC(scan_tmp, ftc::kScanMaxBlocks);
  FTC_ALLOC(bitmap, nwords);
  w.colsum_words = (((int64_t)(grid->nx + ftc::kColBlock - 1) / ftc::kColBlock) * grid->ny *
                        ((grid->nz + ftc::kSlab - 1) / ftc::kSlab) + 31) / 32;
  FTC_ALLOC(colsum, w.colsum_words);
  FTC_ALLOC(word_off, nwords + 1);
  FTC_ALLOC(band_off, nwords + 1);
  w.queue_cap = 2 * P + 1024;  // candidates that need clipping can outnumber pieces
  FTC_ALLOC(pair_cell, P + w.queue_cap);
  FTC_ALLOC(pair_tri, P + w.queue_cap);
  FTC_ALLOC(pair_flux, P + w.queue_cap);
  FTC_ALLOC(pair_vol, P + w.queue_cap);
  FTC_ALLOC(tmp_rec, 4 * P);
  FTC_ALLOC(cell_ids, Cc);
  FTC_ALLOC(offsets, Cc + 1);
  FTC_ALLOC(pair_local, P + w.queue_cap);
  FTC_ALLOC(tri_ids, P);
  FTC_ALLOC(piece_flux, P);
  FTC_ALLOC(piece_vol, P);
  FTC_ALLOC(cell_flux, Cc);
  FTC_ALLOC(cell_vol, Cc);
  FTC_ALLOC(vt_off, Vc + 1);
  FTC_ALLOC(vt_cursor, Vc);
  FTC_ALLOC(vt_loc, 3 * Tc);
  FTC_ALLOC(vt_ids, 3 * Tc);
  FTC_ALLOC(tri4, 4 * Tc);
  FTC_ALLOC(vtx4, 4 * Vc);
  FTC_ALLOC(ovf_cells, Cc);
  FTC_ALLOC(vcell, Vc);
  FTC_ALLOC(vb_off, Cc + 1);
  FTC_ALLOC(vb_cursor, Cc);
  FTC_ALLOC(vb_loc, Vc);
  FTC_ALLOC(vb_rec, 4 * Vc);
  FTC_ALLOC(stray, Vc);
  FTC_ALLOC(frame_n, 3 * Cc);
  FTC_ALLOC(best_d2, Cc);
  FTC_ALLOC(best_v, Cc);
  FTC_ALLOC(best_inc, 2 * Cc);
  FTC_ALLOC(sel_cells, Cc);
  FTC_ALLOC(r_tn, 4 * (int64_t)nt_capacity);
  FTC_ALLOC(r_vG, nv_capacity);
  FTC_ALLOC(r_vV, nv_capacity);
  FTC_ALLOC(r_rt, nt_capacity);
  FTC_ALLOC(r_vflag, nv_capacity);
  FTC_ALLOC(r_estate, 3 * (int64_t)nt_capacity);
  FTC_ALLOC(r_elist, 3 * (int64_t)nt_capacity);
  FTC_ALLOC(quad_nodes, ftc::kQuadNodes);
#undef FTC_ALLOC
  w.timing = 0;
  int nev = 0;
  for (int k = 0; k < FTC_KERNEL_COUNT && e == hipSuccess; ++k) {
    w.ev_used[k] = 0;
    e = hipEventCreate(&w.ev_start[k]);
    if (e == hipSuccess) {
      e = hipEventCreate(&w.ev_stop[k]);
      if (e != hipSuccess) (void)hipEventDestroy(w.ev_start[k]);
    }
    if (e == hipSuccess) ++nev;
  }
  if (e == hipSuccess) {
    double nodes[ftc::kQuadNodes];
    ftc::paraboloid_nodes(nodes);
    e = hipMemcpy(w.quad_nodes, nodes, sizeof(nodes), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(w.counters, 0, sizeof(int32_t) * ftc::C_COUNT);
  // per-vertex and per-cell counts of the PPIC pre-passes start at zero and
  // are back at zero after every call
  if (e == hipSuccess) e = hipMemset(w.vt_cursor, 0, sizeof(int32_t) * Vc);
  if (e == hipSuccess) e = hipMemset(w.vb_cursor, 0, sizeof(int32_t) * Cc);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    for (int k = 0; k < nev; ++k) {
      (void)hipEventDestroy(w.ev_start[k]);
      (void)hipEventDestroy(w.ev_stop[k]);
    }
    for (int q = 0; q < n; ++q) (void)hipFree(reg[q]);
    delete o;
    return e == hipErrorOutOfMemory ? FTC_ENOMEM : FTC_EHIP;
  }
  static_assert(offsetof(ftc_cells_owner, ws) == 0, "owner layout");
  *out = &o->ws;
  return FTC_OK;
}

void ftc_cells_destroy(ftc_cells* cells) {
  if (!cells) return;
  ftc_cells_owner* o = reinterpret_cast<ftc_cells_owner*>(cells);
  (void)hipDeviceSynchronize();
  for (int k = 0; k < FTC_KERNEL_COUNT; ++k) {
    (void)hipEventDestroy(o->ws.ev_start[k]);
    (void)hipEventDestroy(o->ws.ev_stop[k]);
  }
  for (int q = 0; q < o->nbuf; ++q) (void)hipFree(o->buffers[q]);
  delete o;
}

ftc_status ftc_build_cell_lists(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid)) return FTC_EINVAL;
  if (mesh->nv > cells->nv_cap || mesh->nt > cells->nt_cap) return FTC_EINVAL;
  if (!on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_cell_lists(cells, to_mesh(mesh), (hipStream_t)stream));
}

ftc_status ftc_cells_count(const ftc_cells* cells, int32_t* n_interfacial, int64_t* n_pairs, void* stream) {
  if (!cells || !on_device(cells)) return FTC_EINVAL;
  int32_t h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(h, cells->counters, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return FTC_EHIP;
  // clamped to the capacities: past them the lists are truncated (and
  // FTC_ECAPACITY is latched), so no reader goes past a buffer
  if (n_interfacial) *n_interfacial = std::min<int32_t>(h[ftc::C_NIF], cells->cell_cap);
  if (n_pairs) *n_pairs = std::min<int64_t>(h[ftc::C_NPAIRS], cells->pair_cap);
  return FTC_OK;
}

ftc_status ftc_cells_view(const ftc_cells* cells, const int32_t** cell_ids, const int32_t** offsets,
                          const int32_t** tri_ids, const int32_t** d_counts) {
  if (!cells) return FTC_EINVAL;
  if (cell_ids) *cell_ids = cells->cell_ids;
  if (offsets) *offsets = cells->offsets;
  if (tri_ids) *tri_ids = cells->tri_ids;
  if (d_counts) *d_counts = cells->counters;
  return FTC_OK;
}

ftc_status ftc_volume_fraction(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, double* alpha_if,
                               double* alpha_dense, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid)) return FTC_EINVAL;
  if (mesh->nv > cells->nv_cap || mesh->nt > cells->nt_cap || (!alpha_if && !alpha_dense)) return FTC_EINVAL;
  if (!on_device(cells)) return FTC_EINVAL;
  return hip_status(
      ftc::launch_volume_fraction(cells, to_mesh(mesh), alpha_if, alpha_dense, (hipStream_t)stream));
}

ftc_status ftc_ppic_curvature(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                              const ftc_ppic_params* params, double* kappa, double* nx, double* ny, double* nz,
                              double* coeff, int32_t* cell_status, int32_t* diag, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid)) return FTC_EINVAL;
  if (mesh->nv > cells->nv_cap || mesh->nt > cells->nt_cap || !kappa || !nx || !ny || !nz) return FTC_EINVAL;
  // the vertex adjacency and closest vertices come from the last build
  if (mesh->nv != cells->built_nv || mesh->nt != cells->built_nt) return FTC_EINVAL;
  ftc::PPICParams p{2.5, 3, 24, 1.1, 16, 0};
  if (params) {
    p = ftc::PPICParams{params->delta_over_h, params->rings,    params->n_min,
                        params->grow,         params->max_iter, params->precision};
    if (!(p.delta_over_h > 0.0) || !isfinite(p.delta_over_h) || p.rings < 1 || p.rings > 4 || p.n_min < 1 ||
        !(p.grow > 1.0) || !isfinite(p.grow) || p.max_iter < 0 || p.max_iter > 64 || p.mixed < 0 ||
        p.mixed > 1)
      return FTC_EINVAL;
  }
  if (!on_device(cells)) return FTC_EINVAL;
  const ftc_status st = hip_status(
      ftc::launch_ppic(cells, to_mesh(mesh), p, kappa, nx, ny, nz, coeff, cell_status, diag, (hipStream_t)stream));
  cells->ppic_build = st == FTC_OK ? cells->builds : -1;
  return st;
}

ftc_status ftc_csf_force(const ftc_cells* cells, const ftc_grid* grid, const double* alpha_dense, const double* kappa,
                         double sigma, double* fx, double* fy, double* fz, void* stream) {
  if (!cells || !grid_valid(grid) || !same_grid(cells->grid, grid) || !alpha_dense || !kappa || !fx || !fy || !fz ||
      !isfinite(sigma))
    return FTC_EINVAL;
  if (!on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_csf(cells, alpha_dense, kappa, sigma, fx, fy, fz, (hipStream_t)stream));
}

ftc_status ftc_csf_force_band(ftc_cells* cells, const ftc_grid* grid, const double* alpha_dense,
                              const double* kappa, const double* nx, const double* ny, const double* nz, double sigma,
                              int32_t band_capacity, int32_t* band_ids, double* kappa_band, double* fx, double* fy,
                              double* fz, int32_t* d_n_band, void* stream) {
  if (!cells || !grid_valid(grid) || !same_grid(cells->grid, grid) || !alpha_dense || !kappa || !nx || !ny || !nz ||
      !band_ids || !kappa_band || !fx || !fy || !fz || !d_n_band || band_capacity <= 0 || !isfinite(sigma))
    return FTC_EINVAL;
  if (!on_device(cells)) return FTC_EINVAL;
  const ftc_status st = hip_status(ftc::launch_csf_band(cells, alpha_dense, kappa, nx, ny, nz, sigma, band_capacity,
                                                        band_ids, kappa_band, fx, fy, fz, d_n_band,
                                                        (hipStream_t)stream));
  if (st == FTC_OK) {
    cells->band_build = cells->builds;
    cells->band_cap = band_capacity;
  }
  return st;
}

ftc_status ftc_paraboloid_cell(const ftc_cells* cells, const ftc_grid* grid, const double* coeff,
                               double* alpha_paraboloid, double* kappa_cell, double* normal_cell, void* stream) {
  if (!cells || !grid_valid(grid) || !same_grid(cells->grid, grid) || !coeff || !alpha_paraboloid)
    return FTC_EINVAL;
  if (!on_device(cells) || cells->builds == 0 || cells->ppic_build != cells->builds) return FTC_EINVAL;
  return hip_status(
      ftc::launch_paraboloid_cell(cells, coeff, alpha_paraboloid, kappa_cell, normal_cell, (hipStream_t)stream));
}

ftc_status ftc_surface_tension_flux(ftc_cells* cells, const ftc_grid* grid, const double* alpha_dense,
                                    const double* kappa, int32_t band_capacity, const int32_t* band_ids,
                                    const double* kappa_band, const int32_t* d_n_band, double rho_a, double rho_b,
                                    double sigma, double* flux_if, double* flux_band, void* stream) {
  if (!cells || !grid_valid(grid) || !same_grid(cells->grid, grid) || !alpha_dense || !kappa || !band_ids ||
      !kappa_band || !d_n_band || !flux_if || !flux_band || band_capacity <= 0 || !isfinite(sigma) ||
      !(rho_a > 0.0) || !(rho_b > 0.0) || !isfinite(rho_a) || !isfinite(rho_b))
    return FTC_EINVAL;
  if (!on_device(cells) || cells->builds == 0 || cells->band_build != cells->builds ||
      band_capacity != cells->band_cap)
    return FTC_EINVAL;
  return hip_status(ftc::launch_face_flux(cells, alpha_dense, kappa, band_capacity, band_ids, kappa_band, d_n_band,
                                          rho_a, rho_b, sigma, flux_if, flux_band, (hipStream_t)stream));
}

ftc_status ftc_interp_vertex_velocity(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, const double* U,
                                      const double* V, const double* W, double* ux, double* uy, double* uz,
                                      void* stream) {
  if (!cells || !grid_valid(grid) || !mesh || mesh->nv <= 0 || !mesh->x || !mesh->y || !mesh->z || !U || !V || !W ||
      !ux || !uy || !uz)
    return FTC_EINVAL;
  if (!on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_interp(cells, to_grid(grid), to_mesh(mesh), U, V, W, ux, uy, uz, (hipStream_t)stream));
}

ftc_status ftc_advect_vertices_rk4(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, const double* U,
                                   const double* V, const double* W, double dt, double* x_out, double* y_out,
                                   double* z_out, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh || mesh->nv <= 0 || !mesh->x || !mesh->y || !mesh->z || !U || !V || !W ||
      !x_out || !y_out || !z_out || !isfinite(dt))
    return FTC_EINVAL;
  if (!on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_advect_rk4(cells, to_grid(grid), to_mesh(mesh), U, V, W, dt, x_out, y_out, z_out,
                                           (hipStream_t)stream));
}

ftc_status ftc_curvature_features(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                  const double* alpha_dense, float* features, int32_t* final_flags, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid) || !alpha_dense || !features)
    return FTC_EINVAL;
  if (mesh->nv != cells->built_nv || mesh->nt != cells->built_nt || !on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_features(cells, to_mesh(mesh), alpha_dense, features, final_flags,
                                         (hipStream_t)stream));
}

ftc_status ftc_mlp_forward(const float* theta, const float* X, int64_t rows, const int32_t* idx, const int32_t* sym,
                           int32_t n, float* y, void* stream) {
  if (!theta || !X || rows <= 0 || n < 0 || !y) return FTC_EINVAL;
  if (n == 0) return FTC_OK;
  return hip_status(ftc::launch_mlp_forward(theta, X, rows, idx, sym, n, y, (hipStream_t)stream));
}

ftc_status ftc_mlp_loss_grad(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                             const int32_t* sym, const float* t, int32_t n, float* grad, float* loss, float* work,
                             void* stream) {
  if (!theta || !X || rows <= 0 || !t || n <= 0 || !grad || !work) return FTC_EINVAL;
  return hip_status(ftc::launch_mlp_loss_grad(theta, X, rows, idx, sym, t, n, grad, loss, work, (hipStream_t)stream));
}

ftc_status ftc_mlp_loss_grad_static(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                                    const int32_t* sym, const float* t, int32_t n, float* grad, float* loss,
                                    void* stream) {
  if (!theta || !X || rows <= 0 || !t || n <= 0 || !grad) return FTC_EINVAL;
  return hip_status(ftc::launch_mlp_loss_grad_static(theta, X, rows, idx, sym, t, n, grad, loss, (hipStream_t)stream));
}

ftc_status ftc_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream) {
  if (!theta || !m || !v || !grad || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return FTC_EINVAL;
  return hip_status(ftc::launch_mlp_adam(theta, m, v, grad, step, lr, beta1, beta2, eps, (hipStream_t)stream));
}

ftc_status ftc_learned_curvature(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                 const double* alpha_dense, const float* theta, double bound,
                                 const ftc_ppic_params* params, double* kappa, double* nx, double* ny, double* nz,
                                 float* spread, int32_t* cell_status, int32_t* d_n_fallback, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid) || !alpha_dense || !theta ||
      !kappa || !nx || !ny || !nz || !(bound >= 0.0))
    return FTC_EINVAL;
  if (mesh->nv != cells->built_nv || mesh->nt != cells->built_nt) return FTC_EINVAL;
  ftc::PPICParams p{2.5, 3, 24, 1.1, 16, 0};
  if (params) {
    p = ftc::PPICParams{params->delta_over_h, params->rings,    params->n_min,
                        params->grow,         params->max_iter, params->precision};
    if (!(p.delta_over_h > 0.0) || !isfinite(p.delta_over_h) || p.rings < 1 || p.rings > 4 || p.n_min < 1 ||
        !(p.grow > 1.0) || !isfinite(p.grow) || p.max_iter < 0 || p.max_iter > 64 || p.mixed < 0 ||
        p.mixed > 1)
      return FTC_EINVAL;
  }
  if (!on_device(cells)) return FTC_EINVAL;
  cells->ppic_build = -1;  // PPIC runs for the fallback cells only
  return hip_status(ftc::launch_surrogate(cells, to_mesh(mesh), alpha_dense, theta, (float)bound, p, kappa, nx, ny,
                                          nz, spread, cell_status, d_n_fallback, (hipStream_t)stream));
}

ftc_status ftc_front_roughness(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, double* gl_mag,
                               double* rough, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid) || !gl_mag || !rough)
    return FTC_EINVAL;
  if (mesh->nv != cells->built_nv || mesh->nt != cells->built_nt || !on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_roughness(cells, to_mesh(mesh), gl_mag, rough, (hipStream_t)stream));
}

ftc_status ftc_smooth_rough_edges(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, const double* gl_mag,
                                  const double* rough, double gl_threshold, double rough_threshold, int32_t max_rounds,
                                  double* x_out, double* y_out, double* z_out, int32_t* d_counts, void* stream) {
  if (!cells || !grid_valid(grid) || !mesh_valid(mesh) || !same_grid(cells->grid, grid) || !gl_mag || !rough || !x_out ||
      !y_out || !z_out || !d_counts || max_rounds < 0 || max_rounds > 4096 || isnan(gl_threshold) ||
      isnan(rough_threshold))
    return FTC_EINVAL;
  if (mesh->nv != cells->built_nv || mesh->nt != cells->built_nt || !on_device(cells)) return FTC_EINVAL;
  return hip_status(ftc::launch_smooth(cells, to_mesh(mesh), gl_mag, rough, gl_threshold, rough_threshold, max_rounds,
                                       x_out, y_out, z_out, d_counts, (hipStream_t)stream));
}

ftc_status ftc_get_tuning(const ftc_cells* cells, ftc_tuning* out) {
  if (!cells || !out) return FTC_EINVAL;
  out->ring_lanes = cells->tune.ring_lanes;
  out->column_chunks = cells->tune.column_chunks;
  out->ring_blocks = cells->tune.ring_blocks;
  out->queue_chunk = cells->tune.queue_chunk;
  return FTC_OK;
}

ftc_status ftc_set_tuning(ftc_cells* cells, const ftc_tuning* in) {
  if (!cells || !in) return FTC_EINVAL;
  const int32_t L = in->ring_lanes;
  if ((L != 4 && L != 8 && L != 16 && L != 32 && L != 64) ||
      (in->column_chunks != 4 && in->column_chunks != 8 && in->column_chunks != 16) || in->ring_blocks < 0 ||
      in->ring_blocks > 65536 || in->queue_chunk < 0 || in->queue_chunk > 64)
    return FTC_EINVAL;
  cells->tune.ring_lanes = in->ring_lanes;
  cells->tune.column_chunks = in->column_chunks;
  cells->tune.ring_blocks = in->ring_blocks;
  cells->tune.queue_chunk = in->queue_chunk;
  return FTC_OK;
}

ftc_status ftc_last_device_error(ftc_cells* cells, int32_t* code, void* stream) {
  if (!cells || !code || !on_device(cells)) return FTC_EINVAL;
  int32_t err = 0;
  const int32_t zero = 0;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&err, cells->counters + ftc::C_ERR, sizeof(err), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpyAsync(cells->counters + ftc::C_ERR, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return FTC_EHIP;
  if (err & ftc::ERR_CAPACITY)
    *code = FTC_ECAPACITY;
  else if (err & ftc::ERR_DOMAIN)
    *code = FTC_EDOMAIN;
  else if (err & ftc::ERR_MESH)
    *code = FTC_EMESH;
  else
    *code = FTC_OK;
  return FTC_OK;
}

ftc_status ftc_set_timing(ftc_cells* cells, int32_t enable) {
  if (!cells) return FTC_EINVAL;
  cells->timing = enable ? 1 : 0;
  return FTC_OK;
}

ftc_status ftc_kernel_time(const ftc_cells* cells, int32_t kernel, float* ms) {
  if (!cells || !ms || kernel < 0 || kernel >= FTC_KERNEL_COUNT || !cells->ev_used[kernel]) return FTC_EINVAL;
  hipError_t e = hipEventSynchronize(cells->ev_stop[kernel]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, cells->ev_start[kernel], cells->ev_stop[kernel]);
  return e == hipSuccess ? FTC_OK : FTC_EHIP;
}

const char* ftc_status_str(int32_t status) {
  switch (status) {
    case FTC_OK: return "ok";
    case FTC_EINVAL: return "invalid argument";
    case FTC_EDOMAIN: return "front vertex outside the grid margin";
    case FTC_EMESH: return "front not closed or not outward oriented";
    case FTC_ECAPACITY: return "workspace capacity exceeded";
    case FTC_ENOMEM: return "device allocation failed";
    case FTC_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

}  // extern "C"
