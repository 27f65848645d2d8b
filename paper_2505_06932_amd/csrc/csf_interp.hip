// csf_interp.hip -- CSF source on the interfacial cells (paper Eq. csf), its
// band mode, the divergence-preserving interpolation of staggered face
// velocities to the front vertices and the RK4 step of the vertices through
// it (paper section 3.1).  Both are gather kernels bound by
// memory traffic: one thread per interfacial cell, one thread per vertex.
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kT = 64;  // one wavefront per workgroup: small launches spread over every CU

__global__ __launch_bounds__(kT) void k_csf(Grid g, const int32_t* cell_ids, const double* alpha,
                                            const double* kappa, double sigma, double* fx, double* fy, double* fz,
                                            int32_t cell_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap);
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  const double inv2h = 1.0 / (2.0 * g.h);
  for (int32_t c = blockIdx.x * kT + threadIdx.x; c < nif; c += gridDim.x * kT) {
    const int64_t lin = cell_ids[c];
    // interfacial cells lie at least two cells inside the grid, so every
    // neighbour exists
    const double gx = (alpha[lin + 1] - alpha[lin - 1]) * inv2h;
    const double gy = (alpha[lin + sy] - alpha[lin - sy]) * inv2h;
    const double gz = (alpha[lin + sz] - alpha[lin - sz]) * inv2h;
    const double sk = sigma * kappa[c];
    fx[c] = sk * gx;
    fy[c] = sk * gy;
    fz[c] = sk * gz;
  }
}

// Band mode: per band cell (face neighbour of an interfacial cell, not
// interfacial), the weighted average of the finite curvatures of the
// interfacial cells among its 26 neighbours (block order, x fastest) with
// weights |s.n| / |s|, s = (di, dj, dk) h the offset to the neighbour and n
// its interface normal; the plain mean if every weight vanishes, NaN if
// there is no such neighbour.  Then sigma kappa_bar grad(alpha).  A band
// cell is at least one cell inside the grid, so all its neighbours exist.
__global__ __launch_bounds__(kT) void k_csf_band(Grid g, const uint32_t* bitmap, const int32_t* word_off,
                                                 const double* alpha, const double* kappa, const double* nx,
                                                 const double* ny, const double* nz, double sigma,
                                                 const int32_t* band_ids, const int32_t* n_band, int32_t band_cap,
                                                 double* kappa_band, double* fx, double* fy, double* fz,
                                                 int32_t cell_cap) {
  const int32_t nb = min(*n_band, band_cap);
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  const double inv2h = 1.0 / (2.0 * g.h);
  for (int32_t b = blockIdx.x * kT + threadIdx.x; b < nb; b += gridDim.x * kT) {
    const int64_t lin = band_ids[b];
    double sw = 0.0, swk = 0.0, sk = 0.0;
    int32_t nq = 0;
    for (int dk = -1; dk <= 1; ++dk)
      for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
          if (di == 0 && dj == 0 && dk == 0) continue;
          const int32_t q = cell_rank(bitmap, word_off, lin + di + dj * sy + dk * sz);
          if (q < 0 || q >= cell_cap) continue;
          const double kq = kappa[q];
          if (!isfinite(kq)) continue;
          const double sn = (double)di * nx[q] + (double)dj * ny[q] + (double)dk * nz[q];
          const double w = fabs(sn) / sqrt((double)(di * di + dj * dj + dk * dk));
          sw += w;
          swk += kq * w;
          sk += kq;
          ++nq;
        }
    const double kb = nq == 0 ? NAN : (sw > 0.0 ? swk / sw : sk / (double)nq);
    const double gx = (alpha[lin + 1] - alpha[lin - 1]) * inv2h;
    const double gy = (alpha[lin + sy] - alpha[lin - sy]) * inv2h;
    const double gz = (alpha[lin + sz] - alpha[lin - sz]) * inv2h;
    kappa_band[b] = kb;
    fx[b] = sigma * kb * gx;
    fy[b] = sigma * kb * gy;
    fz[b] = sigma * kb * gz;
  }
}

// The curvature the CSF source uses in cell `lin` (paper section 3.3): the
// PPIC curvature of an interfacial cell, kappa_bar of a band cell (NaN if its
// row lies beyond the lists written); false for any other cell, which
// carries no surface force.
__device__ inline bool carried_kappa(const BandWords& B, const int32_t* word_off, const int32_t* band_off,
                                     int64_t lin, const double* kappa, int32_t nif, const double* kappa_band,
                                     int32_t nb, double& k) {
  const int64_t w = lin >> 5;
  const uint32_t bit = 1u << (lin & 31), below = bit - 1u;
  const uint32_t iw = B.I[w];
  if (iw & bit) {
    const int32_t r = word_off[w] + __popc(iw & below);
    k = r < nif ? kappa[r] : NAN;
    return true;
  }
  const uint32_t bw = B.word(w);
  if (bw & bit) {
    const int32_t r = band_off[w] + __popc(bw & below);
    k = r < nb ? kappa_band[r] : NAN;
    return true;
  }
  return false;
}

// k g / rho along one axis: the CSF source of a cell over its density, g the
// central difference of alpha.  One expression for both sides of a face, so
// that the two cells sharing it compute the same value.
__device__ inline double source_over_rho(double k, double a_plus, double a_minus, double inv2h, double rho) {
  return k * ((a_plus - a_minus) * inv2h) / rho;
}

// Surface-tension part of the face flux of the momentum-weighted
// interpolation (paper section 3.3, Eq. mwi_disc) divided by d_f A_f, for the
// six faces of every interfacial and band cell: one thread per cell.  Face
// between P (lower) and Q (upper) along axis d:
//   sigma [kbar_f (alpha_Q - alpha_P) / h - rho*_f / 2 (k_P g_P / rho_P + k_Q g_Q / rho_Q)],
// rho = rho_a + alpha (rho_b - rho_a), rho*_f the harmonic mean of rho_P and
// rho_Q, kbar_f the mean curvature of the cells of the two that carry one,
// the source terms only for those.  Listed cells are at least one cell
// inside the grid and so are the cells carrying a curvature: every alpha
// read exists.
__global__ __launch_bounds__(kT) void k_face_flux(Grid g, BandWords B, const int32_t* word_off,
                                                  const int32_t* band_off, const int32_t* cell_ids,
                                                  const double* alpha, const double* kappa, const int32_t* band_ids,
                                                  const double* kappa_band, const int32_t* n_band, int32_t band_cap,
                                                  double rho_a, double rho_b, double sigma, double* flux_if,
                                                  double* flux_band, int32_t cell_cap, const int32_t* counters) {
  const int32_t nif = min(counters[C_NIF], cell_cap), nb = min(*n_band, band_cap);
  const int64_t st[3] = {1, (int64_t)g.nx, (int64_t)g.nx * g.ny};
  const double inv_h = 1.0 / g.h, inv2h = 1.0 / (2.0 * g.h), drho = rho_b - rho_a;
  for (int32_t r = blockIdx.x * kT + threadIdx.x; r < nif + nb; r += gridDim.x * kT) {
    const bool in_band = r >= nif;
    const int32_t row = in_band ? r - nif : r;
    const int64_t c = in_band ? band_ids[row] : cell_ids[row];
    const double kc = in_band ? kappa_band[row] : kappa[row];
    double* out = in_band ? flux_band + row : flux_if + row;
    const int64_t ostride = in_band ? band_cap : cell_cap;
    const double ac = alpha[c], rc = rho_a + ac * drho;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t s = st[d];
      const double tc = source_over_rho(kc, alpha[c + s], alpha[c - s], inv2h, rc);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int64_t n = side ? c + s : c - s;
        double kn = 0.0;
        const bool carries = carried_kappa(B, word_off, band_off, n, kappa, nif, kappa_band, nb, kn);
        const double an = alpha[n], rn = rho_a + an * drho;
        const double tn = carries ? source_over_rho(kn, alpha[n + s], alpha[n - s], inv2h, rn) : 0.0;
        const double kf = carries ? 0.5 * (kc + kn) : kc;
        const double aP = side ? ac : an, aQ = side ? an : ac;
        const double rP = side ? rc : rn, rQ = side ? rn : rc;
        const double tP = side ? tc : tn, tQ = side ? tn : tc;
        const double rs = 2.0 * rP * rQ / (rP + rQ);
        out[(2 * d + side) * ostride] = sigma * (kf * (aQ - aP) * inv_h - 0.5 * rs * (tP + tQ));
      }
    }
  }
}

// The divergence-preserving interpolant at (x, y, z), in the half-open cell
// holding it; false (and nothing written) if the point is not finite or the
// cell is not at least one cell inside the grid.
__device__ inline bool interp_at(const Grid& g, const double* U, const double* V, const double* W, double x,
                                 double y, double z, double out[3]) {
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) return false;
  const int64_t i = cell_index(x, g.x0, g.h), j = cell_index(y, g.y0, g.h), k = cell_index(z, g.z0, g.h);
  if (!(i >= 1 && j >= 1 && k >= 1 && i <= g.nx - 2 && j <= g.ny - 2 && k <= g.nz - 2)) return false;
  const int64_t nx = g.nx, ny = g.ny;
  // strides of the three staggered arrays (x fastest)
  const int64_t uy_s = nx + 1, uz_s = (nx + 1) * ny;
  const int64_t vy_s = nx, vz_s = nx * (ny + 1);
  const int64_t wy_s = nx, wz_s = nx * ny;
  const int64_t u0 = i + uy_s * j + uz_s * k;  // U face (i, j, k): lower x face
  const int64_t v0 = i + vy_s * j + vz_s * k;  // V face (i, j, k): lower y face
  const int64_t w0 = i + wy_s * j + wz_s * k;  // W face (i, j, k): lower z face
  const double h = g.h, i2h = 1.0 / (2.0 * h);

  const double Um = U[u0], Up = U[u0 + 1];
  const double Vm = V[v0], Vp = V[v0 + vy_s];
  const double Wm = W[w0], Wp = W[w0 + wz_s];
  // transverse gradients on each face from the faces of the same orientation
  // in the neighbouring cells
  const double Uy_m = (U[u0 + uy_s] - U[u0 - uy_s]) * i2h;
  const double Uy_p = (U[u0 + 1 + uy_s] - U[u0 + 1 - uy_s]) * i2h;
  const double Uz_m = (U[u0 + uz_s] - U[u0 - uz_s]) * i2h;
  const double Uz_p = (U[u0 + 1 + uz_s] - U[u0 + 1 - uz_s]) * i2h;
  const double Vx_m = (V[v0 + 1] - V[v0 - 1]) * i2h;
  const double Vx_p = (V[v0 + vy_s + 1] - V[v0 + vy_s - 1]) * i2h;
  const double Vz_m = (V[v0 + vz_s] - V[v0 - vz_s]) * i2h;
  const double Vz_p = (V[v0 + vy_s + vz_s] - V[v0 + vy_s - vz_s]) * i2h;
  const double Wx_m = (W[w0 + 1] - W[w0 - 1]) * i2h;
  const double Wx_p = (W[w0 + wz_s + 1] - W[w0 + wz_s - 1]) * i2h;
  const double Wy_m = (W[w0 + wy_s] - W[w0 - wy_s]) * i2h;
  const double Wy_p = (W[w0 + wz_s + wy_s] - W[w0 + wz_s - wy_s]) * i2h;

  const double xm = g.x0 + (double)i * h, xp = g.x0 + (double)(i + 1) * h;
  const double ym = g.y0 + (double)j * h, yp = g.y0 + (double)(j + 1) * h;
  const double zm = g.z0 + (double)k * h, zp = g.z0 + (double)(k + 1) * h;
  const double ax = x - xm, bx = xp - x, ay = y - ym, by = yp - y, az = z - zm, bz = zp - z;
  const double cx = x - 0.5 * (xm + xp), cy = y - 0.5 * (ym + yp), cz = z - 0.5 * (zm + zp);
  const double dx = xp - xm, dy = yp - ym, dz = zp - zm;

  out[0] = (ax * (Up + cy * Uy_p + cz * Uz_p) + bx * (Um + cy * Uy_m + cz * Uz_m)) / dx +
           bx * ax / (2.0 * dx) * (Vx_p - Vx_m + Wx_p - Wx_m);
  out[1] = (ay * (Vp + cx * Vx_p + cz * Vz_p) + by * (Vm + cx * Vx_m + cz * Vz_m)) / dy +
           by * ay / (2.0 * dy) * (Uy_p - Uy_m + Wy_p - Wy_m);
  out[2] = (az * (Wp + cx * Wx_p + cy * Wy_p) + bz * (Wm + cx * Wx_m + cy * Wy_m)) / dz +
           bz * az / (2.0 * dz) * (Uz_p - Uz_m + Vz_p - Vz_m);
  return true;
}

__global__ __launch_bounds__(kT) void k_interp(Grid g, Mesh m, const double* U, const double* V, const double* W,
                                               double* ux, double* uy, double* uz, int32_t* counters) {
  const int32_t v = blockIdx.x * kT + threadIdx.x;
  if (v >= m.nv) return;
  double u[3];
  if (!interp_at(g, U, V, W, m.x[v], m.y[v], m.z[v], u)) {
    atomicOr(&counters[C_ERR], ERR_DOMAIN);
    u[0] = u[1] = u[2] = NAN;
  }
  ux[v] = u[0];
  uy[v] = u[1];
  uz[v] = u[2];
}

// One classical fourth-order Runge-Kutta step of dx/dt = u(x) per vertex,
// the face velocities fixed over the step: k1 = u(x), k2 = u(x + dt/2 k1),
// k3 = u(x + dt/2 k2), k4 = u(x + dt k3), x' = x + dt/6 (k1 + 2 k2 + 2 k3 +
// k4).  A stage point outside the admissible cells gives NaN and latches
// ERR_DOMAIN.  Each thread reads its vertex before writing it, so the output
// may be the input arrays.
__global__ __launch_bounds__(kT) void k_advect_rk4(Grid g, Mesh m, const double* U, const double* V,
                                                   const double* W, double dt, double* xo, double* yo, double* zo,
                                                   int32_t* counters) {
  const int32_t v = blockIdx.x * kT + threadIdx.x;
  if (v >= m.nv) return;
  const double p[3] = {m.x[v], m.y[v], m.z[v]};
  double k1[3], k2[3], k3[3], k4[3], s[3];
  bool ok = interp_at(g, U, V, W, p[0], p[1], p[2], k1);
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = p[d] + (0.5 * dt) * k1[d];
  ok = ok && interp_at(g, U, V, W, s[0], s[1], s[2], k2);
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = p[d] + (0.5 * dt) * k2[d];
  ok = ok && interp_at(g, U, V, W, s[0], s[1], s[2], k3);
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = p[d] + dt * k3[d];
  ok = ok && interp_at(g, U, V, W, s[0], s[1], s[2], k4);
  double o[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) o[d] = ok ? p[d] + (dt / 6.0) * (((k1[d] + 2.0 * k2[d]) + 2.0 * k3[d]) + k4[d]) : NAN;
  if (!ok) atomicOr(&counters[C_ERR], ERR_DOMAIN);
  xo[v] = o[0];
  yo[v] = o[1];
  zo[v] = o[2];
}

}  // namespace

hipError_t launch_csf(const ftc_cells* ws, const double* alpha, const double* kappa, double sigma, double* fx,
                      double* fy, double* fz, hipStream_t s) {
  time_start(ws, FTC_KERNEL_CSF, s);
  hipLaunchKernelGGL(k_csf, dim3(grid_blocks(ws->cell_cap, kT, 4096)), dim3(kT), 0, s, ws->grid, ws->cell_ids, alpha,
                     kappa, sigma, fx, fy, fz, ws->cell_cap, ws->counters);
  time_stop(ws, FTC_KERNEL_CSF, s);
  return hipGetLastError();
}

hipError_t launch_csf_band(const ftc_cells* ws, const double* alpha, const double* kappa, const double* nx,
                           const double* ny, const double* nz, double sigma, int32_t band_cap, int32_t* band_ids,
                           double* kappa_band, double* fx, double* fy, double* fz, int32_t* n_band, hipStream_t s) {
  const Grid& g = ws->grid;
  hipError_t e = scan_band_emit(ws->bitmap, ws->nwords, ws->ncell, g.nx, (int64_t)g.nx * g.ny, ws->band_off,
                                ws->scan_tmp, n_band, band_ids, band_cap, ws->counters, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_csf_band, dim3(grid_blocks(band_cap, kT, 4096)), dim3(kT), 0, s, g, ws->bitmap, ws->word_off,
                     alpha, kappa, nx, ny, nz, sigma, band_ids, n_band, band_cap, kappa_band, fx, fy, fz,
                     ws->cell_cap);
  return hipGetLastError();
}

hipError_t launch_face_flux(const ftc_cells* ws, const double* alpha, const double* kappa, int32_t band_cap,
                            const int32_t* band_ids, const double* kappa_band, const int32_t* n_band, double rho_a,
                            double rho_b, double sigma, double* flux_if, double* flux_band, hipStream_t s) {
  const Grid& g = ws->grid;
  const BandWords B{ws->bitmap, ws->nwords, ws->ncell, g.nx, (int64_t)g.nx * g.ny};
  hipLaunchKernelGGL(k_face_flux, dim3(grid_blocks((int64_t)ws->cell_cap + band_cap, kT, 4096)), dim3(kT), 0, s, g, B,
                     ws->word_off, ws->band_off, ws->cell_ids, alpha, kappa, band_ids, kappa_band, n_band, band_cap,
                     rho_a, rho_b, sigma, flux_if, flux_band, ws->cell_cap, ws->counters);
  return hipGetLastError();
}

hipError_t launch_advect_rk4(const ftc_cells* ws, const Grid& g, const Mesh& m, const double* U, const double* V,
                             const double* W, double dt, double* xo, double* yo, double* zo, hipStream_t s) {
  hipLaunchKernelGGL(k_advect_rk4, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, U, V, W, dt, xo, yo, zo,
                     ws->counters);
  return hipGetLastError();
}

hipError_t launch_interp(const ftc_cells* ws, const Grid& g, const Mesh& m, const double* U, const double* V,
                         const double* W, double* ux, double* uy, double* uz, hipStream_t s) {
  time_start(ws, FTC_KERNEL_INTERP, s);
  hipLaunchKernelGGL(k_interp, dim3(grid_blocks(m.nv, kT)), dim3(kT), 0, s, g, m, U, V, W, ux, uy, uz,
                     ws->counters);
  time_stop(ws, FTC_KERNEL_INTERP, s);
  return hipGetLastError();
}

}  // namespace ftc
