/*
 * ftc_oracle.h -- FP64 CPU oracle for the sharp front-tracking coupling
 * (Gorges, Evrard, Chiodi, van Wachem, Denner, "Sharp front tracking with
 * geometric interface reconstruction", arXiv 2505.06932).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the HIP
 * library is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no source, header or
 * helper with the HIP library.
 *
 * Every pointer here is host memory owned by the caller.  Return values:
 * 0 = ok, -1 = invalid argument, -2 = vertex outside the grid margin,
 * -3 = inconsistent (open or inverted) front, -4 = output capacity too small.
 */
#ifndef FTC_ORACLE_H
#define FTC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int32_t nx, ny, nz; double x0, y0, z0, h; } ora_grid;
typedef struct {
  int32_t nv, nt;
  const double *x, *y, *z;
  const int32_t *t0, *t1, *t2;
} ora_mesh;
typedef struct {
  double delta_over_h; /* Wendland support radius in cells (paper: 2.5)    */
  int32_t rings;       /* triangle rings around the closest vertex (3)      */
  int32_t n_min;       /* minimum triangles with non-zero weight (24)       */
  double grow;         /* support growth factor per adjustment (1.1)        */
  int32_t max_iter;    /* maximum number of support adjustments (16)        */
} ora_ppic_params;

/* Number of (triangle, cell) candidates: sum over triangles of the cells of
   their bounding box.  An upper bound on the number of pieces. */
int64_t ora_candidate_bound(const ora_grid* g, const ora_mesh* m);

/* Cell lists (paper sec. 3.2, interfacial cells): all (cell, triangle) pairs
   whose intersection has positive area, sorted by linear cell id, then by
   triangle id.  Returns the number of pairs, or -4 if it exceeds cap, or -2
   if a vertex leaves the grid minus a 2-cell margin. */
int64_t ora_cell_lists(const ora_grid* g, const ora_mesh* m, int64_t cap,
                       int64_t* pair_cell, int32_t* pair_tri);

/* Exact volume fraction of every cell (paper sec. 3.2, definition of the
   discrete indicator), by the divergence theorem along columns of the given
   axis (0 = x, 1 = y, 2 = z).  alpha[ncell], is_if[ncell] (1 = interfacial).
   Returns 0, -2 or -3. */
int32_t ora_volume_fraction(const ora_grid* g, const ora_mesh* m, int32_t axis,
                            double* alpha, uint8_t* is_if);

/* Clip one triangle against one closed cell and return its integrals
   (diagnostic entry point for tests): out[0] = area-weighted n_axis
   (the piece's projected area), out[1] = integral of (x_axis - lo) n_axis.
   Returns 1 if the piece counts (positive area under the half-open rule). */
int32_t ora_piece(const ora_grid* g, const double tri[9], int32_t i, int32_t j,
                  int32_t k, int32_t axis, double out[2]);

/* PPIC curvature (paper sec. 3.2, volume fit) for the listed cells.
   Outputs per cell: kappa, interface normal nrm[3], paraboloid coefficients
   coeff[6] in the local frame (world units), status (bit0 = rank-deficient
   fit), and the discrete decisions diag[4] = {closest vertex, ring size,
   triangles with non-zero weight, support adjustments}.  Any output may be
   NULL.  Returns 0 or -1. */
int32_t ora_ppic(const ora_grid* g, const ora_mesh* m, const ora_ppic_params* p,
                 int64_t ncell, const int64_t* cell_ids, double* kappa,
                 double* nrm, double* coeff, int32_t* status, int32_t* diag);

/* The support of one cell's volume fit (paper sec. 3.2, Eq. Wendland), for
   tests: the ring triangles in ascending order (tri_out), the squared
   distances of their centres to the cell centre (d2_out) and their Wendland
   weights (w_out), at most cap of each, and the final support radius
   (*delta_out), exactly as ora_ppic computes them for the cell with linear
   id cell_id.  Returns the ring size (entries past cap are not written) or
   -1. */
int32_t ora_ppic_support(const ora_grid* g, const ora_mesh* m, const ora_ppic_params* p,
                         int64_t cell_id, int32_t cap, int32_t* tri_out, double* d2_out,
                         double* w_out, double* delta_out);

/* Input of the learned curvature surrogate: per listed cell, the front
   vertex closest to the cell centre (lowest index on ties) and its squared
   distance, and that vertex's normal, the normalised sum of the cross
   products (c1 - c0) x (c2 - c0) of its incident triangles in ascending
   triangle order (the frame normal of the volume fit, paper sec. 3.2).
   Any output may be NULL.  Returns 0 or -1. */
int32_t ora_frame_normal(const ora_grid* g, const ora_mesh* m, int64_t ncell,
                         const int64_t* cell_ids, int32_t* vstar, double* best_d2,
                         double* nrm);

/* One volume fit (paper Eqs. volumefit / volumefit2) in a given frame:
   frame[9] = {t1, t2, n} (rows), origin xc[3], scale h; tri[9*ntri] the
   triangles' corners in world coordinates, w[ntri] their weights.
   Writes a[6] (world units) and returns the rank status (0 = ok). */
int32_t ora_fit(const double frame[9], const double xc[3], double h, int32_t ntri,
                const double* tri, const double* w, double a[6]);

/* Mean curvature (kappa = 2H, positive for a sphere seen from outside) of the
   paraboloid z = a1 + a2 x + a3 y + a4 x^2 + a5 xy + a6 y^2 at (0, 0). */
double ora_kappa(const double a[6]);

/* CSF source (paper Eq. csf) sigma * kappa * grad(alpha) on the listed cells,
   central differences on the dense alpha field.  f[3*ncell]. */
int32_t ora_csf(const ora_grid* g, const double* alpha, int64_t ncell,
                const int64_t* cell_ids, const double* kappa, double sigma,
                double* f);

/* BAND mode of the CSF source (paper sec. 3.3, weighted curvature
   smoothing): the cells sharing a face with an interfacial cell and not
   interfacial themselves, ascending linear id, with the weighted average
   kappa_bar of the finite curvatures of the interfacial cells among their
   26 neighbours (weights |s.n|/|s|, plain mean if they all vanish, NaN
   if there is none) and the source sigma kappa_bar grad(alpha).
   cell_ids ascending; nrm[3*ncell] the interface normals.  Writes the first
   `cap` band cells; returns their total number, -1 or -2 (a band cell on
   the grid boundary). */
int64_t ora_csf_band(const ora_grid* g, const double* alpha, int64_t ncell,
                     const int64_t* cell_ids, const double* kappa, const double* nrm,
                     double sigma, int64_t cap, int64_t* band_ids, double* kappa_band,
                     double* f);

/* Divergence-preserving interpolation (paper sec. 3.1) of the staggered face
   velocities to the points (x, y, z)[n]; u[3*n].  Returns 0 or -2. */
int32_t ora_interp(const ora_grid* g, int32_t n, const double* x, const double* y,
                   const double* z, const double* U, const double* V,
                   const double* W, double* u);

/* One classical fourth-order Runge-Kutta step of dx/dt = u(x) for the points
   (x, y, z)[n], u the divergence-preserving interpolant of the fixed face
   velocities; out[3*n] the new positions.  Returns 0, or -2 if a stage
   point left the admissible cells (that point's output is NaN). */
int32_t ora_advect_rk4(const ora_grid* g, int32_t n, const double* x, const double* y,
                       const double* z, const double* U, const double* V,
                       const double* W, double dt, double* out);

/* The same polynomial evaluated in a given cell (i, j, k) at any point. */
void ora_interp_in_cell(const ora_grid* g, int32_t i, int32_t j, int32_t k,
                        double x, double y, double z, const double* U,
                        const double* V, const double* W, double u[3]);

/* Threads the oracle's parallel loops use (OpenMP), for reporting. */
int32_t ora_threads(void);
/* Threads of the following calls (n <= 0: one per processor). */
void ora_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
