/*
 * ftc.h -- C ABI of the MI355X (gfx950) library for the sharp front-tracking
 * coupling restricted to interfacial cells (Gorges, Evrard, Chiodi,
 * van Wachem, Denner, "Sharp front tracking with geometric interface
 * reconstruction", arXiv 2505.06932, section 3).
 *
 * Conventions for every call below
 * --------------------------------
 * - Pointers are DEVICE memory owned by the caller unless marked [host].
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   Calls only validate host-side arguments and enqueue kernels on `stream`;
 *   none allocates, frees or synchronises (except ftc_cells_count and
 *   ftc_last_device_error, which say so), so a sequence of calls can be
 *   captured into a HIP graph.
 * - Grid: cubic cells of edge h; cell (i,j,k) is the half-open box
 *   [x0+i*h, x0+(i+1)*h) x [y0+j*h, ...) x [z0+k*h, ...), linear id
 *   i + nx*(j + ny*k).  Dense cell fields are FP64 [nz][ny][nx].
 * - Front: closed triangulated surface, vertices as FP64 SoA x,y,z[nv],
 *   triangles as int32 corner indices t0,t1,t2[nt], counter-clockwise seen
 *   from outside (normals point away from the enclosed fluid, the fluid
 *   where the indicator is 1, paper section 2).  Every vertex must lie at
 *   least 2 cells inside the grid.
 * - Per-interfacial-cell outputs are indexed like the cell list
 *   (ascending linear cell id) and sized to the workspace cell capacity.
 * - Return values are ftc_status codes.  Host-detectable argument errors
 *   return immediately and enqueue nothing.  Conditions only the device can
 *   see (front outside the grid margin, open front, capacity overflow) are
 *   latched in the workspace and read by ftc_last_device_error; when one is
 *   latched the outputs of that call are unspecified but no write goes past
 *   any buffer.
 * - No C++ exception crosses this boundary.
 */
#ifndef FTC_H
#define FTC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FTC_OK = 0,
  FTC_EINVAL = -1,    /* bad argument (null pointer, size <= 0, h <= 0, ...) */
  FTC_EDOMAIN = -2,   /* a vertex lies outside the grid minus a 2-cell margin */
  FTC_EMESH = -3,     /* front is not closed or not outward oriented          */
  FTC_ECAPACITY = -4, /* more pairs or cells than the workspace holds         */
  FTC_ENOMEM = -5,    /* device allocation failed (ftc_cells_create only)     */
  FTC_EHIP = -6       /* a HIP runtime call failed                            */
} ftc_status;

typedef struct {
  int32_t nx, ny, nz; /* cells per axis, each > 4                       */
  double x0, y0, z0;  /* grid origin (lower corner of cell (0,0,0))      */
  double h;           /* cell edge, > 0                                  */
} ftc_grid;

typedef struct {
  int32_t nv, nt;              /* vertex and triangle counts, > 0        */
  const double *x, *y, *z;     /* [nv] device                            */
  const int32_t *t0, *t1, *t2; /* [nt] device, corner indices in [0, nv) */
} ftc_mesh;

/* Volume-fit parameters (paper section 3.2, after Eq. Wendland): Wendland
   support radius delta = delta_over_h * h (paper: 2.5), the `rings`-ring of
   triangles around the closest front vertex (paper: 3), the support grown by
   the factor `grow` at most `max_iter` times until at least `n_min`
   triangles carry non-zero weight (paper: "24 to 48").  precision: 0 forms
   and solves the weighted normal equations in double precision; 1 forms and
   factors them in single precision and refines the solution twice with
   double-precision residuals of the same triangles (the curvature then
   agrees with the double-precision solution to about cond(M)^3 times the
   single-precision roundoff cubed; a single-precision pivot at or below
   1e-6 of the trace flags the cell rank deficient).  Cells taken by the
   wide ring shape are always solved in double precision. */
typedef struct {
  double delta_over_h;
  int32_t rings;
  int32_t n_min;
  double grow;
  int32_t max_iter;
  int32_t precision;
} ftc_ppic_params;

/* Per-cell status bits written by ftc_ppic_curvature. */
#define FTC_CELL_RANK 1u     /* normal equations singular: kappa, n, coeff = NaN */
#define FTC_CELL_OVERFLOW 2u /* ring larger than the kernel's stencil limit      */
#define FTC_CELL_SURROGATE 4u /* curvature from the learned surrogate (ftc_learned_curvature) */

/* Opaque workspace: the cell lists and every scratch buffer the calls use,
   allocated once for one grid and maximum front sizes. */
typedef struct ftc_cells ftc_cells;

/* Allocate a workspace on the current HIP device for `grid` [host] and fronts
   of up to nv_capacity vertices and nt_capacity triangles, holding up to
   pair_capacity (cell, triangle) pieces and cell_capacity interfacial
   cells (candidates that must be clipped, up to twice pair_capacity, are
   queued internally).  Device memory is about 116 B x pairs + 1.1 kB x cells
   + 104 B x triangles + 84 B x vertices + 3 nx*ny*nz/8 B (about 110 MB for a
   128^3 grid with 82k triangles, 1.4 GB for 512^3 with 2M triangles).
   Returns FTC_EINVAL, FTC_ENOMEM or FTC_OK; *out is NULL on failure. */
ftc_status ftc_cells_create(ftc_cells** out, const ftc_grid* grid, int32_t nv_capacity,
                            int32_t nt_capacity, int64_t pair_capacity, int32_t cell_capacity);

/* Free a workspace (synchronises the device first).  NULL is a no-op. */
void ftc_cells_destroy(ftc_cells* cells);

/* Build the interfacial-cell lists (paper section 3.2: the interfacial cells
   are those containing the front; sections 1 and 3: the coupling is
   restricted to them).  A (cell, triangle) pair exists when the triangle's
   intersection with the closed cell has positive area; a triangle lying
   exactly in a grid plane belongs to the cell above that plane.  Result, in
   the workspace: interfacial cells in ascending linear id and, per cell, its
   triangles in ascending id (CSR), together with each piece's two surface
   integrals used by ftc_volume_fraction (clipping happens once, here).  The
   same launches prepare what ftc_ppic_curvature needs from the front: each
   vertex's incident triangles, the vertices binned by interfacial cell and
   the closest front vertex of every interfacial cell.
   `grid` must equal the workspace's grid.
   Latches FTC_EDOMAIN or FTC_ECAPACITY on the device. */
ftc_status ftc_build_cell_lists(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                void* stream);

/* Copy the interfacial-cell and pair counts of the last build to the host,
   each clamped to its capacity (a build that exceeded one has latched
   FTC_ECAPACITY and its lists are truncated).  Synchronises `stream`. */
ftc_status ftc_cells_count(const ftc_cells* cells, int32_t* n_interfacial /*[host]*/,
                           int64_t* n_pairs /*[host]*/, void* stream);

/* Device pointers into the workspace: cell_ids[cell_capacity],
   offsets[cell_capacity+1], tri_ids[pair_capacity], and d_counts[2] =
   {interfacial cells, pairs} (int32, device), valid until the next build.
   Any output pointer may be NULL. */
ftc_status ftc_cells_view(const ftc_cells* cells, const int32_t** cell_ids, const int32_t** offsets,
                          const int32_t** tri_ids, const int32_t** d_counts);

/* Exact volume fraction alpha_C = |Omega cap C| / h^3 (paper section 3.2,
   definition of the discrete indicator; polyhedron intersection; full and
   empty cells), where Omega is the region enclosed by the triangulated
   front.  By the divergence theorem along z columns: for an interfacial
   cell, the sum over its pieces p of the integral of (z - z_lo) n_z dA plus
   h times the wetted area of its upper face, which is the sum of the
   integrals of n_z dA over all pieces strictly above it in the column.
   Cells without pieces get 0 or 1 from the same column sum.
   alpha_if[cell_capacity]: alpha of each interfacial cell (cell-list order).
   alpha_dense[nx*ny*nz] or NULL: every cell of the grid is written.
   Latches FTC_EMESH if a column sum is not 0 or h^2 where no piece is
   (open or inverted front).  Uses the pieces of the last
   ftc_build_cell_lists on the same workspace (mesh must be that front). */
ftc_status ftc_volume_fraction(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                               double* alpha_if, double* alpha_dense, void* stream);

/* PPIC curvature (paper section 3.2): for each interfacial cell, the front
   vertex closest to the cell centre (lowest index on ties), its area-weighted
   normal n, tangents completing a right-handed frame; the ring neighbourhood
   of triangles around that vertex; Wendland weights of the triangle-centre
   distances (Eq. Wendland) with the support grown per `params`; the weighted
   least-squares volume fit of the paraboloid z = a1 + a2 x + a3 y + a4 x^2 +
   a5 xy + a6 y^2 (Eqs. volumefit, volumefit2) in that frame; then at the
   frame origin the mean curvature kappa = 2H (positive for a sphere seen from
   outside, kappa = 2/r; section 4.1 and appendix A) and the interface normal.
   Outputs (each [cell_capacity], cell-list order): kappa; nx, ny, nz (unit
   interface normal, outward); coeff [6][cell_capacity] or NULL (a1..a6 in
   world units, frame origin at the cell centre); cell_status or NULL
   (FTC_CELL_* bits); diag [4][cell_capacity] or NULL (closest vertex, ring
   triangle count, triangles with non-zero weight, support adjustments).
   `params` [host] NULL means the paper's values {2.5, 3, 24, 1.1, 16}.
   Uses the closest vertices and vertex adjacency of the last
   ftc_build_cell_lists on the same workspace: mesh must be that front
   (FTC_EINVAL if its vertex or triangle count differs, or before any
   build). */
ftc_status ftc_ppic_curvature(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                              const ftc_ppic_params* params, double* kappa, double* nx, double* ny,
                              double* nz, double* coeff, int32_t* cell_status, int32_t* diag,
                              void* stream);

/* The cell quantities of the fitted paraboloid (paper section 3.2): the
   volume fraction alpha = |cell below the paraboloid| / |cell|, and the
   curvature and normal integrated over the part of the paraboloid inside
   the cell.  For every interfacial cell, the paraboloid is zeta = a1 + a2 xi
   + a3 eta + a4 xi^2 + a5 xi eta + a6 eta^2 of the last ftc_ppic_curvature
   on this workspace, in its frame (t1, t2, n) with origin at the cell
   centre, n the frame normal of that call (kept in the workspace); the
   liquid lies below the surface (zeta smaller).
   coeff [6][cell_capacity] as that call wrote it.  Outputs, cell-list order:
   alpha_paraboloid [cell_capacity]; kappa_cell [cell_capacity] or NULL, the
   area-weighted mean of kappa = 2H over the surface inside the cell (same
   sign convention as ftc_ppic_curvature); normal_cell [3][cell_capacity] or
   NULL, the normalised integral of the unit normal (pointing out of the
   liquid) over that surface.  The volume is exact in one tangential
   direction and a 16-node Gauss rule between exact breakpoints in the other
   (about 1e-14); when kappa_cell or normal_cell is asked for, that rule has
   24 nodes (for the normal integral; alpha then agrees with the volume-only
   call to about 1e-13, not bit for bit) and the area and curvature add an
   8-node rule between the breakpoints in the first direction.  NaN for a
   cell whose fit failed, and kappa_cell and
   normal_cell NaN where the paraboloid does not cross the cell (and where
   rounding would split the surface inside the cell into more than four
   runs of eta intervals, which exact arithmetic excludes).
   FTC_EINVAL unless ftc_ppic_curvature (not the learned curvature) ran after
   the last ftc_build_cell_lists. */
ftc_status ftc_paraboloid_cell(const ftc_cells* cells, const ftc_grid* grid, const double* coeff,
                               double* alpha_paraboloid, double* kappa_cell, double* normal_cell, void* stream);

/* Continuum surface force (paper section 3.3, Eq. csf): S = sigma kappa
   grad(alpha) on the interfacial cells only, grad(alpha) by central
   differences of the dense alpha field (alpha_dense[nx*ny*nz]) with spacing
   h.  fx, fy, fz [cell_capacity], cell-list order. */
ftc_status ftc_csf_force(const ftc_cells* cells, const ftc_grid* grid, const double* alpha_dense,
                         const double* kappa, double sigma, double* fx, double* fy, double* fz,
                         void* stream);

/* Band mode of the continuum surface force (paper section 3.3, weighted
   curvature smoothing in the neighbours of interfacial cells): for every
   cell P that shares a face with an interfacial cell and is not interfacial
   itself, kappa_bar_P = sum_Q kappa_Q w_Q / sum_Q w_Q over the interfacial
   cells Q among P's 26 neighbours whose kappa is finite, with
   w_Q = |s_Q . n_Q| / |s_Q|, s_Q from P's centre to Q's and n_Q the
   interface normal of Q (nx, ny, nz from ftc_ppic_curvature); the plain
   mean of those kappa_Q if every w_Q is 0, NaN if there is no such Q.  The
   source is S_P = sigma kappa_bar_P grad(alpha)_P (central differences of
   alpha_dense, as ftc_csf_force; the interfacial cells keep their own kappa
   and source from ftc_csf_force).  Outputs, each [band_capacity], in
   ascending linear cell id: band_ids (linear ids), kappa_band, fx, fy, fz;
   *d_n_band [device int32] receives the number of band cells, which may
   exceed band_capacity (six times the interfacial cell count always
   suffices); then FTC_ECAPACITY is latched and only the first
   band_capacity are written.  Uses the interfacial cells of the last
   build. */
ftc_status ftc_csf_force_band(ftc_cells* cells, const ftc_grid* grid, const double* alpha_dense,
                              const double* kappa, const double* nx, const double* ny, const double* nz,
                              double sigma, int32_t band_capacity, int32_t* band_ids, double* kappa_band,
                              double* fx, double* fy, double* fz, int32_t* d_n_band, void* stream);

/* Surface-tension part of the face flux of the momentum-weighted
   interpolation (paper section 3.3, Eq. mwi_disc), divided by the solver's
   coefficients d_f A_f, for the six faces of every interfacial and band
   cell.  For the face between cells P (lower) and Q (upper) along axis d,
   oriented along +d:
     sigma [kbar_f (alpha_Q - alpha_P) / h
            - rho*_f / 2 (k_P g_P / rho_P + k_Q g_Q / rho_Q)],
   rho_C = rho_a + alpha_C (rho_b - rho_a) (the mixture density, section 2),
   rho*_f = 2 rho_P rho_Q / (rho_P + rho_Q) (harmonic, section 2), g_C the
   d-component of the central-difference gradient of alpha_dense, k_C the
   curvature the CSF source uses in C (kappa of an interfacial cell,
   kappa_band of a band cell) and no source in any other cell, kbar_f the mean
   of k_P and k_Q over those of the two cells that carry a curvature.  With a
   constant curvature and p = sigma k alpha it equals the pressure term of the
   same flux (force balance).  kappa [cell_capacity] as from
   ftc_ppic_curvature; band_ids, kappa_band [band_capacity] and d_n_band
   [device int32] as written by the last ftc_csf_force_band on this
   workspace, which must follow its last ftc_build_cell_lists, with the same
   band_capacity (FTC_EINVAL otherwise).  rho_a, rho_b > 0.  Outputs flux_if [6][cell_capacity]
   (cell-list order) and flux_band [6][band_capacity] (band order); slot 2d
   holds the face towards C - e_d, slot 2d + 1 the face towards C + e_d, so a
   face shared by two listed cells has the same value in both rows.  A NaN
   curvature propagates to the faces it touches. */
ftc_status ftc_surface_tension_flux(ftc_cells* cells, const ftc_grid* grid, const double* alpha_dense,
                                    const double* kappa, int32_t band_capacity, const int32_t* band_ids,
                                    const double* kappa_band, const int32_t* d_n_band, double rho_a,
                                    double rho_b, double sigma, double* flux_if, double* flux_band,
                                    void* stream);

/* Divergence-preserving interpolation (paper section 3.1) of staggered
   normal face velocities to the front vertices: inside the cell holding the
   vertex, linear interpolation between opposite faces plus transverse-
   gradient terms (central differences over the neighbouring faces of the
   same orientation) and the quadratic correction that makes the
   interpolant's divergence equal the cell's discrete divergence.
   U[nz][ny][nx+1], V[nz][ny+1][nx], W[nz+1][ny][nx] (x fastest).
   ux, uy, uz [mesh->nv].  A vertex whose cell is within 1 cell of the grid
   boundary gets NaN and latches FTC_EDOMAIN.  `cells` supplies the error
   latch only. */
ftc_status ftc_interp_vertex_velocity(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                      const double* U, const double* V, const double* W, double* ux,
                                      double* uy, double* uz, void* stream);

/* One classical fourth-order Runge-Kutta step of the front vertices through
   the interpolated velocity (paper section 3.1: the vertices are advected in
   a Lagrangian manner, dx/dt = u(x), with the fourth-order Runge-Kutta
   scheme), the face velocities held fixed over the step:
   k1 = u(x), k2 = u(x + dt/2 k1), k3 = u(x + dt/2 k2), k4 = u(x + dt k3),
   x' = x + dt/6 (k1 + 2 k2 + 2 k3 + k4), u the interpolant of
   ftc_interp_vertex_velocity.  x_out, y_out, z_out [mesh->nv] may be the
   mesh's own coordinate arrays (each vertex is read before it is written).
   A vertex whose stage point lies within 1 cell of the grid boundary gets
   NaN and latches FTC_EDOMAIN.  `cells` supplies the error latch only. */
ftc_status ftc_advect_vertices_rk4(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                   const double* U, const double* V, const double* W, double dt,
                                   double* x_out, double* y_out, double* z_out, void* stream);

/* Read and clear the device-latched error of the workspace: *code [host]
   receives FTC_OK or the first of FTC_ECAPACITY, FTC_EDOMAIN, FTC_EMESH
   that was latched.  Synchronises `stream`. */
ftc_status ftc_last_device_error(ftc_cells* cells, int32_t* code, void* stream);

/* Kernel timing, for measurement only.  While enabled, every call records a
   HIP event on its stream immediately before and after its dominant kernel;
   ftc_kernel_time then returns the interval of the last such launch.  Keep
   it disabled while capturing a graph (event records are not captured). */
typedef enum {
  FTC_KERNEL_TRI_PIECES = 0,  /* cell lists: per-triangle clip and integrals  */
  FTC_KERNEL_PIECE_RANK = 1,  /* cell lists: piece order, closest vertices    */
  FTC_KERNEL_COLUMNS = 2,     /* volume fraction: column pass and dense field */
  FTC_KERNEL_PPIC = 3,        /* PPIC: ring, fit, curvature (both shapes)     */
  FTC_KERNEL_CSF = 4,         /* CSF force                                    */
  FTC_KERNEL_INTERP = 5,      /* vertex velocity interpolation                */
  FTC_KERNEL_SURROGATE = 6,   /* learned curvature with its PPIC fallback     */
  FTC_KERNEL_COUNT = 7
} ftc_kernel;

/* Enable (1) or disable (0) the timing events of a workspace. */
ftc_status ftc_set_timing(ftc_cells* cells, int32_t enable);

/* Milliseconds of the last timed launch of `kernel` (an ftc_kernel value),
   into *ms [host]; waits for that launch to finish.  FTC_EINVAL if the kernel
   was never timed. */
ftc_status ftc_kernel_time(const ftc_cells* cells, int32_t kernel, float* ms);

/* Static text for a status code. */
const char* ftc_status_str(int32_t status);

/* ------------------------------------------------------------------------
   Learned curvature surrogate (an extension of the PPIC fit of paper section
   3.2: the network learns kappa h from what the fit sees).

   Feature row of an interfacial cell, FTC_MLP_FEATURES floats: the volume
   fractions of the 3x3x3 block of cells centred on it, entry
   q = 9 (dk+1) + 3 (dj+1) + (di+1) for the cell (i+di, j+dj, k+dk) (0 outside
   the grid), then the fit's frame normal (the normalised sum of the cross
   products (c1 - c0) x (c2 - c0) of the incident triangles of the front
   vertex closest to the cell centre, in ascending triangle order), then two
   zeros.

   Network: 30 -> 64 -> 64 -> 1 with tanh hidden units, parameters theta
   (FTC_MLP_PARAMS floats, device): W1 [64][30] row-major, b1 [64],
   W2 [64][64] row-major, b2 [64], w3 [64], b3.  Evaluated with weights and
   hidden activations rounded to bfloat16 and single-precision sums; every
   input x enters as bf16(x) plus bf16(x - bf16(x)).

   Cube symmetries: sym in [0, 48) is permutation sym / 8 of the axes (in
   lexicographic order) with axis a negated where bit a of sym % 8 is set,
   (P x)_a = sign_a x_perm[a]; a feature row mapped by it holds the fractions
   alpha'(d) = alpha(P^T d) and the normal P n.
   ------------------------------------------------------------------------ */
#define FTC_MLP_FEATURES 32
#define FTC_MLP_PARAMS 6209
/* work buffer of ftc_mlp_loss_grad, floats (256 partial rows) */
#define FTC_MLP_WORK_FLOATS (256 * (FTC_MLP_PARAMS + 3))

/* Feature rows of the interfacial cells of the last build:
   features[cell_capacity][FTC_MLP_FEATURES] (device, row c for compact cell
   c), from the dense volume fractions alpha_dense [nz][ny][nx] (device,
   ftc_volume_fraction's output).  final_flags [cell_capacity] (device, or
   NULL): 0 if the cell's closest front vertex lies within 1.5 h of its
   centre, else 1 (its normal is then 0).  The mesh must be the one of the
   last build. */
ftc_status ftc_curvature_features(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                  const double* alpha_dense, float* features, int32_t* final_flags,
                                  void* stream);

/* Network outputs y[n] (device) for the rows X[rows][FTC_MLP_FEATURES]
   (device): sample s reads row idx[s] (or s if idx is NULL) mapped by cube
   symmetry sym[s] (or none if sym is NULL).  A sample whose row lies outside
   [0, rows) reads zeros; a symmetry outside [0, 48) is taken as 0. */
ftc_status ftc_mlp_forward(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                           const int32_t* sym, int32_t n, float* y, void* stream);

/* Mean squared error (1/n) sum_s (y_s - t[row_s])^2 over a batch of n
   samples chosen as in ftc_mlp_forward, and its gradient grad[FTC_MLP_PARAMS]
   (device) with respect to theta; loss (device, one float) may be NULL.  The
   backward pass rounds dz to bfloat16 before each product, takes the
   derivative of tanh from the rounded activation and sums in single
   precision; partial sums of up to 256 workgroups are added in workgroup
   order.  work: FTC_MLP_WORK_FLOATS floats of device memory owned by the
   caller (overwritten).  n must be positive. */
ftc_status ftc_mlp_loss_grad(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                             const int32_t* sym, const float* t, int32_t n, float* grad, float* loss,
                             float* work, void* stream);

/* ftc_mlp_loss_grad for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving or training loops, harnesses that
   forbid hipMalloc): the same arguments without `work`, and the same
   results bit for bit.  The partial rows live in a fixed scratch array of
   the library, FTC_MLP_WORK_FLOATS floats (6.4 MB) on each device that
   calls it, held until the process ends; its address is resolved on the
   first call on each device (that call may return FTC_EHIP if the runtime
   cannot resolve it).  The call allocates and frees nothing.  Any n > 0 is
   accepted: at most 256 workgroups write partial rows, each its whole row,
   so the scratch never needs clearing.  Calls that overlap on one device
   (concurrent streams or host threads) share the scratch and race; order
   them on one stream. */
ftc_status ftc_mlp_loss_grad_static(const float* theta, const float* X, int64_t rows, const int32_t* idx,
                                    const int32_t* sym, const float* t, int32_t n, float* grad, float* loss,
                                    void* stream);

/* One Adam step (Kingma and Ba, ICLR 2015) on theta, with first and second
   moments m, v (device, FTC_MLP_PARAMS floats each, zero before step 1) and
   bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
   theta -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
   step counts from 1. */
ftc_status ftc_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream);

/* Curvature of every interfacial cell of the last build by the surrogate,
   with PPIC where it is not trusted.  For each cell the network is evaluated
   on its feature row mapped by four cube symmetries (0, 17, 24, 7: identity,
   quarter turn about z, cyclic exchange of the axes, point reflection); the
   estimate of kappa h is their mean ((y0 + y1) + (y2 + y3)) / 4 and the error
   estimate their spread (max - min).  A cell with spread <= bound and a
   closest vertex within 1.5 h gets kappa = mean / h, the frame normal in
   (nx, ny, nz) and cell_status FTC_CELL_SURROGATE; every other cell is
   computed by ftc_ppic_curvature's kernels (params as there; coefficients
   and decisions are not written) and gets its status.  spread
   [cell_capacity] (device float, or NULL) receives every cell's spread.
   d_n_fallback (device, one int32, or NULL) receives the number of cells
   handed to PPIC.  Outputs have cell_capacity entries (device).  The mesh
   must be the one of the last build. */
ftc_status ftc_learned_curvature(const ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh,
                                 const double* alpha_dense, const float* theta, double bound,
                                 const ftc_ppic_params* params, double* kappa, double* nx, double* ny, double* nz,
                                 float* spread, int32_t* cell_status, int32_t* d_n_fallback, void* stream);

/* ------------------------------------------------------------------------
   Local roughness detection and smoothing of the front (paper section 3.4).
   Both calls use the vertex adjacency of the last build (the mesh must be
   that build's) and treat the front as closed and consistently oriented.
   ------------------------------------------------------------------------ */

/* Per vertex (device arrays of nv doubles): gl_mag, the length of the
   geometric Laplacian x_i - sum_j w_ij x_j / sum_j w_ij over the one-ring,
   w_ij = 1 / |x_i - x_j|; rough, the dihedral roughness max(R^1, R^2),
   where R_e = 1 - n1 . n2 on each edge (unit normals of its two triangles),
   G_i and V_i are the mean and the population variance of R_e over the edges
   at i, R_t = sum G V / sum V over a triangle's corners (the mean of the G if
   every V is 0), and R^l_i is the mean of A_t R_t over the triangles of the
   l-ring of i (A_t the area; the two-ring holds the triangles with a corner
   in i's one-ring or at i). */
ftc_status ftc_front_roughness(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, double* gl_mag,
                               double* rough, void* stream);

/* Volume-conserving smoothing of the rough edges (paper section 3.4, after
   Kuprat et al. 2001, algorithm 4).  A vertex is rough when gl_mag >
   gl_threshold and rough > rough_threshold (the paper takes 1.2 to 1.5 times
   the maxima on the initial front); an edge is smoothed when both its ends
   are rough.  Its ends move to the simultaneous Laplacian positions
   x1s = (S2 + n2 S1) / (n1 n2 - 1), x2s = (x1s + S2) / n2 (n_i the one-ring
   sizes, S_i the one-ring sums without the other end), plus the least common
   displacement that keeps the enclosed volume: -c g / |g|^2 with
   g = A1 + A2 + y x (d1 - d2), c = d1.A1 + d2.A2 + d1.(d2 x y), d_i = x_is - x_i,
   A_i the sum of (a - x_i) x (b - x_i) over the triangles (x_i, a, b) at end
   i and y the difference of the far corners of the triangles holding the
   half-edges x1 -> x2 and x2 -> x1 (the enclosed volume then changes by
   exactly 0; the text prints the last term of c as d1.(y x d1), which
   vanishes identically).  Edges are processed in up to max_rounds rounds: in
   each, an edge is taken unless a pending edge ordered before it has an end
   within one ring of it; edges are ordered by (fmix32(id), id), fmix32 the
   32-bit finalizer of MurmurHash3 and id = 3 t + k for the half-edge a -> b,
   a < b, at corners k, k+1 of triangle t; an edge with g = 0 is left in place.
   New positions go to x_out, y_out, z_out (device, nv each; the mesh's
   positions where nothing moved).  d_counts (device, 3 int32): edges
   listed, edges moved, edges still pending after the rounds. */
ftc_status ftc_smooth_rough_edges(ftc_cells* cells, const ftc_grid* grid, const ftc_mesh* mesh, const double* gl_mag,
                                  const double* rough, double gl_threshold, double rough_threshold, int32_t max_rounds,
                                  double* x_out, double* y_out, double* z_out, int32_t* d_counts, void* stream);

/* ------------------------------------------------------------------------
   Launch shapes of a workspace, for fronts of different sizes and
   triangle-per-cell counts (an autotuner on top chooses them by timing:
   paper_2505_06932_amd/tune.py).  Every choice gives the same cell lists,
   decisions and PPIC results; the column chunking changes the order in
   which fluxes are summed, so volume fractions may differ in the last bits.
     ring_lanes    : lanes per interfacial cell in the fast PPIC shape, 4, 8,
                     16, 32 or 64 (64 / ring_lanes cells per wavefront);
     column_chunks : z-chunks (wavefronts) per 64-column block of the
                     volume-fraction column pass, 4, 8 or 16;
     ring_blocks   : workgroups of the fast PPIC shape, 0 for one per group of
                     cells (or, with a work queue, as many as the chip holds
                     at once), else a persistent grid of that many (<= 65536);
     queue_chunk   : 0 to split the cell groups statically over the
                     workgroups, else the number of groups (1 to 64) a
                     workgroup takes at a time from a work queue (one range
                     per XCD, taken in order, the others' ranges afterwards).
   Defaults: 8 lanes, 16 chunks for nz <= 256 and 4 above, one workgroup
   per group, no queue (the fastest shapes measured on fronts of 28k to 179k
   interfacial cells on 128^3 to 512^3).
   ------------------------------------------------------------------------ */
typedef struct {
  int32_t ring_lanes;
  int32_t column_chunks;
  int32_t ring_blocks;
  int32_t queue_chunk;
} ftc_tuning;

ftc_status ftc_get_tuning(const ftc_cells* cells, ftc_tuning* out /*[host]*/);
/* FTC_EINVAL (nothing changed) for a value outside the lists above. */
ftc_status ftc_set_tuning(ftc_cells* cells, const ftc_tuning* in /*[host]*/);

#ifdef __cplusplus
}
#endif
#endif
