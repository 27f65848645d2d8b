/*
 * ftc_oracle.c -- FP64 CPU oracle for the sharp front-tracking coupling on
 * interfacial cells (arXiv 2505.06932, section 3).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously-correct reference the
 * HIP library is compared with.  Nothing in the product path may load it.
 * It shares no code with the HIP library.  Build with -ffp-contract=off so
 * that every product and sum below is rounded exactly as written.
 *
 * What each part follows:
 *   cell lists       -- sec. 3.2: the interfacial cells are the cells the
 *                       front passes through; a (cell, triangle) pair exists
 *                       when their intersection has positive area.
 *   volume fraction  -- sec. 3.2, definition of the discrete indicator
 *                       alpha_C = |Omega_b cap C| / V_C with Omega_b the fluid
 *                       enclosed by the triangulated front (indicator of
 *                       sec. 2), evaluated exactly by the divergence theorem;
 *                       full and empty cells follow from the same column sums.
 *   PPIC curvature   -- sec. 3.2: local frame at the cell centre with the
 *                       normal of the closest front vertex, paraboloid
 *                       P(x,y), volume fit over the 3-ring (Eq. volumefit),
 *                       Wendland weights (Eq. Wendland) with delta = 2.5 dx
 *                       grown until enough triangles weigh in, normal
 *                       equations (Eq. volumefit2); mean curvature kappa = 2H
 *                       as in sec. 4.1 (kappa = 2/r for a sphere) and
 *                       appendix A.
 *   CSF              -- sec. 3.3, Eq. csf: S = sigma kappa grad(alpha).
 *   interpolation    -- sec. 3.1: the divergence-preserving polynomial for
 *                       u-bar; v-bar and w-bar by the same rule.
 */
#include "ftc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* grid geometry                                                            */
/* ------------------------------------------------------------------------ */

/* Coordinate of grid plane i along an axis with origin x0 and spacing h. */
static double plane_at(double x0, int64_t i, double h) { return x0 + (double)i * h; }

/* Index of the half-open cell [plane(i), plane(i+1)) containing x, exact with
   respect to the planes as computed by plane_at. */
static int64_t cell_of(double x, double x0, double h) {
  int64_t i = (int64_t)floor((x - x0) / h);
  while (plane_at(x0, i, h) > x) --i;
  while (plane_at(x0, i + 1, h) <= x) ++i;
  return i;
}

static int dims_of(const ora_grid* g, int d) { return d == 0 ? g->nx : (d == 1 ? g->ny : g->nz); }
static double org_of(const ora_grid* g, int d) { return d == 0 ? g->x0 : (d == 1 ? g->y0 : g->z0); }

static int grid_ok(const ora_grid* g) {
  return g && g->nx > 4 && g->ny > 4 && g->nz > 4 && g->h > 0.0 && isfinite(g->h) &&
         isfinite(g->x0) && isfinite(g->y0) && isfinite(g->z0);
}

/* Every vertex must lie at least two cells inside the grid. */
static int mesh_in_margin(const ora_grid* g, const ora_mesh* m) {
  for (int32_t v = 0; v < m->nv; ++v) {
    const double p[3] = {m->x[v], m->y[v], m->z[v]};
    for (int d = 0; d < 3; ++d) {
      double lo = plane_at(org_of(g, d), 2, g->h);
      double hi = plane_at(org_of(g, d), dims_of(g, d) - 2, g->h);
      if (!(p[d] >= lo && p[d] < hi)) return 0;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* triangle / cell clipping                                                 */
/* ------------------------------------------------------------------------ */

typedef struct { int n; double v[12][3]; } poly_t;

/* Point where segment p-q crosses the plane x_d = c.  The segment is taken
   from its endpoint with the smaller x_d, so the point does not depend on the
   direction in which the polygon walks the edge. */
/* A convex polygon cut by one plane gains at most one corner (nine after six
   planes); the capacity checks below only guard memory. */
static void cross_point(const double* p, const double* q, int d, double c, double* r) {
  const double* a = p[d] < q[d] ? p : q;
  const double* b = p[d] < q[d] ? q : p;
  double t = (c - a[d]) / (b[d] - a[d]);
  for (int e = 0; e < 3; ++e) r[e] = (e == d) ? c : a[e] + t * (b[e] - a[e]);
}

/* Sutherland-Hodgman step: keep x_d >= c (upper = 0) or x_d <= c (upper = 1). */
static void clip_half(const poly_t* in, poly_t* out, int d, double c, int upper) {
  out->n = 0;
  for (int e = 0; e < in->n; ++e) {
    const double* p = in->v[e];
    const double* q = in->v[(e + 1) % in->n];
    int pin = upper ? (p[d] <= c) : (p[d] >= c);
    int qin = upper ? (q[d] <= c) : (q[d] >= c);
    if (out->n + 2 > 12) break;
    if (pin && qin) {
      memcpy(out->v[out->n++], q, sizeof(double) * 3);
    } else if (pin) {
      if (p[d] != c) cross_point(p, q, d, c, out->v[out->n++]);
    } else if (qin) {
      if (q[d] != c) cross_point(p, q, d, c, out->v[out->n++]);
      memcpy(out->v[out->n++], q, sizeof(double) * 3);
    }
  }
}

/* Clip triangle tri (3 corners) to the closed box of cell (i, j, k).  Returns
   1 and the polygon if the piece has positive area under the half-open cell
   rule: a triangle lying exactly in a cell's upper plane belongs to the next
   cell, and a polygon with fewer than three corners or a zero vector area is
   no piece. */
static int clip_to_cell(const ora_grid* g, const double tri[3][3], const int64_t ijk[3], poly_t* out) {
  poly_t a, b;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = plane_at(org_of(g, d), ijk[d], g->h);
    hi[d] = plane_at(org_of(g, d), ijk[d] + 1, g->h);
    if (tri[0][d] == hi[d] && tri[1][d] == hi[d] && tri[2][d] == hi[d]) return 0;
  }
  a.n = 3;
  memcpy(a.v, tri, sizeof(double) * 9);
  poly_t* src = &a;
  poly_t* dst = &b;
  for (int d = 0; d < 3; ++d) {
    clip_half(src, dst, d, lo[d], 0);
    if (dst->n == 0) return 0;
    { poly_t* s = src; src = dst; dst = s; }
    clip_half(src, dst, d, hi[d], 1);
    if (dst->n == 0) return 0;
    { poly_t* s = src; src = dst; dst = s; }
  }
  if (src->n < 3) return 0;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  const double* q0 = src->v[0];
  for (int j = 1; j + 1 < src->n; ++j) {
    double ux = src->v[j][0] - q0[0], uy = src->v[j][1] - q0[1], uz = src->v[j][2] - q0[2];
    double vx = src->v[j + 1][0] - q0[0], vy = src->v[j + 1][1] - q0[1], vz = src->v[j + 1][2] - q0[2];
    sx += uy * vz - uz * vy;
    sy += uz * vx - ux * vz;
    sz += ux * vy - uy * vx;
  }
  if (sx == 0.0 && sy == 0.0 && sz == 0.0) return 0;
  *out = *src;
  return 1;
}

/* Integrals over a piece for columns along axis d, with (a, b) the other two
   axes in cyclic order: flux = integral of n_d dA (fan of signed projected
   triangles), vol = integral of (x_d - lo_d) n_d dA (exact: x_d is linear on
   the piece, so its mean over each fan triangle is the corner mean). */
static void piece_integrals(const poly_t* p, int d, double lo_d, double* flux, double* vol) {
  int a = (d + 1) % 3, b = (d + 2) % 3;
  const double* q0 = p->v[0];
  double f = 0.0, v = 0.0;
  for (int j = 1; j + 1 < p->n; ++j) {
    const double* q1 = p->v[j];
    const double* q2 = p->v[j + 1];
    double A = 0.5 * ((q1[a] - q0[a]) * (q2[b] - q0[b]) - (q2[a] - q0[a]) * (q1[b] - q0[b]));
    f += A;
    v += A * ((q0[d] + q1[d] + q2[d]) / 3.0 - lo_d);
  }
  *flux = f;
  *vol = v;
}

static void load_tri(const ora_mesh* m, int32_t t, double tri[3][3]) {
  const int32_t c[3] = {m->t0[t], m->t1[t], m->t2[t]};
  for (int r = 0; r < 3; ++r) {
    tri[r][0] = m->x[c[r]];
    tri[r][1] = m->y[c[r]];
    tri[r][2] = m->z[c[r]];
  }
}

static void tri_cell_range(const ora_grid* g, const double tri[3][3], int64_t lo[3], int64_t hi[3]) {
  for (int d = 0; d < 3; ++d) {
    double mn = tri[0][d], mx = tri[0][d];
    for (int r = 1; r < 3; ++r) {
      if (tri[r][d] < mn) mn = tri[r][d];
      if (tri[r][d] > mx) mx = tri[r][d];
    }
    lo[d] = cell_of(mn, org_of(g, d), g->h);
    hi[d] = cell_of(mx, org_of(g, d), g->h);
  }
}

static int mesh_ok(const ora_mesh* m) {
  if (!m || m->nv <= 0 || m->nt <= 0 || !m->x || !m->y || !m->z || !m->t0 || !m->t1 || !m->t2) return 0;
  for (int32_t t = 0; t < m->nt; ++t) {
    if (m->t0[t] < 0 || m->t0[t] >= m->nv || m->t1[t] < 0 || m->t1[t] >= m->nv || m->t2[t] < 0 ||
        m->t2[t] >= m->nv)
      return 0;
  }
  return 1;
}

int64_t ora_candidate_bound(const ora_grid* g, const ora_mesh* m) {
  if (!grid_ok(g) || !mesh_ok(m)) return -1;
  int64_t total = 0;
  for (int32_t t = 0; t < m->nt; ++t) {
    double tri[3][3];
    int64_t lo[3], hi[3];
    load_tri(m, t, tri);
    tri_cell_range(g, tri, lo, hi);
    total += (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  }
  return total;
}

typedef struct { int64_t cell; int32_t tri; } pair_t;

static int pair_cmp(const void* a, const void* b) {
  const pair_t* p = (const pair_t*)a;
  const pair_t* q = (const pair_t*)b;
  if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
  return (p->tri > q->tri) - (p->tri < q->tri);
}

int64_t ora_cell_lists(const ora_grid* g, const ora_mesh* m, int64_t cap, int64_t* pair_cell,
                       int32_t* pair_tri) {
  if (!grid_ok(g) || !mesh_ok(m) || cap < 0) return -1;
  if (!mesh_in_margin(g, m)) return -2;
  int64_t bound = ora_candidate_bound(g, m);
  pair_t* pairs = (pair_t*)malloc(sizeof(pair_t) * (size_t)(bound > 0 ? bound : 1));
  if (!pairs) return -1;
  int64_t n = 0;
  for (int32_t t = 0; t < m->nt; ++t) {
    double tri[3][3];
    int64_t lo[3], hi[3];
    load_tri(m, t, tri);
    tri_cell_range(g, tri, lo, hi);
    for (int64_t k = lo[2]; k <= hi[2]; ++k)
      for (int64_t j = lo[1]; j <= hi[1]; ++j)
        for (int64_t i = lo[0]; i <= hi[0]; ++i) {
          int64_t ijk[3] = {i, j, k};
          poly_t p;
          if (clip_to_cell(g, tri, ijk, &p)) {
            pairs[n].cell = i + (int64_t)g->nx * (j + (int64_t)g->ny * k);
            pairs[n].tri = t;
            ++n;
          }
        }
  }
  qsort(pairs, (size_t)n, sizeof(pair_t), pair_cmp);
  if (n > cap) {
    free(pairs);
    return -4;
  }
  for (int64_t q = 0; q < n; ++q) {
    pair_cell[q] = pairs[q].cell;
    pair_tri[q] = pairs[q].tri;
  }
  free(pairs);
  return n;
}

int32_t ora_piece(const ora_grid* g, const double tri_in[9], int32_t i, int32_t j, int32_t k, int32_t axis,
                  double out[2]) {
  double tri[3][3];
  memcpy(tri, tri_in, sizeof(double) * 9);
  int64_t ijk[3] = {i, j, k};
  poly_t p;
  out[0] = out[1] = 0.0;
  if (!clip_to_cell(g, tri, ijk, &p)) return 0;
  double lo = plane_at(org_of(g, axis), ijk[axis], g->h);
  piece_integrals(&p, axis, lo, &out[0], &out[1]);
  return 1;
}

/* ------------------------------------------------------------------------ */
/* volume fraction                                                          */
/* ------------------------------------------------------------------------ */

int32_t ora_volume_fraction(const ora_grid* g, const ora_mesh* m, int32_t axis, double* alpha,
                            uint8_t* is_if) {
  if (!grid_ok(g) || !mesh_ok(m) || axis < 0 || axis > 2 || !alpha || !is_if) return -1;
  if (!mesh_in_margin(g, m)) return -2;
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz, ncell = nx * ny * nz;
  const double h = g->h;
  double* flux = (double*)calloc((size_t)ncell, sizeof(double));
  double* vloc = (double*)calloc((size_t)ncell, sizeof(double));
  if (!flux || !vloc) {
    free(flux);
    free(vloc);
    return -1;
  }
  memset(is_if, 0, (size_t)ncell);
  /* Surface part: every piece's two integrals, accumulated per cell in
     ascending triangle order. */
  for (int32_t t = 0; t < m->nt; ++t) {
    double tri[3][3];
    int64_t lo[3], hi[3];
    load_tri(m, t, tri);
    tri_cell_range(g, tri, lo, hi);
    for (int64_t k = lo[2]; k <= hi[2]; ++k)
      for (int64_t j = lo[1]; j <= hi[1]; ++j)
        for (int64_t i = lo[0]; i <= hi[0]; ++i) {
          int64_t ijk[3] = {i, j, k};
          poly_t p;
          if (!clip_to_cell(g, tri, ijk, &p)) continue;
          double f, v;
          piece_integrals(&p, axis, plane_at(org_of(g, axis), ijk[axis], h), &f, &v);
          int64_t c = i + nx * (j + ny * k);
          flux[c] += f;
          vloc[c] += v;
          is_if[c] = 1;
        }
  }
  /* Column part.  With F = (x_d - lo_d) e_d (divergence 1), the volume of
     Omega_b in cell C is the surface integral over the pieces in C plus h
     times the wetted area W of C's upper face; F . n vanishes on the lower and
     side faces.  With F = e_d (divergence 0) on the part of the column above
     C, W equals the sum of the n_d-fluxes of all pieces strictly above C. */
  const int a = (axis + 1) % 3, b = (axis + 2) % 3;
  const int64_t n_d = dims_of(g, axis), n_a = dims_of(g, a), n_b = dims_of(g, b);
  const int64_t stride[3] = {1, nx, nx * ny};
  int32_t status = 0;
#pragma omp parallel for schedule(static) reduction(min : status)
  for (int64_t line = 0; line < n_a * n_b; ++line) {
    int64_t ia = line % n_a, ib = line / n_a;
    double W = 0.0;
    for (int64_t id = n_d - 1; id >= 0; --id) {
      int64_t c = ia * stride[a] + ib * stride[b] + id * stride[axis];
      if (is_if[c]) {
        alpha[c] = (vloc[c] + h * W) / (h * h * h);
      } else {
        double r = W / (h * h);
        double rr = round(r);
        if (fabs(r - rr) > 1e-9 || (rr != 0.0 && rr != 1.0)) status = -3;
        alpha[c] = rr;
      }
      W += flux[c];
    }
    if (fabs(W / (h * h)) > 1e-9) status = -3; /* the column must close */
  }
  free(flux);
  free(vloc);
  return status;
}

/* ------------------------------------------------------------------------ */
/* PPIC curvature                                                           */
/* ------------------------------------------------------------------------ */

double ora_kappa(const double a[6]) {
  /* Graph z = P(x, y): 2H = [(1+P_y^2) P_xx - 2 P_x P_y P_xy + (1+P_x^2) P_yy]
     / (1+P_x^2+P_y^2)^(3/2) at the origin, with P_x = a2, P_y = a3,
     P_xx = 2 a4, P_xy = a5, P_yy = 2 a6.  The frame normal points out of the
     fluid, so a sphere bends towards -n and kappa = -2H = 2/r > 0. */
  double gx = a[1], gy = a[2];
  double num = 2.0 * a[3] * (1.0 + gy * gy) - 2.0 * gx * gy * a[4] + 2.0 * a[5] * (1.0 + gx * gx);
  double s = 1.0 + gx * gx + gy * gy;
  return -num / (s * sqrt(s));
}

/* Weighted least squares by Householder QR: rows sqrt(w_t) m_t against
   sqrt(w_t) V_t, with m_t the six moments and V_t the volume under the
   triangle's plane over the projected triangle.  Returns 0, or 1 if the fit
   is rank deficient. */
int32_t ora_fit(const double frame[9], const double xc[3], double h, int32_t ntri, const double* tri,
                const double* w, double a_out[6]) {
  const double* t1 = frame;
  const double* t2 = frame + 3;
  const double* nn = frame + 6;
  double* A = (double*)malloc(sizeof(double) * 6 * (size_t)(ntri > 0 ? ntri : 1));
  double* rhs = (double*)malloc(sizeof(double) * (size_t)(ntri > 0 ? ntri : 1));
  int32_t rows = 0;
  double trace = 0.0;
  for (int32_t t = 0; t < ntri; ++t) {
    if (!(w[t] > 0.0)) continue;
    double xi[3], eta[3], zeta[3];
    for (int r = 0; r < 3; ++r) {
      double dx = tri[9 * t + 3 * r + 0] - xc[0];
      double dy = tri[9 * t + 3 * r + 1] - xc[1];
      double dz = tri[9 * t + 3 * r + 2] - xc[2];
      xi[r] = (dx * t1[0] + dy * t1[1] + dz * t1[2]) / h;
      eta[r] = (dx * t2[0] + dy * t2[1] + dz * t2[2]) / h;
      zeta[r] = (dx * nn[0] + dy * nn[1] + dz * nn[2]) / h;
    }
    /* Signed area of the projected triangle Gamma_t and the integrals of
       {1, x, y, x^2, xy, y^2} over it by the edge-midpoint rule, which is
       exact for quadratics. */
    double area = 0.5 * ((xi[1] - xi[0]) * (eta[2] - eta[0]) - (xi[2] - xi[0]) * (eta[1] - eta[0]));
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int e = 0; e < 3; ++e) {
      double mx = 0.5 * (xi[e] + xi[(e + 1) % 3]);
      double my = 0.5 * (eta[e] + eta[(e + 1) % 3]);
      s[0] += 1.0;
      s[1] += mx;
      s[2] += my;
      s[3] += mx * mx;
      s[4] += mx * my;
      s[5] += my * my;
    }
    /* Integral of the triangle's plane g_t over Gamma_t: g_t is linear, so
       it is the area times the mean corner height. */
    double vol = area * (zeta[0] + zeta[1] + zeta[2]) / 3.0;
    double sw = sqrt(w[t]);
    for (int c = 0; c < 6; ++c) {
      double mc = area * s[c] / 3.0;
      A[6 * rows + c] = sw * mc;
      trace += w[t] * mc * mc;
    }
    rhs[rows] = sw * vol;
    ++rows;
  }
  int32_t status = 0;
  double ahat[6] = {0, 0, 0, 0, 0, 0};
  if (rows < 6) {
    status = 1;
  } else {
    double R[6][6];
    for (int k = 0; k < 6; ++k) {
      double norm2 = 0.0;
      for (int32_t r = k; r < rows; ++r) norm2 += A[6 * r + k] * A[6 * r + k];
      double nrm = sqrt(norm2);
      double x0 = A[6 * k + k];
      double alpha = x0 >= 0.0 ? -nrm : nrm;
      if (nrm == 0.0) {
        R[k][k] = 0.0;
        for (int c = k + 1; c < 6; ++c) R[k][c] = A[6 * k + c];
        continue;
      }
      /* v = x - alpha e1, stored in place of column k */
      A[6 * k + k] = x0 - alpha;
      double vnorm2 = norm2 - x0 * x0 + (x0 - alpha) * (x0 - alpha);
      for (int c = k + 1; c < 6; ++c) {
        double dot = 0.0;
        for (int32_t r = k; r < rows; ++r) dot += A[6 * r + k] * A[6 * r + c];
        double f = 2.0 * dot / vnorm2;
        for (int32_t r = k; r < rows; ++r) A[6 * r + c] -= f * A[6 * r + k];
      }
      {
        double dot = 0.0;
        for (int32_t r = k; r < rows; ++r) dot += A[6 * r + k] * rhs[r];
        double f = 2.0 * dot / vnorm2;
        for (int32_t r = k; r < rows; ++r) rhs[r] -= f * A[6 * r + k];
      }
      R[k][k] = alpha;
      for (int c = k + 1; c < 6; ++c) R[k][c] = A[6 * k + c];
    }
    for (int k = 0; k < 6; ++k)
      if (R[k][k] * R[k][k] <= 1e-14 * trace) status = 1;
    if (!status) {
      for (int k = 5; k >= 0; --k) {
        double s = rhs[k];
        for (int c = k + 1; c < 6; ++c) s -= R[k][c] * ahat[c];
        ahat[k] = s / R[k][k];
      }
    }
  }
  free(A);
  free(rhs);
  if (status) {
    for (int c = 0; c < 6; ++c) a_out[c] = NAN;
    return status;
  }
  /* Back to world units: z = h zeta(x/h, y/h). */
  a_out[0] = h * ahat[0];
  a_out[1] = ahat[1];
  a_out[2] = ahat[2];
  a_out[3] = ahat[3] / h;
  a_out[4] = ahat[4] / h;
  a_out[5] = ahat[5] / h;
  return 0;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Vertex -> incident triangles, ascending triangle id: *off[nv + 1] and
   *ids[3 nt], allocated here (free both). */
static void vertex_triangles(const ora_mesh* m, int32_t** off, int32_t** ids) {
  const int32_t nv = m->nv, nt = m->nt;
  int32_t* vt_off = (int32_t*)calloc((size_t)nv + 1, sizeof(int32_t));
  int32_t* vt_ids = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)nt);
  int32_t* fill = (int32_t*)calloc((size_t)nv, sizeof(int32_t));
  for (int32_t t = 0; t < nt; ++t) {
    vt_off[m->t0[t] + 1]++;
    vt_off[m->t1[t] + 1]++;
    vt_off[m->t2[t] + 1]++;
  }
  for (int32_t v = 0; v < nv; ++v) vt_off[v + 1] += vt_off[v];
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t c[3] = {m->t0[t], m->t1[t], m->t2[t]};
    for (int r = 0; r < 3; ++r) vt_ids[vt_off[c[r]] + fill[c[r]]++] = t;
  }
  free(fill);
  *off = vt_off;
  *ids = vt_ids;
}

/* Per-thread working storage of the PPIC steps for one cell. */
typedef struct {
  int32_t *tmark, *vmark, *tlist, *vlist, *vnext;
  double *d2, *wts, *tri;
  int32_t stamp;
} ppic_scratch;

static void scratch_init(ppic_scratch* s, int32_t nv, int32_t nt) {
  s->tmark = (int32_t*)calloc((size_t)nt, sizeof(int32_t));
  s->vmark = (int32_t*)calloc((size_t)nv, sizeof(int32_t));
  s->tlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)nt);
  s->vlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)nv);
  s->vnext = (int32_t*)malloc(sizeof(int32_t) * (size_t)nv);
  s->d2 = (double*)malloc(sizeof(double) * (size_t)nt);
  s->wts = (double*)malloc(sizeof(double) * (size_t)nt);
  s->tri = (double*)malloc(sizeof(double) * 9 * (size_t)nt);
  s->stamp = 0;
}

static void scratch_free(ppic_scratch* s) {
  free(s->tmark);
  free(s->vmark);
  free(s->tlist);
  free(s->vlist);
  free(s->vnext);
  free(s->d2);
  free(s->wts);
  free(s->tri);
}

/* The PPIC steps for the cell with linear id cid.  Leaves the ring
   triangles (ascending) in s->tlist[0, *ntl_out), their centre distances
   squared in s->d2, their weights in s->wts and the support radius in
   *delta_out; writes kappa, the interface normal, the coefficients, the
   status and diag[4] = {closest vertex, ring size, triangles with non-zero
   weight, support adjustments}. */
static void ppic_cell(const ora_grid* g, const ora_mesh* m, const ora_ppic_params* prm, const int32_t* vt_off,
                      const int32_t* vt_ids, int64_t cid, ppic_scratch* s, int32_t* ntl_out, double* delta_out,
                      double* kap_out, double ni[3], double co[6], int32_t* st_out, int32_t diag[4]) {
  const int32_t nv = m->nv;
  const double h = g->h;
  int32_t *tmark = s->tmark, *vmark = s->vmark, *tlist = s->tlist, *vlist = s->vlist, *vnext = s->vnext;
  double *d2 = s->d2, *wts = s->wts, *tri = s->tri;
  int64_t i = cid % g->nx, j = (cid / g->nx) % g->ny, k = cid / ((int64_t)g->nx * g->ny);
  double xc[3] = {g->x0 + ((double)i + 0.5) * h, g->y0 + ((double)j + 0.5) * h,
                  g->z0 + ((double)k + 0.5) * h};
  /* 1. closest front vertex (lowest index on ties) */
  double best = DBL_MAX;
  int32_t vs = -1;
  for (int32_t v = 0; v < nv; ++v) {
    double dx = m->x[v] - xc[0], dy = m->y[v] - xc[1], dz = m->z[v] - xc[2];
    double dd = dx * dx + dy * dy + dz * dz;
    if (dd < best) {
      best = dd;
      vs = v;
    }
  }
  /* 2. its normal: area-weighted sum of the incident triangle normals */
  double n[3] = {0, 0, 0};
  for (int32_t e = vt_off[vs]; e < vt_off[vs + 1]; ++e) {
    double tr[3][3];
    load_tri(m, vt_ids[e], tr);
    double ux = tr[1][0] - tr[0][0], uy = tr[1][1] - tr[0][1], uz = tr[1][2] - tr[0][2];
    double wx = tr[2][0] - tr[0][0], wy = tr[2][1] - tr[0][1], wz = tr[2][2] - tr[0][2];
    n[0] += uy * wz - uz * wy;
    n[1] += uz * wx - ux * wz;
    n[2] += ux * wy - uy * wx;
  }
  double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  n[0] /= nl;
  n[1] /= nl;
  n[2] /= nl;
  /* 3. tangents completing a right-handed orthonormal frame (Duff et al.,
     "Building an orthonormal basis, revisited", JCGT 2017) */
  double sg = copysign(1.0, n[2]);
  double ca = -1.0 / (sg + n[2]);
  double cb = n[0] * n[1] * ca;
  double frame[9] = {1.0 + sg * n[0] * n[0] * ca, sg * cb, -sg * n[0],
                     cb, sg + n[1] * n[1] * ca, -n[1],
                     n[0], n[1], n[2]};
  /* 4. ring neighbourhood: T_1 = triangles at the vertex, T_{r+1} =
     triangles sharing a vertex with T_r */
  ++s->stamp;
  int32_t nvl = 1, ntl = 0;
  vlist[0] = vs;
  vmark[vs] = s->stamp;
  for (int32_t r = 1; r <= prm->rings; ++r) {
    ntl = 0;
    ++s->stamp;
    for (int32_t a = 0; a < nvl; ++a)
      for (int32_t e = vt_off[vlist[a]]; e < vt_off[vlist[a] + 1]; ++e) {
        int32_t t = vt_ids[e];
        if (tmark[t] != s->stamp) {
          tmark[t] = s->stamp;
          tlist[ntl++] = t;
        }
      }
    if (r == prm->rings) break;
    int32_t nn2 = 0;
    for (int32_t a = 0; a < ntl; ++a) {
      const int32_t c[3] = {m->t0[tlist[a]], m->t1[tlist[a]], m->t2[tlist[a]]};
      for (int q = 0; q < 3; ++q)
        if (vmark[c[q]] != s->stamp) {
          vmark[c[q]] = s->stamp;
          vnext[nn2++] = c[q];
        }
    }
    memcpy(vlist, vnext, sizeof(int32_t) * (size_t)nn2);
    nvl = nn2;
  }
  qsort(tlist, (size_t)ntl, sizeof(int32_t), cmp_i32);
  /* 5. distances of the triangle centres to the cell centre */
  for (int32_t a = 0; a < ntl; ++a) {
    double tr[3][3];
    load_tri(m, tlist[a], tr);
    memcpy(tri + 9 * a, tr, sizeof(double) * 9);
    double cx = (tr[0][0] + tr[1][0] + tr[2][0]) / 3.0;
    double cy = (tr[0][1] + tr[1][1] + tr[2][1]) / 3.0;
    double cz = (tr[0][2] + tr[1][2] + tr[2][2]) / 3.0;
    double dx = cx - xc[0], dy = cy - xc[1], dz = cz - xc[2];
    d2[a] = dx * dx + dy * dy + dz * dz;
  }
  /* 6. support radius: grow until enough triangles have non-zero weight */
  double delta = prm->delta_over_h * h;
  int32_t it = 0, cnt = 0;
  for (;;) {
    double lim = delta * delta;
    cnt = 0;
    for (int32_t a = 0; a < ntl; ++a) cnt += d2[a] < lim;
    if (cnt >= prm->n_min || cnt == ntl || it == prm->max_iter) break;
    delta = delta * prm->grow;
    ++it;
  }
  /* 7. Wendland C2 weights */
  double lim = delta * delta;
  for (int32_t a = 0; a < ntl; ++a) {
    if (d2[a] < lim) {
      double qq = sqrt(d2[a]) / delta;
      double om = 1.0 - qq;
      wts[a] = (1.0 + 4.0 * qq) * (om * om) * (om * om);
    } else {
      wts[a] = 0.0;
    }
  }
  /* 8. volume fit, curvature and interface normal */
  int32_t st = ora_fit(frame, xc, h, ntl, tri, wts, co);
  *kap_out = st ? NAN : ora_kappa(co);
  ni[0] = ni[1] = ni[2] = NAN;
  if (!st) {
    for (int d = 0; d < 3; ++d) ni[d] = frame[6 + d] - co[1] * frame[d] - co[2] * frame[3 + d];
    double l = sqrt(ni[0] * ni[0] + ni[1] * ni[1] + ni[2] * ni[2]);
    for (int d = 0; d < 3; ++d) ni[d] /= l;
  }
  *st_out = st;
  *ntl_out = ntl;
  *delta_out = delta;
  diag[0] = vs;
  diag[1] = ntl;
  diag[2] = cnt;
  diag[3] = it;
}

static int ppic_params_ok(const ora_ppic_params* prm) {
  return prm && prm->rings >= 1 && prm->n_min >= 1 && prm->delta_over_h > 0.0 && prm->grow > 1.0 &&
         prm->max_iter >= 0;
}

int32_t ora_ppic(const ora_grid* g, const ora_mesh* m, const ora_ppic_params* prm, int64_t ncell,
                 const int64_t* cell_ids, double* kappa, double* nrm, double* coeff, int32_t* status,
                 int32_t* diag) {
  if (!grid_ok(g) || !mesh_ok(m) || !ppic_params_ok(prm) || ncell < 0 || (ncell > 0 && !cell_ids)) return -1;
  int32_t *vt_off, *vt_ids;
  vertex_triangles(m, &vt_off, &vt_ids);
#pragma omp parallel
  {
    ppic_scratch s;
    scratch_init(&s, m->nv, m->nt);
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < ncell; ++q) {
      int32_t ntl, st, dg[4];
      double delta, kap, ni[3], co[6];
      ppic_cell(g, m, prm, vt_off, vt_ids, cell_ids[q], &s, &ntl, &delta, &kap, ni, co, &st, dg);
      if (kappa) kappa[q] = kap;
      if (nrm)
        for (int d = 0; d < 3; ++d) nrm[3 * q + d] = ni[d];
      if (coeff)
        for (int c = 0; c < 6; ++c) coeff[6 * q + c] = co[c];
      if (status) status[q] = st;
      if (diag)
        for (int d = 0; d < 4; ++d) diag[4 * q + d] = dg[d];
    }
    scratch_free(&s);
  }
  free(vt_off);
  free(vt_ids);
  return 0;
}

int32_t ora_ppic_support(const ora_grid* g, const ora_mesh* m, const ora_ppic_params* prm, int64_t cell_id,
                         int32_t cap, int32_t* tri_out, double* d2_out, double* w_out, double* delta_out) {
  if (!grid_ok(g) || !mesh_ok(m) || !ppic_params_ok(prm) || cap < 0 || !tri_out || !d2_out || !w_out ||
      !delta_out || cell_id < 0 || cell_id >= (int64_t)g->nx * g->ny * g->nz)
    return -1;
  int32_t *vt_off, *vt_ids;
  vertex_triangles(m, &vt_off, &vt_ids);
  ppic_scratch s;
  scratch_init(&s, m->nv, m->nt);
  int32_t ntl, st, dg[4];
  double kap, ni[3], co[6];
  ppic_cell(g, m, prm, vt_off, vt_ids, cell_id, &s, &ntl, delta_out, &kap, ni, co, &st, dg);
  for (int32_t a = 0; a < ntl && a < cap; ++a) {
    tri_out[a] = s.tlist[a];
    d2_out[a] = s.d2[a];
    w_out[a] = s.wts[a];
  }
  scratch_free(&s);
  free(vt_off);
  free(vt_ids);
  return ntl;
}

/* ------------------------------------------------------------------------ */
/* CSF                                                                      */
/* ------------------------------------------------------------------------ */

int32_t ora_frame_normal(const ora_grid* g, const ora_mesh* m, int64_t ncell,
                         const int64_t* cell_ids, int32_t* vstar, double* best_d2,
                         double* nrm) {
  if (!grid_ok(g) || !mesh_ok(m) || ncell < 0 || (ncell > 0 && !cell_ids)) return -1;
  const double h = g->h;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < ncell; ++q) {
    int64_t cid = cell_ids[q];
    int64_t i = cid % g->nx, j = (cid / g->nx) % g->ny, k = cid / ((int64_t)g->nx * g->ny);
    double xc[3] = {g->x0 + ((double)i + 0.5) * h, g->y0 + ((double)j + 0.5) * h,
                    g->z0 + ((double)k + 0.5) * h};
    double best = DBL_MAX;
    int32_t vs = -1;
    for (int32_t v = 0; v < m->nv; ++v) {
      double dx = m->x[v] - xc[0], dy = m->y[v] - xc[1], dz = m->z[v] - xc[2];
      double dd = dx * dx + dy * dy + dz * dz;
      if (dd < best) {
        best = dd;
        vs = v;
      }
    }
    /* the incident triangles of vs in ascending order: a scan of all triangles */
    double n[3] = {0, 0, 0};
    for (int32_t t = 0; t < m->nt; ++t) {
      if (m->t0[t] != vs && m->t1[t] != vs && m->t2[t] != vs) continue;
      double tr[3][3];
      load_tri(m, t, tr);
      double ux = tr[1][0] - tr[0][0], uy = tr[1][1] - tr[0][1], uz = tr[1][2] - tr[0][2];
      double wx = tr[2][0] - tr[0][0], wy = tr[2][1] - tr[0][1], wz = tr[2][2] - tr[0][2];
      n[0] += uy * wz - uz * wy;
      n[1] += uz * wx - ux * wz;
      n[2] += ux * wy - uy * wx;
    }
    double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (vstar) vstar[q] = vs;
    if (best_d2) best_d2[q] = best;
    if (nrm)
      for (int d = 0; d < 3; ++d) nrm[3 * q + d] = n[d] / nl;
  }
  return 0;
}

int32_t ora_csf(const ora_grid* g, const double* alpha, int64_t ncell, const int64_t* cell_ids,
                const double* kappa, double sigma, double* f) {
  if (!grid_ok(g) || !alpha || ncell < 0 || (ncell > 0 && (!cell_ids || !kappa || !f))) return -1;
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
  for (int64_t q = 0; q < ncell; ++q) {
    int64_t c = cell_ids[q];
    int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    if (i < 1 || j < 1 || k < 1 || i > nx - 2 || j > ny - 2 || k > nz - 2) return -2;
    double gx = (alpha[c + 1] - alpha[c - 1]) / (2.0 * g->h);
    double gy = (alpha[c + nx] - alpha[c - nx]) / (2.0 * g->h);
    double gz = (alpha[c + nx * ny] - alpha[c - nx * ny]) / (2.0 * g->h);
    f[3 * q + 0] = sigma * kappa[q] * gx;
    f[3 * q + 1] = sigma * kappa[q] * gy;
    f[3 * q + 2] = sigma * kappa[q] * gz;
  }
  return 0;
}

/* BAND mode (paper sec. 3.3): the curvature of a cell next to the interface
   is the average of the curvatures of the interfacial cells around it,
   weighted by how well the offset to each lines up with its interface
   normal: kappa_bar_P = sum_Q kappa_Q w_Q / sum_Q w_Q, w_Q = |s_Q . n_Q| /
   |s_Q|, s_Q from the centre of P to the centre of Q.  Read here as: P runs
   over the cells sharing a face with an interfacial cell without being
   interfacial, Q over the interfacial cells among P's 26 neighbours (block
   order, x fastest) whose curvature is finite; sum w_Q = 0 falls back to the
   plain mean, no such Q gives NaN.  s_Q = (di, dj, dk) h, so
   w_Q = |di n_x + dj n_y + dk n_z| / sqrt(di^2 + dj^2 + dk^2). */
static int64_t find_cell(const int64_t* ids, int64_t n, int64_t c) {
  int64_t lo = 0, hi = n - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (ids[mid] == c) return mid;
    if (ids[mid] < c) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int64_t ora_csf_band(const ora_grid* g, const double* alpha, int64_t ncell, const int64_t* cell_ids,
                     const double* kappa, const double* nrm, double sigma, int64_t cap, int64_t* band_ids,
                     double* kappa_band, double* f) {
  if (!grid_ok(g) || !alpha || ncell < 0 || cap < 0 || (ncell > 0 && (!cell_ids || !kappa || !nrm)) ||
      (cap > 0 && (!band_ids || !kappa_band || !f)))
    return -1;
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz, ntot = nx * ny * nz;
  for (int64_t q = 1; q < ncell; ++q)
    if (cell_ids[q] <= cell_ids[q - 1]) return -1; /* ascending, as the cell lists give them */
  unsigned char* mark = (unsigned char*)calloc((size_t)ntot, 1);
  if (!mark) return -1;
  for (int64_t q = 0; q < ncell; ++q) mark[cell_ids[q]] = 1;
  for (int64_t q = 0; q < ncell; ++q) {
    const int64_t c = cell_ids[q];
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    const int64_t nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
    for (int e = 0; e < 6; ++e) {
      const int64_t a = nb[e][0], b = nb[e][1], d = nb[e][2];
      if (a < 0 || b < 0 || d < 0 || a >= nx || b >= ny || d >= nz) continue;
      const int64_t cn = a + nx * (b + ny * d);
      if (mark[cn] == 0) mark[cn] = 2;
    }
  }
  int64_t nb_out = 0;
  int bad = 0;
  for (int64_t c = 0; c < ntot; ++c) {
    if (mark[c] != 2) continue;
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    if (i < 1 || j < 1 || k < 1 || i > nx - 2 || j > ny - 2 || k > nz - 2) { bad = 1; break; }
    double sw = 0.0, swk = 0.0, sk = 0.0;
    int64_t nq = 0;
    for (int dk = -1; dk <= 1; ++dk)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          if (di == 0 && dj == 0 && dk == 0) continue;
          const int64_t cq = (i + di) + nx * ((j + dj) + ny * (k + dk));
          if (mark[cq] != 1) continue;
          const int64_t q = find_cell(cell_ids, ncell, cq);
          if (q < 0 || !isfinite(kappa[q])) continue;
          const double sn = (double)di * nrm[3 * q] + (double)dj * nrm[3 * q + 1] + (double)dk * nrm[3 * q + 2];
          const double w = fabs(sn) / sqrt((double)(di * di + dj * dj + dk * dk));
          sw += w;
          swk += kappa[q] * w;
          sk += kappa[q];
          ++nq;
        }
    double kb;
    if (nq == 0) kb = NAN;
    else if (sw > 0.0) kb = swk / sw;
    else kb = sk / (double)nq;
    if (nb_out < cap) {
      const double gx = (alpha[c + 1] - alpha[c - 1]) / (2.0 * g->h);
      const double gy = (alpha[c + nx] - alpha[c - nx]) / (2.0 * g->h);
      const double gz = (alpha[c + nx * ny] - alpha[c - nx * ny]) / (2.0 * g->h);
      band_ids[nb_out] = c;
      kappa_band[nb_out] = kb;
      f[3 * nb_out + 0] = sigma * kb * gx;
      f[3 * nb_out + 1] = sigma * kb * gy;
      f[3 * nb_out + 2] = sigma * kb * gz;
    }
    ++nb_out;
  }
  free(mark);
  return bad ? -2 : nb_out;
}

/* ------------------------------------------------------------------------ */
/* divergence-preserving interpolation                                      */
/* ------------------------------------------------------------------------ */

void ora_interp_in_cell(const ora_grid* g, int32_t i, int32_t j, int32_t k, double x, double y, double z,
                        const double* U, const double* V, const double* W, double u[3]) {
  const int64_t nx = g->nx, ny = g->ny;
  const double h = g->h;
#define UF(a, b, c) U[(int64_t)(a) + (nx + 1) * ((int64_t)(b) + ny * (int64_t)(c))]
#define VF(a, b, c) V[(int64_t)(a) + nx * ((int64_t)(b) + (ny + 1) * (int64_t)(c))]
#define WF(a, b, c) W[(int64_t)(a) + nx * ((int64_t)(b) + ny * (int64_t)(c))]
  /* normal velocities on the six faces */
  double Um = UF(i, j, k), Up = UF(i + 1, j, k);
  double Vm = VF(i, j, k), Vp = VF(i, j + 1, k);
  double Wm = WF(i, j, k), Wp = WF(i, j, k + 1);
  /* transverse gradients on each face: central differences over the faces of
     the same orientation in the neighbouring cells */
  double Uy_m = (UF(i, j + 1, k) - UF(i, j - 1, k)) / (2.0 * h);
  double Uy_p = (UF(i + 1, j + 1, k) - UF(i + 1, j - 1, k)) / (2.0 * h);
  double Uz_m = (UF(i, j, k + 1) - UF(i, j, k - 1)) / (2.0 * h);
  double Uz_p = (UF(i + 1, j, k + 1) - UF(i + 1, j, k - 1)) / (2.0 * h);
  double Vx_m = (VF(i + 1, j, k) - VF(i - 1, j, k)) / (2.0 * h);
  double Vx_p = (VF(i + 1, j + 1, k) - VF(i - 1, j + 1, k)) / (2.0 * h);
  double Vz_m = (VF(i, j, k + 1) - VF(i, j, k - 1)) / (2.0 * h);
  double Vz_p = (VF(i, j + 1, k + 1) - VF(i, j + 1, k - 1)) / (2.0 * h);
  double Wx_m = (WF(i + 1, j, k) - WF(i - 1, j, k)) / (2.0 * h);
  double Wx_p = (WF(i + 1, j, k + 1) - WF(i - 1, j, k + 1)) / (2.0 * h);
  double Wy_m = (WF(i, j + 1, k) - WF(i, j - 1, k)) / (2.0 * h);
  double Wy_p = (WF(i, j + 1, k + 1) - WF(i, j - 1, k + 1)) / (2.0 * h);
#undef UF
#undef VF
#undef WF
  double xm = g->x0 + (double)i * h, xp = g->x0 + (double)(i + 1) * h;
  double ym = g->y0 + (double)j * h, yp = g->y0 + (double)(j + 1) * h;
  double zm = g->z0 + (double)k * h, zp = g->z0 + (double)(k + 1) * h;
  double xb = 0.5 * (xm + xp), yb = 0.5 * (ym + yp), zb = 0.5 * (zm + zp);
  double dx = xp - xm, dy = yp - ym, dz = zp - zm;
  u[0] = (x - xm) / dx * (Up + (y - yb) * Uy_p + (z - zb) * Uz_p) +
         (xp - x) / dx * (Um + (y - yb) * Uy_m + (z - zb) * Uz_m) +
         (xp - x) * (x - xm) / (2.0 * dx) * (Vx_p - Vx_m + Wx_p - Wx_m);
  u[1] = (y - ym) / dy * (Vp + (x - xb) * Vx_p + (z - zb) * Vz_p) +
         (yp - y) / dy * (Vm + (x - xb) * Vx_m + (z - zb) * Vz_m) +
         (yp - y) * (y - ym) / (2.0 * dy) * (Uy_p - Uy_m + Wy_p - Wy_m);
  u[2] = (z - zm) / dz * (Wp + (x - xb) * Wx_p + (y - yb) * Wy_p) +
         (zp - z) / dz * (Wm + (x - xb) * Wx_m + (y - yb) * Wy_m) +
         (zp - z) * (z - zm) / (2.0 * dz) * (Uz_p - Uz_m + Vz_p - Vz_m);
}

int32_t ora_interp(const ora_grid* g, int32_t n, const double* x, const double* y, const double* z,
                   const double* U, const double* V, const double* W, double* u) {
  if (!grid_ok(g) || n < 0 || (n > 0 && (!x || !y || !z || !U || !V || !W || !u))) return -1;
  for (int32_t q = 0; q < n; ++q) {
    if (!(isfinite(x[q]) && isfinite(y[q]) && isfinite(z[q]))) return -2;
    int64_t i = cell_of(x[q], g->x0, g->h), j = cell_of(y[q], g->y0, g->h), k = cell_of(z[q], g->z0, g->h);
    if (i < 1 || j < 1 || k < 1 || i > g->nx - 2 || j > g->ny - 2 || k > g->nz - 2) return -2;
  }
#pragma omp parallel for schedule(static)
  for (int32_t q = 0; q < n; ++q) {
    int64_t i = cell_of(x[q], g->x0, g->h), j = cell_of(y[q], g->y0, g->h), k = cell_of(z[q], g->z0, g->h);
    ora_interp_in_cell(g, (int32_t)i, (int32_t)j, (int32_t)k, x[q], y[q], z[q], U, V, W, u + 3 * q);
  }
  return 0;
}

/* One classical fourth-order Runge-Kutta step (paper sec. 3.1: the front
   vertices move with the interpolated velocity, dx/dt = u(x)) with the face
   velocities held fixed over the step:
     k1 = u(x), k2 = u(x + dt/2 k1), k3 = u(x + dt/2 k2), k4 = u(x + dt k3),
     x' = x + dt/6 (k1 + 2 k2 + 2 k3 + k4),
   each u the divergence-preserving interpolant in the cell holding the stage
   point.  A vertex whose stage point leaves the admissible cells (index 1 to
   n - 2 on every axis) gets NaN and the call returns -2. */
static int stage_velocity(const ora_grid* g, const double p[3], const double* U, const double* V, const double* W,
                          double u[3]) {
  if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) return 0;
  const int64_t i = cell_of(p[0], g->x0, g->h), j = cell_of(p[1], g->y0, g->h), k = cell_of(p[2], g->z0, g->h);
  if (i < 1 || j < 1 || k < 1 || i > g->nx - 2 || j > g->ny - 2 || k > g->nz - 2) return 0;
  ora_interp_in_cell(g, (int32_t)i, (int32_t)j, (int32_t)k, p[0], p[1], p[2], U, V, W, u);
  return 1;
}

int32_t ora_advect_rk4(const ora_grid* g, int32_t n, const double* x, const double* y, const double* z,
                       const double* U, const double* V, const double* W, double dt, double* out) {
  if (!grid_ok(g) || n < 0 || !isfinite(dt) || (n > 0 && (!x || !y || !z || !U || !V || !W || !out))) return -1;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int32_t q = 0; q < n; ++q) {
    const double p[3] = {x[q], y[q], z[q]};
    double k1[3], k2[3], k3[3], k4[3], s[3];
    int ok = stage_velocity(g, p, U, V, W, k1);
    for (int d = 0; d < 3; ++d) s[d] = p[d] + (0.5 * dt) * k1[d];
    ok = ok && stage_velocity(g, s, U, V, W, k2);
    for (int d = 0; d < 3; ++d) s[d] = p[d] + (0.5 * dt) * k2[d];
    ok = ok && stage_velocity(g, s, U, V, W, k3);
    for (int d = 0; d < 3; ++d) s[d] = p[d] + dt * k3[d];
    ok = ok && stage_velocity(g, s, U, V, W, k4);
    for (int d = 0; d < 3; ++d)
      out[3 * q + d] = ok ? p[d] + (dt / 6.0) * (((k1[d] + 2.0 * k2[d]) + 2.0 * k3[d]) + k4[d]) : NAN;
    if (!ok) bad = 1;
  }
  return bad ? -2 : 0;
}

int32_t ora_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}
