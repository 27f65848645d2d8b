/* Runs the oracle's native entry points on a front read from a file, for a
   build with AddressSanitizer and UndefinedBehaviorSanitizer (test
   infrastructure only).  The file holds the grid, the mesh and the face
   velocities as written by tests/test_sanitizers.py:
     int32 nx ny nz, float64 x0 y0 z0 h, int32 nv nt, float64 x[nv] y[nv]
     z[nv], int32 t0[nt] t1[nt] t2[nt], float64 U[(nx+1)ny nz]
     V[nx(ny+1)nz] W[nx ny(nz+1)].
   Prints one line of checksums per call; exits non-zero on a failed call. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ftc_oracle.h"

static void* take(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

static double sum(const double* a, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (a[i] == a[i]) s += a[i];
  return s;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  ora_grid g;
  int32_t* dims = (int32_t*)take(f, 3 * sizeof(int32_t));
  double* org = (double*)take(f, 4 * sizeof(double));
  g.nx = dims[0];
  g.ny = dims[1];
  g.nz = dims[2];
  g.x0 = org[0];
  g.y0 = org[1];
  g.z0 = org[2];
  g.h = org[3];
  int32_t* sz = (int32_t*)take(f, 2 * sizeof(int32_t));
  const int32_t nv = sz[0], nt = sz[1];
  double* x = (double*)take(f, sizeof(double) * (size_t)nv);
  double* y = (double*)take(f, sizeof(double) * (size_t)nv);
  double* z = (double*)take(f, sizeof(double) * (size_t)nv);
  int32_t* t0 = (int32_t*)take(f, sizeof(int32_t) * (size_t)nt);
  int32_t* t1 = (int32_t*)take(f, sizeof(int32_t) * (size_t)nt);
  int32_t* t2 = (int32_t*)take(f, sizeof(int32_t) * (size_t)nt);
  const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
  double* U = (double*)take(f, sizeof(double) * (size_t)((g.nx + 1) * (int64_t)g.ny * g.nz));
  double* V = (double*)take(f, sizeof(double) * (size_t)(g.nx * (int64_t)(g.ny + 1) * g.nz));
  double* W = (double*)take(f, sizeof(double) * (size_t)(g.nx * (int64_t)g.ny * (g.nz + 1)));
  fclose(f);
  ora_mesh m = {nv, nt, x, y, z, t0, t1, t2};

  /* cell lists */
  const int64_t cap = ora_candidate_bound(&g, &m);
  int64_t* pc = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
  int32_t* pt = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  const int64_t np = ora_cell_lists(&g, &m, cap, pc, pt);
  if (np < 0) return 3;
  int64_t nif = 0, tsum = 0;
  int64_t* cells = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
  for (int64_t p = 0; p < np; ++p) {
    tsum += pt[p];
    if (p == 0 || pc[p] != pc[p - 1]) cells[nif++] = pc[p];
  }
  printf("cell_lists pairs %lld cells %lld tri_sum %lld\n", (long long)np, (long long)nif, (long long)tsum);

  /* volume fractions along each axis */
  double* alpha = (double*)malloc(sizeof(double) * (size_t)ncell);
  uint8_t* isif = (uint8_t*)malloc((size_t)ncell);
  for (int32_t axis = 0; axis < 3; ++axis) {
    if (ora_volume_fraction(&g, &m, axis, alpha, isif) != 0) return 4;
    printf("volume_fraction axis %d sum %.17g\n", axis, sum(alpha, ncell));
  }

  /* PPIC, its support, the CSF source in both modes */
  ora_ppic_params prm = {2.5, 3, 24, 1.1, 16};
  const int64_t nc = nif;
  double* kap = (double*)malloc(sizeof(double) * (size_t)nc);
  double* nrm = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  double* co = (double*)malloc(sizeof(double) * 6 * (size_t)nc);
  int32_t* st = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
  int32_t* dg = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)nc);
  if (ora_ppic(&g, &m, &prm, nc, cells, kap, nrm, co, st, dg) != 0) return 5;
  int64_t dsum = 0;
  for (int64_t q = 0; q < 4 * nc; ++q) dsum += dg[q];
  printf("ppic kappa_sum %.17g normal_sum %.17g diag_sum %lld\n", sum(kap, nc), sum(nrm, 3 * nc), (long long)dsum);
  int32_t tri[4096];
  double d2[4096], w[4096], delta;
  const int32_t ntl = ora_ppic_support(&g, &m, &prm, cells[0], 4096, tri, d2, w, &delta);
  if (ntl < 0) return 6;
  printf("ppic_support ring %d weight_sum %.17g delta %.17g\n", ntl, sum(w, ntl < 4096 ? ntl : 4096), delta);
  double* force = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  if (ora_csf(&g, alpha, nc, cells, kap, 1.0, force) != 0) return 7;
  printf("csf sum %.17g\n", sum(force, 3 * nc));
  const int64_t bcap = 6 * nc;
  int64_t* bid = (int64_t*)malloc(sizeof(int64_t) * (size_t)bcap);
  double* kb = (double*)malloc(sizeof(double) * (size_t)bcap);
  double* fb = (double*)malloc(sizeof(double) * 3 * (size_t)bcap);
  const int64_t nb = ora_csf_band(&g, alpha, nc, cells, kap, nrm, 1.0, bcap, bid, kb, fb);
  if (nb < 0) return 8;
  printf("csf_band cells %lld kappa_sum %.17g\n", (long long)nb, sum(kb, nb));

  /* interpolation and one RK4 step of every vertex */
  double* u = (double*)malloc(sizeof(double) * 3 * (size_t)nv);
  if (ora_interp(&g, nv, x, y, z, U, V, W, u) != 0) return 9;
  printf("interp sum %.17g\n", sum(u, 3 * (int64_t)nv));
  if (ora_advect_rk4(&g, nv, x, y, z, U, V, W, 1e-3, u) != 0) return 10;
  printf("advect_rk4 sum %.17g\n", sum(u, 3 * (int64_t)nv));

  free(pc);
  free(pt);
  free(cells);
  free(alpha);
  free(isif);
  free(kap);
  free(nrm);
  free(co);
  free(st);
  free(dg);
  free(force);
  free(bid);
  free(kb);
  free(fb);
  free(u);
  free(x);
  free(y);
  free(z);
  free(t0);
  free(t1);
  free(t2);
  free(U);
  free(V);
  free(W);
  free(dims);
  free(org);
  free(sz);
  return 0;
}
