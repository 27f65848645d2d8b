// Host build of the library's candidate classification and clipping
// (paper_2505_06932_amd/csrc/ftc_device.hpp, compiled for the CPU) against
// the oracle's per-piece clip: whether a (triangle, cell) pair has a piece,
// and its two integrals, must agree bit for bit.  Both builds of the clip
// are checked: the one with kMaxPoly corner slots, and the six-slot one the
// clipping kernel runs first, with its candidates over capacity clipped
// again by the former as the kernel does.  Test infrastructure only.
//
// usage: clip_vs_oracle <triangles> <seed>     seeded degenerate-heavy triangles
//        clip_vs_oracle --mesh <file>          the triangles of a mesh: the file
//          holds "nx ny nz x0 y0 z0 h", then the triangle count, then one
//          triangle per line as nine coordinates
// Prints "candidates <n> kept <k> redone <r> differences <d>" and exits
// with d != 0.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>

#include "ftc_device.hpp"
#include "ftc_oracle.h"

using namespace ftc;

static bool same(double a, double b) { return std::memcmp(&a, &b, sizeof(double)) == 0; }

namespace {

struct Tally {
  long cand = 0, kept = 0, redone = 0, diff = 0;
};

Grid make_grid(int32_t nx, int32_t ny, int32_t nz, double x0, double y0, double z0, double h) {
  Grid g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.x0 = x0;
  g.y0 = y0;
  g.z0 = z0;
  g.h = h;
  g.dnx = FastDiv((uint32_t)nx);
  g.dny = FastDiv((uint32_t)ny);
  g.dncol = FastDiv((uint32_t)nx * (uint32_t)ny);
  return g;
}

// Every cell of the triangle's bounding box grown by one cell: the library's
// class and piece (both clip builds) against the oracle's piece.
void check_triangle(const Grid& g, const Tri& T, long it, int mode, Tally& n) {
  static PolyLDS<1> L;
  static PolyLDS<1, 6> L6;
  const ora_grid og{g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.h};
  const double org[3] = {g.x0, g.y0, g.z0};
  double tri[9];
  for (int r = 0; r < 3; ++r)
    for (int d = 0; d < 3; ++d) tri[3 * r + d] = T.v[r][d];
  int64_t lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    const double mn = std::fmin(std::fmin(T.v[0][d], T.v[1][d]), T.v[2][d]);
    const double mx = std::fmax(std::fmax(T.v[0][d], T.v[1][d]), T.v[2][d]);
    lo[d] = (int64_t)std::floor((mn - org[d]) / g.h) - 1;
    hi[d] = (int64_t)std::floor((mx - org[d]) / g.h) + 1;
  }
  for (int64_t k = lo[2]; k <= hi[2]; ++k)
    for (int64_t j = lo[1]; j <= hi[1]; ++j)
      for (int64_t i = lo[0]; i <= hi[0]; ++i) {
        ++n.cand;
        Piece pc{false, 0.0, 0.0, false}, p6{false, 0.0, 0.0, false};
        const int cls = classify_candidate(g, T, i, j, k);
        if (cls == 1) pc = p6 = whole_piece(T, grid_plane(g.z0, k, g.h));
        if (cls == 2) {
          const uint32_t skip = inside_mask(g, T, i, j, k);
          pc = clip_piece(g, T, i, j, k, L, 0, skip);
          p6 = clip_piece(g, T, i, j, k, L6, 0, skip);
          if (p6.over_cap) {
            ++n.redone;
            p6 = clip_piece(g, T, i, j, k, L, 0, skip);
          }
        }
        double out[2];
        const bool ok = ora_piece(&og, tri, (int32_t)i, (int32_t)j, (int32_t)k, 2, out) != 0;
        n.kept += ok ? 1 : 0;
        for (int b = 0; b < 2; ++b) {
          const Piece& r = b ? p6 : pc;
          if (ok != r.keep || (ok && (!same(out[0], r.flux) || !same(out[1], r.vol)))) {
            if (n.diff < 5)
              std::printf("difference (%s slots): triangle %ld mode %d cell %ld %ld %ld class %d oracle %d %.17g "
                          "%.17g library %d %.17g %.17g\n",
                          b ? "six" : "nine", it, mode, (long)i, (long)j, (long)k, cls, (int)ok, out[0], out[1],
                          (int)r.keep, r.flux, r.vol);
            ++n.diff;
          }
        }
      }
}

int run_mesh(const char* path, Tally& n) {
  FILE* f = std::fopen(path, "r");
  if (!f) {
    std::printf("cannot open %s\n", path);
    return 2;
  }
  int nx, ny, nz;
  long nt;
  double x0, y0, z0, h;
  if (std::fscanf(f, "%d %d %d %lf %lf %lf %lf %ld", &nx, &ny, &nz, &x0, &y0, &z0, &h, &nt) != 8) {
    std::fclose(f);
    std::printf("bad header in %s\n", path);
    return 2;
  }
  const Grid g = make_grid(nx, ny, nz, x0, y0, z0, h);
  for (long t = 0; t < nt; ++t) {
    Tri T;
    for (int r = 0; r < 3; ++r)
      for (int d = 0; d < 3; ++d)
        if (std::fscanf(f, "%lf", &T.v[r][d]) != 1) {
          std::fclose(f);
          std::printf("short triangle list in %s\n", path);
          return 2;
        }
    check_triangle(g, T, t, -1, n);
  }
  std::fclose(f);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  Tally n;
  if (argc > 2 && std::strcmp(argv[1], "--mesh") == 0) {
    const int rc = run_mesh(argv[2], n);
    if (rc) return rc;
    std::printf("candidates %ld kept %ld redone %ld differences %ld\n", n.cand, n.kept, n.redone, n.diff);
    return n.diff != 0;
  }
  const long nt = argc > 1 ? std::atol(argv[1]) : 100000;
  const unsigned seed = argc > 2 ? (unsigned)std::atoi(argv[2]) : 1u;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const double hs[] = {1.0 / 32, 1.0 / 128, 0.1, 1.0 / 7, 0.25, 1.0 / 512, 3.0};
  for (long it = 0; it < nt; ++it) {
    const double h = hs[rng() % 7];
    const double x0 = (rng() % 3 == 0) ? 0.0 : (U(rng) - 0.5) * 4;
    const double y0 = (rng() % 3 == 0) ? 0.0 : (U(rng) - 0.5) * 4;
    const double z0 = (rng() % 3 == 0) ? 0.0 : (U(rng) - 0.5) * 4;
    const Grid g = make_grid(64, 64, 64, x0, y0, z0, h);
    const double org[3] = {g.x0, g.y0, g.z0};
    const int64_t b[3] = {(int64_t)(rng() % 20) + 5, (int64_t)(rng() % 20) + 5, (int64_t)(rng() % 20) + 5};
    // kinds of triangles: general, corners on grid planes, corners on quarter
    // points, collinear or repeated corners, tiny, large, lying in a grid plane
    const int mode = (int)(rng() % 8);
    const double span = mode == 5 ? 0.05 : (mode == 6 ? 3.0 : 1.5);
    Tri T;
    for (int r = 0; r < 3; ++r)
      for (int d = 0; d < 3; ++d) {
        double x = org[d] + ((double)b[d] + U(rng) * span - (span - 1.0) / 2) * g.h;
        if (mode == 1 || (mode == 2 && rng() % 2)) x = org[d] + (double)(b[d] + (int64_t)(rng() % 3) - 1) * g.h;
        if (mode == 3 && rng() % 2) x = org[d] + ((double)b[d] + 0.25 * (double)(rng() % 5)) * g.h;
        T.v[r][d] = x;
      }
    if (mode == 4) {
      const double t = (rng() % 2) ? 0.5 : U(rng);
      for (int d = 0; d < 3; ++d) T.v[2][d] = T.v[0][d] + t * (T.v[1][d] - T.v[0][d]);
    }
    if (mode == 7) {
      const int d = (int)(rng() % 3);
      const double x = org[d] + (double)(b[d] + (int64_t)(rng() % 2)) * g.h;
      for (int r = 0; r < 3; ++r) T.v[r][d] = x;
    }
    check_triangle(g, T, it, mode, n);
  }
  std::printf("candidates %ld kept %ld redone %ld differences %ld\n", n.cand, n.kept, n.redone, n.diff);
  return n.diff != 0;
}
