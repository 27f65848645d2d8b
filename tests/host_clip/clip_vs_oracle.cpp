// Host build of the library's candidate classification and clipping
// (paper_2505_06932_amd/csrc/ftc_device.hpp, compiled for the CPU) against
// the oracle's per-piece clip: whether a (triangle, cell) pair has a piece,
// and its two integrals, must agree bit for bit.  Both builds of the clip
// are checked: the one with kMaxPoly corner slots, and the six-slot one the
// clipping kernel runs first, with its candidates over capacity clipped
// again by the former as the kernel does.  Test infrastructure only.
//
// usage: clip_vs_oracle <triangles> <seed>
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

int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 100000;
  const unsigned seed = argc > 2 ? (unsigned)std::atoi(argv[2]) : 1u;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  PolyLDS<1> L;
  PolyLDS<1, 6> L6;
  long cand = 0, kept = 0, redone = 0, diff = 0;
  const double hs[] = {1.0 / 32, 1.0 / 128, 0.1, 1.0 / 7, 0.25, 1.0 / 512, 3.0};
  for (long it = 0; it < n; ++it) {
    Grid g{};
    g.h = hs[rng() % 7];
    g.nx = g.ny = g.nz = 64;
    g.dnx = FastDiv(64);
    g.dny = FastDiv(64);
    g.dncol = FastDiv(64 * 64);
    g.x0 = (rng() % 3 == 0) ? 0.0 : (U(rng) - 0.5) * 4;
    g.y0 = (rng() % 3 == 0) ? 0.0 : (U(rng) - 0.5) * 4;
    g.z0 = (rng() % 3 == 0) ? 0.0 : (U(rng) - 0.5) * 4;
    const ora_grid og{g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.h};
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
          ++cand;
          Piece pc{false, 0.0, 0.0, false}, p6{false, 0.0, 0.0, false};
          const int cls = classify_candidate(g, T, i, j, k);
          if (cls == 1) pc = p6 = whole_piece(T, grid_plane(g.z0, k, g.h));
          if (cls == 2) {
            const uint32_t skip = inside_mask(g, T, i, j, k);
            pc = clip_piece(g, T, i, j, k, L, 0, skip);
            p6 = clip_piece(g, T, i, j, k, L6, 0, skip);
            if (p6.over_cap) {
              ++redone;
              p6 = clip_piece(g, T, i, j, k, L, 0, skip);
            }
          }
          double out[2];
          const bool ok = ora_piece(&og, tri, (int32_t)i, (int32_t)j, (int32_t)k, 2, out) != 0;
          kept += ok ? 1 : 0;
          for (int b = 0; b < 2; ++b) {
            const Piece& r = b ? p6 : pc;
            if (ok != r.keep || (ok && (!same(out[0], r.flux) || !same(out[1], r.vol)))) {
              if (diff < 5)
                std::printf("difference (%s slots): triangle %ld mode %d cell %ld %ld %ld class %d oracle %d %.17g "
                            "%.17g library %d %.17g %.17g\n",
                            b ? "six" : "nine", it, mode, (long)i, (long)j, (long)k, cls, (int)ok, out[0], out[1],
                            (int)r.keep, r.flux, r.vol);
              ++diff;
            }
          }
        }
  }
  std::printf("candidates %ld kept %ld redone %ld differences %ld\n", cand, kept, redone, diff);
  return diff != 0;
}
