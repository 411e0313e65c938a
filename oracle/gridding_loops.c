/* Sums over the kernel nodes of the FP64 gridding NUFFT, as plain loops.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle; nothing in the product
 * path links or calls it.  It computes exactly what oracle/gridding.py's
 * Grid.interp and Grid.spread compute (step 4 of type 2 and step 1 of
 * type 1 of the gridding NUFFT), for several grids at once and fast enough
 * for full-size comparisons: the node indices and weights come from the
 * caller (Grid.nodes), so this file holds only the triple sum.
 *
 * Layouts: a grid is [nfz][nfy][nfx] complex, interleaved (re, im) doubles;
 * P grids follow each other.  l0 is [m][3] int64 first nodes in (x, y, z)
 * order (wrapped mod nf here); w is [m][3][W] weights, rows x, y, z.
 */
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t wrap(int64_t v, int64_t n) {
  int64_t r = v % n;
  return r < 0 ? r + n : r;
}

/* out[p][j] = sum_{az, ay, ax} G_p[l0z+az][l0y+ay][l0x+ax] wz[az] wy[ay] wx[ax]
 * (complex, interleaved); one thread per point, no shared writes. */
void oracle_interp(const double *G, int64_t P, int64_t nfz, int64_t nfy, int64_t nfx,
                   int64_t W, const int64_t *l0, const double *w, int64_t m, double *out) {
  const int64_t cells = nfz * nfy * nfx;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    const double *wx = w + (j * 3 + 0) * W;
    const double *wy = w + (j * 3 + 1) * W;
    const double *wz = w + (j * 3 + 2) * W;
    for (int64_t p = 0; p < P; ++p) {
      const double *g = G + 2 * p * cells;
      double re = 0.0, im = 0.0;
      for (int64_t az = 0; az < W; ++az) {
        const int64_t lz = wrap(l0[j * 3 + 2] + az, nfz);
        for (int64_t ay = 0; ay < W; ++ay) {
          const int64_t ly = wrap(l0[j * 3 + 1] + ay, nfy);
          for (int64_t ax = 0; ax < W; ++ax) {
            const int64_t lx = wrap(l0[j * 3 + 0] + ax, nfx);
            const double wt = wz[az] * wy[ay] * wx[ax];
            const int64_t c = (lz * nfy + ly) * nfx + lx;
            re += g[2 * c] * wt;
            im += g[2 * c + 1] * wt;
          }
        }
      }
      out[2 * (p * m + j)] = re;
      out[2 * (p * m + j) + 1] = im;
    }
  }
}

/* H_p[l0z+az][l0y+ay][l0x+ax] += v[p][j] wz[az] wy[ay] wx[ax] for every point
 * j, onto H as given.  The z planes are split between threads, and each
 * thread walks all points in order and adds only into its own planes, so a
 * cell receives its terms in point order whatever the thread count. */
void oracle_spread(const double *v, int64_t P, int64_t nfz, int64_t nfy, int64_t nfx,
                   int64_t W, const int64_t *l0, const double *w, int64_t m, double *H) {
  const int64_t cells = nfz * nfy * nfx;
#pragma omp parallel
  {
    int nt = 1, t = 0;
#ifdef _OPENMP
    nt = omp_get_num_threads();
    t = omp_get_thread_num();
#endif
    const int64_t z0 = nfz * t / nt, z1 = nfz * (t + 1) / nt;
    for (int64_t j = 0; j < m; ++j) {
      const double *wx = w + (j * 3 + 0) * W;
      const double *wy = w + (j * 3 + 1) * W;
      const double *wz = w + (j * 3 + 2) * W;
      for (int64_t az = 0; az < W; ++az) {
        const int64_t lz = wrap(l0[j * 3 + 2] + az, nfz);
        if (lz < z0 || lz >= z1) continue;
        for (int64_t ay = 0; ay < W; ++ay) {
          const int64_t ly = wrap(l0[j * 3 + 1] + ay, nfy);
          for (int64_t ax = 0; ax < W; ++ax) {
            const int64_t lx = wrap(l0[j * 3 + 0] + ax, nfx);
            const double wt = wz[az] * wy[ay] * wx[ax];
            const int64_t c = (lz * nfy + ly) * nfx + lx;
            for (int64_t p = 0; p < P; ++p) {
              H[2 * (p * cells + c)] += v[2 * (p * m + j)] * wt;
              H[2 * (p * cells + c) + 1] += v[2 * (p * m + j) + 1] * wt;
            }
          }
        }
      }
    }
  }
}
