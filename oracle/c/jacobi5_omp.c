/*
 * CPU oracle, all host cores -- TEST INFRASTRUCTURE (used by the tests and by
 * the benchmark's CPU-baseline leg only; the library never links it).
 *
 * The Jacobi 5-point loop of the benchmark's stencil workload (the paper's
 * sec. 6.2 names a 2D stencil kernel; the update and residual are those of
 * the float32-order serial oracle, oracle/bodies.py `jacobi5`), written as
 * the OpenMP loop the paper's programming models would express: a
 * `parallel for` over rows with a static schedule and a `reduction(max:)`
 * of the update norm, one sweep after another. Per point, in float32:
 * u1 = ((N + S) + (W + E)) * 0.25 on the interior, boundary copied; the
 * sweep's residual is the max over the interior of |(double) u1 - (double) u0|.
 * Built with -ffp-contract=off so no multiply-add is fused: each result is
 * identical to the serial oracle's, in any thread count.
 *
 * jacobi5_omp(u, tmp, rows, cols, sweeps, res, threads): u (rows x cols,
 * row-major) holds the initial grid and receives the final one; tmp is a
 * scratch grid of the same size; res gets
 * `sweeps` residuals; threads <= 0 means every available core. Returns the
 * thread count used.
 */
#include <math.h>
#include <omp.h>
#include <string.h>

int jacobi5_omp(float *u, float *tmp, long rows, long cols, int sweeps, double *res, int threads) {
  if (threads <= 0) threads = omp_get_max_threads();
  const long n = cols;
  float *a = u, *b = tmp;
  memcpy(b, a, (size_t)rows * (size_t)cols * sizeof(float));
  for (int k = 0; k < sweeps; ++k) {
    double r = 0.0;
#pragma omp parallel for schedule(static) reduction(max : r) num_threads(threads)
    for (long i = 1; i < rows - 1; ++i) {
      const float *up = a + (i - 1) * n, *mid = a + i * n, *dn = a + (i + 1) * n;
      float *out = b + i * n;
      for (long j = 1; j < n - 1; ++j) {
        const float v = ((up[j] + dn[j]) + (mid[j - 1] + mid[j + 1])) * 0.25f;
        out[j] = v;
        const double d = fabs((double)v - (double)mid[j]);
        if (d > r) r = d;
      }
    }
    res[k] = r;
    float *t = a;
    a = b;
    b = t;
  }
  if (a != u) memcpy(u, a, (size_t)rows * (size_t)cols * sizeof(float));
  return threads;
}
