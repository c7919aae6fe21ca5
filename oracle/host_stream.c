/*
 * Host memory bandwidth probe for the CPU baseline -- TEST INFRASTRUCTURE
 * ONLY (see oracle.h).  The triad kernel of McCalpin's STREAM benchmark,
 * a[i] = b[i] + s c[i], timed on the OpenMP threads.
 */
#include "oracle.h"

#include <stdlib.h>
#include <time.h>

static double now_s(void)
{
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

double orc_stream_triad(int64_t n, int32_t reps)
{
  const size_t bytes = (size_t)n * sizeof(double);
  const size_t padded = (bytes + 63) / 64 * 64;
  double *a = (double *)aligned_alloc(64, padded);
  double *b = (double *)aligned_alloc(64, padded);
  double *c = (double *)aligned_alloc(64, padded);
  if (!a || !b || !c) {
    free(a); free(b); free(c);
    return -1.0;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    a[i] = 0.0;
    b[i] = 1.0;
    c[i] = 2.0;
  }
  const double s = 3.0;
  double best = 0.0;
  for (int32_t r = 0; r < reps; ++r) {
    const double t0 = now_s();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) a[i] = b[i] + s * c[i];
    const double dt = now_s() - t0;
    const double gbs = 3.0 * (double)bytes / dt / 1e9;
    if (gbs > best) best = gbs;
  }
  volatile double sink = a[n / 2];  /* the result is used */
  (void)sink;
  free(a); free(b); free(c);
  return best;
}
