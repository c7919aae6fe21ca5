// Dense variant of the SP2 step (placeholder until the MFMA kernels land).
#include <string>

#include "../../include/ellsp2.h"

extern "C" int dense_x2(const void *d_A, void *d_C, int32_t N, int32_t mode, void *hip_stream)
{
  (void)d_A; (void)d_C; (void)N; (void)mode; (void)hip_stream;
  return ELL_EINVAL;
}

extern "C" int dense_sp2_solve(const double *d_H, int32_t N, double *d_D, int32_t mode, const sp2_params_t *p,
                               sp2_report_t *r, void *hip_stream)
{
  (void)d_H; (void)N; (void)d_D; (void)mode; (void)p; (void)r; (void)hip_stream;
  return ELL_EINVAL;
}
