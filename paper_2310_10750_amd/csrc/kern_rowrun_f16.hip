// Row-run and LDS-resident kernels, storage half_t / arithmetic float.
// horizons of the multifidelity study's other models (FP32 arithmetic only)
#define NLCH_ROWRUN_EXTRA_R2(X) X(121) X(144) X(484) X(576)
#include "kern_rowrun_dispatch.h"

NLCH_ROWRUN_UNIT(f16, nlch::half_t, float)
