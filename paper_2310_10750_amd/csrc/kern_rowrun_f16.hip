// Row-run and LDS-resident kernels, storage half_t / arithmetic float.
#include "kern_rowrun_dispatch.h"

NLCH_ROWRUN_UNIT(f16, nlch::half_t, float)
