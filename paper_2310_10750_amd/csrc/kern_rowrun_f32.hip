// Row-run and LDS-resident kernels, storage float / arithmetic float.
#include "kern_rowrun_dispatch.h"

NLCH_ROWRUN_UNIT(f32, float, float)
