// Row-run and LDS-resident kernels, storage double / arithmetic double.
#include "kern_rowrun_dispatch.h"

NLCH_ROWRUN_UNIT(f64, double, double)
