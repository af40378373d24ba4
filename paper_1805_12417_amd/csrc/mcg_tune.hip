// SpMV lanes-per-row autotuner.
#include "mcg_internal.h"

int mcg_autotune_lanes(mcg_solver *, hipStream_t) { return MCG_OK; }
