// Second-level preconditioners beyond the diagonal ones: incomplete
// LDL^T(0) with level-scheduled sweeps, and the learned C C^T factor.
#include "mcg_internal.h"

int mcg_ildl0_create(mcg_pc *, double, hipStream_t) { return MCG_EINVAL; }
int mcg_cct_create(mcg_pc *, const mcg_csr_t *, hipStream_t) { return MCG_EINVAL; }
void mcg_pc_release_extra(mcg_pc *) {}
template <typename T>
void mcg_ildl0_apply(const mcg_pc *, const T *, T *, DevState *, int, hipStream_t) {}
template <typename T>
void mcg_cct_apply(const mcg_pc *, const T *, T *, DevState *, int, hipStream_t) {}
template void mcg_ildl0_apply<double>(const mcg_pc *, const double *, double *, DevState *, int, hipStream_t);
template void mcg_ildl0_apply<float>(const mcg_pc *, const float *, float *, DevState *, int, hipStream_t);
template void mcg_cct_apply<double>(const mcg_pc *, const double *, double *, DevState *, int, hipStream_t);
template void mcg_cct_apply<float>(const mcg_pc *, const float *, float *, DevState *, int, hipStream_t);
