// ms_step_v6.hip -- step kernels for models with at most 6 via-points per
// muscle (one translation unit per via-point bound, compiled in parallel).
#include "ms_step_kernel.h"

namespace ms {
template hipError_t launch_nvia<6>(const Tables &, const KModel &, const KRun &, int, int, hipStream_t);
template hipError_t launch_muscle<6>(const KModel &, const KRun &, const KSplit &, int, int, hipStream_t);
}  // namespace ms
