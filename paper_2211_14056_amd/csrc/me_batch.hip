// Dispatch of the persistent mixed-batch kernel over precision.
#include "internal.h"

namespace mf {

template <typename R, int MODE> hipError_t launch_batch_one(const BatchArgs& a, int waves_per_cu, int n_cu, hipStream_t s);

hipError_t launch_batch(const BatchArgs& a, int precision, int waves_per_cu, int n_cu, hipStream_t s)
{
    if (a.ntiles == 0) return hipSuccess;
    switch (precision) {
    case 0: return launch_batch_one<double, 0>(a, waves_per_cu, n_cu, s);
    case 1: return launch_batch_one<float, 0>(a, waves_per_cu, n_cu, s);
    case 2: return launch_batch_one<float, 2>(a, waves_per_cu, n_cu, s);   // BF16 matrix cores
    case 3: return launch_batch_one<float, 1>(a, waves_per_cu, n_cu, s);   // FP32 matrix cores
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mf
