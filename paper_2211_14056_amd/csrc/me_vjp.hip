// Dispatch of the derivative kernel over process and working precision.
#include "internal.h"

namespace mf {

template <int PROC, typename R> hipError_t launch_vjp_batch_one(const VjpBatchArgs& a, hipStream_t s);

hipError_t launch_vjp_batch(const VjpBatchArgs& a, int precision, hipStream_t s)
{
    if (a.ntiles == 0) return hipSuccess;
    const bool f64 = precision == 0;
    switch (a.job.proc) {
    case GG_TT: return f64 ? launch_vjp_batch_one<GG_TT, double>(a, s) : launch_vjp_batch_one<GG_TT, float>(a, s);
    case GG_TTG: return f64 ? launch_vjp_batch_one<GG_TTG, double>(a, s) : launch_vjp_batch_one<GG_TTG, float>(a, s);
    case GG_TTGG:
        return f64 ? launch_vjp_batch_one<GG_TTGG, double>(a, s) : launch_vjp_batch_one<GG_TTGG, float>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mf
