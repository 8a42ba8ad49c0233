// Dispatch of the derivative kernel over process and working precision.
#include "internal.h"

namespace mf {

template <int PROC, typename R> hipError_t launch_vjp_one(const VjpJob& j, hipStream_t s);

hipError_t launch_vjp(const VjpJob& j, int precision, hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    const bool f64 = precision == 0;
    switch (j.proc) {
    case GG_TT: return f64 ? launch_vjp_one<GG_TT, double>(j, s) : launch_vjp_one<GG_TT, float>(j, s);
    case GG_TTG: return f64 ? launch_vjp_one<GG_TTG, double>(j, s) : launch_vjp_one<GG_TTG, float>(j, s);
    case GG_TTGG: return f64 ? launch_vjp_one<GG_TTGG, double>(j, s) : launch_vjp_one<GG_TTGG, float>(j, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mf
