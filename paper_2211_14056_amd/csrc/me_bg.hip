// g g -> t tbar g g g: the table-driven recursion (me_bg.h) with 16, 32 or 64 lanes per
// event, in FP64 and FP32.  Lanes per event trade the width of the levels of the
// recursion (a level holds 5 to 120 independent nodes) against LDS per workgroup and
// events in flight: the layout sweep of this kernel (the paper studies the block size of
// its kernels, sect. 3, Fig. 3).
#include "internal.h"
#include "me_common.h"

#include "generated/me_bg_k5.inc"
#include "me_bg.h"

namespace mf {
namespace {

template <typename R, int LPE>
hipError_t launch_lpe(const MeJob& j, double mt, double coupling, hipStream_t s)
{
    constexpr int EPB = 64 / LPE;
    const unsigned grid = (unsigned)((j.n + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_me_bg<5, R, LPE>), dim3(grid), dim3(64), 0, s, j.p, j.n, static_cast<R*>(j.out), mt,
                       coupling);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_r(const MeJob& j, double mt, double coupling, int lpe, hipStream_t s)
{
    switch (lpe) {
    case 16: return launch_lpe<R, 16>(j, mt, coupling, s);
    case 32: return launch_lpe<R, 32>(j, mt, coupling, s);
    case 0:
    case 64: return launch_lpe<R, 64>(j, mt, coupling, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_ttggg(const MeJob& j, int precision, double mt, double coupling, int lanes_per_event,
                        hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    if (precision == 0) return launch_r<double>(j, mt, coupling, lanes_per_event, s);
    if (precision == 1) return launch_r<float>(j, mt, coupling, lanes_per_event, s);
    return hipErrorInvalidValue;
}

}  // namespace mf
