// g g -> t tbar g g with four lanes per event (lanes 4j..4j+3 of a wave share
// event j), an option for the FP64 kernel.  With one lane per event the FP64
// working set (24 partial amplitudes and 34 multi-gluon currents per helicity
// configuration) is about twice the register file and spills to memory.  The
// quad form divides the colour orderings by their first gluon.  Each lane
// relabels the gluons so that its own orderings are (0, x, y, z) in slot
// labels: slot j holds gluon (j + sub) mod 4, so the code is identical for the
// four lanes.  The colour quadratic form is completed with the amplitudes of
// the other lanes of the quad, read by DPP.  The generated body and the
// argument of the split are in gen/lane_split.py.
//
// Gluon labels: 0 and 1 are the beams (legs 0 and 1, incoming, polarisation
// eps), 2 and 3 are legs 4 and 5 (outgoing, polarisation eps*).  Momenta enter
// the recursion in the incoming convention.
#include "internal.h"
#include "me_common.h"

#include "generated/me_gg_ttgg_quad.inc"

namespace mf {
namespace {

constexpr int kQuadEvents = 16;     // events per one-wave workgroup

__global__ __launch_bounds__(64) void k_me_ttgg_quad(const double* __restrict__ p, int64_t n,
                                                     double* __restrict__ out, double mt, double coupling)
{
    __shared__ double smem[me_gg_ttgg_quad_slots * 64];
    const int sub = threadIdx.x & 3;
    const int64_t e = (int64_t)blockIdx.x * kQuadEvents + (threadIdx.x >> 2);
    if (e >= n) return;             // the four lanes of a quad leave together
    double kin[4][4], pt[4], ptb[4];
    double eu[4][3], ew[4][2];
    int hb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int g = (j + sub) & 3;
        const int leg = g < 2 ? g : g + 2;
        double pl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pl[c] = p[(int64_t)(leg * 4 + c) * n + e];
        const double sgn = g < 2 ? 1.0 : -1.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) kin[j][c] = sgn * pl[c];
        // eps* = -lam u + i w for an outgoing gluon; an incoming one has eps = -lam u - i w
        pol_basis<double, double>(pl, eu[j], ew[j]);
        ew[j][0] *= -sgn;
        ew[j][1] *= -sgn;
        hb[j] = g;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        pt[c] = p[(int64_t)(2 * 4 + c) * n + e];
        ptb[c] = p[(int64_t)(3 * 4 + c) * n + e];
    }
    HelicitySum<double> hs;
    me_gg_ttgg_split<double, double>(kin, pt, ptb, eu, ew, hb, mt, hs, smem + threadIdx.x);
    double acc = hs.acc;
    acc += quad_rot<1>(acc);
    acc += quad_rot<2>(acc);
    if (sub == 0) out[e] = acc * coupling * me_gg_ttgg_quad_norm_noalpha();
}

}  // namespace

hipError_t launch_ttgg_quad(const MeJob& j, double mt, double coupling, hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    const int64_t blocks = (j.n + kQuadEvents - 1) / kQuadEvents;
    hipLaunchKernelGGL(k_me_ttgg_quad, dim3((unsigned)blocks), dim3(64), 0, s, j.p, j.n,
                       static_cast<double*>(j.out), mt, coupling);
    return hipGetLastError();
}

}  // namespace mf
