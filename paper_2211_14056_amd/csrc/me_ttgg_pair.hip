// g g -> t tbar g g with two lanes per event (lanes 2j, 2j+1 of a wave share
// event j): the default FP64 kernel.  With one lane per event the FP64 working
// set is about twice the register file and spills heavily; two lanes halve the
// colour orderings and amplitudes each lane holds.  Lane sub relabels the
// gluons by the involution sigma = (0 1)(2 3): slot j holds gluon j ^ sub, so
// the beams stay in slots 0 and 1 (their momenta keep their zero components)
// and the code is identical for the two lanes.  Each lane takes the 12
// orderings that start with slot 0 or 2; gluon currents are computed once per
// {c, sigma(c)} pair and exchanged, and the colour quadratic form is completed
// with the partner lane's amplitudes, both by DPP.  The generated body is
// emitted by gen/lane_split.py (emit_pair).
//
// Gluon labels: 0 and 1 are the beams (legs 0 and 1, incoming), 2 and 3 are
// legs 4 and 5 (outgoing, polarisation eps*).  Momenta enter the recursion in
// the incoming convention.
#include "internal.h"
#include "me_common.h"

#include "generated/me_gg_ttgg_pair.inc"

namespace mf {
namespace {

constexpr int kPairEvents = 32;     // events per one-wave workgroup

__global__ __launch_bounds__(64) void k_me_ttgg_pair(const double* __restrict__ p, int64_t n,
                                                     double* __restrict__ out, double mt, double coupling)
{
    __shared__ double smem[me_gg_ttgg_pair_slots * 64];
    const int sub = threadIdx.x & 1;
    const int64_t e = (int64_t)blockIdx.x * kPairEvents + (threadIdx.x >> 1);
    if (e >= n) return;             // the two lanes of a pair leave together
    double kin[4][4], pt[4], ptb[4];
    double eu[2][3], ew[2][2], zs[2];
    int hb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int g = j ^ sub;
        const int leg = g < 2 ? g : g + 2;
        double pl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pl[c] = p[(int64_t)(leg * 4 + c) * n + e];
        const double sgn = g < 2 ? 1.0 : -1.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) kin[j][c] = sgn * pl[c];
        if (j >= 2) pol_basis<double, double>(pl, eu[j - 2], ew[j - 2]);
        hb[j] = g;
    }
    // beam slots: z direction of the gluon they hold (gluon 0 along +z, gluon 1 along -z)
    zs[0] = sub ? -1.0 : 1.0;
    zs[1] = -zs[0];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        pt[c] = p[(int64_t)(2 * 4 + c) * n + e];
        ptb[c] = p[(int64_t)(3 * 4 + c) * n + e];
    }
    HelicitySum<double> hs;
    me_gg_ttgg_pair<double, double>(kin, pt, ptb, eu, ew, zs, hb, mt, hs, smem + threadIdx.x);
    double acc = hs.acc;
    acc += pair_swap(acc);
    if (sub == 0) out[e] = acc * coupling * me_gg_ttgg_pair_norm_noalpha();
}

}  // namespace

hipError_t launch_ttgg_pair(const MeJob& j, double mt, double coupling, hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    const int64_t blocks = (j.n + kPairEvents - 1) / kPairEvents;
    hipLaunchKernelGGL(k_me_ttgg_pair, dim3((unsigned)blocks), dim3(64), 0, s, j.p, j.n,
                       static_cast<double*>(j.out), mt, coupling);
    return hipGetLastError();
}

}  // namespace mf
