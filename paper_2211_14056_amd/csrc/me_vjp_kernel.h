// Derivative kernel: vector-Jacobian product of |M|^2 with respect to the
// uniforms x (through the Vegas map and the phase space) and (m_t, alpha_s).
//
// The paper's custom operator has no derivative (sect. 2).  Here the
// derivative is computed in the kernel by forward (tangent) mode along each
// of the d + 1 inputs x_1..x_d, m_t: the phase space and the whole generated
// helicity/colour recursion are re-run with Dual scalars, one direction per
// pass, so every intermediate current is recomputed in registers for every
// helicity and nothing is stored in memory.  With d + 1 <= 9 directions this
// costs about 3(d+1) forward evaluations but keeps the register footprint at
// twice the forward one; a reverse sweep would need the whole per-helicity
// tape (~10^4 values for gg -> ttbar gg) live at once.  The alpha_s
// derivative is exact: |M|^2 is proportional to alpha_s^k for k gluons.
#pragma once
#include "internal.h"
#include "me_common.h"
#include "ps_core.h"

#include "generated/me_gg_tt.inc"
#include "generated/me_gg_ttg.inc"
#include "generated/me_gg_ttgg.inc"

namespace mf {

template <int PROC, typename R>   // R = double or float: working type of the recursion
__global__ __launch_bounds__(256) void k_me_vjp(VjpJob j)
{
    constexpr int NEXT = PROC == GG_TT ? 4 : (PROC == GG_TTG ? 5 : 6);
    constexpr int NOUT = NEXT - 2;
    constexpr int D = 3 * NOUT - 4;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= j.n) return;
    const int64_t n = j.n;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = j.x[k * n + e];
    const double gbar = j.grad_me[e];
    const double rs = j.sqrt_s;
    double me_val = 0.0;
    typedef Dual<double> KT;
    typedef Dual<R> DR;
#pragma unroll 1
    for (int dir = 0; dir <= D; ++dir) {
        KT y[D];
        double jac = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const KT xk(x[k], k == dir ? 1.0 : 0.0);
            if (j.edges) vegas_map1(xk, j.edges + k * (j.nb + 1), j.nb, y[k], jac);
            else y[k] = xk;
        }
        const KT mt(j.mt, dir == D ? 1.0 : 0.0);
        KT m[NOUT];
#pragma unroll
        for (int i = 0; i < NOUT; ++i) m[i] = i < 2 ? mt : KT(0.0);
        KT P[NOUT][4];
        rambo_event<NOUT, KT>(y, rs, m, P, nullptr);
        KT pe[NEXT][4];
        const double E = 0.5 * rs;
        pe[0][0] = KT(E); pe[0][1] = KT(0.0); pe[0][2] = KT(0.0); pe[0][3] = KT(E);
        pe[1][0] = KT(E); pe[1][1] = KT(0.0); pe[1][2] = KT(0.0); pe[1][3] = KT(-E);
#pragma unroll
        for (int i = 0; i < NOUT; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) pe[i + 2][c] = P[i][c];
        HelicitySum<DR> hs;
        double norm;
        if constexpr (PROC == GG_TT) {
            me_gg_tt_body<DR, KT>(pe, mt, hs);
            norm = me_gg_tt_norm_noalpha();
        } else if constexpr (PROC == GG_TTG) {
            me_gg_ttg_body<DR, KT>(pe, mt, hs);
            norm = me_gg_ttg_norm_noalpha();
        } else {
            me_gg_ttgg_body<DR, KT>(pe, mt, hs);
            norm = me_gg_ttgg_norm_noalpha();
        }
        const double scale = j.coupling * norm;
        me_val = (double)hs.acc.v * scale;
        const double deriv = (double)hs.acc.t * scale;
        if (dir < D) j.grad_x[dir * n + e] = gbar * deriv;
        else j.grad_theta[2 * e] = gbar * deriv;
    }
    j.grad_theta[2 * e + 1] = gbar * (NEXT - 2) * me_val / j.alpha_s;
    if (j.me_out) {
        if (j.me_f32) static_cast<float*>(j.me_out)[e] = (float)me_val;
        else static_cast<double*>(j.me_out)[e] = me_val;
    }
}

template <int PROC, typename R>
hipError_t launch_vjp_one(const VjpJob& j, hipStream_t s)
{
    const int block = 256;
    const unsigned grid = (unsigned)((j.n + block - 1) / block);
    hipLaunchKernelGGL((k_me_vjp<PROC, R>), dim3(grid), dim3(block), 0, s, j);
    return hipGetLastError();
}

}  // namespace mf
