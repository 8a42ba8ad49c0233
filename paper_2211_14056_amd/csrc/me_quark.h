// Matrix elements of the processes with two quark lines (q qbar -> t tbar (+g, +gg),
// q g -> t tbar q (+g)): one lane per event.
//
// The generated traits (generated/me_qq_*.inc, me_qg_*.inc; gen/quark_lines.py) hold the
// helicity configurations, the leg kinds, the leg subsets whose off-shell currents the
// diagrams use, and the straight-line body of one helicity configuration: every Feynman
// diagram from the external wavefunctions, summed into colour-flow amplitudes and contracted
// with the colour matrix (the paper's generated code, sect. 2, Fig. 2).  Per event the
// momentum sums and propagator denominators of those subsets are formed once in FP64 and
// rounded; the helicity loop then rebuilds the external wavefunctions of each configuration.
#pragma once
#include "me_common.h"

namespace mf {

// eps(k, l) = -l u - i w for an incoming gluon, eps*(k, l) = -l u + i w for an outgoing one
// (u, w the transverse basis divided by sqrt 2; time component 0)
template <typename R>
__device__ __forceinline__ void gluon_pol(const double* k, int l, bool incoming, cplx<R> e[4])
{
    R u[3], w[2];
    pol_basis<R, double>(k, u, w);
    const R lr = R(l), s = incoming ? R(-1) : R(1);
    e[0] = {R(0), R(0)};
    e[1] = {-lr * u[0], s * w[0]};
    e[2] = {-lr * u[1], s * w[1]};
    e[3] = {-lr * u[2], R(0)};
}

// |M|^2 of one event without the couplings: (4 pi alpha_s)^(n-2) multiplies it
template <class T, typename R>
__device__ __forceinline__ double quark_event(const double (&pe)[T::NEXT][4], double mt)
{
    R K[5 * T::NSUB];
#pragma unroll
    for (int s = 0; s < T::NSUB; ++s) {
        double P[4] = {0.0, 0.0, 0.0, 0.0};
        int cnt = 0;
#pragma unroll
        for (int l = 0; l < T::NEXT; ++l)
            if (T::SUB_MASK[s] >> l & 1) {
                ++cnt;
                const double sg = l < 2 ? 1.0 : -1.0;          // incoming momenta
#pragma unroll
                for (int c = 0; c < 4; ++c) P[c] += sg * pe[l][c];
            }
        const double m = T::SUB_TOP[s] ? mt : 0.0;
        const double den = P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3] - m * m;
#pragma unroll
        for (int c = 0; c < 4; ++c) K[5 * s + c] = R(P[c]);
        K[5 * s + 4] = cnt > 1 ? R(1.0 / den) : R(0);      // external legs carry no propagator
    }
    R acc = R(0);
#pragma unroll 1
    for (int h = 0; h < T::NHEL; ++h) {
        cplx<R> W[4 * T::NEXT];
#pragma unroll
        for (int l = 0; l < T::NEXT; ++l) {
            const int lam = T::hel(h, l);
            const double m = T::MASSIVE[l] ? mt : 0.0;
            switch (T::KIND[l]) {
            case 0: u_spinor<R, double>(pe[l], m, lam, W + 4 * l); break;
            case 1: vbar_spinor<R, double>(pe[l], m, lam, W + 4 * l); break;
            case 2: ubar_spinor<R, double>(pe[l], m, lam, W + 4 * l); break;
            case 3: v_spinor<R, double>(pe[l], m, lam, W + 4 * l); break;
            case 4: gluon_pol<R>(pe[l], lam, true, W + 4 * l); break;
            default: gluon_pol<R>(pe[l], lam, false, W + 4 * l); break;
            }
        }
        acc += T::template body<R>(W, K, R(mt));
    }
    return double(acc) * T::NORM;
}

}  // namespace mf
