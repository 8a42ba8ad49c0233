// Per-event derivative of |M|^2 with respect to the uniforms x (through the
// Vegas map and the phase space) and to m_t at fixed x.  The paper's custom
// operator has none (sect. 2).
//
// Reverse sweep over the amplitude recursion, forward tangents over the
// kinematics:
//  1. FP64 kinematics: Vegas map, phase space, then the inputs z of the
//     recursion (propagator denominators, momenta, polarisation bases,
//     spinors; emitted by the process compiler as <proc>_kin) rounded to the
//     working type R.
//  2. <proc>_adjoint: for every helicity configuration the currents, quark
//     line and colour sum are evaluated forward and swept backwards at once,
//     recomputing the gluon currents for their own sweep, so no current is
//     stored; it returns |M|^2 and zbar = d|M|^2/dz.  Its cost is about three
//     forward evaluations whatever the number of inputs.
//  3. The kinematics again, with DualN tangents along CH of the d + 1 inputs
//     (x_1..x_d, m_t) per pass: every z component, as it is formed, is
//     contracted with zbar, so d|M|^2/dinput = sum_z zbar_z dz/dinput.  The
//     kinematic map has d + 1 <= 9 inputs and ~80 outputs, so forward tangents
//     are its cheap direction; the root solves carry implicit-function
//     derivatives (one Newton step in tangent arithmetic from the converged
//     root).
// The alpha_s derivative needs none of this: |M|^2 is proportional to
// alpha_s^k for k gluons.
#pragma once
#include "dualn.h"
#include "me_common.h"
#include "ps_core.h"

namespace mf {

// The generated functions of the gg -> t tbar + (K-2) g process with K gluons: the
// process compiler emits the specialisation AdjProc<K> beside them, with
//   NZ       number of kinematic inputs z,
//   kin      z from the momenta and m_t (KT = double or DualN), handed to out.put,
//   adjoint  |M|^2 (no couplings, no normalisation) and zbar = d|M|^2/dz.
template <int K> struct AdjProc;

// z <- kinematic inputs rounded to the working type
template <typename R, int NZ>
struct KinStore {
    R (&z)[NZ];
    __device__ __forceinline__ void put(int s, double v) { z[s] = R(v); }
};

// g[k] += zbar . dz/d(direction k) for each kinematic input as it is formed
// (zbar of slot s at zb[s * ZS])
template <typename R, int ZS, int CH>
struct KinContract {
    const R* zb;
    double g[CH];
    __device__ __forceinline__ void put(int s, const DualN<double, CH>& v)
    {
        const double w = double(zb[s * ZS]);
#pragma unroll
        for (int k = 0; k < CH; ++k) g[k] = fma(w, v.t[k], g[k]);
    }
};

// Event momenta (beams along +-z with E = rs/2, then the outgoing momenta).
template <int NOUT, typename KT>
__device__ __forceinline__ void event_momenta(const KT (&P)[NOUT][4], double rs, KT (&pe)[NOUT + 2][4])
{
    const double E = 0.5 * rs;
    pe[0][0] = KT(E); pe[0][1] = KT(0.0); pe[0][2] = KT(0.0); pe[0][3] = KT(E);
    pe[1][0] = KT(E); pe[1][1] = KT(0.0); pe[1][2] = KT(0.0); pe[1][3] = KT(-E);
#pragma unroll
    for (int i = 0; i < NOUT; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) pe[i + 2][c] = P[i][c];
}

// |M|^2 without couplings and normalisation (me) and its derivatives grad[0..D-1]
// along x and grad[D] along m_t, for the uniforms x of one event.  edges: Vegas
// grid [D][nb + 1] or null (identity map).  CH: tangent directions per
// kinematic pass (ceil((D + 1)/CH) passes).  zb: the adjoint's accumulators,
// max(NZ, NZB) slots at stride ZS (the first NZ hold zbar on return), owned by
// the caller: registers of the lane (ZS = 1) or its column of an LDS array.
template <int K, typename R, int CH, int ZS>
__device__ __forceinline__ void vjp_event(const double (&x)[3 * K - 4], const double* edges, int nb, double rs,
                                          double mt, double& me, double (&grad)[3 * K - 3], R* zb)
{
    constexpr int NOUT = K, NEXT = K + 2, D = 3 * K - 4;
    typedef AdjProc<K> A;
    constexpr int NZ = A::NZ;
    {
        double y[D];
        double jac = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (edges) vegas_map1(x[k], edges + k * (nb + 1), nb, y[k], jac);
            else y[k] = x[k];
        }
        double m[NOUT];
#pragma unroll
        for (int i = 0; i < NOUT; ++i) m[i] = i < 2 ? mt : 0.0;
        double P[NOUT][4];
        rambo_event<NOUT, double>(y, rs, m, P, nullptr);
        double pe[NEXT][4];
        event_momenta<NOUT, double>(P, rs, pe);
        R z[NZ];
        KinStore<R, NZ> st{z};
        A::kin(pe, mt, st);
        R acc = R(0);
        A::template adjoint<R, ZS>(z, zb, acc);
        me = double(acc);
    }
    typedef DualN<double, CH> DN;
    // one pass at a time: unrolled, the passes' tangent values were live together and spilled
#pragma unroll 1
    for (int c0 = 0; c0 <= D; c0 += CH) {
        DN y[D];
        double jac = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const DN xk = DN::seed(x[k], k - c0);
            if (edges) vegas_map1(xk, edges + k * (nb + 1), nb, y[k], jac);
            else y[k] = xk;
        }
        const DN mtd = DN::seed(mt, D - c0);
        DN m[NOUT];
#pragma unroll
        for (int i = 0; i < NOUT; ++i) m[i] = i < 2 ? mtd : DN(0.0);
        DN P[NOUT][4];
        rambo_event<NOUT, DN>(y, rs, m, P, nullptr);
        DN pe[NEXT][4];
        event_momenta<NOUT, DN>(P, rs, pe);
        KinContract<R, ZS, CH> kc{zb, {}};
        A::kin(pe, mtd, kc);
#pragma unroll
        for (int i = 0; i <= D; ++i)           // constant indices: grad stays in registers
#pragma unroll
            for (int k = 0; k < CH; ++k)
                if (c0 + k == i) grad[i] = kc.g[k];
    }
}

}  // namespace mf
