// Derivative kernel: vector-Jacobian product of |M|^2 with respect to the
// uniforms x (through the Vegas map and the phase space) and (m_t, alpha_s).
//
// The paper's custom operator has no derivative (sect. 2).  One lane per
// event runs vjp_event (me_vjp_event.h): a reverse sweep over the generated
// helicity/colour recursion, recomputing the currents of every helicity
// instead of storing them, and forward tangents over the few kinematic inputs.
// The alpha_s derivative is exact: |M|^2 is proportional to alpha_s^k for k
// gluons.
#pragma once
#include "internal.h"
#include "me_common.h"
#include "ps_core.h"

#include "generated/me_gg_tt_adj.inc"
#include "generated/me_gg_ttg_adj.inc"
#include "generated/me_gg_ttgg_adj.inc"
#include "me_vjp_event.h"

namespace mf {

// tangent directions per kinematic pass, one pass at a time.  Measured on 4e6
// gg -> ttbar g events (whole derivative): FP32 recursion 8.27 ms with three
// directions per pass, 8.96 with two, 10.76 with one; FP64 recursion (whose adjoint
// still spills) 38.5 ms with one direction per pass, 40.4 with two, 42.2 with three.
// gg -> ttbar gg, FP32, 2^18 events: 28.7 ms with three, 29.0 with two, 35.9 with one.
template <typename R> constexpr int vjp_tangent_width() { return sizeof(R) == 8 ? 1 : 3; }

// derivative of event e of request q (shared settings in j)
template <int PROC, typename R>
__device__ __forceinline__ void vjp_one_event(const VjpJob& j, const VjpReq& q, int64_t e)
{
    constexpr int K = PROC == GG_TT ? 2 : (PROC == GG_TTG ? 3 : 4);
    constexpr int D = 3 * K - 4;
    const int64_t n = q.n;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = q.x[k * n + e];
    double me, g[D + 1];
    typedef AdjProc<K> A;
    constexpr int NS = A::NZB > A::NZ ? A::NZB : A::NZ;
    if constexpr (A::NZB > 0 && A::NZB * 64 * sizeof(R) <= 40960) {
        // accumulators in LDS, slot s of lane l at zbl[s * 64 + l] (one-wave blocks), where they
        // leave four waves per compute unit (40 KB of the 160 KB each).  gg -> ttbar gg in FP64
        // (42 KB) keeps them in registers: 72.8 ms instead of 82.8 on 2^18 events, despite more spill.
        __shared__ R zbl[A::NZB * 64];
        vjp_event<K, R, vjp_tangent_width<R>(), 64>(x, j.edges, j.nb, j.sqrt_s, j.mt, me, g, zbl + threadIdx.x);
    } else {
        R zbr[NS];
        vjp_event<K, R, vjp_tangent_width<R>(), 1>(x, j.edges, j.nb, j.sqrt_s, j.mt, me, g, zbr);
    }
    const double scale = j.coupling * AdjProc<K>::norm;
    const double gbar = q.grad_me[e];
    const double gs = gbar * scale;
#pragma unroll
    for (int k = 0; k < D; ++k) q.grad_x[k * n + e] = gs * g[k];
    const double me_val = me * scale;
    q.grad_theta[2 * e] = gs * g[D];
    q.grad_theta[2 * e + 1] = gbar * K * me_val / j.alpha_s;
    if (q.me_out) {
        if (j.me_f32) static_cast<float*>(q.me_out)[e] = (float)me_val;
        else static_cast<double*>(q.me_out)[e] = me_val;
    }
}

// requests of one process: block b serves 64-event tile b of the request table
template <int PROC, typename R>
__global__ __launch_bounds__(64) void k_me_vjp_batch(VjpBatchArgs a)
{
    const int64_t tile = blockIdx.x;
    int r = 0;
    while (r + 1 < a.nreq && a.req[r + 1].tile_begin <= tile) ++r;
    const VjpReq& q = a.req[r];
    const int64_t e = (tile - q.tile_begin) * 64 + threadIdx.x;
    if (e >= q.n) return;
    vjp_one_event<PROC, R>(a.job, q, e);
}

template <int PROC, typename R>
hipError_t launch_vjp_batch_one(const VjpBatchArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((k_me_vjp_batch<PROC, R>), dim3((unsigned)a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace mf
