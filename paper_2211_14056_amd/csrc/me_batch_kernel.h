// Persistent mixed-batch matrix-element kernel: one launch serves up to 64
// requests of different processes and sizes.
//
// The paper launches one set of kernels per process and batch (sect. 2) and
// notes that how the work is spread over the device matters (sect. 3, Fig. 3).
// Here a fixed grid of one-wave workgroups (a multiple of the compute-unit
// count) pops 64-event tiles from a device counter.  Tiles are numbered with
// the most expensive process first (the host orders the requests by cost), so
// the long gg -> ttbar gg tiles start early and the cheap ones fill the tail.
// Each tile is one wave: the wave runs the fused body of that tile's process
// (VALU or matrix-core colour), lanes past the end of a request recompute its
// last event and do not store.  Every wave leaves the loop when the counter
// passes the tile count.  The request table travels in the kernel arguments,
// so a captured graph replays it as is.
#pragma once
#include "internal.h"
#include "me_common.h"

#include "generated/me_gg_tt.inc"
#include "generated/me_gg_ttg.inc"
#include "generated/me_gg_ttgg.inc"
#include "me_mfma_colour.h"

namespace mf {

template <int NEXT>
__device__ __forceinline__ void load_event_b(const double* __restrict__ p, int64_t n, int64_t e, double (&pe)[NEXT][4])
{
#pragma unroll
    for (int l = 0; l < NEXT; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) pe[l][c] = p[(l * 4 + c) * n + e];
}

// MODE: 0 = VALU colour (R = float or double), 1 = FP32 matrix cores, 2 = BF16 matrix cores (R = float)
template <typename R, int MODE>
__global__ __launch_bounds__(64) void k_me_batch(BatchArgs a)
{
    constexpr int SLOTS = (MODE != 0) ? me_gg_ttgg_amps_slots
                                      : (sizeof(R) == 4 ? me_gg_ttgg_lds32_slots : me_gg_ttgg_lds64_slots);
    __shared__ R smem[SLOTS * 64];
    const int lane = threadIdx.x;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(a.counter, 1u);
        const int64_t tile = (int64_t)__shfl(t, 0);
        if (tile >= a.ntiles) break;
        int r = 0;
        while (r + 1 < a.nreq && a.req[r + 1].tile_begin <= tile) ++r;
        const BatchReq q = a.req[r];
        const int64_t e0 = (tile - q.tile_begin) * 64 + lane;
        const int64_t e = e0 < q.n ? e0 : q.n - 1;
        double me = 0.0;
        if (q.proc == GG_TT) {
            double pe[4][4];
            load_event_b<4>(q.p, q.n, e, pe);
            if constexpr (MODE == 0) {
                HelicitySum<R> hs;
                me_gg_tt_body<R>(pe, a.mt, hs);
                me = (double)hs.acc;
            } else {
                MfmaColour<2, MODE - 1> sink;
                sink.init(me_gg_tt_cnum);
                me_gg_tt_amps<float>(pe, a.mt, sink);
                me = (double)sink.acc;
            }
            me *= a.coupling[GG_TT] * me_gg_tt_norm_noalpha();
        } else if (q.proc == GG_TTG) {
            double pe[5][4];
            load_event_b<5>(q.p, q.n, e, pe);
            if constexpr (MODE == 0) {
                HelicitySum<R> hs;
                me_gg_ttg_body<R>(pe, a.mt, hs);
                me = (double)hs.acc;
            } else {
                MfmaColour<6, MODE - 1> sink;
                sink.init(me_gg_ttg_cnum);
                me_gg_ttg_amps<float>(pe, a.mt, sink);
                me = (double)sink.acc;
            }
            me *= a.coupling[GG_TTG] * me_gg_ttg_norm_noalpha();
        } else {
            double pe[6][4];
            load_event_b<6>(q.p, q.n, e, pe);
            if constexpr (MODE == 0) {
                HelicitySum<R> hs;
                if constexpr (sizeof(R) == 4)
                    me_gg_ttgg_body_lds32<R>(pe, a.mt, hs, smem + lane);
                else
                    me_gg_ttgg_body_lds64<R>(pe, a.mt, hs, smem + lane);
                me = (double)hs.acc;
            } else {
                MfmaColour<24, MODE - 1> sink;
                sink.init(me_gg_ttgg_cnum);
                me_gg_ttgg_amps<float>(pe, a.mt, sink, reinterpret_cast<float*>(smem) + lane);
                me = (double)sink.acc;
            }
            me *= a.coupling[GG_TTGG] * me_gg_ttgg_norm_noalpha();
        }
        if (e0 < q.n) static_cast<R*>(q.out)[e0] = (R)me;
    }
}

static __global__ void k_batch_reset(unsigned* counter) { *counter = 0u; }

template <typename R, int MODE>
hipError_t launch_batch_one(const BatchArgs& a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, a.counter);
    hipLaunchKernelGGL((k_me_batch<R, MODE>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace mf
