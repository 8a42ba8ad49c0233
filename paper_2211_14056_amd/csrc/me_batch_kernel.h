// Persistent mixed-batch matrix-element kernels: one launch per process class
// serves all requests of that process in a call (up to 64 per launch).
//
// The paper launches one set of kernels per process and batch (sect. 2) and
// notes that how the work is spread over the device matters (sect. 3, Fig. 3).
// Here a fixed grid of one-wave workgroups (a multiple of the compute-unit
// count) pops tiles of 64 x batch_chunk(process) events from a device
// counter.  The host launches the
// process classes most expensive first.  Within a launch, each tile is one wave
// running the fused body of the process (VALU or matrix-core colour).  Lanes past
// the end of a request recompute its last event and do not store.  Every wave leaves the loop when the counter
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

// |M|^2 of event e of request q without couplings and normalisation.
// MODE: 0 = VALU colour (R = float or double), 1 = FP32 matrix cores, 2 = BF16 matrix cores (R = float)
template <typename R, int MODE, int PROC>
__device__ __forceinline__ double batch_event(const BatchReq& q, int64_t e, double mt, R* lds)
{
    if constexpr (PROC == GG_TT) {
        double pe[4][4];
        load_event_b<4>(q.p, q.n, e, pe);
        if constexpr (MODE == 0) {
            HelicitySum<R> hs;
            me_gg_tt_body<R>(pe, mt, hs);
            return (double)hs.acc;
        } else {
            MfmaColour<2, MODE - 1> sink;
            sink.init(me_gg_tt_cnum);
            me_gg_tt_amps<float>(pe, mt, sink);
            return (double)sink.acc;
        }
    } else if constexpr (PROC == GG_TTG) {
        double pe[5][4];
        load_event_b<5>(q.p, q.n, e, pe);
        if constexpr (MODE == 0) {
            HelicitySum<R> hs;
            me_gg_ttg_body<R>(pe, mt, hs);
            return (double)hs.acc;
        } else {
            MfmaColour<6, MODE - 1> sink;
            sink.init(me_gg_ttg_cnum);
            me_gg_ttg_amps<float>(pe, mt, sink);
            return (double)sink.acc;
        }
    } else {
        double pe[6][4];
        load_event_b<6>(q.p, q.n, e, pe);
        if constexpr (MODE == 0) {
            HelicitySum<R> hs;
            if constexpr (sizeof(R) == 4)
                me_gg_ttgg_body_lds32<R>(pe, mt, hs, lds);
            else
                me_gg_ttgg_body_lds64<R>(pe, mt, hs, lds);
            return (double)hs.acc;
        } else {
            MfmaColour<24, MODE - 1> sink;
            sink.init(me_gg_ttgg_cnum);
            me_gg_ttgg_amps<float>(pe, mt, sink, reinterpret_cast<float*>(lds));
            return (double)sink.acc;
        }
    }
}

template <int PROC>
constexpr double batch_norm()
{
    return PROC == GG_TT ? me_gg_tt_norm_noalpha() : PROC == GG_TTG ? me_gg_ttg_norm_noalpha() : me_gg_ttgg_norm_noalpha();
}

// One persistent launch per process present in the batch: the kernel is
// specialised for the process, so its registers and LDS (and with them the
// number of waves per compute unit) are those of that process alone.
template <typename R, int MODE, int PROC>
__global__ __launch_bounds__(64) void k_me_batch(BatchArgs a)
{
    constexpr int SLOTS = PROC != GG_TTGG ? 1
                          : (MODE != 0) ? me_gg_ttgg_amps_slots
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
        const int chunk = PROC == GG_TTGG ? 1 : a.chunk[PROC];
        const int64_t base = (tile - q.tile_begin) * (64 * chunk);
        for (int c = 0; c < chunk && base + 64 * c < q.n; ++c) {
            const int64_t e0 = base + 64 * c + lane;
            const int64_t e = e0 < q.n ? e0 : q.n - 1;
            const double me =
                batch_event<R, MODE, PROC>(q, e, a.mt, smem + lane) * a.coupling[PROC] * batch_norm<PROC>();
            if (e0 < q.n) static_cast<R*>(q.out)[e0] = (R)me;
        }
    }
}

// The same work as one plain grid: block b serves tile b, found in the request
// table.  Used for gg -> ttbar gg with matrix-core colour: there it compiles to
// the same code as the single-request kernel.  The persistent loop does not: it
// shifts the register allocation of the large body, which costs 11%.
template <typename R, int MODE, int PROC>
__global__ __launch_bounds__(64) void k_me_batch_grid(BatchArgs a)
{
    constexpr int SLOTS = PROC != GG_TTGG ? 1
                          : (MODE != 0) ? me_gg_ttgg_amps_slots
                                        : (sizeof(R) == 4 ? me_gg_ttgg_lds32_slots : me_gg_ttgg_lds64_slots);
    __shared__ R smem[SLOTS * 64];
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    int r = 0;
    while (r + 1 < a.nreq && a.req[r + 1].tile_begin <= tile) ++r;
    const BatchReq q = a.req[r];
    const int chunk = PROC == GG_TTGG ? 1 : a.chunk[PROC];
    const int64_t base = (tile - q.tile_begin) * (64 * chunk);
    for (int c = 0; c < chunk && base + 64 * c < q.n; ++c) {
        const int64_t e0 = base + 64 * c + lane;
        const int64_t e = e0 < q.n ? e0 : q.n - 1;
        const double me = batch_event<R, MODE, PROC>(q, e, a.mt, smem + lane) * a.coupling[PROC] * batch_norm<PROC>();
        if (e0 < q.n) static_cast<R*>(q.out)[e0] = (R)me;
    }
}

static __global__ void k_batch_reset(unsigned* counter) { *counter = 0u; }

template <typename R, int MODE, int PROC>
hipError_t launch_batch_proc(const BatchArgs& a, int waves_per_cu, int n_cu, hipStream_t s)
{
    if (PROC == GG_TTGG && MODE != 0) {
        hipLaunchKernelGGL((k_me_batch_grid<R, MODE, PROC>), dim3((unsigned)a.ntiles), dim3(64), 0, s, a);
        return hipGetLastError();
    }
    if (waves_per_cu <= 0) {
        // as many one-wave blocks per compute unit as the kernel's registers and LDS allow
        static int fit = 0;
        if (fit == 0) {
            int blocks = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_me_batch<R, MODE, PROC>, 64, 0);
            if (e != hipSuccess) return e;
            fit = blocks > 0 ? blocks : 1;
        }
        waves_per_cu = fit;
    }
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, a.counter);
    hipLaunchKernelGGL((k_me_batch<R, MODE, PROC>), dim3(waves_per_cu * n_cu), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename R, int MODE>
hipError_t launch_batch_one(const BatchArgs& a, int waves_per_cu, int n_cu, hipStream_t s)
{
    switch (a.req[0].proc) {
    case GG_TT: return launch_batch_proc<R, MODE, GG_TT>(a, waves_per_cu, n_cu, s);
    case GG_TTG: return launch_batch_proc<R, MODE, GG_TTG>(a, waves_per_cu, n_cu, s);
    case GG_TTGG: return launch_batch_proc<R, MODE, GG_TTGG>(a, waves_per_cu, n_cu, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mf
