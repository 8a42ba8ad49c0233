// Matrix element with the colour contraction on the matrix cores.
//
// Per event and helicity the colour-summed square is a quadratic form in the
// colour-ordered partial amplitudes, |M|^2_h = Re(A^dagger C A) = a^T C' a + b^T C' b
// (a, b the real and imaginary parts, C' = den * C an integer matrix, exact
// in FP32 and in BF16).  Batched over events this is a dense contraction
// D = C' V with one column of V per (event, helicity, re/im), followed by the
// column dot products v . D -- the only place in the path where matrix cores
// apply.
//
// Layout.  Each lane of a wave64 owns the amplitude vectors of its event
// (32 colour slots, ordering index s < NC, zero padding above).  A 32x32
// MFMA takes a column from two lanes: slots 0..15 from lane n and slots
// 16..31 from lane n+32.  One v_permlane32_swap per slot pair (j, 16+j)
// exchanges the upper half of the low lanes' vectors with the lower half of
// the high lanes' vectors, after which every lane holds the B operand for two
// 32-column MFMA sets: set A = vectors of lanes 0..31, set B = lanes 32..63.
// The colour slots are laid out so that the rows of D a lane receives belong
// to the same 16 slots as the K entries it supplied, so v . D is a 16-term
// local dot product plus one more swap to add the two halves.  No LDS, no
// shuffles through memory.
//
// Modes: FP32 MFMA (32x32x2, K = 32 in 16 instructions per set) and BF16
// MFMA (32x32x16, amplitudes split into hi + mid + lo BF16 terms, colour
// matrix exact in BF16), both accumulating in FP32.
#include "internal.h"
#include "me_common.h"

#include "generated/me_gg_tt.inc"
#include "generated/me_gg_ttg.inc"
#include "generated/me_gg_ttgg.inc"
#include "me_mfma_colour.h"

namespace mf {
namespace {

constexpr double kPi = 3.141592653589793238463;

template <int NEXT>
__device__ __forceinline__ void load_event(const double* __restrict__ p, int64_t n, int64_t e, double (&pe)[NEXT][4])
{
#pragma unroll
    for (int l = 0; l < NEXT; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) pe[l][c] = p[(l * 4 + c) * n + e];
}

// All 64 lanes of a wave take part in every MFMA, so lanes past the end of
// the batch recompute the last event and do not store.
template <int PROC, int MODE>
__global__ __launch_bounds__(256) void k_me_mfma(const double* __restrict__ p, int64_t n, float* __restrict__ out,
                                                 double mt, double coupling)
{
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = e0 < n ? e0 : n - 1;
    if constexpr (PROC == GG_TT) {
        double pe[4][4];
        load_event<4>(p, n, e, pe);
        MfmaColour<2, MODE> sink;
        sink.init(me_gg_tt_cnum);
        me_gg_tt_amps<float>(pe, mt, sink);
        if (e0 < n) out[e0] = (float)((double)sink.acc * coupling * me_gg_tt_norm_noalpha());
    } else if constexpr (PROC == GG_TTG) {
        double pe[5][4];
        load_event<5>(p, n, e, pe);
        MfmaColour<6, MODE> sink;
        sink.init(me_gg_ttg_cnum);
        me_gg_ttg_amps<float>(pe, mt, sink);
        if (e0 < n) out[e0] = (float)((double)sink.acc * coupling * me_gg_ttg_norm_noalpha());
    }
}

// gg -> ttbar gg: one wave per block, its multi-gluon currents parked in the
// wave's LDS columns (the launch bound of one wave lets the compiler plan the
// register file for exactly one wave per SIMD)
template <int MODE>
__global__ __launch_bounds__(64) void k_me_mfma_ttgg(const double* __restrict__ p, int64_t n,
                                                     float* __restrict__ out, double mt, double coupling)
{
    __shared__ float smem[me_gg_ttgg_amps_slots * 64];
    const int64_t e0 = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t e = e0 < n ? e0 : n - 1;
    double pe[6][4];
    load_event<6>(p, n, e, pe);
    MfmaColour<24, MODE> sink;
    sink.init(me_gg_ttgg_cnum);
    me_gg_ttgg_amps<float>(pe, mt, sink, smem + threadIdx.x);
    if (e0 < n) out[e0] = (float)((double)sink.acc * coupling * me_gg_ttgg_norm_noalpha());
}

template <int MODE>
hipError_t launch_mode(const MeJob& j, double mt, double coupling, int block, hipStream_t s)
{
    const unsigned grid = (unsigned)((j.n + block - 1) / block);
    float* out = static_cast<float*>(j.out);
    switch (j.proc) {
    case GG_TT: hipLaunchKernelGGL((k_me_mfma<GG_TT, MODE>), dim3(grid), dim3(block), 0, s, j.p, j.n, out, mt, coupling); break;
    case GG_TTG: hipLaunchKernelGGL((k_me_mfma<GG_TTG, MODE>), dim3(grid), dim3(block), 0, s, j.p, j.n, out, mt, coupling); break;
    case GG_TTGG: {
        const unsigned g64 = (unsigned)((j.n + 63) / 64);
        hipLaunchKernelGGL((k_me_mfma_ttgg<MODE>), dim3(g64), dim3(64), 0, s, j.p, j.n, out, mt, coupling);
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_matrix_element_mfma(const MeJob& j, int precision, double mt, double coupling, int block,
                                      hipStream_t s)
{
    if (block <= 0 || block % 64) block = 256;
    if (precision == 3) return launch_mode<0>(j, mt, coupling, block, s);
    if (precision == 2) return launch_mode<1>(j, mt, coupling, block, s);
    return hipErrorInvalidValue;
}

}  // namespace mf
