// Colour quadratic form on the matrix cores (see me_mfma.hip for the layout).
#pragma once
#include <hip/hip_runtime.h>

namespace mf {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// Slot held in accumulator row t (t = 4 i + jj) of a lane in half hb:
// MFMA output row r = 8 i + 4 hb + jj  <->  colour slot 16 hb + t.
__device__ __forceinline__ int slot_of_row(int r) { return 16 * ((r >> 2) & 1) + 4 * (r >> 3) + (r & 3); }

// BF16 mode with at most 8 orderings: one 32x32x8 MFMA per term, K = 8 with no
// padding beyond it.  Lane half hb supplies slots 4 hb + e (e < 4), and a lane's
// accumulator rows t < 4 hold those slots (the other rows are zero rows).
__device__ __forceinline__ int slot_of_row_k8(int r)
{
    const int t = 4 * (r >> 3) + (r & 3);
    return t < 4 ? 4 * ((r >> 2) & 1) + t : 32 + t;
}

__device__ __forceinline__ short bf16_bits(float v) { return __builtin_bit_cast(short, (__bf16)v); }

__device__ __forceinline__ void swap_halves(float& lo_keep, float& hi_keep)
{
    // lanes 32..63 of the first operand <-> lanes 0..31 of the second
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo_keep), __float_as_uint(hi_keep), false, false);
    lo_keep = __uint_as_float(r[0]);
    hi_keep = __uint_as_float(r[1]);
}

template <int NC, int MODE>   // MODE 0: FP32 MFMA, 1: BF16 x3 MFMA
struct MfmaColour {
    static_assert(NC <= 32, "colour orderings must fit 32 slots");
    float a[2][NC][2];        // [antitop helicity][ordering][re, im], filled by the generated body
    float acc = 0.0f;         // this lane's helicity sum
    // BF16 mode for at most 8 orderings: one 32x32x8 block (only one MFMA shape per
    // accumulator: an MFMA reading another shape's result needs wait states that
    // the compiler did not always insert)
    static constexpr bool K8 = MODE == 1 && NC <= 8;
    float cA[16];             // colour numerators in A-operand layout (FP32 mode)
    bf16x8 cB[2];             // same, BF16 mode: chunk c, element e
    shortx4 cB8;              // same, BF16 mode with at most 8 orderings (bf16 bit patterns)

    __device__ __forceinline__ void init(const short (*cnum)[NC])
    {
        const int lane = threadIdx.x & 63, hb = lane >> 5;
        if constexpr (K8) {
            const int sr = slot_of_row_k8(lane & 31);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int sc = 4 * hb + e;
                cB8[e] = bf16_bits((sr < NC && sc < NC) ? (float)cnum[sr][sc] : 0.0f);
            }
            return;
        }
        const int sr = slot_of_row(lane & 31);
        if constexpr (MODE == 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int sc = 16 * hb + j;
                cA[j] = (sr < NC && sc < NC) ? (float)cnum[sr][sc] : 0.0f;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int sc = 16 * hb + 8 * c + e;
                    cB[c][e] = (__bf16)((sr < NC && sc < NC) ? (float)cnum[sr][sc] : 0.0f);
                }
        }
    }

    __device__ __forceinline__ void flush_k8()
    {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int part = 0; part < 2; ++part) {
                // X: set A (events of lanes 0..31), Y: set B (lanes 32..63)
                float X[4], Y[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    X[e] = (e < NC) ? a[h][e][part] : 0.0f;
                    Y[e] = (4 + e < NC) ? a[h][4 + e][part] : 0.0f;
                    swap_halves(X[e], Y[e]);
                }
                shortx4 hA, mA, lA, hB, mB, lB;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const __bf16 xa = (__bf16)X[e], xb = (__bf16)Y[e];
                    const float ra = X[e] - (float)xa, rb = Y[e] - (float)xb;
                    const __bf16 ma = (__bf16)ra, mb = (__bf16)rb;
                    hA[e] = __builtin_bit_cast(short, xa);
                    mA[e] = __builtin_bit_cast(short, ma);
                    lA[e] = bf16_bits(ra - (float)ma);
                    hB[e] = __builtin_bit_cast(short, xb);
                    mB[e] = __builtin_bit_cast(short, mb);
                    lB[e] = bf16_bits(rb - (float)mb);
                }
                floatx16 DA = {0}, DB = {0};
                DA = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(cB8, lA, DA, 0, 0, 0);
                DA = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(cB8, mA, DA, 0, 0, 0);
                DA = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(cB8, hA, DA, 0, 0, 0);
                DB = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(cB8, lB, DB, 0, 0, 0);
                DB = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(cB8, mB, DB, 0, 0, 0);
                DB = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(cB8, hB, DB, 0, 0, 0);
                float pA = 0.0f, pB = 0.0f;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    pA = fmaf(X[t], DA[t], pA);
                    pB = fmaf(Y[t], DB[t], pB);
                }
                swap_halves(pA, pB);
                acc += pA + pB;
            }
        }
    }

    __device__ __forceinline__ void flush()
    {
        if constexpr (K8) {
            flush_k8();
            return;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int part = 0; part < 2; ++part) {
                float R1[16], R2[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    R1[j] = (j < NC) ? a[h][j][part] : 0.0f;
                    R2[j] = (16 + j < NC) ? a[h][16 + j][part] : 0.0f;
                    swap_halves(R1[j], R2[j]);
                }
                floatx16 DA = {0}, DB = {0};
                if constexpr (MODE == 0) {
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        DA = __builtin_amdgcn_mfma_f32_32x32x2f32(cA[j], R1[j], DA, 0, 0, 0);
                        DB = __builtin_amdgcn_mfma_f32_32x32x2f32(cA[j], R2[j], DB, 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        bf16x8 hA, mA, lA, hB, mB, lB;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const float va = R1[8 * c + e], vb = R2[8 * c + e];
                            const __bf16 ha = (__bf16)va, hbv = (__bf16)vb;
                            const float ra = va - (float)ha, rb = vb - (float)hbv;
                            const __bf16 ma = (__bf16)ra, mb = (__bf16)rb;
                            hA[e] = ha; mA[e] = ma; lA[e] = (__bf16)(ra - (float)ma);
                            hB[e] = hbv; mB[e] = mb; lB[e] = (__bf16)(rb - (float)mb);
                        }
                        DA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cB[c], lA, DA, 0, 0, 0);
                        DA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cB[c], mA, DA, 0, 0, 0);
                        DA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cB[c], hA, DA, 0, 0, 0);
                        DB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cB[c], lB, DB, 0, 0, 0);
                        DB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cB[c], mB, DB, 0, 0, 0);
                        DB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cB[c], hB, DB, 0, 0, 0);
                    }
                }
                float pA = 0.0f, pB = 0.0f;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    pA = fmaf(R1[t], DA[t], pA);
                    pB = fmaf(R2[t], DB[t], pB);
                }
                swap_halves(pA, pB);
                acc += pA + pB;
            }
        }
    }
};

}  // namespace mf
