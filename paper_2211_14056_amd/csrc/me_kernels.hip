// Matrix-element kernels: one lane per event, the helicity sum (half of the
// gluon-helicity configurations evaluated, their reverses supplied by the
// reversal symmetry), the colour-ordered recursion and the colour contraction
// fused in registers.
//
// The paper's custom operator launches one GPU kernel per spinor, vertex and
// propagator, passing every intermediate through device memory (sect. 2),
// and identifies the memory footprint of the calculation as what limits the
// GPU for processes with many diagrams (sect. 2, discussion of Table 1).
// Here the per-event state (wavefunctions, off-shell currents, partial
// amplitudes) never leaves the register file: a launch reads 32 B per
// external leg per event and writes one number per event.
//
// The per-process bodies are emitted by paper_2211_14056_amd/gen from the
// process definition (me_<process>.inc).
#include "internal.h"
#include "me_common.h"

#include "generated/me_gg_tt.inc"
#include "generated/me_gg_ttg.inc"
#include "generated/me_gg_ttgg.inc"

namespace mf {
namespace {

constexpr double kPi = 3.141592653589793238463;

// e-(p0) e+(p1) -> mu-(p2) mu+(p3) through an s-channel photon (massless QED):
// A = [vbar(p1) gamma^mu u(p0)] [ubar(p2) gamma_mu v(p3)], |M|^2 = e^4/s^2 |A|^2,
// summed over the 16 helicities and averaged by 1/4.
template <typename R>
__device__ __forceinline__ void spinor_current(const cplx<R> a[4], const cplx<R> b[4], cplx<R> j[4])
{
    // a (row) gamma^mu b (column), chiral representation:
    // gamma^0 swaps the 2-blocks; gamma^k = [[0, s^k], [-s^k, 0]].
    auto mul = [](cplx<R> x, cplx<R> y) { return cplx<R>{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re}; };
    auto add = [](cplx<R> x, cplx<R> y) { return cplx<R>{x.re + y.re, x.im + y.im}; };
    auto sub = [](cplx<R> x, cplx<R> y) { return cplx<R>{x.re - y.re, x.im - y.im}; };
    // j0 = a0 b2 + a1 b3 + a2 b0 + a3 b1
    j[0] = add(add(mul(a[0], b[2]), mul(a[1], b[3])), add(mul(a[2], b[0]), mul(a[3], b[1])));
    // s^1 = [[0,1],[1,0]]: upper(a) s1 lower(b) - lower(a) s1 upper(b)
    j[1] = sub(add(mul(a[0], b[3]), mul(a[1], b[2])), add(mul(a[2], b[1]), mul(a[3], b[0])));
    // s^2 = [[0,-i],[i,0]]
    {
        const cplx<R> t = sub(sub(mul(a[1], b[2]), mul(a[0], b[3])), sub(mul(a[3], b[0]), mul(a[2], b[1])));
        j[2] = cplx<R>{-t.im, t.re};   // i * t
    }
    // s^3 = diag(1,-1)
    j[3] = sub(sub(mul(a[0], b[2]), mul(a[1], b[3])), sub(mul(a[2], b[0]), mul(a[3], b[1])));
}

template <typename R>
__device__ __forceinline__ double me_ee_mumu(const double (&p)[4][4], double alpha)
{
    double s = 0.0;
    {
        const double P0 = p[0][0] + p[1][0], P1 = p[0][1] + p[1][1];
        const double P2 = p[0][2] + p[1][2], P3 = p[0][3] + p[1][3];
        s = P0 * P0 - P1 * P1 - P2 * P2 - P3 * P3;
    }
    R tot = R(0);
    for (int h = 0; h < 16; ++h) {
        const int l0 = (h & 8) ? 1 : -1, l1 = (h & 4) ? 1 : -1, l2 = (h & 2) ? 1 : -1, l3 = (h & 1) ? 1 : -1;
        cplx<R> u0[4], vb1[4], ub2[4], v3[4], jin[4], jout[4];
        u_spinor<R>(p[0], 0.0, l0, u0);
        vbar_spinor<R>(p[1], 0.0, l1, vb1);
        ubar_spinor<R>(p[2], 0.0, l2, ub2);
        v_spinor<R>(p[3], 0.0, l3, v3);
        spinor_current<R>(vb1, u0, jin);
        spinor_current<R>(ub2, v3, jout);
        R re = jin[0].re * jout[0].re - jin[0].im * jout[0].im;
        R im = jin[0].re * jout[0].im + jin[0].im * jout[0].re;
        for (int c = 1; c < 4; ++c) {
            re -= jin[c].re * jout[c].re - jin[c].im * jout[c].im;
            im -= jin[c].re * jout[c].im + jin[c].im * jout[c].re;
        }
        tot += re * re + im * im;
    }
    const double e2 = 4.0 * kPi * alpha;
    return (double)tot * e2 * e2 / (s * s) / 4.0;
}

template <int NEXT>
__device__ __forceinline__ void load_event(const double* __restrict__ p, int64_t n, int64_t e, double (&pe)[NEXT][4])
{
#pragma unroll
    for (int l = 0; l < NEXT; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) pe[l][c] = p[(l * 4 + c) * n + e];
}

template <int PROC, typename R>
__global__ __launch_bounds__(256) void k_me_valu(const double* __restrict__ p, int64_t n, R* __restrict__ out,
                                                 double mt, double coupling)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if constexpr (PROC == EE_MUMU) {
        double pe[4][4];
        load_event<4>(p, n, e, pe);
        out[e] = R(me_ee_mumu<R>(pe, coupling));
    } else if constexpr (PROC == GG_TT) {
        double pe[4][4];
        load_event<4>(p, n, e, pe);
        HelicitySum<R> hs;
        me_gg_tt_body<R>(pe, mt, hs);
        out[e] = R((double)hs.acc * coupling * me_gg_tt_norm_noalpha());
    } else if constexpr (PROC == GG_TTG) {
        double pe[5][4];
        load_event<5>(p, n, e, pe);
        HelicitySum<R> hs;
        me_gg_ttg_body<R>(pe, mt, hs);
        out[e] = R((double)hs.acc * coupling * me_gg_ttg_norm_noalpha());
    }
}

// gg -> ttbar gg: one wave per block; the multi-gluon currents are parked in
// this wave's LDS columns (one per lane, stride 64) between the gluon-current
// block and the quark line.
template <typename R>
__global__ __launch_bounds__(64) void k_me_ttgg(const double* __restrict__ p, int64_t n, R* __restrict__ out,
                                                double mt, double coupling)
{
    constexpr int SLOTS = sizeof(R) == 4 ? me_gg_ttgg_lds32_slots : me_gg_ttgg_lds64_slots;
    __shared__ R smem[SLOTS * 64];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double pe[6][4];
    load_event<6>(p, n, e, pe);
    HelicitySum<R> hs;
    if constexpr (sizeof(R) == 4)
        me_gg_ttgg_body_lds32<R>(pe, mt, hs, smem + threadIdx.x);
    else
        me_gg_ttgg_body_lds64<R>(pe, mt, hs, smem + threadIdx.x);
    out[e] = R((double)hs.acc * coupling * me_gg_ttgg_norm_noalpha());
}

template <typename R>
hipError_t launch_valu(const MeJob& j, double mt, double coupling, int block, hipStream_t s)
{
    const unsigned grid = (unsigned)((j.n + block - 1) / block);
    R* out = static_cast<R*>(j.out);
    switch (j.proc) {
    case EE_MUMU: hipLaunchKernelGGL((k_me_valu<EE_MUMU, R>), dim3(grid), dim3(block), 0, s, j.p, j.n, out, mt, coupling); break;
    case GG_TT: hipLaunchKernelGGL((k_me_valu<GG_TT, R>), dim3(grid), dim3(block), 0, s, j.p, j.n, out, mt, coupling); break;
    case GG_TTG: hipLaunchKernelGGL((k_me_valu<GG_TTG, R>), dim3(grid), dim3(block), 0, s, j.p, j.n, out, mt, coupling); break;
    case GG_TTGG: {
        const unsigned g64 = (unsigned)((j.n + 63) / 64);
        hipLaunchKernelGGL((k_me_ttgg<R>), dim3(g64), dim3(64), 0, s, j.p, j.n, out, mt, coupling);
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool precision_available(int precision) { return precision >= 0 && precision <= 3; }

hipError_t launch_matrix_element(const MeJob& j, int precision, double mt, double alpha_s, double alpha,
                                 int block, hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    // coupling factor: alpha for e+e- (the kernel applies e^4), (4 pi alpha_s)^k for QCD
    double coupling = alpha;
    if (j.proc != EE_MUMU) {
        coupling = 1.0;
        const double g2 = 4.0 * kPi * alpha_s;
        for (int i = 0; i < n_gluons(j.proc); ++i) coupling *= g2;
    }
    if (j.proc == GG_TTGGG) {
        if (precision > 1) return hipErrorInvalidValue;          // no matrix-core colour form
        return launch_ttggg(j, precision, mt, coupling, block, s);
    }
    if (quark_proc(j.proc)) return launch_quark(j, precision, mt, coupling, block, s);
    if (j.proc == GG_TTGG && precision == 0 && block == TTGG_QUAD_LAYOUT)
        return launch_ttgg_quad(j, mt, coupling, s);
    if (j.proc == GG_TTGG && precision == 0 && (block <= 0 || block == TTGG_PAIR_LAYOUT))
        return launch_ttgg_pair(j, mt, coupling, s);
    if (block <= 0) block = 256;
    switch (precision) {
    case 0: return launch_valu<double>(j, mt, coupling, block, s);
    case 1: return launch_valu<float>(j, mt, coupling, block, s);
    case 2:
    case 3:
        if (j.proc == EE_MUMU) return hipErrorInvalidValue;    // no colour to contract
        return launch_matrix_element_mfma(j, precision, mt, coupling, block, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mf
