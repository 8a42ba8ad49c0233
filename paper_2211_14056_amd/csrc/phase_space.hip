// Phase-space kernel: RNG -> Vegas map -> RAMBO on diet -> massive rescaling
// -> cuts, one lane per event, FP64 throughout (momentum conservation and mass
// shells are kept to FP64 rounding).
//
// The paper samples events in parallel along the event axis and integrates
// with Vegas (sect. 1); it does not describe its phase-space generator.  The
// sampler is RAMBO on diet (S. Plaetzer, arXiv:1308.2922: 3n-4 uniforms,
// constant weight) followed by the massive rescaling of RAMBO (R. Kleiss,
// W. J. Stirling, S. D. Ellis, Comput. Phys. Commun. 40 (1986) 359).
//
// Uniform assignment: the n-2 intermediate-mass numbers first, then one
// (cos theta, phi) pair per emission.  Outgoing order: t, tbar, gluons (or
// mu-, mu+).  Incoming partons along +z and -z with E = sqrt(s)/2.
// All reads and writes are SoA with the event index fastest (coalesced).
#include "internal.h"
#include "rng.h"

#include "ps_core.h"

namespace mf {
namespace {

template <int NOUT>
__global__ __launch_bounds__(256) void k_phase_space(PsArgs a)
{
    constexpr int D = 3 * NOUT - 4;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int64_t n = a.n;
    // ---- uniforms
    double x[D];
    if (a.x) {
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = a.x[k * n + e];
    } else {
        const uint64_t base = a.offset + (a.offset_dev ? *a.offset_dev : 0ull);
        event_uniforms<D>(a.seed, base + (uint64_t)e, x);
    }
    if (a.x_out) {
#pragma unroll
        for (int k = 0; k < D; ++k) a.x_out[k * n + e] = x[k];
    }
    // ---- Vegas map
    double y[D];
    double jac = 1.0;
    if (a.edges) {
        const int nb = a.nb;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = x[k] * nb;
            const int i = vegas_bin(t, nb);
            const double* ed = a.edges + k * (nb + 1);
            const double lo = ed[i], wdt = ed[i + 1] - lo;
            y[k] = lo + (t - i) * wdt;
            jac *= nb * wdt;
            if (a.bin_idx) a.bin_idx[k * n + e] = (int16_t)i;
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            y[k] = x[k];
            if (a.bin_idx) {
                a.bin_idx[k * n + e] = (int16_t)vegas_bin(x[k] * a.nb, a.nb);
            }
        }
    }
    // ---- RAMBO on diet + massive rescaling
    const double rs = a.sqrt_s;
    double P[NOUT][4];
    double wgt = 0.0;
    const bool ok = rambo_event<NOUT, double>(y, rs, a.m_out, P, &wgt);
    if (!ok && a.fail_count) atomicAdd(a.fail_count, 1ull);
    // ---- cuts on the final gluons (outgoing index >= 2 for the gg processes)
    if (a.pass) a.pass[e] = gluon_cuts<NOUT>(P, 0.0, a.pt_min, a.eta_max, a.dr_min) ? 1 : 0;
    // ---- outputs: incoming legs then outgoing, [leg][comp][event]
    const double E = 0.5 * rs;
    const double inc[2][4] = {{E, 0.0, 0.0, E}, {E, 0.0, 0.0, -E}};
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) a.p[(l * 4 + c) * n + e] = inc[l][c];
#pragma unroll
    for (int i = 0; i < NOUT; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) a.p[((i + 2) * 4 + c) * n + e] = P[i][c];
    a.w[e] = wgt;
    if (a.jac) a.jac[e] = jac;
}

}  // namespace

hipError_t launch_phase_space(const PsArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int block = 256;
    const unsigned grid = (unsigned)((a.n + block - 1) / block);
    switch (n_out(a.proc)) {
    case 2: hipLaunchKernelGGL(k_phase_space<2>, dim3(grid), dim3(block), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_phase_space<3>, dim3(grid), dim3(block), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_phase_space<4>, dim3(grid), dim3(block), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_phase_space<5>, dim3(grid), dim3(block), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
