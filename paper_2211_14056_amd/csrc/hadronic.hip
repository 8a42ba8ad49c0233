// Hadronic events: parton densities convoluted with the partonic phase space.
//
// The paper's workload is pp -> t tbar + jets (sect. 3, Table 1): the partonic matrix
// element weighted with parton densities interpolated from grids (sect. 1).  One parton
// channel per launch, parton 1 with density grid, parton 2 with density grid_b:
//   k_pdf_eval         x f(x, Q^2) for arrays of points (pdf.h);
//   k_phase_space_pp   two more uniforms per event give tau = tau0^(1 - u_tau)
//                      (tau0 = (2 m_t)^2 / S) and the rapidity y = (u_y - 1/2) ln(1/tau),
//                      x1,2 = sqrt(tau) e^(+-y), s_hat = tau S; the partonic event is made in
//                      its c.m. frame at sqrt(s_hat) (ps_core.h), the cuts are applied in the
//                      lab frame (light-parton pseudorapidities shifted by y), and the weight is
//                        w = tau ln(1/tau0) ln(1/tau) f_a(x1) f_b(x2) W (S / s_hat)
//                      at mu_F = m_t, so that the Vegas step with sqrt(s) = sqrt(S) forms
//                      F = (hbar c)^2 / (2 s_hat) J f_a f_b W ME Theta.
// One lane per event, FP64, SoA in and out as in the partonic phase-space kernel.
#include "internal.h"
#include "pdf.h"
#include "ps_core.h"
#include "rng.h"

namespace mf {
namespace {

__global__ __launch_bounds__(256) void k_pdf_eval(PdfGrid g, int64_t n, const double* x, const double* q2,
                                                  double* out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    out[e] = pdf_xf(g, x[e], q2[e]);
}

template <int NOUT>
__global__ __launch_bounds__(256) void k_phase_space_pp(PpArgs a)
{
    constexpr int D = 3 * NOUT - 4;
    constexpr int DH = D + 2;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int64_t n = a.n;
    double x[DH];
    if (a.x) {
#pragma unroll
        for (int k = 0; k < DH; ++k) x[k] = a.x[k * n + e];
    } else {
        const uint64_t base = a.offset + (a.offset_dev ? *a.offset_dev : 0ull);
        event_uniforms<DH>(a.seed, base + (uint64_t)e, x);
    }
    if (a.x_out) {
#pragma unroll
        for (int k = 0; k < DH; ++k) a.x_out[k * n + e] = x[k];
    }
    double y[DH];
    double jac = 1.0;
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        if (a.edges) {
            const int i = vegas_map1(x[k], a.edges + k * (a.nb + 1), a.nb, y[k], jac);
            if (a.bin_idx) a.bin_idx[k * n + e] = (int16_t)i;
        } else {
            y[k] = x[k];
            if (a.bin_idx) a.bin_idx[k * n + e] = (int16_t)vegas_bin(x[k] * a.nb, a.nb);
        }
    }
    // ---- hadronic variables
    const double ltau0 = log(a.tau0);
    const double tau = exp((1.0 - y[0]) * ltau0);
    const double lti = -log(tau);
    const double yb = (y[1] - 0.5) * lti;
    const double sq = sqrt(tau);
    const double x1 = sq * exp(yb), x2 = sq * exp(-yb);
    const double shat = tau * a.S;
    const double rs = sqrt(shat);
    const double jh = tau * (-ltau0) * lti;
    // ---- partonic event in its c.m. frame
    double P[NOUT][4];
    double wgt = 0.0;
    const bool ok = rambo_event<NOUT, double>(y + 2, rs, a.m_out, P, &wgt);
    if (!ok && a.fail_count) atomicAdd(a.fail_count, 1ull);
    // ---- cuts in the lab frame (massless gluons: eta_lab = eta + y)
    if (a.pass) a.pass[e] = gluon_cuts<NOUT>(P, yb, a.pt_min, a.eta_max, a.dr_min) ? 1 : 0;
    // ---- parton densities and weight
    const double f1 = pdf_xf(a.grid, x1, a.mu2) / x1;
    const double f2 = pdf_xf(a.grid_b, x2, a.mu2) / x2;
    const double w = jh * f1 * f2 * wgt * (a.S / shat);
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
    a.w[e] = w;
    if (a.jac) a.jac[e] = jac;
    if (a.x12) {
        a.x12[e] = x1;
        a.x12[n + e] = x2;
    }
}

}  // namespace

hipError_t launch_pdf_eval(const PdfGrid& g, int64_t n, const double* x, const double* q2, double* out,
                           hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_pdf_eval, dim3(grid), dim3(256), 0, s, g, n, x, q2, out);
    return hipGetLastError();
}

hipError_t launch_phase_space_pp(const PpArgs& a, int n_out, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    switch (n_out) {
    case 2: hipLaunchKernelGGL(k_phase_space_pp<2>, dim3(grid), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_phase_space_pp<3>, dim3(grid), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_phase_space_pp<4>, dim3(grid), dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_phase_space_pp<5>, dim3(grid), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
