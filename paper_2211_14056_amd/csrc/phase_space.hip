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

namespace mf {
namespace {

constexpr double kTwoPi = 6.283185307179586476925;

__device__ __forceinline__ void boost_from_rest(const double p[4], const double Q[4], double M, double out[4])
{
    // p given in the rest frame of Q (invariant mass M, known from the
    // recursion rather than recomputed from Q, which would cancel for a
    // strongly boosted light system) -> frame where Q has momentum Q
    const double qp = Q[1] * p[1] + Q[2] * p[2] + Q[3] * p[3];
    const double E = (Q[0] * p[0] + qp) / M;
    const double fac = (p[0] + E) / (Q[0] + M);
    out[0] = E;
    out[1] = p[1] + Q[1] * fac;
    out[2] = p[2] + Q[2] * fac;
    out[3] = p[3] + Q[3] * fac;
}

// Solve u = (a+1) rho^a - a rho^(a+1) for rho = r^2 in [0,1] (increasing):
// safeguarded Newton inside a shrinking bracket.
__device__ double solve_mass_ratio(double u, int a)
{
    double lo = 0.0, hi = 1.0;
    double rho = (a == 1) ? 1.0 - sqrt(1.0 - u) : pow(u / (a + 1), 1.0 / a);
    if (!(rho > 0.0 && rho < 1.0)) rho = 0.5;
    for (int it = 0; it < 100; ++it) {
        const double ra = pow(rho, a - 1);
        const double f = ((a + 1) - a * rho) * ra * rho - u;
        if (f == 0.0) break;                       // exact root
        if (f > 0.0) hi = rho; else lo = rho;
        const double df = a * (a + 1) * ra * (1.0 - rho);
        double nr = rho - f / df;
        if (!(nr >= lo && nr <= hi)) nr = 0.5 * (lo + hi);
        if (fabs(nr - rho) <= 2.5e-16 * rho || hi - lo <= 2.5e-16 * hi) { rho = nr; break; }
        rho = nr;
    }
    return sqrt(rho);
}

template <int NOUT>
__global__ __launch_bounds__(256) void k_phase_space(PsArgs a)
{
    constexpr int D = 3 * NOUT - 4;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int64_t n = a.n;
    // ---- a1: uniforms
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
    // ---- a2: Vegas map
    double y[D];
    double jac = 1.0;
    if (a.edges) {
        const int nb = a.nb;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = x[k] * nb;
            int i = (int)floor(t);
            i = i > nb - 1 ? nb - 1 : i;
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
                int i = (int)floor(x[k] * a.nb);
                a.bin_idx[k * n + e] = (int16_t)(i > a.nb - 1 ? a.nb - 1 : i);
            }
        }
    }
    // ---- a3: massless momenta (RAMBO on diet)
    const double rs = a.sqrt_s;
    double M[NOUT];
    M[0] = rs;
#pragma unroll
    for (int i = 2; i < NOUT; ++i) M[i - 1] = solve_mass_ratio(y[i - 2], NOUT - i) * M[i - 2];
    M[NOUT - 1] = 0.0;
    double P[NOUT][4];
    double Q[4] = {rs, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i < NOUT; ++i) {
        const double Mi = M[i - 1], Mn = M[i];
        const double q = (Mi * Mi - Mn * Mn) / (2.0 * Mi);
        const double cth = 2.0 * y[(NOUT - 2) + 2 * (i - 1)] - 1.0;
        const double ph = kTwoPi * y[(NOUT - 2) + 2 * (i - 1) + 1];
        const double sth = sqrt(fmax(1.0 - cth * cth, 0.0));
        double sph, cph;
        sincos(ph, &sph, &cph);
        const double nv[3] = {sth * cph, sth * sph, cth};
        const double pr[4] = {q, q * nv[0], q * nv[1], q * nv[2]};
        const double Qr[4] = {sqrt(q * q + Mn * Mn), -q * nv[0], -q * nv[1], -q * nv[2]};
        double Qn[4];
        boost_from_rest(pr, Q, Mi, P[i - 1]);
        boost_from_rest(Qr, Q, Mi, Qn);
#pragma unroll
        for (int c = 0; c < 4; ++c) Q[c] = Qn[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) P[NOUT - 1][c] = Q[c];
    // massless volume (2pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!)
    double wgt = 1.0;
    {
        const double s = rs * rs;
        double v = 1.0;
        for (int i = 0; i < 3 * NOUT - 4; ++i) v /= kTwoPi;
        for (int i = 0; i < NOUT - 1; ++i) v *= 0.5 * 3.141592653589793238463;
        for (int i = 0; i < NOUT - 2; ++i) v *= s;
        double f = 1.0;
        for (int i = 2; i <= NOUT - 1; ++i) f *= i;
        for (int i = 2; i <= NOUT - 2; ++i) f *= i;
        wgt = v / f;
    }
    // ---- massive rescaling: sum sqrt(m^2 + xi^2 E^2) = sqrt(s)
    double msum = 0.0;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) msum += a.m_out[i];
    if (msum > 0.0) {
        double lo = 0.0, hi = 1.0;
        double xi = sqrt(fmax(1.0 - (msum / rs) * (msum / rs), 0.0));
        bool ok = false;
        for (int it = 0; it < 50; ++it) {
            double F = -rs, dF = 0.0;
#pragma unroll
            for (int i = 0; i < NOUT; ++i) {
                const double E = P[i][0];
                const double r = sqrt(a.m_out[i] * a.m_out[i] + xi * xi * E * E);
                F += r;
                dF += xi * E * E / r;
            }
            if (F == 0.0) { ok = true; break; }     // exact root
            if (F > 0.0) hi = xi; else lo = xi;
            double nx = xi - F / dF;
            if (!(nx >= lo && nx <= hi)) nx = 0.5 * (lo + hi);
            const double dx = fabs(nx - xi);
            xi = nx;
            if (dx <= 1e-15 * xi) { ok = true; break; }
        }
        if (!ok) {
            wgt = 0.0;
            if (a.fail_count) atomicAdd(a.fail_count, 1ull);
        }
        double sk = 0.0, pk = 1.0, s2 = 0.0;
#pragma unroll
        for (int i = 0; i < NOUT; ++i) {
            const double E = P[i][0];
            const double k0 = sqrt(a.m_out[i] * a.m_out[i] + xi * xi * E * E);
            P[i][0] = k0;
            P[i][1] *= xi; P[i][2] *= xi; P[i][3] *= xi;
            const double ka = sqrt(P[i][1] * P[i][1] + P[i][2] * P[i][2] + P[i][3] * P[i][3]);
            sk += ka;
            pk *= ka / k0;
            s2 += ka * ka / k0;
        }
        double fac = 1.0;
        for (int i = 0; i < 2 * NOUT - 3; ++i) fac *= sk / rs;
        wgt *= fac * pk * rs / s2;
    }
    // ---- a4: cuts on the final gluons (outgoing index >= 2 for the gg processes)
    bool pass = true;
    if (a.pass) {
        double eta_[2] = {0.0, 0.0}, phi_[2] = {0.0, 0.0};
        int ng = 0;
#pragma unroll
        for (int i = 2; i < NOUT; ++i) {
            const double pt = sqrt(P[i][1] * P[i][1] + P[i][2] * P[i][2]);
            const double pa = sqrt(pt * pt + P[i][3] * P[i][3]);
            const double eta = atanh(P[i][3] / pa);
            pass = pass && (pt > a.pt_min) && (fabs(eta) < a.eta_max);
            eta_[ng] = eta;
            phi_[ng] = atan2(P[i][2], P[i][1]);
            ++ng;
        }
        if (ng == 2) {
            double dphi = phi_[0] - phi_[1];
            // wrap into [-pi, pi): same convention as remainder(x + pi, 2 pi) - pi
            dphi = dphi + 3.141592653589793238463;
            dphi = dphi - kTwoPi * floor(dphi / kTwoPi);
            dphi = dphi - 3.141592653589793238463;
            const double deta = eta_[0] - eta_[1];
            pass = pass && (sqrt(deta * deta + dphi * dphi) > a.dr_min);
        }
        a.pass[e] = pass ? 1 : 0;
    }
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
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
