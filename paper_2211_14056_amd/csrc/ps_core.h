// Phase-space core shared by the phase-space kernel (KT = double) and the
// derivative kernel (KT = DualN<double, N>, tangents along N inputs): Vegas map,
// RAMBO on diet
// (S. Plaetzer, arXiv:1308.2922) and the massive rescaling of RAMBO
// (R. Kleiss, W. J. Stirling, S. D. Ellis, Comput. Phys. Commun. 40 (1986) 359).
//
// The two one-dimensional root solves (intermediate mass ratio, rescaling
// factor xi) run on FP64 values with a safeguarded Newton iteration; one more
// Newton step is then taken in KT arithmetic from the converged root, which
// leaves the value unchanged to rounding and carries the implicit-function
// derivative when KT carries tangents.
#pragma once
#include <hip/hip_runtime.h>

#include "dual.h"
#include "dualn.h"

namespace mf {

constexpr double kTwoPiPs = 6.283185307179586476925;
constexpr double kPiPs = 3.141592653589793238463;

__device__ __forceinline__ void ps_sincos(double x, double& s, double& c) { sincos(x, &s, &c); }
template <typename T>
__device__ __forceinline__ void ps_sincos(Dual<T> x, Dual<T>& s, Dual<T>& c)
{
    T sv, cv;
    sincos(x.v, &sv, &cv);
    s = Dual<T>(sv, cv * x.t);
    c = Dual<T>(cv, -sv * x.t);
}

template <typename T, int N>
__device__ __forceinline__ void ps_sincos(const DualN<T, N>& x, DualN<T, N>& s, DualN<T, N>& c)
{
    T sv, cv;
    sincos(x.v, &sv, &cv);
    s.v = sv;
    c.v = cv;
    for (int k = 0; k < N; ++k) {
        s.t[k] = cv * x.t[k];
        c.t[k] = -sv * x.t[k];
    }
}

template <typename KT>
__device__ __forceinline__ void boost_from_rest(const KT p[4], const KT Q[4], KT M, KT out[4])
{
    // p given in the rest frame of Q (invariant mass M, known from the
    // recursion rather than recomputed from Q, which would cancel for a
    // strongly boosted light system) -> frame where Q has momentum Q
    const KT qp = Q[1] * p[1] + Q[2] * p[2] + Q[3] * p[3];
    const KT E = (Q[0] * p[0] + qp) / M;
    const KT fac = (p[0] + E) / (Q[0] + M);
    out[0] = E;
    out[1] = p[1] + Q[1] * fac;
    out[2] = p[2] + Q[2] * fac;
    out[3] = p[3] + Q[3] * fac;
}

// Root rho of u = (a+1) rho^a - a rho^(a+1) on [0, 1] (increasing), FP64.
__device__ inline double solve_mass_ratio_sq(double u, int a)
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
    return rho;
}

// Vegas map of one uniform: y = e_i + (x nb - i)(e_{i+1} - e_i); returns the bin.
// The bin is clamped to [0, nb) before any edge is read, so a uniform outside
// [0, 1) uses the first or last bin (extrapolated linearly) and a NaN uniform
// bin 0 with y = NaN: the edge reads stay in bounds whatever the caller passes.
__device__ __forceinline__ int vegas_bin(double t, int nb)
{
    return (int)fmin(fmax(floor(t), 0.0), double(nb - 1));    // fmax drops a NaN
}

template <typename KT>
__device__ __forceinline__ int vegas_map1(KT x, const double* ed, int nb, KT& y, double& jac)
{
    const KT t = x * double(nb);
    const int i = vegas_bin(kval(t), nb);
    const double lo = ed[i], wdt = ed[i + 1] - lo;
    y = (t - double(i)) * wdt + lo;
    jac *= nb * wdt;
    return i;
}

// Massless momenta from the phase-space uniforms y[3 NOUT - 4], massive
// rescaling with masses m[NOUT]; P[i] outgoing momenta in the c.m. frame.
// Returns false if the rescaling did not converge.  If wgt != nullptr the
// phase-space weight is returned too (FP64 only).
template <int NOUT, typename KT>
__device__ __forceinline__ bool rambo_event(const KT* y, double rs, const KT* m, KT (&P)[NOUT][4], double* wgt)
{
    KT M[NOUT];
    M[0] = KT(rs);
#pragma unroll
    for (int i = 2; i < NOUT; ++i) {
        const int a = NOUT - i;
        const KT u = y[i - 2];
        const double r0 = sqrt(solve_mass_ratio_sq(kval(u), a));
        // implicit-function step in r: G(r, u) = (a+1) r^(2a) - a r^(2a+2) - u,
        // dG/dr = 2a(a+1) r^(2a-1) (1 - r^2)
        const double r2a = pow(r0, 2 * a);
        const double G0 = (a + 1) * r2a - a * r2a * r0 * r0;
        const double dG = 2.0 * a * (a + 1) * pow(r0, 2 * a - 1) * (1.0 - r0 * r0);
        const KT r = (u - G0) / dG + r0;
        M[i - 1] = r * M[i - 2];
    }
    M[NOUT - 1] = KT(0.0);
    KT Q[4] = {KT(rs), KT(0.0), KT(0.0), KT(0.0)};
#pragma unroll
    for (int i = 1; i < NOUT; ++i) {
        const KT Mi = M[i - 1], Mn = M[i];
        const KT q = (Mi * Mi - Mn * Mn) / (Mi * 2.0);
        const KT cth = y[(NOUT - 2) + 2 * (i - 1)] * 2.0 - 1.0;
        const KT ph = y[(NOUT - 2) + 2 * (i - 1) + 1] * kTwoPiPs;
        const KT sth = sqrt(fmax(1.0 - cth * cth, 0.0));
        KT sph, cph;
        ps_sincos(ph, sph, cph);
        const KT nv[3] = {sth * cph, sth * sph, cth};
        const KT pr[4] = {q, q * nv[0], q * nv[1], q * nv[2]};
        const KT Qr[4] = {sqrt(q * q + Mn * Mn), -(q * nv[0]), -(q * nv[1]), -(q * nv[2])};
        KT Qn[4];
        boost_from_rest(pr, Q, Mi, P[i - 1]);
        boost_from_rest(Qr, Q, Mi, Qn);
#pragma unroll
        for (int c = 0; c < 4; ++c) Q[c] = Qn[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) P[NOUT - 1][c] = Q[c];
    if (wgt) {
        // massless volume (2pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!)
        const double s = rs * rs;
        double v = 1.0;
        for (int i = 0; i < 3 * NOUT - 4; ++i) v /= kTwoPiPs;
        for (int i = 0; i < NOUT - 1; ++i) v *= 0.5 * kPiPs;
        for (int i = 0; i < NOUT - 2; ++i) v *= s;
        double f = 1.0;
        for (int i = 2; i <= NOUT - 1; ++i) f *= i;
        for (int i = 2; i <= NOUT - 2; ++i) f *= i;
        *wgt = v / f;
    }
    // massive rescaling: sum sqrt(m^2 + xi^2 E^2) = sqrt(s)
    double msum = 0.0;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) msum += kval(m[i]);
    if (!(msum > 0.0)) return true;
    double lo = 0.0, hi = 1.0;
    double xi = sqrt(fmax(1.0 - (msum / rs) * (msum / rs), 0.0));
    bool ok = false;
    // F(0) = sum m - sqrt(s) < 0 <= F(1) brackets the root; at or below threshold there is
    // none and the event fails
    for (int it = 0; msum < rs && it < 50; ++it) {
        double F = -rs, dF = 0.0;
#pragma unroll
        for (int i = 0; i < NOUT; ++i) {
            const double E = kval(P[i][0]), mi = kval(m[i]);
            const double r = sqrt(mi * mi + xi * xi * E * E);
            F += r;
            dF += xi * E * E / r;
        }
        // converged when the residual is at the rounding level of its own evaluation (NOUT
        // square roots of size up to sqrt(s)): near threshold (xi -> 0) F'(xi) -> 0, so the
        // Newton step there is rounding noise and a step-size test alone would never pass
        if (fabs(F) <= 4.5e-16 * NOUT * rs) { ok = true; break; }
        if (F > 0.0) hi = xi; else lo = xi;
        if (hi - lo <= 4.5e-16 * hi) { ok = true; break; }     // bracket at the last bits
        double nx = xi - F / dF;
        if (!(nx >= lo && nx <= hi)) nx = 0.5 * (lo + hi);
        const double dx = fabs(nx - xi);
        xi = nx;
        if (dx <= 1e-15 * xi) { ok = true; break; }
    }
    // implicit-function step in KT: xi <- xi0 - F(xi0)/F'(xi0)
    KT F = KT(-rs);
    double dF = 0.0;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
        const KT r = sqrt(m[i] * m[i] + P[i][0] * P[i][0] * (xi * xi));
        F = F + r;
        dF += xi * kval(P[i][0]) * kval(P[i][0]) / kval(r);
    }
    const KT xik = dF > 0.0 ? KT(xi) - F / dF : KT(xi);
    double sk = 0.0, pk = 1.0, s2 = 0.0;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
        const KT E = P[i][0];
        const KT k0 = sqrt(m[i] * m[i] + xik * xik * E * E);
        P[i][0] = k0;
        P[i][1] = P[i][1] * xik;
        P[i][2] = P[i][2] * xik;
        P[i][3] = P[i][3] * xik;
        if (wgt) {
            const double kx = kval(P[i][1]), ky = kval(P[i][2]), kz = kval(P[i][3]), e0 = kval(k0);
            const double ka = sqrt(kx * kx + ky * ky + kz * kz);
            sk += ka;
            pk *= ka / e0;
            s2 += ka * ka / e0;
        }
    }
    if (wgt) {
        double fac = 1.0;
        for (int i = 0; i < 2 * NOUT - 3; ++i) fac *= sk / rs;
        *wgt *= fac * pk * rs / s2;
        if (!ok) *wgt = 0.0;
    }
    return ok;
}

// Generation cuts on the final gluons (outgoing particles 2 .. NOUT-1; the tops are not
// cut): pT > pt_min and |eta + y| < eta_max for each, Delta R > dr_min for every pair, with
// eta = atanh(pz/|p|) and Delta phi wrapped into [-pi, pi).  y shifts the pseudorapidities
// (a longitudinal boost of massless particles; 0 in the c.m. frame).  Strict inequalities.
template <int NOUT>
__device__ __forceinline__ bool gluon_cuts(const double (&P)[NOUT][4], double y, double pt_min, double eta_max,
                                           double dr_min)
{
    constexpr int NG = NOUT > 2 ? NOUT - 2 : 1;
    double eta_[NG], phi_[NG];
    bool pass = true;
#pragma unroll
    for (int i = 2; i < NOUT; ++i) {
        const double pt = sqrt(P[i][1] * P[i][1] + P[i][2] * P[i][2]);
        const double pa = sqrt(pt * pt + P[i][3] * P[i][3]);
        const double eta = atanh(P[i][3] / pa) + y;
        pass = pass && (pt > pt_min) && (fabs(eta) < eta_max);
        eta_[i - 2] = eta;
        phi_[i - 2] = atan2(P[i][2], P[i][1]);
    }
#pragma unroll
    for (int i = 0; i + 2 < NOUT; ++i)
#pragma unroll
        for (int j = i + 1; j + 2 < NOUT; ++j) {
            // wrap into [-pi, pi): the convention of remainder(x + pi, 2 pi) - pi
            double dphi = phi_[i] - phi_[j] + 3.141592653589793238463;
            dphi = dphi - kTwoPiPs * floor(dphi / kTwoPiPs) - 3.141592653589793238463;
            const double deta = eta_[i] - eta_[j];
            pass = pass && (sqrt(deta * deta + dphi * dphi) > dr_min);
        }
    return pass;
}

}  // namespace mf
