// Device helpers shared by the matrix-element kernels: complex pairs and the
// external wavefunctions (HELAS conventions, chiral Dirac representation;
// H. Murayama, I. Watanabe, K. Hagiwara, KEK-91-11).  The paper builds each
// matrix element from such external-state routines plus vertices and
// propagators (sect. 2, Fig. 2); it does not print their form.
//
// All wavefunctions are evaluated in the kinematic type KT (double, or the
// tangent types of dual.h / dualn.h in the derivative kernel) and rounded once
// to the kernel's working type R.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dual.h"

template <typename R>
struct cplx {
    R re, im;
};

// Two-component helicity eigenstate chi_lam(p) of sigma.p_hat (eigenvalue lam):
//   chi_+ = (|p|+pz, px + i py)/sqrt(2|p|(|p|+pz)),  chi_- = (-px + i py, |p|+pz)/(same)
// with |p|+pz evaluated as pT^2/(|p|-pz) when pz < 0 (no cancellation), the
// limits chi_+ = (0,1), chi_- = (-1,0) for p along -z, and chi along +z at rest.
template <typename KT>
__device__ __forceinline__ void helicity_chi(const KT* p, int lam, KT c[4])
{
    const KT px = p[1], py = p[2], pz = p[3];
    const KT pt2 = px * px + py * py;
    const KT pa = sqrt(pt2 + pz * pz);
    if (kval(pa) == 0.0) {
        c[0] = KT(lam > 0 ? 1.0 : 0.0); c[1] = KT(0.0);
        c[2] = KT(lam > 0 ? 0.0 : 1.0); c[3] = KT(0.0);
        return;
    }
    const KT s = (kval(pz) >= 0.0) ? pa + pz : pt2 / (pa - pz);
    if (kval(s) == 0.0) {
        c[0] = KT(lam > 0 ? 0.0 : -1.0); c[1] = KT(0.0);
        c[2] = KT(lam > 0 ? 1.0 : 0.0);  c[3] = KT(0.0);
        return;
    }
    const KT inv = KT(1.0) / sqrt(KT(2.0) * pa * s);
    if (lam > 0) {
        c[0] = s * inv;   c[1] = KT(0.0);
        c[2] = px * inv;  c[3] = py * inv;
    } else {
        c[0] = -px * inv; c[1] = py * inv;
        c[2] = s * inv;   c[3] = KT(0.0);
    }
}

// omega_+ = sqrt(E + |p|), omega_- = m / omega_+ (= sqrt(E - |p|) on shell).
template <typename KT>
__device__ __forceinline__ void omegas(const KT* p, KT m, KT& wp, KT& wm)
{
    const KT pa = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    wp = sqrt(p[0] + pa);
    wm = m / wp;
}

// Row spinor ubar(p, lam) = u^dagger gamma^0 with u = (w_{-lam} chi, w_{lam} chi):
//   ubar = (w_{lam} chi^*, w_{-lam} chi^*).
template <typename R, typename KT>
__device__ __forceinline__ void ubar_spinor(const KT* p, KT m, int lam, cplx<R> out[4])
{
    KT c[4], wp, wm;
    helicity_chi(p, lam, c);
    omegas(p, m, wp, wm);
    const KT a = lam > 0 ? wp : wm;   // w_{lam}
    const KT b = lam > 0 ? wm : wp;   // w_{-lam}
    out[0] = {cvt<R>(a * c[0]), cvt<R>(-a * c[1])};
    out[1] = {cvt<R>(a * c[2]), cvt<R>(-a * c[3])};
    out[2] = {cvt<R>(b * c[0]), cvt<R>(-b * c[1])};
    out[3] = {cvt<R>(b * c[2]), cvt<R>(-b * c[3])};
}

// Column spinor u(p, lam) = (w_{-lam} chi_lam, w_{lam} chi_lam).
template <typename R, typename KT>
__device__ __forceinline__ void u_spinor(const KT* p, KT m, int lam, cplx<R> out[4])
{
    KT c[4], wp, wm;
    helicity_chi(p, lam, c);
    omegas(p, m, wp, wm);
    const KT a = lam > 0 ? wm : wp;   // w_{-lam}
    const KT b = lam > 0 ? wp : wm;   // w_{lam}
    out[0] = {cvt<R>(a * c[0]), cvt<R>(a * c[1])};
    out[1] = {cvt<R>(a * c[2]), cvt<R>(a * c[3])};
    out[2] = {cvt<R>(b * c[0]), cvt<R>(b * c[1])};
    out[3] = {cvt<R>(b * c[2]), cvt<R>(b * c[3])};
}

// Column spinor v(p, lam) = (-lam w_{lam} chi_{-lam}, lam w_{-lam} chi_{-lam}).
template <typename R, typename KT>
__device__ __forceinline__ void v_spinor(const KT* p, KT m, int lam, cplx<R> out[4])
{
    KT c[4], wp, wm;
    helicity_chi(p, -lam, c);
    omegas(p, m, wp, wm);
    const KT a = double(-lam) * (lam > 0 ? wp : wm);   // -lam w_{lam}
    const KT b = double(lam) * (lam > 0 ? wm : wp);    //  lam w_{-lam}
    out[0] = {cvt<R>(a * c[0]), cvt<R>(a * c[1])};
    out[1] = {cvt<R>(a * c[2]), cvt<R>(a * c[3])};
    out[2] = {cvt<R>(b * c[0]), cvt<R>(b * c[1])};
    out[3] = {cvt<R>(b * c[2]), cvt<R>(b * c[3])};
}

// Row spinor vbar(p, lam) = v^dagger gamma^0.
template <typename R, typename KT>
__device__ __forceinline__ void vbar_spinor(const KT* p, KT m, int lam, cplx<R> out[4])
{
    cplx<R> v[4];
    v_spinor<R>(p, m, lam, v);
    out[0] = {v[2].re, -v[2].im};
    out[1] = {v[3].re, -v[3].im};
    out[2] = {v[0].re, -v[0].im};
    out[3] = {v[1].re, -v[1].im};
}

// Transverse basis of a massless vector boson's polarisation, divided by sqrt 2:
//   u = e1/sqrt2 = (cos th cos ph, cos th sin ph, -sin th)/sqrt2
//   w = e2/sqrt2 = (-sin ph, cos ph, 0)/sqrt2            (phi = 0 when pT = 0)
// so that eps(k, l) = -l u - i w and eps*(k, l) = -l u + i w.
template <typename R, typename KT>
__device__ __forceinline__ void pol_basis(const KT* k, R u[3], R w[2])
{
    const KT kx = k[1], ky = k[2], kz = k[3];
    const KT kt = sqrt(kx * kx + ky * ky);
    const KT ka = sqrt(kt * kt + kz * kz);
    const bool has_t = kval(kt) > 0.0;
    const KT cph = has_t ? kx / kt : KT(1.0);
    const KT sph = has_t ? ky / kt : KT(0.0);
    const KT cth = kz / ka, sth = kt / ka;
    const double r = 0.70710678118654752440;
    u[0] = cvt<R>(r * cth * cph);
    u[1] = cvt<R>(r * cth * sph);
    u[2] = cvt<R>(-r * sth);
    w[0] = cvt<R>(-r * sph);
    w[1] = cvt<R>(r * cph);
}

// Declares a value as changed by an empty asm statement: values derived from
// it cannot be hoisted out of the enclosing loop, so they are recomputed
// there instead of occupying registers across the loop.  No instruction.
__device__ __forceinline__ void opaque(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(double& x) { asm volatile("" : "+v"(x)); }
template <typename T> __device__ __forceinline__ void opaque(Dual<T>& x) { opaque(x.v); opaque(x.t); }

// Value held by lane (i + M) mod 4 of this lane's quad (lanes 4j..4j+3), by a
// DPP quad permutation.  Every lane of the quad must be active.
template <int M>
__device__ __forceinline__ int quad_rot_bits(int x)
{
    constexpr int ctrl = ((0 + M) & 3) | (((1 + M) & 3) << 2) | (((2 + M) & 3) << 4) | (((3 + M) & 3) << 6);
    return __builtin_amdgcn_update_dpp(0, x, ctrl, 0xF, 0xF, false);
}
template <int M>
__device__ __forceinline__ float quad_rot(float x)
{
    return __builtin_bit_cast(float, quad_rot_bits<M>(__builtin_bit_cast(int, x)));
}
template <int M>
__device__ __forceinline__ double quad_rot(double x)
{
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)quad_rot_bits<M>((int)(unsigned)v);
    const unsigned hi = (unsigned)quad_rot_bits<M>((int)(unsigned)(v >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Value held by the other lane of this lane's pair (lanes 2j, 2j+1), by a DPP
// quad permutation [1, 0, 3, 2].  Both lanes of the pair must be active.
__device__ __forceinline__ int pair_swap_bits(int x) { return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float pair_swap(float x)
{
    return __builtin_bit_cast(float, pair_swap_bits(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double pair_swap(double x)
{
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)pair_swap_bits((int)(unsigned)v);
    const unsigned hi = (unsigned)pair_swap_bits((int)(unsigned)(v >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Helicity-sum accumulator used by the VALU colour path.
template <typename R>
struct HelicitySum {
    R acc = R(0);
    __device__ __forceinline__ void add(R a, R b) { acc += a + b; }
};
