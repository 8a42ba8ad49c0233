// Vector forward-mode (tangent) arithmetic: DualN<T, N> = value + sum_k eps_k t[k],
// eps_j eps_k = 0, i.e. the value of a scalar and its derivatives along N input
// directions at once.
//
// The derivative kernel carries the kinematics (Vegas map, phase space, the
// wavefunctions and propagator denominators the amplitude recursion reads)
// through this type with one direction per uniform and one for m_t.  Every
// transcendental or division is evaluated once on the value; each direction
// costs only the linear rule, so N directions cost far less than N separate
// passes.  Each operation is the exact first-order rule of its scalar
// counterpart: the tangents are the directional derivatives of the same
// floating-point program.
#pragma once
#include <hip/hip_runtime.h>

#include "dual.h"

template <typename T, int N>
struct DualN {
    T v;
    T t[N];
    __host__ __device__ DualN() : v(T(0))
    {
        for (int k = 0; k < N; ++k) t[k] = T(0);
    }
    __host__ __device__ DualN(double x) : v(T(x))
    {
        for (int k = 0; k < N; ++k) t[k] = T(0);
    }
    // value x with unit tangent along direction dir (none if dir is outside [0, N))
    __host__ __device__ static DualN seed(T x, int dir)
    {
        DualN r(x);
        for (int k = 0; k < N; ++k) r.t[k] = k == dir ? T(1) : T(0);
        return r;
    }
};

#define DN_TEMPLATE template <typename T, int N> __host__ __device__ __forceinline__ DualN<T, N>

DN_TEMPLATE operator+(const DualN<T, N>& a, const DualN<T, N>& b)
{
    DualN<T, N> r;
    r.v = a.v + b.v;
    for (int k = 0; k < N; ++k) r.t[k] = a.t[k] + b.t[k];
    return r;
}
DN_TEMPLATE operator-(const DualN<T, N>& a, const DualN<T, N>& b)
{
    DualN<T, N> r;
    r.v = a.v - b.v;
    for (int k = 0; k < N; ++k) r.t[k] = a.t[k] - b.t[k];
    return r;
}
DN_TEMPLATE operator-(const DualN<T, N>& a)
{
    DualN<T, N> r;
    r.v = -a.v;
    for (int k = 0; k < N; ++k) r.t[k] = -a.t[k];
    return r;
}
DN_TEMPLATE operator*(const DualN<T, N>& a, const DualN<T, N>& b)
{
    DualN<T, N> r;
    r.v = a.v * b.v;
    for (int k = 0; k < N; ++k) r.t[k] = fma(a.v, b.t[k], a.t[k] * b.v);
    return r;
}
DN_TEMPLATE operator/(const DualN<T, N>& a, const DualN<T, N>& b)
{
    DualN<T, N> r;
    const T inv = T(1) / b.v;
    r.v = a.v * inv;
    for (int k = 0; k < N; ++k) r.t[k] = (a.t[k] - r.v * b.t[k]) * inv;
    return r;
}
// with plain scalars
DN_TEMPLATE operator*(double s, const DualN<T, N>& a)
{
    DualN<T, N> r;
    r.v = T(s) * a.v;
    for (int k = 0; k < N; ++k) r.t[k] = T(s) * a.t[k];
    return r;
}
DN_TEMPLATE operator*(const DualN<T, N>& a, double s) { return s * a; }
DN_TEMPLATE operator/(const DualN<T, N>& a, double s)
{
    DualN<T, N> r;
    r.v = a.v / T(s);
    for (int k = 0; k < N; ++k) r.t[k] = a.t[k] / T(s);
    return r;
}
DN_TEMPLATE operator/(double s, const DualN<T, N>& a)
{
    DualN<T, N> r;
    r.v = T(s) / a.v;
    const T f = -r.v / a.v;
    for (int k = 0; k < N; ++k) r.t[k] = f * a.t[k];
    return r;
}
DN_TEMPLATE operator+(const DualN<T, N>& a, double s)
{
    DualN<T, N> r = a;
    r.v = a.v + T(s);
    return r;
}
DN_TEMPLATE operator+(double s, const DualN<T, N>& a) { return a + s; }
DN_TEMPLATE operator-(const DualN<T, N>& a, double s)
{
    DualN<T, N> r = a;
    r.v = a.v - T(s);
    return r;
}
DN_TEMPLATE operator-(double s, const DualN<T, N>& a)
{
    DualN<T, N> r;
    r.v = T(s) - a.v;
    for (int k = 0; k < N; ++k) r.t[k] = -a.t[k];
    return r;
}
DN_TEMPLATE sqrt(const DualN<T, N>& a)
{
    DualN<T, N> r;
    r.v = sqrt(a.v);
    const T h = T(0.5) / r.v;
    for (int k = 0; k < N; ++k) r.t[k] = a.t[k] * h;
    return r;
}
DN_TEMPLATE fmax(const DualN<T, N>& a, double b) { return a.v >= T(b) ? a : DualN<T, N>(b); }

#undef DN_TEMPLATE

template <typename T, int N>
__host__ __device__ __forceinline__ DualN<T, N>& operator+=(DualN<T, N>& a, const DualN<T, N>& b)
{
    a = a + b;
    return a;
}

template <typename T, int N> __host__ __device__ __forceinline__ T kval(const DualN<T, N>& x) { return x.v; }

// conversion from the kinematic types (the tangents travel with the value)
template <typename T, int N> struct Cvt<DualN<T, N>> {
    __host__ __device__ static __forceinline__ DualN<T, N> from(const DualN<T, N>& x) { return x; }
    __host__ __device__ static __forceinline__ DualN<T, N> from(double x) { return DualN<T, N>(x); }
};
