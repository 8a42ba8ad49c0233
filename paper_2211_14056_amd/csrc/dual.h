// Forward-mode (tangent) arithmetic: Dual<T> = value + eps * tangent, eps^2 = 0.
//
// One input direction at a time.  The derivative kernel carries the kinematics
// through the several-direction form DualN (dualn.h); the phase-space and
// wavefunction code is written for either.  Every operation below is the exact
// first-order rule of its scalar counterpart, so the tangent of the output is
// the directional derivative of the same floating-point program.
#pragma once
#include <hip/hip_runtime.h>

template <typename T>
struct Dual {
    T v, t;
    __host__ __device__ constexpr Dual() : v(T(0)), t(T(0)) {}
    __host__ __device__ constexpr Dual(double x) : v(T(x)), t(T(0)) {}
    __host__ __device__ constexpr Dual(T x, T dx) : v(x), t(dx) {}
    template <typename U>
    __host__ __device__ explicit constexpr Dual(const Dual<U>& o) : v(T(o.v)), t(T(o.t)) {}
};

template <typename T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.t + b.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.t - b.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, fma(a.v, b.t, a.t * b.v)}; }
template <typename T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b)
{
    const T q = a.v / b.v;
    return {q, (a.t - q * b.t) / b.v};
}
template <typename T> __device__ __forceinline__ Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { a = a + b; return a; }
template <typename T> __device__ __forceinline__ Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { a = a - b; return a; }
template <typename T> __device__ __forceinline__ Dual<T>& operator*=(Dual<T>& a, Dual<T> b) { a = a * b; return a; }
// mixed with plain scalars
template <typename T> __device__ __forceinline__ Dual<T> operator*(double s, Dual<T> a) { return {T(s) * a.v, T(s) * a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, double s) { return {T(s) * a.v, T(s) * a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, double s) { return {a.v + T(s), a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator+(double s, Dual<T> a) { return {a.v + T(s), a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, double s) { return {a.v - T(s), a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(double s, Dual<T> a) { return {T(s) - a.v, -a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, double s) { return {a.v / T(s), a.t / T(s)}; }
template <typename T> __device__ __forceinline__ Dual<T> operator/(double s, Dual<T> a)
{
    const T q = T(s) / a.v;
    return {q, -q * a.t / a.v};
}

template <typename T> __device__ __forceinline__ Dual<T> fma(Dual<T> a, Dual<T> b, Dual<T> c)
{
    return {fma(a.v, b.v, c.v), fma(a.v, b.t, fma(a.t, b.v, c.t))};
}
template <typename T> __device__ __forceinline__ Dual<T> sqrt(Dual<T> a)
{
    const T s = sqrt(a.v);
    return {s, a.t / (T(2) * s)};
}
template <typename T> __device__ __forceinline__ Dual<T> sin(Dual<T> a) { return {sin(a.v), cos(a.v) * a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> cos(Dual<T> a) { return {cos(a.v), -sin(a.v) * a.t}; }
template <typename T> __device__ __forceinline__ Dual<T> fmax(Dual<T> a, double b) { return a.v >= T(b) ? a : Dual<T>(b); }

// value of a scalar for comparisons and branch decisions
__device__ __forceinline__ double kval(double x) { return x; }
__device__ __forceinline__ float kval(float x) { return x; }
template <typename T> __device__ __forceinline__ T kval(Dual<T> x) { return x.v; }

// conversion between kinematic and working types (value and tangent rounded separately)
template <typename R> struct Cvt {
    template <typename K> __device__ static __forceinline__ R from(K x) { return R(x); }
};
template <typename T> struct Cvt<Dual<T>> {
    template <typename U> __device__ static __forceinline__ Dual<T> from(Dual<U> x) { return Dual<T>(T(x.v), T(x.t)); }
    __device__ static __forceinline__ Dual<T> from(double x) { return Dual<T>(x); }
};
template <typename R, typename K> __device__ __forceinline__ R cvt(K x) { return Cvt<R>::from(x); }
