// Parton density from a tabulated grid: x f(x, Q^2) by cubic Hermite interpolation in
// ln x and then in ln Q^2 (the grid interpolation the paper's generator runs on the
// device before the matrix element, sect. 1; it does not print the scheme).  Node slopes
// are the mean of the two adjacent secant slopes inside the grid and the one secant slope
// at its ends; (x, Q^2) outside the grid is clamped to its edge.  The grid (a few tens of
// KB) stays in the L2 cache; every point reads 16 node values.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mf {

// i with t[i] <= s < t[i+1], in [0, n - 2] (binary search; s is inside [t0, t_{n-1}])
__device__ __forceinline__ int pdf_cell(const double* t, int n, double s)
{
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t[mid] <= s) lo = mid;
        else hi = mid;
    }
    return lo;
}

// slope at node k of values v(k) (a functor) at nodes t
template <typename V>
__device__ __forceinline__ double pdf_slope(const double* t, int n, int k, const V& v)
{
    if (k == 0) return (v(1) - v(0)) / (t[1] - t[0]);
    if (k == n - 1) return (v(n - 1) - v(n - 2)) / (t[n - 1] - t[n - 2]);
    return 0.5 * ((v(k + 1) - v(k)) / (t[k + 1] - t[k]) + (v(k) - v(k - 1)) / (t[k] - t[k - 1]));
}

__device__ __forceinline__ double pdf_hermite(double vi, double vj, double mi, double mj, double h, double u)
{
    const double u2 = u * u, u3 = u2 * u;
    return (2 * u3 - 3 * u2 + 1) * vi + (u3 - 2 * u2 + u) * h * mi + (-2 * u3 + 3 * u2) * vj + (u3 - u2) * h * mj;
}

// x f(x, Q^2)
__device__ __forceinline__ double pdf_xf(const PdfGrid& g, double x, double q2)
{
    const double t = fmin(fmax(log(x), g.lx[0]), g.lx[g.nx - 1]);
    const double s = fmin(fmax(log(q2), g.lq[0]), g.lq[g.nq - 1]);
    const int i = pdf_cell(g.lx, g.nx, t);
    const int j = pdf_cell(g.lq, g.nq, s);
    const double hx = g.lx[i + 1] - g.lx[i], ux = (t - g.lx[i]) / hx;
    // the rows j-1 .. j+2 that exist, interpolated in ln x
    double row[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int jj = j - 1 + r;
        row[r] = 0.0;
        if (jj < 0 || jj >= g.nq) continue;
        const double* v = g.v + (int64_t)jj * g.nx;
        auto val = [&](int k) { return v[k]; };
        row[r] = pdf_hermite(v[i], v[i + 1], pdf_slope(g.lx, g.nx, i, val), pdf_slope(g.lx, g.nx, i + 1, val), hx, ux);
    }
    // node slopes at j and j + 1 from the rows (the pdf_slope rule, written out so the rows
    // stay in registers)
    const double hq = g.lq[j + 1] - g.lq[j], uq = (s - g.lq[j]) / hq;
    const double sec = (row[2] - row[1]) / hq;
    const double mj = j == 0 ? sec : 0.5 * (sec + (row[1] - row[0]) / (g.lq[j] - g.lq[j - 1]));
    const double mj1 = j + 1 == g.nq - 1 ? sec : 0.5 * ((row[3] - row[2]) / (g.lq[j + 2] - g.lq[j + 1]) + sec);
    return pdf_hermite(row[1], row[2], mj, mj1, hq, uq);
}

}  // namespace mf
