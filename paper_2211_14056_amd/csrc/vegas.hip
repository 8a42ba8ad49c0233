// Vegas accumulation and grid refinement.
//
// The paper integrates with Vegas (sect. 1, G. P. Lepage 1978/1980); the
// refinement used here is Lepage's: per dimension a histogram of F^2 over the
// bins of the current grid, smoothed over neighbouring bins, compressed by
// r = ((1 - rho)/(-ln rho))^alpha and rebinned so that every new bin holds the
// same share of sum r.
//
// Accumulation is deterministic (fixed reduction order for any run):
//  * each block walks a fixed set of 256-event chunks (grid-stride with a
//    grid size that depends only on n);
//  * per wave, lane k < d owns the histogram row of dimension k in LDS and
//    adds the wave's 64 events in lane order;
//  * block partials (sum F, sum F^2, histogram) go to a cell-major workspace,
//    and one workgroup sums them (a wave per cell, fixed lane order and a
//    fixed butterfly) and then refines the grid.
// F = flux * w * J_vegas * ME for events that pass the cuts and have a weight
// that is neither 0 nor NaN (0 otherwise) is formed here from the phase-space weight, the Vegas Jacobian
// and the matrix element, so it never round-trips through memory unless the
// caller asks for it.
#include <mutex>

#include "internal.h"

namespace mf {
namespace {

constexpr int VB = 256;           // threads per block
constexpr int WAVES = VB / 64;
constexpr int MAXD = VEGAS_MAX_D;
constexpr int MAXNB = 64;
static_assert(2 + MAXD * MAXNB == VEGAS_MAX_CELLS, "workspace size");

// MD: histogram rows held in LDS (8 serves the partonic processes up to four final-state
// particles with a small footprint; 16 the hadronic and larger ones)
template <int MD>
__global__ __launch_bounds__(VB) void k_vegas_accumulate(VegasArgs a)
{
    __shared__ double hist[WAVES][MD][MAXNB];
    __shared__ double fsq[WAVES][64];
    __shared__ short bins[WAVES][MD][64];
    __shared__ double red[2][VB];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int d = a.d, nb = a.nb;
    for (int c = lane; c < MD * MAXNB; c += 64) hist[wv][c / MAXNB][c % MAXNB] = 0.0;
    double sf = 0.0, sf2 = 0.0;
    const int64_t n = a.n;
    for (int64_t chunk = blockIdx.x; chunk * VB < n; chunk += gridDim.x) {
        const int64_t e = chunk * VB + tid;
        double F = 0.0;
        if (e < n) {
            const double me = a.me_f32 ? (double)static_cast<const float*>(a.me)[e]
                                       : static_cast<const double*>(a.me)[e];
            const bool ps = a.pass ? a.pass[e] != 0 : true;
            const double jac = a.jac ? a.jac[e] : 1.0;
            const double w = a.w[e];
            // an event outside the cuts or without weight (a failed phase-space solve
            // gives 0, NaN uniforms NaN) contributes exactly 0, whatever its |M|^2 holds;
            // a negative weight (a parton density below zero) counts as it is
            F = (ps && w == w && w != 0.0) ? a.flux * w * jac * me : 0.0;
            if (a.F) a.F[e] = F;
        }
        sf += F;
        sf2 += F * F;
        fsq[wv][lane] = F * F;
        for (int k = 0; k < d; ++k) bins[wv][k][lane] = (e < n) ? a.bin_idx[k * n + e] : (short)-1;
        __syncthreads();
        if (lane < d) {
            for (int l = 0; l < 64; ++l) {
                const int b = bins[wv][lane][l];
                if (b >= 0 && b < nb) hist[wv][lane][b] += fsq[wv][l];
            }
        }
        __syncthreads();
    }
    red[0][tid] = sf;
    red[1][tid] = sf2;
    __syncthreads();
    for (int s = VB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
        }
        __syncthreads();
    }
    // partials are cell-major, [cell][block], so the final reduction reads them coalesced
    const int64_t nblk = gridDim.x;
    double* out = a.partials + blockIdx.x;
    if (tid == 0) {
        out[0] = red[0][0];
        out[nblk] = red[1][0];
    }
    for (int c = tid; c < d * nb; c += VB) {
        const int k = c / nb, b = c % nb;
        double s = 0.0;
        for (int w = 0; w < WAVES; ++w) s += hist[w][k][b];
        out[(2 + c) * nblk] = s;
    }
}

__device__ void refine_dim(const double* h, double* edges, int nb, double alpha)
{
    // a histogram without weight, or with a non-finite entry (an infinite or NaN
    // integrand value), leaves the grid of this dimension as it is
    bool any = false, finite = true;
    for (int i = 0; i < nb; ++i) {
        any = any || (h[i] > 0.0);
        finite = finite && isfinite(h[i]);
    }
    if (!any || !finite) return;
    double hb[MAXNB], r[MAXNB], old[MAXNB + 1];
    hb[0] = (h[0] + h[1]) / 2.0;
    hb[nb - 1] = (h[nb - 2] + h[nb - 1]) / 2.0;
    for (int i = 1; i < nb - 1; ++i) hb[i] = (h[i - 1] + h[i] + h[i + 1]) / 3.0;
    double tot = 0.0;
    for (int i = 0; i < nb; ++i) tot += hb[i];
    double rsum = 0.0;
    for (int i = 0; i < nb; ++i) {
        const double rho = hb[i] / tot;
        double v;
        if (rho <= 0.0) v = 0.0;
        else if (rho >= 1.0) v = 1.0;
        else v = pow((1.0 - rho) / (-log(rho)), alpha);
        r[i] = v;
        rsum += v;
    }
    for (int i = 0; i <= nb; ++i) old[i] = edges[i];
    const double delta = rsum / nb;
    double cum = 0.0;
    int i = 0;
    for (int e = 1; e < nb; ++e) {
        const double target = e * delta;
        while (i < nb && cum + r[i] < target) {
            cum += r[i];
            ++i;
        }
        if (i >= nb) {
            edges[e] = old[nb];
            continue;
        }
        edges[e] = r[i] > 0.0 ? old[i] + (target - cum) / r[i] * (old[i + 1] - old[i]) : old[i];
    }
    edges[0] = 0.0;
    edges[nb] = 1.0;
}

__global__ __launch_bounds__(64) void k_vegas_reduce(VegasArgs a)
{
    // one wave per cell (cell = blockIdx.x): lane l sums blocks l, l+64, ... in
    // order, then a fixed xor-butterfly adds the 64 lane sums (same order every run)
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const double* src = a.partials + (int64_t)c * a.nblk;
    double s = 0.0;
    for (int b = lane; b < a.nblk; b += 64) s += src[b];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) a.acc[c] = a.accumulate ? a.acc[c] + s : s;
}

__global__ __launch_bounds__(64) void k_vegas_update(VegasArgs a)
{
    // after the reduction: refine the grid (one lane per dimension) and advance
    // the event counter of the random-number stream
    if (a.update_edges && threadIdx.x < a.d) {
        const int k = threadIdx.x;
        refine_dim(a.acc + 2 + k * a.nb, a.edges + k * (a.nb + 1), a.nb, a.alpha);
    }
    if (a.rng_counter && threadIdx.x == 0) *a.rng_counter += (uint64_t)a.n;
}

}  // namespace

// Block partials of mf_vegas_refine_noalloc: a library-owned array of the largest size
// any call needs (VEGAS_PARTIALS_MAX doubles, 8.4 MB), one copy per device, held until
// the process ends.  Every call writes all the cells it reads, so nothing needs clearing.
// In host code `scratch` only names the symbol; kernels get the device address found by
// vegas_static_partials.
static __device__ __align__(256) double scratch[VEGAS_PARTIALS_MAX];

hipError_t vegas_static_partials(double** out)
{
    // device address of the current device's copy, looked up once per device with that
    // device current, then kept
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static double* ptr[MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double*>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

int vegas_blocks(int64_t n)
{
    int64_t b = (n + VB - 1) / VB;
    if (b > VEGAS_MAX_BLOCKS) b = VEGAS_MAX_BLOCKS;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_vegas(const VegasArgs& a, hipStream_t s)
{
    if (a.d > MAXD || a.nb > MAXNB || a.nb < 2) return hipErrorInvalidValue;
    // n = 0 still runs the accumulation: every block then writes zero partials
    if (a.d <= 8) hipLaunchKernelGGL(k_vegas_accumulate<8>, dim3(a.nblk), dim3(VB), 0, s, a);
    else hipLaunchKernelGGL(k_vegas_accumulate<MAXD>, dim3(a.nblk), dim3(VB), 0, s, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_vegas_reduce, dim3(2 + a.d * a.nb), dim3(64), 0, s, a);
    err = hipGetLastError();
    if (err != hipSuccess || !(a.update_edges || a.rng_counter)) return err;
    hipLaunchKernelGGL(k_vegas_update, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace mf
