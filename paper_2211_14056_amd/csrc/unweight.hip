// Unweighting: from weighted events to a sample of unit-weight events
// (hit-or-miss acceptance; the event generators the paper serves, sect. 1).
//
// Event e is kept iff u_e * w_max < w_e (FP64), u_e the Philox4x32-10 uniform
// of counter (e_lo, e_hi, 0, 1) and key = seed; non-positive and NaN weights
// are never kept; a kept weight above w_max carries the factor w_e / w_max.
// Kept events are written in increasing event order (stream compaction with a
// fixed partition, so the output does not depend on scheduling):
//  1. k_uw_max      w_max = the largest positive weight (unless the caller gives
//                   one): per-wave maxima, one atomicMax per wave on the bit
//                   pattern (positive doubles order like their bits);
//  2. k_uw_count    block b owns the contiguous event range [b L, (b+1) L) and
//                   counts its kept events;
//  3. k_uw_scan     one workgroup turns the block counts into block offsets;
//  4. k_uw_write    each block recounts its range chunk by chunk (ballot and
//                   popcount give each lane its rank) and writes index, factor
//                   and momenta of its kept events from its offset on.
// The uniforms are recomputed in steps 2 and 4 (ten Philox rounds) rather than
// stored.  Workspace: the handle's Vegas partials (a word for w_max, 2 x 1024
// block counts and offsets).
#include "internal.h"
#include "rng.h"

namespace mf {
namespace {

constexpr int UB = 256;                 // threads per block
constexpr int UMAX_BLOCKS = 1024;

__device__ __forceinline__ double acceptance_uniform(uint64_t seed, uint64_t ev)
{
    uint32_t c[4] = {(uint32_t)ev, (uint32_t)(ev >> 32), 0u, 1u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return u64_to_unit(((uint64_t)c[1] << 32) | c[0]);
}

__device__ __forceinline__ bool kept(const UnweightArgs& a, int64_t e, double wmax)
{
    const double w = a.w[e];
    return w > 0.0 && acceptance_uniform(a.seed, a.offset + (uint64_t)e) * wmax < w;
}

__global__ void k_uw_init(UnweightArgs a)
{
    // the reference maximum: the caller's, or 0 before the batch maximum is taken
    unsigned long long* wm = reinterpret_cast<unsigned long long*>(a.work);
    *wm = a.w_max > 0.0 ? __double_as_longlong(a.w_max) : 0ull;
}

__global__ __launch_bounds__(UB) void k_uw_max(UnweightArgs a)
{
    double m = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * UB + threadIdx.x; e < a.n; e += (int64_t)gridDim.x * UB) {
        const double w = a.w[e];
        if (w > m) m = w;                   // NaN and non-positive weights never enter
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s));
    if ((threadIdx.x & 63) == 0 && m > 0.0)
        atomicMax(reinterpret_cast<unsigned long long*>(a.work), (unsigned long long)__double_as_longlong(m));
}

__device__ __forceinline__ double ref_max(const UnweightArgs& a)
{
    return __longlong_as_double((long long)*reinterpret_cast<const unsigned long long*>(a.work));
}

__device__ __forceinline__ void block_range(const UnweightArgs& a, int64_t& lo, int64_t& hi)
{
    const int64_t L = (a.n + gridDim.x - 1) / gridDim.x;
    lo = (int64_t)blockIdx.x * L;
    hi = lo + L < a.n ? lo + L : a.n;
}

__global__ __launch_bounds__(UB) void k_uw_count(UnweightArgs a)
{
    __shared__ unsigned long long wsum[UB / 64];
    const double wmax = ref_max(a);
    int64_t lo, hi;
    block_range(a, lo, hi);
    unsigned long long c = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += UB) c += kept(a, e, wmax) ? 1 : 0;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) c += __shfl_xor(c, s);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < UB / 64; ++w) t += wsum[w];
        reinterpret_cast<unsigned long long*>(a.work)[1 + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(UMAX_BLOCKS) void k_uw_scan(UnweightArgs a, int nblk)
{
    // exclusive scan of the block counts (one value per thread, Hillis-Steele in LDS)
    __shared__ unsigned long long v[UMAX_BLOCKS];
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(a.work) + 1;
    unsigned long long* off = cnt + UMAX_BLOCKS;
    const int t = threadIdx.x;
    const unsigned long long mine = t < nblk ? cnt[t] : 0ull;
    v[t] = mine;
    __syncthreads();
    for (int s = 1; s < UMAX_BLOCKS; s <<= 1) {
        const unsigned long long add = t >= s ? v[t - s] : 0ull;
        __syncthreads();
        v[t] += add;
        __syncthreads();
    }
    if (t < nblk) off[t] = v[t] - mine;
    if (t == UMAX_BLOCKS - 1) {
        *a.count = v[t];
        if (a.w_max_out) *a.w_max_out = ref_max(a);
    }
}

__global__ __launch_bounds__(UB) void k_uw_write(UnweightArgs a)
{
    __shared__ unsigned long long wtot[UB / 64];
    const double wmax = ref_max(a);
    const unsigned long long* off = reinterpret_cast<const unsigned long long*>(a.work) + 1 + UMAX_BLOCKS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t lo, hi;
    block_range(a, lo, hi);
    unsigned long long base = off[blockIdx.x];
    for (int64_t c0 = lo; c0 < hi; c0 += UB) {
        const int64_t e = c0 + threadIdx.x;
        const bool k = e < hi && kept(a, e, wmax);
        const unsigned long long mask = __ballot(k);
        const unsigned long long below = lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
        if (lane == 0) wtot[wv] = (unsigned long long)__popcll(mask);
        __syncthreads();
        unsigned long long before = 0, total = 0;
        for (int w = 0; w < UB / 64; ++w) {
            before += w < wv ? wtot[w] : 0ull;
            total += wtot[w];
        }
        if (k) {
            const unsigned long long pos = base + before + (unsigned long long)__popcll(below);
            if (pos < (unsigned long long)a.cap) {
                const double w = a.w[e];
                a.idx[pos] = e;
                if (a.fac) a.fac[pos] = w > wmax ? w / wmax : 1.0;
                if (a.p_out)
                    for (int l = 0; l < a.n_ext; ++l)
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            a.p_out[(int64_t)(l * 4 + c) * a.cap + pos] = a.p[(int64_t)(l * 4 + c) * a.n + e];
            }
        }
        base += total;
        __syncthreads();                    // wtot is rewritten by the next chunk
    }
}

}  // namespace

hipError_t launch_unweight(const UnweightArgs& a, hipStream_t s)
{
    const int64_t chunks = (a.n + UB - 1) / UB;
    const int nblk = (int)(chunks < UMAX_BLOCKS ? (chunks < 1 ? 1 : chunks) : UMAX_BLOCKS);
    hipLaunchKernelGGL(k_uw_init, dim3(1), dim3(1), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!(a.w_max > 0.0) && a.n > 0) {
        hipLaunchKernelGGL(k_uw_max, dim3(nblk), dim3(UB), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_uw_count, dim3(nblk), dim3(UB), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_uw_scan, dim3(1), dim3(UMAX_BLOCKS), 0, s, a, nblk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_uw_write, dim3(nblk), dim3(UB), 0, s, a);
    return hipGetLastError();
}

}  // namespace mf
