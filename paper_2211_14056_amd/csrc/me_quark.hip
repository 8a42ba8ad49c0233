// q qbar -> t tbar (+g, +gg) and q g -> t tbar q (+g): one lane per event, FP64 or FP32.
//
// The quark-initiated subprocesses of the paper's pp -> t tbar (+ jets) workload (sect. 3,
// Table 1).  The bodies are generated per process (gen/quark_lines.py): every Feynman diagram,
// colour-flow amplitudes over two generator strings and their colour matrix; the event loop
// (me_quark.h) forms the kinematics once and loops over the helicity configurations.
#include "internal.h"
#include "me_common.h"

#include "generated/me_qq_tt.inc"
#include "generated/me_qq_ttg.inc"
#include "generated/me_qq_ttgg.inc"
#include "generated/me_qg_ttq.inc"
#include "generated/me_qg_ttqg.inc"
#include "me_quark.h"

namespace mf {
namespace {

template <class T, typename R>
__global__ __launch_bounds__(256) void k_me_quark(const double* __restrict__ p, int64_t n, R* __restrict__ out,
                                                  double mt, double coupling)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double pe[T::NEXT][4];
#pragma unroll
    for (int l = 0; l < T::NEXT; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) pe[l][c] = p[(l * 4 + c) * n + e];
    out[e] = R(quark_event<T, R>(pe, mt) * coupling);
}

template <class T, typename R>
hipError_t launch_t(const MeJob& j, double mt, double coupling, int block, hipStream_t s)
{
    const unsigned grid = (unsigned)((j.n + block - 1) / block);
    hipLaunchKernelGGL((k_me_quark<T, R>), dim3(grid), dim3(block), 0, s, j.p, j.n, static_cast<R*>(j.out), mt,
                       coupling);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_r(const MeJob& j, double mt, double coupling, int block, hipStream_t s)
{
    switch (j.proc) {
    case QQ_TT: return launch_t<QL_qq_tt, R>(j, mt, coupling, block, s);
    case QQ_TTG: return launch_t<QL_qq_ttg, R>(j, mt, coupling, block, s);
    case QQ_TTGG: return launch_t<QL_qq_ttgg, R>(j, mt, coupling, block, s);
    case QG_TTQ: return launch_t<QL_qg_ttq, R>(j, mt, coupling, block, s);
    case QG_TTQG: return launch_t<QL_qg_ttqg, R>(j, mt, coupling, block, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_quark(const MeJob& j, int precision, double mt, double coupling, int block, hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    if (block <= 0) block = 256;
    if (precision == 0) return launch_r<double>(j, mt, coupling, block, s);
    if (precision == 1) return launch_r<float>(j, mt, coupling, block, s);
    return hipErrorInvalidValue;
}

}  // namespace mf
