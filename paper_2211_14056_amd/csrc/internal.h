// Internal launch interface between the C-ABI layer (mf_api.cpp) and the
// kernel translation units.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

enum Proc {
    EE_MUMU = 0, GG_TT = 1, GG_TTG = 2, GG_TTGG = 3, GG_TTGGG = 4,
    QQ_TT = 5, QQ_TTG = 6, QQ_TTGG = 7, QG_TTQ = 8, QG_TTQG = 9, NPROC = 10
};

inline int n_ext(int proc)
{
    switch (proc) {
    case GG_TTG: case QQ_TTG: case QG_TTQ: return 5;
    case GG_TTGG: case QQ_TTGG: case QG_TTQG: return 6;
    case GG_TTGGG: return 7;
    default: return 4;
    }
}
// processes with two quark lines (the generated diagram kernels of me_quark.hip)
inline bool quark_proc(int proc) { return proc >= QQ_TT && proc <= QG_TTQG; }
inline int n_out(int proc) { return n_ext(proc) - 2; }
inline int dims(int proc) { return 3 * n_out(proc) - 4; }
inline int n_gluons(int proc) { return proc == EE_MUMU ? 0 : n_ext(proc) - 2; }

struct PsArgs {
    int64_t n;
    int proc, nb;
    const double* x;            // [d][n] or null (generate)
    uint64_t seed, offset;
    const uint64_t* offset_dev; // optional device-side offset added to `offset`
    const double* edges;        // [d][nb+1] or null (identity map)
    double sqrt_s, m_out[5];     // final-state masses, one per outgoing leg (up to 5)
    double pt_min, eta_max, dr_min;
    double* p;                  // [n_ext][4][n]
    double* w;                  // [n]
    uint8_t* pass;              // [n] or null
    int16_t* bin_idx;           // [d][n] or null
    double* jac;                // [n] or null
    double* x_out;              // [d][n] or null
    unsigned long long* fail_count;   // device counter of Newton failures
};

hipError_t launch_phase_space(const PsArgs& a, hipStream_t s);

struct MeJob {
    int proc;
    int64_t n;
    const double* p;   // [n_ext][4][n]
    void* out;         // [n] f64 or f32
};

// precision: 0 = FP64, 1 = FP32 (VALU colour), 2 = FP32 amplitudes + BF16 MFMA colour,
//            3 = FP32 amplitudes + FP32 MFMA colour
hipError_t launch_matrix_element(const MeJob& j, int precision, double mt, double alpha_s,
                                 double alpha, int block, hipStream_t s);
bool precision_available(int precision);
// precisions 2 and 3 (matrix-core colour contraction), gg processes only;
// `coupling` = (4 pi alpha_s)^k
hipError_t launch_matrix_element_mfma(const MeJob& j, int precision, double mt, double coupling, int block,
                                      hipStream_t s);
// g g -> t tbar g g in FP64 with four lanes per event; `coupling` = (4 pi alpha_s)^4
hipError_t launch_ttgg_quad(const MeJob& j, double mt, double coupling, hipStream_t s);
// g g -> t tbar g g g by the table-driven recursion, lanes_per_event in {16, 32, 64}
// (0: 64); precision 0 = FP64, 1 = FP32 (FP64 kinematics, FP32 recursion and colour sum)
hipError_t launch_quark(const MeJob& j, int precision, double mt, double coupling, int block, hipStream_t s);
hipError_t launch_ttggg(const MeJob& j, int precision, double mt, double coupling, int lanes_per_event,
                        hipStream_t s);
// g g -> t tbar g g in FP64 with two lanes per event (the default layout)
hipError_t launch_ttgg_pair(const MeJob& j, double mt, double coupling, hipStream_t s);
// launch-configuration values of mf_set_launch that select the layout of g g -> t tbar g g
// in FP64: two lanes per event (also 0, the default), four lanes per event; other values
// select one lane per event
constexpr int TTGG_PAIR_LAYOUT = 128;
constexpr int TTGG_QUAD_LAYOUT = 256;

constexpr int MAX_BATCH = 64;

struct BatchReq {
    int proc;
    int64_t n;
    const double* p;
    void* out;
    int64_t tile_begin;     // first tile of this request (64 * chunk events per tile)
};

// 64-event waves per tile of the persistent launch (the default; mf_set_batch_tile changes it
// for gg -> ttbar and gg -> ttbar g): cheap processes take several per queue pop, so the
// queue's atomic is not on the critical path
constexpr int batch_chunk(int proc) { return proc == GG_TT ? 16 : proc == GG_TTG ? 4 : 1; }
constexpr int BATCH_CHUNK_MAX = 64;

struct BatchArgs {
    BatchReq req[MAX_BATCH];
    int nreq;
    int64_t ntiles;
    unsigned* counter;      // device tile counter (reset by the launch)
    double mt;
    double coupling[4];     // per process: alpha (e+e-) or (4 pi alpha_s)^k
    int chunk[4];           // per process: 64-event waves per tile (gg -> ttbar gg: always 1)
};

// One persistent launch over requests of one gg process; precision as for
// launch_matrix_element; waves_per_cu one-wave blocks per compute unit
// (<= 0: as many as fit).
hipError_t launch_batch(const BatchArgs& a, int precision, int waves_per_cu, int n_cu, hipStream_t s);

struct VjpJob {
    int proc;
    int64_t n;
    const double* x;            // [d][n]
    const double* grad_me;      // [n]
    double* grad_x;             // [d][n]
    double* grad_theta;         // [n][2]
    void* me_out;               // [n] or null
    int me_f32;
    const double* edges;        // [d][nb+1] or null
    int nb;
    double sqrt_s, mt, alpha_s, coupling;
};

// Derivative requests of one process in one launch: a grid of 64-event
// tiles over the requests (request r owns tiles tile_begin .. tile_begin +
// ceil(n / 64) - 1).  The per-request fields of `job` (n, x, grad_me, grad_x,
// grad_theta, me_out) are ignored; the shared ones are used.
struct VjpReq {
    int64_t n;
    const double* x;
    const double* grad_me;
    double* grad_x;
    double* grad_theta;
    void* me_out;
    int64_t tile_begin;
};
constexpr int VJP_MAX_BATCH = 32;
struct VjpBatchArgs {
    VjpJob job;
    VjpReq req[VJP_MAX_BATCH];
    int nreq;
    int64_t ntiles;
};
static_assert(sizeof(VjpBatchArgs) <= 4096, "kernel arguments");
// precision 0: FP64 recursion; otherwise FP32 recursion (kinematics FP64)
hipError_t launch_vjp_batch(const VjpBatchArgs& a, int precision, hipStream_t s);

struct VegasArgs {
    int64_t n;
    int d, nb;
    double alpha, flux;         // flux = conversion / (2 s)
    const double* w;
    const double* jac;          // may be null
    const void* me;
    int me_f32;
    const uint8_t* pass;        // may be null
    const int16_t* bin_idx;
    double* F;                  // may be null
    double* partials;           // workspace [nblk][2 + d*nb]
    int nblk;
    double* acc;                // [2 + d*nb]
    double* edges;              // [d][nb+1]
    int update_edges;
    int accumulate;             // acc += batch sums instead of acc = batch sums
    uint64_t* rng_counter;      // may be null
};

// tabulated parton density (device arrays): x f at nodes equally or unequally spaced in
// ln x and ln Q^2
struct PdfGrid {
    int nx, nq;
    const double* lx;      // [nx] ln x nodes, increasing
    const double* lq;      // [nq] ln Q^2 nodes, increasing
    const double* v;       // [nq][nx] x f at the nodes
};

// hadronic (gluon-gluon) events; the uniforms are (u_tau, u_y, partonic ...)
struct PpArgs {
    int64_t n;
    int nb;
    const double* x;            // [d + 2][n] or null (generate)
    uint64_t seed, offset;
    const uint64_t* offset_dev;
    const double* edges;        // [d + 2][nb + 1] or null
    double S, tau0, mu2;        // collider energy squared, threshold tau, factorisation scale squared
    double m_out[5];             // final-state masses, one per outgoing leg (up to 5)
    double pt_min, eta_max, dr_min;
    PdfGrid grid, grid_b;       // densities of parton 1 (beam 1) and parton 2 (beam 2)
    double* p;                  // [n_ext][4][n] partonic c.m. frame
    double* w;                  // [n]
    uint8_t* pass;
    int16_t* bin_idx;           // [d + 2][n] or null
    double* jac;
    double* x_out;              // [d + 2][n] or null
    double* x12;                // [2][n] or null: x1, x2
    unsigned long long* fail_count;
};
hipError_t launch_phase_space_pp(const PpArgs& a, int n_out, hipStream_t s);
hipError_t launch_pdf_eval(const PdfGrid& g, int64_t n, const double* x, const double* q2, double* out,
                           hipStream_t s);

struct UnweightArgs {
    int64_t n;
    const double* w;            // [n] event weights
    double w_max;               // reference maximum (> 0), or <= 0: the batch maximum
    uint64_t seed, offset;      // acceptance stream: counter (offset + e, 0, 1)
    int n_ext;                  // legs of p / p_out (0: no momenta)
    const double* p;            // [n_ext][4][n] or null
    int64_t cap;                // capacity of idx / fac / p_out
    int64_t* idx;               // [cap] kept event indices, increasing
    double* fac;                // [cap] weight factors, or null
    double* p_out;              // [n_ext][4][cap] momenta of the kept events, or null
    unsigned long long* count;  // device: number of kept events (may exceed cap)
    double* w_max_out;          // device: the reference maximum used, or null
    double* work;               // workspace (>= 2049 words)
};
hipError_t launch_unweight(const UnweightArgs& a, hipStream_t s);

int vegas_blocks(int64_t n);
// largest workspace of one Vegas call: at most VEGAS_MAX_BLOCKS blocks, each writing
// 2 + d * nb <= 2 + 8 * 64 partial sums
constexpr int VEGAS_MAX_BLOCKS = 1024;
constexpr int VEGAS_MAX_D = 16;
constexpr int VEGAS_MAX_CELLS = 2 + VEGAS_MAX_D * 64;
constexpr size_t VEGAS_PARTIALS_MAX = (size_t)VEGAS_MAX_BLOCKS * VEGAS_MAX_CELLS;
hipError_t launch_vegas(const VegasArgs& a, hipStream_t s);
// device address of the library's static block-partials array (VEGAS_PARTIALS_MAX
// doubles) on the current device
hipError_t vegas_static_partials(double** out);

}  // namespace mf
