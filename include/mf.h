/*
 * mf.h -- C ABI of the MI355X (gfx950) event-parallel matrix-element library.
 *
 * The library evaluates, for batches of Monte Carlo events, the hot path of
 * an event-parallel tree-level generator: phase-space sampling, the
 * spin/colour summed matrix element |M|^2, its derivative, and Vegas grid
 * adaptation.  It corresponds to the custom operator of Carrazza,
 * Cruz-Martinez, Palazzo, "Extending MadFlow: device-specific optimization"
 * (ICHEP 2022): a momentum tensor in, a matrix-element tensor out, launched
 * from a C++ host interface and wrapped for Python (sect. 2, Fig. 2); the
 * derivative the paper left out (sect. 2) is provided by
 * mf_matrix_element_vjp.  Monte Carlo integration is Vegas (sect. 1).
 *
 * Conventions for every entry point
 *  - All array arguments are DEVICE pointers owned by the caller (for
 *    example torch tensors); the library never frees them.  Argument structs
 *    (mf_params, mf_request) are host memory read during the call only.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    default stream).  The status return covers argument validation and
 *    launch errors only; mf_last_error() then gives a message (thread-local).
 *  - Layouts are structure-of-arrays with the event index fastest.
 *    Momenta: p[leg][component][event], component = (E, px, py, pz), legs in
 *    the order of the process (incoming first), FP64.
 *  - n = 0 is a valid no-op (returns MF_OK) except where stated; n above 2^36
 *    events per call or request is rejected (MF_ERR_INVALID_ARG).
 *  - Numerical trouble is not an error: NaN inputs give NaN outputs; an
 *    event whose massive phase-space rescaling does not converge gets
 *    weight 0 and is counted (mf_failures).
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MF_OK = 0,
    MF_ERR_INVALID_ARG = -1,  /* null pointer, negative size, unknown enum, ... */
    MF_ERR_UNSUPPORTED = -2,  /* valid request the library cannot serve */
    MF_ERR_HIP = -3,          /* HIP runtime error (message has the HIP error string) */
    MF_ERR_NO_MEMORY = -4     /* workspace allocation failed */
} mf_status;

/* Processes (legs in momentum-array order):
 *   MF_EE_MUMU : e-(in) e+(in) -> mu-(out) mu+(out), s-channel photon, massless
 *   MF_GG_TT   : g g -> t tbar
 *   MF_GG_TTG  : g g -> t tbar g
 *   MF_GG_TTGG : g g -> t tbar g g
 *   MF_GG_TTGGG: g g -> t tbar g g g (matrix element by the table-driven recursion, one
 *                wavefront per event; MF_FP64 and MF_FP32; no derivative, no persistent batch)
 *   MF_QQ_TT   : q(in) qbar(in) -> t tbar
 *   MF_QQ_TTG  : q qbar -> t tbar g
 *   MF_QQ_TTGG : q qbar -> t tbar g g
 *   MF_QG_TTQ  : q(in) g(in) -> t tbar q(out)
 *   MF_QG_TTQG : q g -> t tbar q g
 *                (q a massless light quark of one flavour; matrix elements from generated
 *                diagram code, one lane per event; MF_FP64 and MF_FP32; no derivative, no
 *                persistent batch)
 * The gg processes are the gluon-initiated channels of the paper's benchmarks
 * (pp -> t tbar (+ g, + g g); sect. 3, Table 1, Figs. 3 and 4), the qq and qg ones its
 * quark-initiated channels. */
typedef enum {
    MF_EE_MUMU = 0, MF_GG_TT = 1, MF_GG_TTG = 2, MF_GG_TTGG = 3, MF_GG_TTGGG = 4,
    MF_QQ_TT = 5, MF_QQ_TTG = 6, MF_QQ_TTGG = 7, MF_QG_TTQ = 8, MF_QG_TTQG = 9
} mf_process;

/* Arithmetic of the matrix element.
 *   MF_FP64           : everything in FP64; output f64.
 *   MF_FP32           : FP64 kinematics, FP32 complex amplitudes, FP32 colour sum; output f32.
 *   MF_FP32_MFMA_BF16 : as MF_FP32 with the colour contraction on BF16 matrix cores
 *                       (colour matrix exact in BF16, amplitudes split in three BF16
 *                       terms, FP32 accumulation); output f32.
 *   MF_FP32_MFMA_F32  : as MF_FP32 with the colour contraction on FP32 matrix cores. */
typedef enum { MF_FP64 = 0, MF_FP32 = 1, MF_FP32_MFMA_BF16 = 2, MF_FP32_MFMA_F32 = 3 } mf_precision;

/* Physics and generation-cut parameters (GeV units).  alpha is used by
 * MF_EE_MUMU only, m_t / alpha_s / cuts by the QCD processes.  Cuts apply to
 * the final-state light partons (gluons and the light quark): pT > pt_min,
 * |eta| < eta_max, and Delta R > dr_min between every pair of them. */
typedef struct {
    double sqrt_s, m_t, alpha_s, alpha, pt_min, eta_max, dr_min;
} mf_params;

/* One batch of events of one process.
 *   proc       an mf_process; reserved: set to 0;
 *   n          number of events (0 is a no-op);
 *   p          [n_ext][4][n] f64 momenta, layout as above (forward only; the
 *              derivative regenerates the momenta from x);
 *   me_out     [n] f64 (MF_FP64) or f32 (other precisions): spin- and colour-
 *              summed |M|^2 averaged over initial helicities/colours, including
 *              the 1/2 for identical final gluons.
 * VJP only:
 *   x          [d][n] f64 uniforms that generated the event (d = 3 n_out - 4),
 *              binned as in mf_phase_space (outside [0, 1): first or last bin),
 *   grad_me    [n] f64 incoming cotangent g,
 *   grad_x     [d][n] f64 out: g * d|M|^2/dx (through the Vegas map and phase space),
 *   grad_theta [n][2] f64 out: g * (d|M|^2/dm_t at fixed x, d|M|^2/dalpha_s). */
typedef struct {
    int32_t proc;
    int32_t reserved;
    int64_t n;
    const double* p;
    void* me_out;
    const double* x;
    const double* grad_me;
    double* grad_x;
    double* grad_theta;
} mf_request;

typedef struct mf_handle_s* mf_handle;

/* Create a handle bound to HIP device `device`; it owns workspace (Vegas
 * reduction partials, about 8.4 MB, the largest any call needs; the Newton
 * failure counter; the tile counter of persistent launches), all allocated
 * here, so no other call allocates, frees or synchronises the device.
 * One handle per thread; calls on one handle from several host threads must
 * be serialised by the caller.  The workspace is shared by the handle's calls:
 * mf_vegas_refine calls, and mf_matrix_element calls with several requests,
 * must not run concurrently on different streams with the same handle (order
 * them with events or use one handle per stream); on one stream they are
 * ordered by the stream.  Errors: MF_ERR_INVALID_ARG for a bad device or NULL
 * out, MF_ERR_NO_MEMORY if the workspace cannot be allocated. */
mf_status mf_create(int device, mf_handle* out);
mf_status mf_destroy(mf_handle h);

/* Text of the last error on this thread ("" if none). */
const char* mf_last_error(void);

/* Number of legs and of uniforms per event for a process (-1 if unknown). */
int mf_process_legs(int proc);
int mf_process_dims(int proc);

/* Launch configuration (what the autotuner sets):
 *   proc >= 0: threads per block for single-request launches of (proc,
 *     precision), 64..256 in steps of 64, 0 = library default.  The
 *     gg -> ttbar gg kernels always run one-wave blocks (their LDS is per wave);
 *     for them the value selects the event layout instead: in FP64, 128 (and 0,
 *     the default) = two lanes per event (colour orderings split in pairs
 *     related by swapping both the beams and the final gluons, currents and
 *     amplitudes exchanged within the pair), 256 = four lanes per event
 *     (orderings split by first gluon, currents shared within the quad),
 *     64 or 192 = one lane per event.  For gg -> ttbar ggg the value is the number of
 *     lanes that share an event: 16, 32 or 64 (0, the default: 64).
 *     proc < 0 leaves the per-process settings unchanged.
 *   batch_waves_per_cu >= 0: one-wave blocks per compute unit in each
 *     persistent launch (0, the default: as many as the process's kernel fits);
 *     < 0 leaves it unchanged.
 *   batch_persistent: 1 = the requests of a call are served by persistent
 *     launches, one per gg process class, each pulling tiles of one or more
 *     64-event waves from a queue (default); 0 = one launch per request;
 *     < 0 = unchanged.
 * Errors: MF_ERR_INVALID_ARG for out-of-range values. */
mf_status mf_set_launch(mf_handle h, int proc, int precision, int block, int batch_waves_per_cu,
                        int batch_persistent);

/* Number of Newton non-convergence events counted by the handle so far
 * (synchronises the handle's device). */
mf_status mf_failures(mf_handle h, uint64_t* count);

/* Tile of the persistent mixed-batch launch (mf_matrix_element with several requests;
 * the paper's study of launch shapes, sect. 3, Fig. 3): each pop of the work queue takes
 * `waves` 64-event waves of one request.  For MF_GG_TT and MF_GG_TTG only (gg -> t tbar g g
 * takes one wave per tile); waves in [1, 64], 0 restores the default (16 for MF_GG_TT, 4
 * for MF_GG_TTG).  Results do not depend on it.  Errors: MF_ERR_INVALID_ARG for another
 * process or waves outside [0, 64]. */
mf_status mf_set_batch_tile(mf_handle h, int proc, int waves);

/*
 * mf_phase_space -- the sampling steps of the path (sect. 1; sect. 3 for the
 * cuts): uniforms, Vegas map, RAMBO-on-diet phase space with massive
 * rescaling, generation cuts.
 *   x          [d][n] uniforms, or NULL to draw them from Philox4x32-10 with
 *              key = seed and counter = (offset + *offset_dev + event, dim/2);
 *              a value outside [0, 1) falls in the first or last Vegas bin
 *              (the map extrapolates linearly) and NaN in bin 0 with NaN
 *              momenta, so no caller value makes an edge read go out of bounds;
 *   offset_dev optional device pointer added to offset (lets a captured graph
 *              advance the stream between replays), may be NULL;
 *   edges      [d][nb+1] Vegas grid, or NULL for the identity map;
 *   p          [n_ext][4][n] out momenta (incoming legs included);
 *   w          [n] out phase-space weight (GeV^(2 n_out - 4));
 *   pass       [n] out cut mask (1 = passes) or NULL;
 *   bin_idx    [d][n] out Vegas bin of each uniform or NULL (needs nb >= 1);
 *   jac        [n] out Vegas Jacobian or NULL;
 *   x_out      [d][n] out copy of the uniforms used, or NULL.
 * Errors: MF_ERR_INVALID_ARG for a bad process, n < 0, NULL p or w, or
 * edges/bin_idx given with nb < 2 or nb > 64.
 */
mf_status mf_phase_space(mf_handle h, int proc, const mf_params* prm, int64_t n,
                         const double* x, uint64_t seed, uint64_t offset, const uint64_t* offset_dev,
                         const double* edges, int nb,
                         double* p, double* w, uint8_t* pass, int16_t* bin_idx, double* jac,
                         double* x_out, void* stream);

/*
 * mf_matrix_element -- the helicity-summed, colour-contracted tree-level |M|^2
 * of each event of each request (sect. 2: the matrix element the paper's
 * generated code evaluates per event).  With n_reqs > 1 and batch_persistent
 * set, the gg requests are served by one persistent launch per process class
 * (mf_set_launch); otherwise one launch per request.  MF_GG_TTGGG requests
 * always take a launch of their own (the table-driven recursion, one wavefront
 * per event; mf_set_launch's block sets its lanes per event).
 * Errors: MF_ERR_INVALID_ARG for n_reqs < 1, NULL reqs/prm, a bad process or
 * precision, n < 0, or NULL p / me_out with n > 0; MF_ERR_UNSUPPORTED for
 * the matrix-core precisions with MF_EE_MUMU or MF_GG_TTGGG.  Every error is
 * found before anything is launched.
 */
mf_status mf_matrix_element(mf_handle h, const mf_request* reqs, int n_reqs, int precision,
                            const mf_params* prm, void* stream);

/*
 * mf_matrix_element_vjp -- vector-Jacobian product of |M|^2 with
 * respect to the uniforms x (through the Vegas map `edges`, which may be NULL
 * for the identity, and the phase space) and to (m_t, alpha_s).  The paper's
 * operator has no derivative (sect. 2); this one is a reverse sweep over the
 * helicity/colour recursion that recomputes every helicity's currents instead
 * of storing them, with forward tangents over the d + 1 kinematic inputs (the
 * sweep's arithmetic is about four forward evaluations, whatever d, plus the
 * phase space and its tangents).  The
 * forward value is written to me_out when it is not NULL (f64 for MF_FP64,
 * f32 otherwise).  The requests of one process are served by one launch (a
 * grid of 64-event tiles over up to 32 requests); all requests share `edges`.
 * Errors: as mf_matrix_element, plus NULL x / grad_me / grad_x / grad_theta,
 * MF_ERR_UNSUPPORTED for MF_EE_MUMU, MF_GG_TTGGG and the quark-initiated
 * processes.
 */
mf_status mf_matrix_element_vjp(mf_handle h, const mf_request* reqs, int n_reqs, int precision,
                                const mf_params* prm, const double* edges, int nb, void* stream);

/*
 * mf_vegas_refine -- the Vegas step (sect. 1): forms F = flux * w * jac * me (events
 * that pass the cuts and have a weight that is neither 0 nor NaN; 0 otherwise) with
 * flux = (hbar c)^2 / (2 s) in pb GeV^2 / GeV^2 (so F is in pb), reduces
 * acc[0] = sum F, acc[1] = sum F^2, acc[2 + k*nb + i] = sum of F^2 over events
 * in bin i of dimension k (deterministic order).  flags:
 *   MF_VEGAS_ACCUMULATE  add this batch's sums to acc instead of overwriting it
 *                        (several batches per Vegas iteration);
 *   MF_VEGAS_REFINE      then refine `edges` in place from acc (Lepage:
 *                        smoothing, damping exponent alpha, rebinning).
 * If rng_counter is not NULL, *rng_counter += n on the device.
 *   w, me      [n] required (me is f32 when me_f32 != 0); jac, pass optional;
 *   bin_idx    [d][n] required; F [n] optional output; acc [2 + d*nb] out.
 * Errors: MF_ERR_INVALID_ARG for d < 1 or d > 16, nb < 2 or nb > 64, n < 0,
 * or a NULL required pointer.  It uses the handle's workspace (allocated by
 * mf_create) and allocates nothing.  F = 0 exactly for an event that fails the
 * cuts or has w = 0 or NaN (a failed phase-space solve, NaN uniforms), whatever its
 * |M|^2; a negative weight counts as it is; a dimension whose histogram holds a
 * non-finite value keeps its grid.
 */
enum { MF_VEGAS_REFINE = 1, MF_VEGAS_ACCUMULATE = 2 };

mf_status mf_vegas_refine(mf_handle h, const mf_params* prm, int64_t n, int d, int nb, double alpha,
                          const double* w, const double* jac, const void* me, int me_f32,
                          const uint8_t* pass, const int16_t* bin_idx, double* F, double* acc,
                          double* edges, int flags, uint64_t* rng_counter, void* stream);

/*
 * mf_vegas_refine_noalloc -- for callers that cannot allocate device memory
 * (code under HIP stream capture, tight serving loops, harnesses that forbid
 * allocation): mf_vegas_refine without a handle and without any allocation.
 * Same arguments, results and errors as mf_vegas_refine (bit-identical
 * results), on the CURRENT device, which `stream` must belong to.  The block
 * partials live in a static device array of the library: 1024 x 1026 doubles
 * (8.4 MB), one copy per device, held until the process ends; every valid
 * (n, d, nb) fits, and a size that would not is rejected with
 * MF_ERR_INVALID_ARG.  All calls on one device share that array: calls that
 * overlap on one GPU (several streams or host threads) race and give wrong
 * sums; order them.  MF_ERR_HIP if the array's address cannot be found.
 */
mf_status mf_vegas_refine_noalloc(const mf_params* prm, int64_t n, int d, int nb, double alpha,
                                  const double* w, const double* jac, const void* me, int me_f32,
                                  const uint8_t* pass, const int16_t* bin_idx, double* F, double* acc,
                                  double* edges, int flags, uint64_t* rng_counter, void* stream);

/*
 * Hadronic events (the paper's workload is pp -> t tbar + jets; sect. 3, Table 1): the
 * partonic processes weighted with parton densities interpolated from a grid (the step
 * before the matrix element, sect. 1).  Built for the gluon-gluon channel.
 *
 * mf_pdf_grid: a tabulated density, device arrays owned by the caller:
 *   log_x [nx], log_q2 [nq]  increasing nodes in ln x and ln Q^2 (nx, nq >= 2);
 *   xf    [nq][nx]           x f(x, Q^2) at the nodes.
 * Interpolation: cubic Hermite in ln x (per Q^2 node), then in ln Q^2 over the nodes
 * j-1 .. j+2 around the cell; node slopes are the mean of the adjacent secant slopes
 * (one secant at the grid ends); points outside the grid take the edge values.
 */
typedef struct {
    int32_t nx, nq;
    const double* log_x;
    const double* log_q2;
    const double* xf;
} mf_pdf_grid;

/* x f(x, Q^2) for n points: x [n], q2 [n] (GeV^2), xf_out [n].
 * Errors: MF_ERR_INVALID_ARG for a NULL or too small grid, n outside [0, 2^36], NULL arrays. */
mf_status mf_pdf_eval(mf_handle h, const mf_pdf_grid* g, int64_t n, const double* x, const double* q2,
                      double* xf_out, void* stream);

/*
 * mf_phase_space_pp -- events of one parton channel of pp collisions at sqrt_S (GeV):
 * parton 1 from beam 1 (+z) with density grid g, parton 2 from beam 2 with density
 * grid g_b (NULL: g as well); for example gg -> t tbar (+ g ...) with the gluon for
 * both, q qbar -> t tbar (+ g ...) with a quark and an antiquark density, q g -> t tbar q
 * (+ g) with a quark and the gluon.  As mf_phase_space with d + 2 uniforms per event,
 * (u_tau, u_y, then the partonic d):
 *   tau = tau0^(1 - u_tau), tau0 = (2 m_t)^2 / S;  y = (u_y - 1/2) ln(1/tau);
 *   x1 = sqrt(tau) e^y, x2 = sqrt(tau) e^-y, s_hat = tau S;
 * the partonic event is generated in its c.m. frame at sqrt(s_hat) (p: parton 1 along +z,
 * E = sqrt(s_hat)/2); the cuts are applied in the lab frame (light-parton pseudorapidities + y);
 *   w = tau ln(1/tau0) ln(1/tau) f_a(x1, m_t^2) f_b(x2, m_t^2) W(s_hat) S / s_hat,
 * so that mf_vegas_refine called with sqrt_s = sqrt_S forms the hadronic integrand
 * (hbar c)^2 / (2 s_hat) J f f W |M|^2 Theta.  edges, bin_idx, x_out have d + 2 rows;
 * x12 [2][n] (x1, x2) optional.  The factorisation scale is m_t.
 * Errors: MF_ERR_INVALID_ARG for MF_EE_MUMU, NULL params, a bad grid, n outside
 * [0, 2^36], NULL p or w, nb outside [2, 64] with edges or bin_idx, unless
 * 0 < 2 m_t < sqrt_S.
 */
mf_status mf_phase_space_pp(mf_handle h, int proc, const mf_params* prm, double sqrt_S, const mf_pdf_grid* g,
                            const mf_pdf_grid* g_b, int64_t n, const double* x, uint64_t seed, uint64_t offset, const uint64_t* offset_dev,
                            const double* edges, int nb, double* p, double* w, uint8_t* pass, int16_t* bin_idx,
                            double* jac, double* x_out, double* x12, void* stream);

/*
 * mf_unweight -- unit-weight event sample from weighted events (hit-or-miss;
 * the event generators of sect. 1): event e is kept iff u_e * w_max < w_e, with
 * u_e the Philox4x32-10 uniform of key = seed, counter = (offset + e, 0, 1) (a
 * stream apart from the phase-space uniforms) and w_max the reference maximum:
 * `w_max` if > 0, else the largest weight of the batch.  Non-positive and NaN
 * weights are never kept.  Kept events are written in increasing event order:
 *   w          [n] weights (for example the F of mf_vegas_refine);
 *   p, n_ext   [n_ext][4][n] momenta to copy for the kept events, or NULL / 0;
 *   cap        capacity of idx, fac and p_out;
 *   idx        [cap] out: kept event indices;
 *   fac        [cap] out: weight factors (w_e / w_max for w_e > w_max, else 1), or NULL;
 *   p_out      [n_ext][4][cap] out: momenta of the kept events, or NULL;
 *   count      device uint64 out: number of kept events (all of them, also when
 *              it exceeds cap: only the first cap are written);
 *   w_max_out  device double out: the reference maximum used, or NULL.
 * Uses the handle's workspace (ordered with the handle's other calls on one
 * stream).  Errors: MF_ERR_INVALID_ARG for n outside [0, 2^36], cap < 0, NULL
 * count, NULL w with n > 0, NULL idx with cap > 0, p_out without p or with n_ext
 * outside [1, 8], NaN w_max.
 */
mf_status mf_unweight(mf_handle h, int64_t n, const double* w, double w_max, uint64_t seed, uint64_t offset,
                      int n_ext, const double* p, int64_t cap, int64_t* idx, double* fac, double* p_out,
                      uint64_t* count, double* w_max_out, void* stream);

/*
 * Graph capture of a sequence of calls (a Vegas iteration: phase space,
 * matrix elements, derivatives, Vegas accumulation and refinement; sect. 1),
 * replayed later with one launch and no host work in between.
 *   mf_graph_begin   starts capturing the work enqueued on `stream` (not the
 *                    default stream) by this thread;
 *   mf_graph_end     ends the capture and instantiates it; *out owns the
 *                    executable graph (free it with mf_graph_destroy);
 *   mf_graph_launch  replays it on `stream`.
 * Every library call is capturable: none allocates, frees or synchronises
 * after mf_create, and counters are reset by kernels, not by memsets.  A
 * replay reads and writes the buffers the captured calls named, with their
 * contents at replay time (a device-side Philox offset, mf_phase_space's
 * offset_dev, advances the random numbers between replays).
 * Errors: MF_ERR_INVALID_ARG for NULL arguments; MF_ERR_HIP for a capture
 * error (for example a call that synchronised during the capture).
 */
typedef struct mf_graph_s* mf_graph;
mf_status mf_graph_begin(mf_handle h, void* stream);
mf_status mf_graph_end(mf_handle h, void* stream, mf_graph* out);
mf_status mf_graph_launch(mf_graph g, void* stream);
mf_status mf_graph_destroy(mf_graph g);

/* 1 if the library serves matrix elements at `precision`, else 0. */
int mf_precision_available(int precision);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
