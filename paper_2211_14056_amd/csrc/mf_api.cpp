// C-ABI layer: argument validation, workspace ownership, kernel launches.
// The public contract is documented in include/mf.h.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/mf.h"
#include "internal.h"

namespace {

thread_local std::string g_err;

mf_status fail(mf_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

mf_status hip_fail(hipError_t e, const char* where)
{
    return fail(MF_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool valid_proc(int p) { return p >= MF_EE_MUMU && p <= MF_QG_TTQG; }

// largest batch a call accepts: keeps every launch grid within 32 bits
constexpr int64_t kMaxEvents = int64_t(1) << 36;

}  // namespace

struct mf_handle_s {
    int device = 0;
    int n_cu = 256;
    double* partials = nullptr;        // Vegas block partials, the largest size any call needs
    unsigned long long* fail_dev = nullptr;
    unsigned* tile_counter = nullptr;  // persistent-batch work queue
    // launch configuration (set by mf_set_launch / the autotuner)
    int block[mf::NPROC][4];           // [process][precision] threads per block, 0 = default
    int batch_waves_per_cu = 0;        // persistent grid = waves_per_cu * n_cu one-wave blocks (0: as many as fit)
    int batch_persistent = 1;          // 0 = one launch per request instead
    int batch_chunk[4] = {1, mf::batch_chunk(mf::GG_TT), mf::batch_chunk(mf::GG_TTG), 1};   // waves per tile
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

const char* mf_last_error(void) { return g_err.c_str(); }

int mf_process_legs(int proc) { return valid_proc(proc) ? mf::n_ext(proc) : -1; }
int mf_process_dims(int proc) { return valid_proc(proc) ? mf::dims(proc) : -1; }

int mf_precision_available(int precision) { return mf::precision_available(precision) ? 1 : 0; }

mf_status mf_create(int device, mf_handle* out)
{
    g_err.clear();
    if (!out) return fail(MF_ERR_INVALID_ARG, "mf_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "mf_create: hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(MF_ERR_INVALID_ARG, "mf_create: device %d out of range (%d devices)", device, count);
    DeviceGuard g(device);
    mf_handle h = new mf_handle_s;
    h->device = device;
    for (auto& r : h->block)
        for (int& b : r) b = 0;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            h->n_cu = prop.multiProcessorCount;
    }
    // all workspace is allocated here, once, at the largest size any call needs, so that
    // no later call allocates, frees or synchronises (a captured graph keeps its pointers)
    e = hipMalloc(&h->fail_dev, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&h->tile_counter, sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc(&h->partials, mf::VEGAS_PARTIALS_MAX * sizeof(double));
    if (e != hipSuccess) {
        if (h->fail_dev) hipFree(h->fail_dev);
        if (h->tile_counter) hipFree(h->tile_counter);
        delete h;
        return fail(MF_ERR_NO_MEMORY, "mf_create: cannot allocate workspace");
    }
    e = hipMemset(h->fail_dev, 0, sizeof(unsigned long long));
    if (e != hipSuccess) {
        hipFree(h->fail_dev);
        hipFree(h->tile_counter);
        hipFree(h->partials);
        delete h;
        return hip_fail(e, "mf_create: hipMemset");
    }
    *out = h;
    return MF_OK;
}

mf_status mf_destroy(mf_handle h)
{
    g_err.clear();
    if (!h) return MF_OK;
    DeviceGuard g(h->device);
    hipDeviceSynchronize();
    if (h->partials) hipFree(h->partials);
    if (h->fail_dev) hipFree(h->fail_dev);
    if (h->tile_counter) hipFree(h->tile_counter);
    delete h;
    return MF_OK;
}

mf_status mf_set_launch(mf_handle h, int proc, int precision, int block, int batch_waves_per_cu,
                        int batch_persistent)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_set_launch: NULL handle");
    if (proc >= 0) {
        if (!valid_proc(proc) || precision < MF_FP64 || precision > MF_FP32_MFMA_F32)
            return fail(MF_ERR_INVALID_ARG, "mf_set_launch: bad process or precision");
        if (proc == MF_GG_TTGGG) {
            if (block != 0 && block != 16 && block != 32 && block != 64)
                return fail(MF_ERR_INVALID_ARG, "mf_set_launch: lanes per event must be 16, 32 or 64 (0 = default)");
        } else if (block != 0 && (block < 64 || block > 256 || block % 64)) {
            return fail(MF_ERR_INVALID_ARG, "mf_set_launch: block must be 64, 128, 192 or 256 (0 = default)");
        }
        h->block[proc][precision] = block;
    }
    if (batch_waves_per_cu >= 0) {
        if (batch_waves_per_cu > 16)
            return fail(MF_ERR_INVALID_ARG, "mf_set_launch: batch_waves_per_cu must be in [0, 16]");
        h->batch_waves_per_cu = batch_waves_per_cu;
    }
    if (batch_persistent >= 0) h->batch_persistent = batch_persistent ? 1 : 0;
    return MF_OK;
}

mf_status mf_set_batch_tile(mf_handle h, int proc, int waves)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_set_batch_tile: NULL handle");
    if (proc != MF_GG_TT && proc != MF_GG_TTG)
        return fail(MF_ERR_INVALID_ARG, "mf_set_batch_tile: process %d has a fixed tile", proc);
    if (waves < 0 || waves > mf::BATCH_CHUNK_MAX)
        return fail(MF_ERR_INVALID_ARG, "mf_set_batch_tile: waves = %d outside [0, %d]", waves, mf::BATCH_CHUNK_MAX);
    h->batch_chunk[proc] = waves ? waves : mf::batch_chunk(proc);
    return MF_OK;
}

mf_status mf_failures(mf_handle h, uint64_t* count)
{
    g_err.clear();
    if (!h || !count) return fail(MF_ERR_INVALID_ARG, "mf_failures: NULL argument");
    DeviceGuard g(h->device);
    unsigned long long v = 0;
    hipError_t e = hipMemcpy(&v, h->fail_dev, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "mf_failures");
    *count = v;
    return MF_OK;
}

mf_status mf_phase_space(mf_handle h, int proc, const mf_params* prm, int64_t n,
                         const double* x, uint64_t seed, uint64_t offset, const uint64_t* offset_dev,
                         const double* edges, int nb,
                         double* p, double* w, uint8_t* pass, int16_t* bin_idx, double* jac,
                         double* x_out, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_phase_space: NULL handle");
    if (!valid_proc(proc)) return fail(MF_ERR_INVALID_ARG, "mf_phase_space: unknown process %d", proc);
    if (!prm) return fail(MF_ERR_INVALID_ARG, "mf_phase_space: NULL params");
    if (n < 0 || n > kMaxEvents)
        return fail(MF_ERR_INVALID_ARG, "mf_phase_space: n = %lld outside [0, 2^36]", (long long)n);
    if (n == 0) return MF_OK;
    if (!p || !w) return fail(MF_ERR_INVALID_ARG, "mf_phase_space: NULL p or w");
    if ((edges || bin_idx) && (nb < 2 || nb > 64))
        return fail(MF_ERR_INVALID_ARG, "mf_phase_space: nb = %d outside [2, 64]", nb);
    if (!(prm->sqrt_s > 0.0)) return fail(MF_ERR_INVALID_ARG, "mf_phase_space: sqrt_s must be > 0");
    const bool qcd = proc != MF_EE_MUMU;
    if (qcd && !(2.0 * prm->m_t < prm->sqrt_s && prm->m_t >= 0.0))
        return fail(MF_ERR_INVALID_ARG, "mf_phase_space: need 0 <= 2 m_t < sqrt_s");
    DeviceGuard g(h->device);
    mf::PsArgs a{};
    a.n = n;
    a.proc = proc;
    a.nb = nb;
    a.x = x;
    a.seed = seed;
    a.offset = offset;
    a.offset_dev = offset_dev;
    a.edges = edges;
    a.sqrt_s = prm->sqrt_s;
    for (int i = 0; i < 5; ++i) a.m_out[i] = 0.0;
    if (qcd) a.m_out[0] = a.m_out[1] = prm->m_t;
    a.pt_min = prm->pt_min;
    a.eta_max = prm->eta_max;
    a.dr_min = prm->dr_min;
    a.p = p;
    a.w = w;
    a.pass = pass;
    a.bin_idx = bin_idx;
    a.jac = jac;
    a.x_out = x_out;
    a.fail_count = h->fail_dev;
    hipError_t e = mf::launch_phase_space(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_phase_space launch");
    return MF_OK;
}

static mf_status check_requests(const char* who, const mf_request* reqs, int n_reqs, int precision,
                                const mf_params* prm, bool vjp)
{
    if (!reqs || n_reqs < 1) return fail(MF_ERR_INVALID_ARG, "%s: need at least one request", who);
    if (!prm) return fail(MF_ERR_INVALID_ARG, "%s: NULL params", who);
    if (precision < MF_FP64 || precision > MF_FP32_MFMA_F32)
        return fail(MF_ERR_INVALID_ARG, "%s: unknown precision %d", who, precision);
    for (int i = 0; i < n_reqs; ++i) {
        const mf_request& r = reqs[i];
        if (!valid_proc(r.proc)) return fail(MF_ERR_INVALID_ARG, "%s: request %d: unknown process %d", who, i, r.proc);
        if (r.n < 0 || r.n > kMaxEvents) return fail(MF_ERR_INVALID_ARG, "%s: request %d: n outside [0, 2^36]", who, i);
        if (r.n == 0) continue;
        if (!r.p && !vjp) return fail(MF_ERR_INVALID_ARG, "%s: request %d: NULL p", who, i);
        if (!vjp && !r.me_out) return fail(MF_ERR_INVALID_ARG, "%s: request %d: NULL me_out", who, i);
        if (vjp && (!r.x || !r.grad_me || !r.grad_x || !r.grad_theta))
            return fail(MF_ERR_INVALID_ARG, "%s: request %d: NULL x/grad_me/grad_x/grad_theta", who, i);
        // no matrix-core colour form without colour (e+e-), for the table-driven recursion or
        // for the two-quark-line diagram code, rejected before anything is launched
        if (!vjp && precision >= MF_FP32_MFMA_BF16
            && (r.proc == MF_EE_MUMU || r.proc == MF_GG_TTGGG || mf::quark_proc(r.proc)))
            return fail(MF_ERR_UNSUPPORTED, "%s: request %d: precision %d not available for process %d", who, i,
                        precision, r.proc);
    }
    return MF_OK;
}

mf_status mf_matrix_element(mf_handle h, const mf_request* reqs, int n_reqs, int precision,
                            const mf_params* prm, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_matrix_element: NULL handle");
    mf_status st = check_requests("mf_matrix_element", reqs, n_reqs, precision, prm, false);
    if (st != MF_OK) return st;
    DeviceGuard g(h->device);
    hipStream_t st_ = static_cast<hipStream_t>(stream);
    // gg requests of a multi-request call go to persistent launches, one per process class
    int order[3] = {MF_GG_TTGG, MF_GG_TTG, MF_GG_TT};   // most expensive first
    bool batched[4096] = {false};
    if (n_reqs > 1 && n_reqs <= 4096 && h->batch_persistent) {
        mf::BatchArgs a{};
        a.counter = h->tile_counter;
        a.mt = prm->m_t;
        for (int p = 0; p < 4; ++p) {
            double c = 1.0;
            for (int k = 0; k < mf::n_gluons(p); ++k) c *= 4.0 * 3.141592653589793238463 * prm->alpha_s;
            a.coupling[p] = c;
            a.chunk[p] = h->batch_chunk[p];
        }
        auto flush = [&]() -> mf_status {
            if (a.nreq == 0) return MF_OK;
            hipError_t e = mf::launch_batch(a, precision, h->batch_waves_per_cu, h->n_cu, st_);
            if (e != hipSuccess) return hip_fail(e, "mf_matrix_element persistent launch");
            a.nreq = 0;
            a.ntiles = 0;
            return MF_OK;
        };
        for (int proc : order) {
            for (int i = 0; i < n_reqs; ++i) {
                const mf_request& r = reqs[i];
                if (r.proc != proc || r.n == 0) continue;
                if (a.nreq == mf::MAX_BATCH) {
                    mf_status s2 = flush();
                    if (s2 != MF_OK) return s2;
                }
                mf::BatchReq& q = a.req[a.nreq++];
                q.proc = r.proc;
                q.n = r.n;
                q.p = r.p;
                q.out = r.me_out;
                q.tile_begin = a.ntiles;
                const int64_t tile = 64 * a.chunk[r.proc];
                a.ntiles += (r.n + tile - 1) / tile;
                batched[i] = true;
            }
            mf_status s1 = flush();     // one launch per process class
            if (s1 != MF_OK) return s1;
        }
    }
    for (int i = 0; i < n_reqs; ++i) {
        if (reqs[i].n == 0 || (i < 4096 && batched[i])) continue;
        mf::MeJob j{reqs[i].proc, reqs[i].n, reqs[i].p, reqs[i].me_out};
        const int blk = h->block[reqs[i].proc][precision];
        hipError_t e = mf::launch_matrix_element(j, precision, prm->m_t, prm->alpha_s, prm->alpha, blk,
                                                 static_cast<hipStream_t>(stream));
        if (e == hipErrorInvalidValue)
            return fail(MF_ERR_UNSUPPORTED, "mf_matrix_element: precision %d not available for process %d",
                        precision, reqs[i].proc);
        if (e != hipSuccess) return hip_fail(e, "mf_matrix_element launch");
    }
    return MF_OK;
}

mf_status mf_matrix_element_vjp(mf_handle h, const mf_request* reqs, int n_reqs, int precision,
                                const mf_params* prm, const double* edges, int nb, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_matrix_element_vjp: NULL handle");
    mf_status st = check_requests("mf_matrix_element_vjp", reqs, n_reqs, precision, prm, true);
    if (st != MF_OK) return st;
    if (edges && (nb < 2 || nb > 64))
        return fail(MF_ERR_INVALID_ARG, "mf_matrix_element_vjp: nb = %d outside [2, 64]", nb);
    for (int i = 0; i < n_reqs; ++i)
        if ((reqs[i].proc == MF_EE_MUMU || reqs[i].proc == MF_GG_TTGGG || mf::quark_proc(reqs[i].proc))
            && reqs[i].n > 0)
            return fail(MF_ERR_UNSUPPORTED, "mf_matrix_element_vjp: no derivative for process %d", reqs[i].proc);
    if (!(2.0 * prm->m_t < prm->sqrt_s && prm->m_t >= 0.0 && prm->alpha_s > 0.0))
        return fail(MF_ERR_INVALID_ARG, "mf_matrix_element_vjp: need 0 <= 2 m_t < sqrt_s and alpha_s > 0");
    DeviceGuard g(h->device);
    // one launch per process class (up to VJP_MAX_BATCH requests each): a grid of 64-event
    // tiles over the class's requests
    const int order[3] = {MF_GG_TTGG, MF_GG_TTG, MF_GG_TT};
    for (int proc : order) {
        mf::VjpBatchArgs a{};
        mf::VjpJob& j = a.job;
        j.proc = proc;
        j.me_f32 = precision != MF_FP64;
        j.edges = edges;
        j.nb = nb;
        j.sqrt_s = prm->sqrt_s;
        j.mt = prm->m_t;
        j.alpha_s = prm->alpha_s;
        double coupling = 1.0;
        for (int k = 0; k < mf::n_gluons(proc); ++k) coupling *= 4.0 * 3.141592653589793238463 * prm->alpha_s;
        j.coupling = coupling;
        auto flush = [&]() -> mf_status {
            if (a.nreq == 0) return MF_OK;
            hipError_t e = mf::launch_vjp_batch(a, precision == MF_FP64 ? 0 : 1, static_cast<hipStream_t>(stream));
            if (e != hipSuccess) return hip_fail(e, "mf_matrix_element_vjp launch");
            a.nreq = 0;
            a.ntiles = 0;
            return MF_OK;
        };
        for (int i = 0; i < n_reqs; ++i) {
            const mf_request& r = reqs[i];
            if (r.proc != proc || r.n == 0) continue;
            if (a.nreq == mf::VJP_MAX_BATCH) {
                mf_status s1 = flush();
                if (s1 != MF_OK) return s1;
            }
            mf::VjpReq& q = a.req[a.nreq++];
            q.n = r.n;
            q.x = r.x;
            q.grad_me = r.grad_me;
            q.grad_x = r.grad_x;
            q.grad_theta = r.grad_theta;
            q.me_out = r.me_out;
            q.tile_begin = a.ntiles;
            a.ntiles += (r.n + 63) / 64;
        }
        mf_status s2 = flush();
        if (s2 != MF_OK) return s2;
    }
    return MF_OK;
}

static mf_status pdf_grid(const char* who, const mf_pdf_grid* g, mf::PdfGrid& out)
{
    if (!g) return fail(MF_ERR_INVALID_ARG, "%s: NULL grid", who);
    if (g->nx < 2 || g->nq < 2) return fail(MF_ERR_INVALID_ARG, "%s: grid needs at least 2 x 2 nodes", who);
    if (!g->log_x || !g->log_q2 || !g->xf) return fail(MF_ERR_INVALID_ARG, "%s: NULL grid array", who);
    out = mf::PdfGrid{g->nx, g->nq, g->log_x, g->log_q2, g->xf};
    return MF_OK;
}

mf_status mf_pdf_eval(mf_handle h, const mf_pdf_grid* g, int64_t n, const double* x, const double* q2,
                      double* xf_out, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_pdf_eval: NULL handle");
    mf::PdfGrid grid;
    mf_status st = pdf_grid("mf_pdf_eval", g, grid);
    if (st != MF_OK) return st;
    if (n < 0 || n > kMaxEvents) return fail(MF_ERR_INVALID_ARG, "mf_pdf_eval: n outside [0, 2^36]");
    if (n > 0 && (!x || !q2 || !xf_out)) return fail(MF_ERR_INVALID_ARG, "mf_pdf_eval: NULL x, q2 or xf_out");
    DeviceGuard dg(h->device);
    hipError_t e = mf::launch_pdf_eval(grid, n, x, q2, xf_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_pdf_eval launch");
    return MF_OK;
}

mf_status mf_phase_space_pp(mf_handle h, int proc, const mf_params* prm, double sqrt_S, const mf_pdf_grid* g,
                            const mf_pdf_grid* g_b, int64_t n, const double* x, uint64_t seed, uint64_t offset, const uint64_t* offset_dev,
                            const double* edges, int nb, double* p, double* w, uint8_t* pass, int16_t* bin_idx,
                            double* jac, double* x_out, double* x12, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: NULL handle");
    if (!valid_proc(proc) || proc == MF_EE_MUMU)
        return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: process %d is not a QCD process", proc);
    if (!prm) return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: NULL params");
    mf::PdfGrid grid, grid_b;
    mf_status st = pdf_grid("mf_phase_space_pp", g, grid);
    if (st != MF_OK) return st;
    st = pdf_grid("mf_phase_space_pp", g_b ? g_b : g, grid_b);
    if (st != MF_OK) return st;
    if (n < 0 || n > kMaxEvents) return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: n outside [0, 2^36]");
    if (n == 0) return MF_OK;
    if (!p || !w) return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: NULL p or w");
    if ((edges || bin_idx) && (nb < 2 || nb > 64))
        return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: nb = %d outside [2, 64]", nb);
    if (!(prm->m_t > 0.0) || !(sqrt_S > 2.0 * prm->m_t))
        return fail(MF_ERR_INVALID_ARG, "mf_phase_space_pp: need 0 < 2 m_t < sqrt_S");
    DeviceGuard dg(h->device);
    mf::PpArgs a{};
    a.n = n;
    a.nb = nb;
    a.x = x;
    a.seed = seed;
    a.offset = offset;
    a.offset_dev = offset_dev;
    a.edges = edges;
    a.S = sqrt_S * sqrt_S;
    a.tau0 = 4.0 * prm->m_t * prm->m_t / a.S;
    a.mu2 = prm->m_t * prm->m_t;
    for (int i = 0; i < 5; ++i) a.m_out[i] = i < 2 ? prm->m_t : 0.0;
    a.pt_min = prm->pt_min;
    a.eta_max = prm->eta_max;
    a.dr_min = prm->dr_min;
    a.grid = grid;
    a.grid_b = grid_b;
    a.p = p;
    a.w = w;
    a.pass = pass;
    a.bin_idx = bin_idx;
    a.jac = jac;
    a.x_out = x_out;
    a.x12 = x12;
    a.fail_count = h->fail_dev;
    hipError_t e = mf::launch_phase_space_pp(a, mf::n_out(proc), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_phase_space_pp launch");
    return MF_OK;
}

mf_status mf_unweight(mf_handle h, int64_t n, const double* w, double w_max, uint64_t seed, uint64_t offset,
                      int n_ext, const double* p, int64_t cap, int64_t* idx, double* fac, double* p_out,
                      uint64_t* count, double* w_max_out, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_unweight: NULL handle");
    if (n < 0 || n > kMaxEvents) return fail(MF_ERR_INVALID_ARG, "mf_unweight: n outside [0, 2^36]");
    if (cap < 0) return fail(MF_ERR_INVALID_ARG, "mf_unweight: negative capacity");
    if (!count) return fail(MF_ERR_INVALID_ARG, "mf_unweight: NULL count");
    if (n > 0 && !w) return fail(MF_ERR_INVALID_ARG, "mf_unweight: NULL w");
    if (cap > 0 && !idx) return fail(MF_ERR_INVALID_ARG, "mf_unweight: NULL idx");
    if (p_out && (!p || n_ext < 1 || n_ext > 8))
        return fail(MF_ERR_INVALID_ARG, "mf_unweight: p_out needs p and 1 <= n_ext <= 8");
    if (!(w_max > 0.0) && w_max != 0.0 && !(w_max < 0.0))
        return fail(MF_ERR_INVALID_ARG, "mf_unweight: w_max is NaN");
    DeviceGuard g(h->device);
    mf::UnweightArgs a{};
    a.n = n;
    a.w = w;
    a.w_max = w_max;
    a.seed = seed;
    a.offset = offset;
    a.n_ext = p_out ? n_ext : 0;
    a.p = p;
    a.cap = cap;
    a.idx = idx;
    a.fac = fac;
    a.p_out = p_out;
    a.count = reinterpret_cast<unsigned long long*>(count);
    a.w_max_out = w_max_out;
    a.work = h->partials;
    hipError_t e = mf::launch_unweight(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_unweight launch");
    return MF_OK;
}

struct mf_graph_s {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

mf_status mf_graph_begin(mf_handle h, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_graph_begin: NULL handle");
    if (!stream) return fail(MF_ERR_INVALID_ARG, "mf_graph_begin: the default stream cannot be captured");
    DeviceGuard g(h->device);
    hipError_t e = hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "mf_graph_begin: hipStreamBeginCapture");
    return MF_OK;
}

mf_status mf_graph_end(mf_handle h, void* stream, mf_graph* out)
{
    g_err.clear();
    if (!h || !stream || !out) return fail(MF_ERR_INVALID_ARG, "mf_graph_end: NULL argument");
    *out = nullptr;
    DeviceGuard g(h->device);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &graph);
    if (e != hipSuccess) return hip_fail(e, "mf_graph_end: hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_fail(e, "mf_graph_end: hipGraphInstantiate");
    }
    mf_graph r = new mf_graph_s;
    r->device = h->device;
    r->graph = graph;
    r->exec = exec;
    *out = r;
    return MF_OK;
}

mf_status mf_graph_launch(mf_graph gr, void* stream)
{
    g_err.clear();
    if (!gr) return fail(MF_ERR_INVALID_ARG, "mf_graph_launch: NULL graph");
    DeviceGuard g(gr->device);
    hipError_t e = hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_graph_launch");
    return MF_OK;
}

mf_status mf_graph_destroy(mf_graph gr)
{
    g_err.clear();
    if (!gr) return MF_OK;
    DeviceGuard g(gr->device);
    if (gr->exec) hipGraphExecDestroy(gr->exec);
    if (gr->graph) hipGraphDestroy(gr->graph);
    delete gr;
    return MF_OK;
}

// validation and kernel arguments shared by mf_vegas_refine and mf_vegas_refine_noalloc
static mf_status vegas_args(const char* who, const mf_params* prm, int64_t n, int d, int nb, double alpha,
                            const double* w, const double* jac, const void* me, int me_f32,
                            const uint8_t* pass, const int16_t* bin_idx, double* F, double* acc,
                            double* edges, int flags, uint64_t* rng_counter, mf::VegasArgs& a)
{
    if (!prm) return fail(MF_ERR_INVALID_ARG, "%s: NULL params", who);
    if (d < 1 || d > mf::VEGAS_MAX_D) return fail(MF_ERR_INVALID_ARG, "%s: d = %d outside [1, 16]", who, d);
    if (nb < 2 || nb > 64) return fail(MF_ERR_INVALID_ARG, "%s: nb = %d outside [2, 64]", who, nb);
    if (n < 0 || n > kMaxEvents) return fail(MF_ERR_INVALID_ARG, "%s: n outside [0, 2^36]", who);
    if (!acc || !edges) return fail(MF_ERR_INVALID_ARG, "%s: NULL acc or edges", who);
    if (n > 0 && (!w || !me || !bin_idx)) return fail(MF_ERR_INVALID_ARG, "%s: NULL w, me or bin_idx", who);
    a = mf::VegasArgs{};
    a.n = n;
    a.d = d;
    a.nb = nb;
    a.alpha = alpha;
    const double s = prm->sqrt_s * prm->sqrt_s;
    a.flux = 0.3893793721e9 / (2.0 * s);
    a.w = w;
    a.jac = jac;
    a.me = me;
    a.me_f32 = me_f32;
    a.pass = pass;
    a.bin_idx = bin_idx;
    a.F = F;
    a.nblk = mf::vegas_blocks(n);
    a.acc = acc;
    a.edges = edges;
    a.update_edges = (flags & MF_VEGAS_REFINE) ? 1 : 0;
    a.accumulate = (flags & MF_VEGAS_ACCUMULATE) ? 1 : 0;
    a.rng_counter = rng_counter;
    return MF_OK;
}

mf_status mf_vegas_refine(mf_handle h, const mf_params* prm, int64_t n, int d, int nb, double alpha,
                          const double* w, const double* jac, const void* me, int me_f32,
                          const uint8_t* pass, const int16_t* bin_idx, double* F, double* acc,
                          double* edges, int flags, uint64_t* rng_counter, void* stream)
{
    g_err.clear();
    if (!h) return fail(MF_ERR_INVALID_ARG, "mf_vegas_refine: NULL handle");
    mf::VegasArgs a;
    mf_status st = vegas_args("mf_vegas_refine", prm, n, d, nb, alpha, w, jac, me, me_f32, pass, bin_idx, F, acc,
                              edges, flags, rng_counter, a);
    if (st != MF_OK) return st;
    DeviceGuard g(h->device);
    a.partials = h->partials;          // VEGAS_PARTIALS_MAX doubles, enough for any n, d, nb
    hipError_t e = mf::launch_vegas(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_vegas_refine launch");
    return MF_OK;
}

mf_status mf_vegas_refine_noalloc(const mf_params* prm, int64_t n, int d, int nb, double alpha,
                                  const double* w, const double* jac, const void* me, int me_f32,
                                  const uint8_t* pass, const int16_t* bin_idx, double* F, double* acc,
                                  double* edges, int flags, uint64_t* rng_counter, void* stream)
{
    g_err.clear();
    mf::VegasArgs a;
    mf_status st = vegas_args("mf_vegas_refine_noalloc", prm, n, d, nb, alpha, w, jac, me, me_f32, pass, bin_idx,
                              F, acc, edges, flags, rng_counter, a);
    if (st != MF_OK) return st;
    const size_t need = (size_t)a.nblk * (size_t)(2 + d * nb);
    if (need > mf::VEGAS_PARTIALS_MAX)
        return fail(MF_ERR_INVALID_ARG, "mf_vegas_refine_noalloc: %zu partial sums exceed the static workspace "
                    "of %zu", need, (size_t)mf::VEGAS_PARTIALS_MAX);
    hipError_t e = mf::vegas_static_partials(&a.partials);
    if (e != hipSuccess) return hip_fail(e, "mf_vegas_refine_noalloc: address of the static workspace");
    e = mf::launch_vegas(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mf_vegas_refine_noalloc launch");
    return MF_OK;
}

}  // extern "C"
