// extern "C" entry points declared in include/wilson.h.  Arguments are validated before
// any device work; no C++ exception crosses this boundary.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <algorithm>

#include "layout_lab.h"
#include "runtime.h"
#include "solver.h"
#include "wilson.h"

using namespace wl;

namespace {

std::mutex g_default_mu;
wilson_ctx *g_default_ctx = nullptr;

void check_dims(const int32_t *dims) {
    WL_CHECK_ARG(dims != nullptr, "dims is NULL");
    long long V = 1;
    for (int k = 0; k < 4; k++) {
        WL_CHECK_ARG(dims[k] >= 2 && dims[k] % 2 == 0, "every lattice extent must be even and >= 2");
        V *= dims[k];
    }
    WL_CHECK_ARG(V / 2 < (1LL << 30), "lattice too large");
}

size_t spinor_doubles(const int32_t *dims, int nrhs) {
    return (size_t)24 * dims[0] * dims[1] * dims[2] * dims[3] * nrhs;
}

// Device view of a caller buffer: device pointers pass through, host buffers are staged.
struct Staged {
    wilson_ctx *ctx;
    const double *user;
    double *dev;
    size_t bytes;
    bool host;
    Staged(wilson_ctx *c, DevBuf &buf, const double *p, size_t n, bool copy_in) : ctx(c), user(p), bytes(n) {
        host = !is_device_ptr(p);
        if (host) {
            dev = static_cast<double *>(ctx->stage(buf, n));
            if (copy_in) WL_HIP(hipMemcpyAsync(dev, p, n, hipMemcpyHostToDevice, ctx->stream));
        } else {
            dev = const_cast<double *>(p);
        }
    }
    void copy_out() {
        if (host) WL_HIP(hipMemcpyAsync(const_cast<double *>(user), dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    }
};

// ---- device memory of the no-allocation solve ---------------------------------------
// One static array per GPU, part of the library's code object: the loader allocates it
// on each device the library is used on, and it stays until the process ends.  Its name
// is only a host-side handle; host code uses the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device when a context is created.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

void *scratch_address(int device) {  // the calling thread's current device must be `device`
    WL_CHECK_ARG(device >= 0 && device < kMaxDevices, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        WL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(WILSON_DEVICE_ERROR, "no device address for the scratch array");
        g_scratch_addr[device] = p;
    }
    return g_scratch_addr[device];
}

wilson_ctx *make_ctx(void *stream) {
    std::unique_ptr<wilson_ctx> c(new wilson_ctx());
    WL_HIP(hipGetDevice(&c->device));
    c->stream = static_cast<hipStream_t>(stream);
    c->lend.create(kMaxRhs);
    c->scratch = scratch_address(c->device);
    return c.release();
}

wilson_ctx *default_ctx() {
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default_ctx) g_default_ctx = make_ctx(nullptr);
    return g_default_ctx;
}

wilson_gauge *load_gauge(wilson_ctx *ctx, const double *U, const int32_t *dims, uint32_t precisions) {
    check_dims(dims);
    WL_CHECK_ARG(U != nullptr, "U is NULL");
    auto *G = new wilson_gauge();
    try {
        G->g = make_geom(dims);
        std::memcpy(G->dims, dims, sizeof G->dims);
        const size_t links = (size_t)72 * dims[0] * dims[1] * dims[2] * dims[3];  // doubles
        DevBuf tmp;
        Staged su(ctx, tmp, U, links * sizeof(double), true);
        // Two-row storage needs exact SU(3) links (to well below the FP64 parity tolerance);
        // anything else is kept in full.  WILSON_RECON=18 forces full storage.
        int recon = 12;
        const char *env = std::getenv("WILSON_RECON");
        if (env && std::strcmp(env, "18") == 0) recon = 18;
        if (recon == 12) {
            if (ctx->flag.size() < sizeof(int)) ctx->flag.alloc(256);
            static const int zero = 0;
            WL_HIP(hipMemcpyAsync(ctx->flag.get(), &zero, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
            WL_HIP(launch_su3_check(su.dev, links / 18, 1e-13, ctx->flag.as<int>(), ctx->stream));
            int bad = 0;
            WL_HIP(hipMemcpyAsync(&bad, ctx->flag.get(), sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            WL_HIP(hipStreamSynchronize(ctx->stream));
            if (bad) recon = 18;
        }
        G->recon = recon;
        for (int prec = 0; prec < 3; prec++) {
            const bool want = prec == P64 || (prec == P32 && (precisions & WILSON_GAUGE_FP32)) ||
                              (prec == P16 && (precisions & WILSON_GAUGE_FP16));
            if (!want) continue;
            G->U[prec].alloc(gauge_bytes(prec, recon, G->g));
            WL_HIP(launch_gauge_pack(G->U[prec].get(), prec, su.dev, G->g, recon, ctx->stream));
        }
        WL_HIP(hipStreamSynchronize(ctx->stream));
    } catch (...) {
        delete G;
        throw;
    }
    return G;
}

int report(const Error &e) {
    set_last_error(e.what());
    return e.code;
}

}  // namespace

#define API_BEGIN try {
#define API_END                                                   \
    }                                                             \
    catch (const Error &e) { return report(e); }                  \
    catch (const std::bad_alloc &) {                              \
        set_last_error("host allocation failed");                 \
        return WILSON_OUT_OF_MEMORY;                              \
    }                                                             \
    catch (const std::exception &e) {                             \
        set_last_error(e.what());                                 \
        return WILSON_DEVICE_ERROR;                               \
    }                                                             \
    catch (...) {                                                 \
        set_last_error("unknown error");                          \
        return WILSON_DEVICE_ERROR;                               \
    }

static void check_solve_args(const double *kappa, const double *tol, int nrhs, const wilson_solve_opts *o) {
    WL_CHECK_ARG(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..64");
    WL_CHECK_ARG(kappa != nullptr && tol != nullptr, "kappa / tol is NULL");
    for (int k = 0; k < nrhs; k++) {
        WL_CHECK_ARG(std::isfinite(kappa[k]) && kappa[k] >= 0.0, "kappa must be finite and >= 0");
        WL_CHECK_ARG(std::isfinite(tol[k]) && tol[k] > 0.0, "tol must be finite and > 0");
    }
    if (o) {
        WL_CHECK_ARG(o->solver == WILSON_SOLVER_BICGSTAB_EO || o->solver == WILSON_SOLVER_CGNR_EO ||
                         o->solver == WILSON_SOLVER_BLOCK_BICGSTAB_EO,
                     "unknown solver");
        if (o->solver == WILSON_SOLVER_BLOCK_BICGSTAB_EO) {
            WL_CHECK_ARG(o->precision == WILSON_FP64, "block BiCGStab runs in FP64 only");
            for (int k = 1; k < nrhs; k++)
                WL_CHECK_ARG(kappa[k] == kappa[0], "block BiCGStab needs one kappa for all right-hand sides");
        }
        WL_CHECK_ARG(o->precision >= WILSON_FP64 && o->precision <= WILSON_FP16_L32, "unknown precision");
        WL_CHECK_ARG(o->maxiter > 0, "maxiter must be > 0");
        WL_CHECK_ARG(o->mixed_update == 0 || o->mixed_update == 1, "mixed_update must be 0 or 1");
        WL_CHECK_ARG(o->mixed_update == 0 || (o->precision != WILSON_FP64 && o->solver == WILSON_SOLVER_BICGSTAB_EO),
                     "reliable updates need a mixed precision and BiCGStab");
        if (o->workspace) {
            WL_CHECK_ARG(reinterpret_cast<uintptr_t>(o->workspace) % 256 == 0, "workspace must be 256-byte aligned");
            WL_CHECK_ARG(is_device_ptr(o->workspace), "workspace must be device memory");
        }
    }
}

static SolveParams params_from(const wilson_solve_opts *o, int maxiter_default) {
    SolveParams p;
    p.maxiter = maxiter_default;
    if (o) {
        p.method = o->solver;
        p.precision = o->precision;
        p.maxiter = o->maxiter;
        p.max_restarts = o->max_restarts < 0 ? 5 : o->max_restarts;
        p.inner_tol = o->inner_tol;
        p.use_x0 = o->use_x0 != 0;
        p.poll_every = o->poll_every > 0 ? o->poll_every : 1;
        p.reliable = o->mixed_update == 1;
        p.workspace = o->workspace;
        p.workspace_bytes = o->workspace_bytes;
    }
    return p;
}

static uint32_t gauge_bits_for(int precision) {
    switch (precision) {
        case WILSON_FP32: return WILSON_GAUGE_FP32;
        case WILSON_FP16: return WILSON_GAUGE_FP16;
        case WILSON_FP16_L32: return WILSON_GAUGE_FP32;
        default: return 0;
    }
}

extern "C" {

const char *wilson_version(void) { return "wilson-mi355x 0.1 (gfx950)"; }

const char *wilson_strerror(int code) {
    switch (code) {
        case WILSON_OK: return "ok";
        case WILSON_NOT_CONVERGED: return "not converged";
        case WILSON_INVALID_ARG: return "invalid argument";
        case WILSON_OUT_OF_MEMORY: return "out of device memory";
        case WILSON_DEVICE_ERROR: return "device (HIP) error";
        case WILSON_BREAKDOWN: return "Krylov breakdown";
        case WILSON_NONFINITE: return "NaN or Inf in input or iterate";
        case WILSON_REJECTED: return "rejected by admission control";
        case WILSON_BUSY: return "slot busy or not ready";
        default: return "unknown status";
    }
}

const char *wilson_last_error(void) { return wl::last_error().c_str(); }

int wilson_context_create(wilson_ctx **ctx, void *hip_stream) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr, "ctx is NULL");
    *ctx = make_ctx(hip_stream);
    return WILSON_OK;
    API_END
}

int wilson_context_destroy(wilson_ctx *ctx) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr, "ctx is NULL");
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &p : ctx->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    ctx->solve_cache.clear();  // their captured graphs first
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return WILSON_OK;
    API_END
}

int wilson_gauge_load(wilson_ctx *ctx, wilson_gauge **g, const double *U, const int32_t dims[4],
                      uint32_t precisions) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr, "ctx / g is NULL");
    *g = load_gauge(ctx, U, dims, precisions);
    return WILSON_OK;
    API_END
}

int wilson_gauge_free(wilson_ctx *ctx, wilson_gauge *g) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr, "ctx / g is NULL");
    WL_HIP(hipStreamSynchronize(ctx->stream));
    // the dslash workspace key names this field; solve workspaces take the field per call
    ctx->dslash_ws.reset();
    ctx->dslash_key.clear();
    delete g;
    return WILSON_OK;
    API_END
}

size_t wilson_gauge_bytes(const wilson_gauge *g) { return g ? g->bytes() : 0; }

int wilson_gauge_attach_clover(wilson_ctx *ctx, wilson_gauge *g, const double *F) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr && F != nullptr, "ctx / g / F is NULL");
    const size_t V = (size_t)g->dims[0] * g->dims[1] * g->dims[2] * g->dims[3];
    DevBuf tmp;
    Staged sf(ctx, tmp, F, V * 144 * 2 * sizeof(double), true);
    DevBuf t[2], ti[2];
    for (int p = 0; p < 2; p++) {
        t[p].alloc(2 * clover_parity_bytes(p, g->g));
        ti[p].alloc(2 * clover_parity_bytes(p, g->g));
    }
    if (ctx->flag.size() < sizeof(int)) ctx->flag.alloc(256);
    static const int zero = 0;
    WL_HIP(hipMemcpyAsync(ctx->flag.get(), &zero, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    WL_HIP(launch_clover_pack(t[P64].get(), ti[P64].get(), t[P32].get(), ti[P32].get(), sf.dev, g->g, 1e-12,
                              ctx->flag.as<int>(), ctx->stream));
    int bad = 0;
    WL_HIP(hipMemcpyAsync(&bad, ctx->flag.get(), sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    if (bad & 1) throw Error(WILSON_INVALID_ARG, "clover term F is not Hermitian or does not commute with gamma5");
    if (bad & 2) throw Error(WILSON_INVALID_ARG, "clover term: 1 + F is singular at some site");
    for (int p = 0; p < 2; p++) {
        g->clovT[p] = std::move(t[p]);
        g->clovTi[p] = std::move(ti[p]);
    }
    return WILSON_OK;
    API_END
}

int wilson_gauge_detach_clover(wilson_ctx *ctx, wilson_gauge *g) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr, "ctx / g is NULL");
    WL_HIP(hipStreamSynchronize(ctx->stream));
    for (int p = 0; p < 2; p++) {
        g->clovT[p].release();
        g->clovTi[p].release();
    }
    return WILSON_OK;
    API_END
}

int wilson_dslash_ex(wilson_ctx *ctx, const wilson_gauge *g, double *out, const double *in, double kappa,
                     int32_t parity, int32_t precision, int32_t nrhs) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr, "ctx / g is NULL");
    WL_CHECK_ARG(out != nullptr && in != nullptr, "out / in is NULL");
    WL_CHECK_ARG(parity >= 0 && parity <= 2, "parity must be 0, 1 or 2");
    WL_CHECK_ARG(!(parity == 2 && out == in), "out == in is not allowed for parity 2");
    WL_CHECK_ARG(std::isfinite(kappa), "kappa must be finite");
    WL_CHECK_ARG(precision >= WILSON_FP64 && precision <= WILSON_FP16_L32, "unknown precision");
    WL_CHECK_ARG(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..64");
    const size_t bytes = spinor_doubles(g->dims, nrhs) * sizeof(double);
    Staged si(ctx, ctx->stage_in, in, bytes, true);
    Staged so(ctx, ctx->stage_out, out, bytes, parity != 2);  // untouched sites keep their contents
    dslash_device(ctx, g, so.dev, si.dev, kappa, parity, precision, nrhs);
    so.copy_out();
    if (si.host || so.host) WL_HIP(hipStreamSynchronize(ctx->stream));
    return WILSON_OK;
    API_END
}

int wilson_dslash(double *out, const double *in, const double *U, double kappa, const int32_t dims[4],
                  int32_t parity) {
    API_BEGIN
    check_dims(dims);
    WL_CHECK_ARG(out && in && U, "NULL argument");
    WL_CHECK_ARG(parity >= 0 && parity <= 2, "parity must be 0, 1 or 2");
    WL_CHECK_ARG(!(parity == 2 && out == in), "out == in is not allowed for parity 2");
    WL_CHECK_ARG(std::isfinite(kappa), "kappa must be finite");
    wilson_ctx *ctx = default_ctx();
    std::lock_guard<std::mutex> lk(g_default_mu);
    wilson_gauge *G = load_gauge(ctx, U, dims, 0);
    try {
        const size_t bytes = spinor_doubles(dims, 1) * sizeof(double);
        Staged si(ctx, ctx->stage_in, in, bytes, true);
        Staged so(ctx, ctx->stage_out, out, bytes, parity != 2);
        dslash_device(ctx, G, so.dev, si.dev, kappa, parity, WILSON_FP64, 1);
        so.copy_out();
        WL_HIP(hipStreamSynchronize(ctx->stream));
    } catch (...) {
        ctx->dslash_ws.reset();
        delete G;
        throw;
    }
    ctx->dslash_ws.reset();
    ctx->dslash_key.clear();
    delete G;
    return WILSON_OK;
    API_END
}

int wilson_solve_ex(wilson_ctx *ctx, const wilson_gauge *g, double *x, const double *b, int32_t nrhs,
                    const double *kappa, const double *tol, const wilson_solve_opts *opts, wilson_solve_info *info) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr, "ctx / g is NULL");
    WL_CHECK_ARG(x != nullptr && b != nullptr, "x / b is NULL");
    WL_CHECK_ARG(x != b, "x and b must be distinct");
    check_solve_args(kappa, tol, nrhs, opts);
    const SolveParams p = params_from(opts, 10000);
    if (p.precision != WILSON_FP64) {
        const uint32_t need = gauge_bits_for(p.precision);
        WL_CHECK_ARG((need & WILSON_GAUGE_FP32) == 0 || g->U[P32].get(), "gauge field has no FP32 copy");
        WL_CHECK_ARG((need & WILSON_GAUGE_FP16) == 0 || g->U[P16].get(), "gauge field has no FP16 copy");
    }
    const size_t bytes = spinor_doubles(g->dims, nrhs) * sizeof(double);
    Staged sb(ctx, ctx->stage_in, b, bytes, true);
    Staged sx(ctx, ctx->stage_out, x, bytes, p.use_x0);
    const int st = solve_device(ctx, g, sx.dev, sb.dev, nrhs, kappa, tol, p, info);
    sx.copy_out();
    WL_HIP(hipStreamSynchronize(ctx->stream));
    return st;
    API_END
}

int wilson_solve_noalloc(wilson_ctx *ctx, const wilson_gauge *g, double *x, const double *b, int32_t nrhs,
                         const double *kappa, const double *tol, const wilson_solve_opts *opts,
                         wilson_solve_info *info) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr && g != nullptr, "ctx / g is NULL");
    WL_CHECK_ARG(x != nullptr && b != nullptr, "x / b is NULL");
    WL_CHECK_ARG(x != b, "x and b must be distinct");
    check_solve_args(kappa, tol, nrhs, opts);
    WL_CHECK_ARG(opts == nullptr || opts->workspace == nullptr,
                 "the no-allocation solve keeps its buffers in the library's scratch array; opts->workspace must be NULL");
    WL_CHECK_ARG(is_device_ptr(x) && is_device_ptr(b), "the no-allocation solve takes device buffers only");
    SolveParams p = params_from(opts, 10000);
    if (p.precision != WILSON_FP64) {
        const uint32_t need = gauge_bits_for(p.precision);
        WL_CHECK_ARG((need & WILSON_GAUGE_FP32) == 0 || g->U[P32].get(), "gauge field has no FP32 copy");
        WL_CHECK_ARG((need & WILSON_GAUGE_FP16) == 0 || g->U[P16].get(), "gauge field has no FP16 copy");
    }
    const size_t need = solve_footprint(g->g, nrhs, p);
    if (need > kScratchBytes)
        throw Error(WILSON_INVALID_ARG, "the solve needs " + std::to_string(need) + " bytes of device memory; the "
                                        "no-allocation solve holds at most " + std::to_string(kScratchBytes) +
                                        " (use wilson_solve_ex)");
    WL_CHECK_ARG(ctx->scratch != nullptr, "no scratch array on this context's device");
    p.workspace = ctx->scratch;
    p.workspace_bytes = kScratchBytes;
    p.no_tune = true;
    // event timing would create events; suspended for the call
    struct TimingOff {
        wilson_ctx *c;
        bool was;
        explicit TimingOff(wilson_ctx *cc) : c(cc), was(cc->timing) { c->timing = false; }
        ~TimingOff() { c->timing = was; }
    } timing_off(ctx);
    const int st = solve_device(ctx, g, x, b, nrhs, kappa, tol, p, info);
    WL_HIP(hipStreamSynchronize(ctx->stream));
    return st;
    API_END
}

int wilson_solve(double *x, const double *b, const double *U, double kappa, const int32_t dims[4], double tol,
                 int32_t maxiter) {
    API_BEGIN
    check_dims(dims);
    WL_CHECK_ARG(x && b && U, "NULL argument");
    WL_CHECK_ARG(maxiter > 0, "maxiter must be > 0");
    WL_CHECK_ARG(x != b, "x and b must be distinct");
    check_solve_args(&kappa, &tol, 1, nullptr);
    wilson_ctx *ctx = default_ctx();
    std::lock_guard<std::mutex> lk(g_default_mu);
    wilson_gauge *G = load_gauge(ctx, U, dims, 0);
    int st;
    try {
        SolveParams p;
        p.maxiter = maxiter;
        const size_t bytes = spinor_doubles(dims, 1) * sizeof(double);
        Staged sb(ctx, ctx->stage_in, b, bytes, true);
        Staged sx(ctx, ctx->stage_out, x, bytes, false);
        st = solve_device(ctx, G, sx.dev, sb.dev, 1, &kappa, &tol, p, nullptr);
        sx.copy_out();
        WL_HIP(hipStreamSynchronize(ctx->stream));
    } catch (...) {
        delete G;
        throw;
    }
    delete G;
    return st;
    API_END
}

size_t wilson_gauge_footprint_bytes(const int32_t dims[4], uint32_t precisions, int32_t link_reals) {
    try {
        check_dims(dims);
        if (link_reals != 12 && link_reals != 18) return 0;
        const Geom g = make_geom(dims);
        size_t b = gauge_bytes(P64, link_reals, g);
        if (precisions & WILSON_GAUGE_FP32) b += gauge_bytes(P32, link_reals, g);
        if (precisions & WILSON_GAUGE_FP16) b += gauge_bytes(P16, link_reals, g);
        return b;
    } catch (...) {
        return 0;
    }
}

int wilson_index_check(const int32_t dims[4]) {
    API_BEGIN
    check_dims(dims);
    std::string first;
    const long long bad = index_check(dims, first);
    if (bad == 0) return WILSON_OK;
    set_last_error(std::to_string(bad) + " index violations; first: " + first);
    return (int)std::min<long long>(bad, 0x7fffffff);
    API_END
}

size_t wilson_footprint_bytes(const int32_t dims[4], int32_t nrhs, const wilson_solve_opts *opts) {
    try {
        check_dims(dims);
        if (nrhs < 1 || nrhs > kMaxRhs) return 0;
        return solve_footprint(make_geom(dims), nrhs, params_from(opts, 10000));
    } catch (...) {
        return 0;
    }
}

int wilson_batch_create(wilson_ctx *ctx, const wilson_gauge *g, int32_t nslots, const wilson_solve_opts *opts,
                        wilson_batch **batch) {
    API_BEGIN
    WL_CHECK_ARG(ctx && g && batch, "NULL argument");
    WL_CHECK_ARG(nslots >= 1 && nslots <= kMaxRhs, "nslots must be in 1..64");
    if (opts) {
        double k = 0.1, t = 1e-10;
        check_solve_args(&k, &t, 1, opts);
        WL_CHECK_ARG(opts->mixed_update == 0, "batches use defect correction (mixed_update 0)");
        WL_CHECK_ARG(opts->solver != WILSON_SOLVER_BLOCK_BICGSTAB_EO,
                     "batches solve each slot on its own (no block solver)");
    }
    *batch = reinterpret_cast<wilson_batch *>(batch_create(ctx, g, nslots, params_from(opts, 10000)));
    return WILSON_OK;
    API_END
}

int wilson_batch_destroy(wilson_batch *batch) {
    API_BEGIN
    WL_CHECK_ARG(batch != nullptr, "batch is NULL");
    batch_destroy(reinterpret_cast<BatchEngine *>(batch));
    return WILSON_OK;
    API_END
}

int wilson_batch_attach(wilson_batch *batch, int32_t slot, const double *b, double kappa, double tol,
                        int32_t maxiter) {
    API_BEGIN
    WL_CHECK_ARG(batch != nullptr && b != nullptr, "NULL argument");
    check_solve_args(&kappa, &tol, 1, nullptr);
    WL_CHECK_ARG(maxiter > 0, "maxiter must be > 0");
    BatchEngine *be = reinterpret_cast<BatchEngine *>(batch);
    wilson_ctx *ctx = batch_ctx(be);
    Staged sb(ctx, ctx->stage_in, b, batch_spinor_bytes(be), true);
    return batch_attach(be, slot, sb.dev, kappa, tol, maxiter);
    API_END
}

int wilson_batch_step(wilson_batch *batch, int32_t iters) {
    API_BEGIN
    WL_CHECK_ARG(batch != nullptr && iters > 0, "bad argument");
    batch_step(reinterpret_cast<BatchEngine *>(batch), iters);
    return WILSON_OK;
    API_END
}

int wilson_batch_poll(wilson_batch *batch, int32_t *state, int32_t *status) {
    API_BEGIN
    WL_CHECK_ARG(batch && state && status, "NULL argument");
    batch_poll(reinterpret_cast<BatchEngine *>(batch), state, status);
    return WILSON_OK;
    API_END
}

int wilson_batch_detach(wilson_batch *batch, int32_t slot, double *x, wilson_solve_info *info) {
    API_BEGIN
    WL_CHECK_ARG(batch != nullptr && x != nullptr, "NULL argument");
    BatchEngine *be = reinterpret_cast<BatchEngine *>(batch);
    wilson_ctx *ctx = batch_ctx(be);
    Staged sx(ctx, ctx->stage_out, x, batch_spinor_bytes(be), false);
    const int st = batch_detach(be, slot, sx.dev, info);
    if (st != WILSON_BUSY) {
        sx.copy_out();
        WL_HIP(hipStreamSynchronize(ctx->stream));
    }
    return st;
    API_END
}

int wilson_timing_enable(wilson_ctx *ctx, int32_t enable) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr, "ctx is NULL");
    ctx->drain_timing();
    for (int k = 0; k < WILSON_KERNEL_COUNT; k++) {
        ctx->t_ms[k] = 0;
        ctx->launches[k] = 0;
        ctx->t_bytes[k] = 0;
    }
    ctx->timing = enable != 0;
    return WILSON_OK;
    API_END
}

int wilson_timing_read(wilson_ctx *ctx, int32_t kernel_class, double *total_ms, int64_t *launches, double *bytes) {
    API_BEGIN
    WL_CHECK_ARG(ctx != nullptr, "ctx is NULL");
    WL_CHECK_ARG(kernel_class >= 0 && kernel_class < WILSON_KERNEL_COUNT, "unknown kernel class");
    ctx->drain_timing();
    if (total_ms) *total_ms = ctx->t_ms[kernel_class];
    if (launches) *launches = ctx->launches[kernel_class];
    if (bytes) *bytes = ctx->t_bytes[kernel_class];
    return WILSON_OK;
    API_END
}

int wilson_layout_hop(wilson_ctx *ctx, double *out, const double *in, const double *U, const int32_t dims[4],
                      double kappa, int32_t parity, int32_t precision, int32_t layout, int32_t link_reals,
                      int32_t reps, double *us_per_launch) {
    API_BEGIN
    WL_CHECK_ARG(ctx && out && in && U, "NULL argument");
    WL_CHECK_ARG(is_device_ptr(out) && is_device_ptr(in) && is_device_ptr(U), "layout hop needs device pointers");
    check_dims(dims);
    WL_CHECK_ARG(parity == 0 || parity == 1, "parity must be 0 or 1");
    WL_CHECK_ARG(precision == WILSON_FP64 || precision == WILSON_FP32, "precision must be WILSON_FP64 or WILSON_FP32");
    WL_CHECK_ARG(layout >= 0 && layout < LAB_LAYOUT_COUNT, "unknown layout");
    WL_CHECK_ARG(link_reals == 12 || link_reals == 18, "link_reals must be 12 or 18");
    WL_CHECK_ARG(reps >= 0 && reps <= 100000, "reps out of range");
    WL_CHECK_ARG(std::isfinite(kappa), "kappa must be finite");
    LabGeom g;
    WL_CHECK_ARG(lab_geom(g, dims, layout), "extents not allowed for this layout (sub-lattice layout: Ly, Lz, Lt "
                                            "multiples of 8)");
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    hipStream_t s = ctx->stream;
    if (link_reals == 12) {
        if (ctx->flag.size() < sizeof(int)) ctx->flag.alloc(256);
        static const int zero = 0;
        WL_HIP(hipMemcpyAsync(ctx->flag.get(), &zero, sizeof(int), hipMemcpyHostToDevice, s));
        WL_HIP(launch_su3_check(U, V * 4, 1e-13, ctx->flag.as<int>(), s));
        int bad = 0;
        WL_HIP(hipMemcpyAsync(&bad, ctx->flag.get(), sizeof(int), hipMemcpyDeviceToHost, s));
        WL_HIP(hipStreamSynchronize(s));
        WL_CHECK_ARG(!bad, "link_reals 12 needs SU(3) links");
    }
    DevBuf fin(lab_spinor_bytes(g, precision)), fout(lab_spinor_bytes(g, precision));
    DevBuf u0(lab_link_bytes(g, precision, link_reals)), u1(lab_link_bytes(g, precision, link_reals));
    WL_HIP(launch_lab_pack_spinor(fin.get(), in, g, layout, precision, 1 - parity, s));
    WL_HIP(launch_lab_pack_links(u0.get(), U, g, layout, precision, link_reals, 0, s));
    WL_HIP(launch_lab_pack_links(u1.get(), U, g, layout, precision, link_reals, 1, s));
    WL_HIP(launch_lab_hop(fout.get(), fin.get(), u0.get(), u1.get(), g, layout, precision, link_reals, parity, -kappa, s));
    double us = 0.0;
    if (reps > 0) {
        hipEvent_t e0, e1;
        WL_HIP(hipEventCreate(&e0));
        WL_HIP(hipEventCreate(&e1));
        WL_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; r++)
            WL_HIP(launch_lab_hop(fout.get(), fin.get(), u0.get(), u1.get(), g, layout, precision, link_reals, parity,
                                  -kappa, s));
        WL_HIP(hipEventRecord(e1, s));
        WL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        WL_HIP(hipEventElapsedTime(&ms, e0, e1));
        WL_HIP(hipEventDestroy(e0));
        WL_HIP(hipEventDestroy(e1));
        us = 1000.0 * ms / reps;
    }
    WL_HIP(launch_lab_zero(out, V * 24, s));
    WL_HIP(launch_lab_unpack_spinor(out, fout.get(), g, layout, precision, parity, s));
    WL_HIP(hipStreamSynchronize(s));
    if (us_per_launch) *us_per_launch = us;
    return WILSON_OK;
    API_END
}

int wilson_stream_copy(wilson_ctx *ctx, void *dst, const void *src, size_t bytes) {
    API_BEGIN
    WL_CHECK_ARG(ctx && dst && src, "NULL argument");
    WL_CHECK_ARG(is_device_ptr(dst) && is_device_ptr(src), "stream copy needs device pointers");
    WL_HIP(launch_stream_copy(dst, src, bytes, ctx->stream));
    return WILSON_OK;
    API_END
}

int wilson_stream_read(wilson_ctx *ctx, const void *src, size_t bytes) {
    API_BEGIN
    WL_CHECK_ARG(ctx && src, "NULL argument");
    WL_CHECK_ARG(is_device_ptr(src), "stream read needs a device pointer");
    if (ctx->flag.size() < 8192 * sizeof(unsigned)) {
        WL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->flag.alloc(8192 * sizeof(unsigned));
    }
    WL_HIP(launch_stream_read(src, bytes, ctx->flag.as<unsigned>(), ctx->stream));
    return WILSON_OK;
    API_END
}

}  // extern "C"
