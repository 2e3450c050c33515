// api.hip - the C ABI of include/bem.h: argument checks, call order,
// workspaces and the orchestration of the kernels of each entry point.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "common.hpp"

namespace bem {

static thread_local std::string g_build_error;

int set_error(bem_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_build_error = buf;
    return code;
}

int ensure(bem_ctx* ctx, DevBuf& b, size_t bytes, hipStream_t stream)
{
    if (bytes <= b.bytes && b.ptr) return BEM_OK;
    if (b.ptr) {
        // kernels already queued may still read the old buffer
        if (hipStreamSynchronize(stream) != hipSuccess) return set_error(ctx, BEM_EHIP, "stream sync before regrow");
        hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        b.ptr = nullptr;
        hipGetLastError();
        return set_error(ctx, BEM_ENOMEM, "hipMalloc of %zu bytes failed", want);
    }
    b.bytes = want;
    return BEM_OK;
}

// The context's second stream (default priority) and its six events (no timing).
int aux_stream(bem_ctx* ctx, hipStream_t* out)
{
    if (!ctx->s2) {
        if (hipStreamCreateWithFlags(&ctx->s2, hipStreamNonBlocking) != hipSuccess) {
            ctx->s2 = nullptr;
            hipGetLastError();
            return set_error(ctx, BEM_EHIP, "second stream");
        }
        for (hipEvent_t& e : ctx->ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                e = nullptr;
                hipGetLastError();
                return set_error(ctx, BEM_EHIP, "stream events");
            }
    }
    *out = ctx->s2;
    return BEM_OK;
}

int check_launch(bem_ctx* ctx, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ctx, BEM_EHIP, "%s: %s", what, hipGetErrorString(e));
    return BEM_OK;
}

static hipEvent_t pool_get(bem_ctx* ctx)
{
    auto& P = ctx->prof.pool;
    if (!P.empty()) {
        hipEvent_t e = P.back();
        P.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        hipGetLastError();
        return nullptr;
    }
    return e;
}

void prof_begin(bem_ctx* ctx, int, hipStream_t s, hipEvent_t* start)
{
    *start = nullptr;
    if (!ctx || !ctx->prof.on) return;
    hipEvent_t e = pool_get(ctx);
    if (e && hipEventRecord(e, s) == hipSuccess) *start = e;
}

void prof_end(bem_ctx* ctx, int tag, hipStream_t s, hipEvent_t start)
{
    if (!ctx || !start) return;
    hipEvent_t e = pool_get(ctx);
    if (!e || hipEventRecord(e, s) != hipSuccess) {
        ctx->prof.pool.push_back(start);
        return;
    }
    ctx->prof.tags.push_back(tag);
    ctx->prof.starts.push_back(start);
    ctx->prof.stops.push_back(e);
}

static void prof_resolve(bem_ctx* ctx)
{
    auto& p = ctx->prof;
    for (size_t i = 0; i < p.tags.size(); ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stops[i]) == hipSuccess && hipEventElapsedTime(&ms, p.starts[i], p.stops[i]) == hipSuccess) {
            p.total_ms[p.tags[i]] += ms;
            p.launches[p.tags[i]] += 1;
        }
        p.pool.push_back(p.starts[i]);
        p.pool.push_back(p.stops[i]);
    }
    p.tags.clear();
    p.starts.clear();
    p.stops.clear();
    hipGetLastError();
}

static void release(DevBuf& b)
{
    if (b.ptr) hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

int check_common(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N)
{
    if (!ctx) return BEM_EINVAL;
    ctx->err.clear();
    if (ctx->state < 2) return set_error(ctx, BEM_ESTATE, "the boundary system is not factored (call bem_factor)");
    if (H < 0 || H > (1 << 20)) return set_error(ctx, BEM_EINVAL, "H = %d out of range", (int)H);
    if ((int64_t)H * ctx->opts.segs_per_handle > (1 << 24)) return set_error(ctx, BEM_EINVAL, "too many segments");
    if (N < 0 || N > ((int64_t)1 << 31)) return set_error(ctx, BEM_EINVAL, "N = %lld out of range", (long long)N);
    if (H > 0 && !theta) return set_error(ctx, BEM_EINVAL, "theta is null");
    if (N > 0 && !x) return set_error(ctx, BEM_EINVAL, "x is null");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, BEM_EHIP, "hipSetDevice(%d)", ctx->device);
    return BEM_OK;
}

// expand + element geometry tables (the element values are not used by callers of this one).
int prepare_forward_tables(bem_ctx* ctx, const double* theta, int32_t H, hipStream_t s)
{
    int rc;
    if ((rc = ensure(ctx, ctx->U, (size_t)ctx->M * 3 * sizeof(double), s))) return rc;
    if ((rc = launch_expand(ctx, theta, H, s))) return rc;
    return launch_pack_elements(ctx, (const double*)ctx->U.ptr, s);
}

// expand -> F -> U -> element table.  Leaves F in ctx->F and U in ctx->U.
int prepare_forward(bem_ctx* ctx, const double* theta, int32_t H, bool mixed, hipStream_t s)
{
    int rc;
    const int K = H * ctx->opts.segs_per_handle;
    if ((rc = ensure(ctx, ctx->F, (size_t)ctx->M * 3 * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->U, (size_t)ctx->M * 3 * sizeof(double), s))) return rc;
    if ((rc = launch_expand(ctx, theta, H, s))) return rc;
    if ((rc = launch_boundary_rhs(ctx, K, (double*)ctx->F.ptr, mixed, s))) return rc;
    if ((rc = launch_boundary_solve(ctx, (const double*)ctx->F.ptr, (double*)ctx->U.ptr, false, s))) return rc;
    return launch_pack_elements(ctx, (const double*)ctx->U.ptr, s);
}

}  // namespace bem

using namespace bem;

extern "C" {

// Shared part of bem_build / bem_build_elements: validate the options, create the context and
// its element table (elems: host [M][4], or null for the unit square), assemble A.
static int build_context(const bem_opts* opts, const double* elems, int M, hipStream_t stream, bem_ctx** out)
{
    g_build_error.clear();
    if (!opts || !out) return set_error(nullptr, BEM_EINVAL, "null opts or out");
    *out = nullptr;
    const bem_opts& o = *opts;
    if (!elems && (o.elems_per_side < 2 || o.elems_per_side > 1024))
        return set_error(nullptr, BEM_EINVAL, "elems_per_side = %d not in [2, 1024]", o.elems_per_side);
    if (o.segs_per_handle < 1 || o.segs_per_handle > 1024)
        return set_error(nullptr, BEM_EINVAL, "segs_per_handle = %d not in [1, 1024]", o.segs_per_handle);
    if (!(o.eps >= 0.0) || !std::isfinite(o.eps)) return set_error(nullptr, BEM_EINVAL, "eps must be finite and >= 0");
    if (!(o.near_factor > 0.0) || !std::isfinite(o.near_factor))
        return set_error(nullptr, BEM_EINVAL, "near_factor must be finite and > 0");
    if (o.tile_rows < 0) return set_error(nullptr, BEM_EINVAL, "tile_rows must be >= 0");
    if (o.handle_model != BEM_HANDLE_CUBIC && o.handle_model != BEM_HANDLE_STRAIGHT)
        return set_error(nullptr, BEM_EINVAL, "handle_model = %d is neither cubic (0) nor straight (1)", o.handle_model);
    if (elems) {
        if (M < 2 || M > 4096) return set_error(nullptr, BEM_EINVAL, "M = %d elements not in [2, 4096]", M);
        for (int i = 0; i < M; ++i) {
            const double* e = elems + 4 * (size_t)i;
            const double dx = e[2] - e[0], dy = e[3] - e[1];
            if (!std::isfinite(e[0]) || !std::isfinite(e[1]) || !std::isfinite(e[2]) || !std::isfinite(e[3]) ||
                !(dx * dx + dy * dy > 0.0))
                return set_error(nullptr, BEM_EINVAL, "element %d is degenerate or not finite", i);
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        hipGetLastError();
        return set_error(nullptr, BEM_EHIP, "no HIP device");
    }
    if (o.device < 0 || o.device >= ndev) return set_error(nullptr, BEM_EINVAL, "device %d not present", o.device);
    if (hipSetDevice(o.device) != hipSuccess) return set_error(nullptr, BEM_EHIP, "hipSetDevice");
    bem_ctx* ctx = new (std::nothrow) bem_ctx();
    if (!ctx) return set_error(nullptr, BEM_ENOMEM, "context allocation");
    ctx->opts = o;
    ctx->device = o.device;
    ctx->per_side = elems ? 0 : o.elems_per_side;
    ctx->M = elems ? M : 4 * o.elems_per_side;
    ctx->model = o.handle_model;
    const bool straight = o.handle_model == BEM_HANDLE_STRAIGHT;
    ctx->npar = straight ? 10 : 20;
    ctx->ngeo = straight ? 4 : 8;
    ctx->ncol = straight ? 2 : 4;
    const size_t ebytes = (size_t)ctx->M * 4 * sizeof(double);
    int rc = ensure(ctx, ctx->egeo, ebytes, stream);
    if (!rc) {
        if (elems) {
            double bb[4] = {elems[0], elems[1], elems[0], elems[1]};
            for (int i = 0; i < 2 * ctx->M; ++i) {
                const double px = elems[2 * i], py = elems[2 * i + 1];
                bb[0] = std::fmin(bb[0], px); bb[1] = std::fmin(bb[1], py);
                bb[2] = std::fmax(bb[2], px); bb[3] = std::fmax(bb[3], py);
            }
            for (int k = 0; k < 4; ++k) ctx->bbox[k] = bb[k];
            if (hipMemcpyAsync(ctx->egeo.ptr, elems, ebytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                rc = set_error(ctx, BEM_EHIP, "element upload");
        } else {
            rc = launch_square_elements(ctx, stream);
        }
    }
    if (!rc) rc = ensure(ctx, ctx->A, (size_t)ctx->M * ctx->M * sizeof(double), stream);
    if (!rc) rc = launch_assemble(ctx, stream);
    if (rc) {
        g_build_error = ctx->err;
        bem_destroy(ctx);
        return rc;
    }
    ctx->state = 1;
    *out = ctx;
    return BEM_OK;
}

int bem_build(const bem_opts* opts, hipStream_t stream, bem_ctx** out)
{
    return build_context(opts, nullptr, 0, stream, out);
}

int bem_build_elements(const bem_opts* opts, const double* elems, int32_t M, hipStream_t stream, bem_ctx** out)
{
    if (!elems) {
        g_build_error = "elems is null";
        return BEM_EINVAL;
    }
    return build_context(opts, elems, M, stream, out);
}

int bem_factor(bem_ctx* ctx, hipStream_t stream)
{
    if (!ctx) return BEM_EINVAL;
    ctx->err.clear();
    if (ctx->state < 1) return set_error(ctx, BEM_ESTATE, "not built");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, BEM_EHIP, "hipSetDevice");
    const int rc = launch_factor(ctx, stream);
    if (rc) return rc;
    ctx->state = 2;
    return BEM_OK;
}

int bem_eval(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N, const double* cbar, void* u,
             bem_prec prec, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, x, N);
    if (rc) return rc;
    if (!cbar) return set_error(ctx, BEM_EINVAL, "cbar is null");
    if (N > 0 && !u) return set_error(ctx, BEM_EINVAL, "u is null");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return set_error(ctx, BEM_EINVAL, "bad precision %d", (int)prec);
    if ((rc = prepare_forward(ctx, theta, H, prec == BEM_PREC_MIXED, stream))) return rc;
    const int K = H * ctx->opts.segs_per_handle;
    if (prec == BEM_PREC_FP64) return launch_sweep_f64(ctx, x, N, K, cbar, (double*)u, stream);
    return launch_sweep_mixed(ctx, x, N, K, cbar, (float*)u, stream);
}

constexpr int64_t kVjpCellOrderMin = 65536;     // samples from which MIXED bem_vjp reorders them

int bem_vjp(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N, const void* gbar, double* grad,
            bem_prec prec, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, x, N);
    if (rc) return rc;
    if (N > 0 && !gbar) return set_error(ctx, BEM_EINVAL, "gbar is null");
    if (H > 0 && !grad) return set_error(ctx, BEM_EINVAL, "grad is null");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return set_error(ctx, BEM_EINVAL, "bad precision %d", (int)prec);
    // MIXED with many samples: visit them cell by cell, so that the near pairs of a wavefront form
    // long runs of one segment (one set of float64 sums per run instead of one per pair)
    if (prec == BEM_PREC_MIXED && H > 0 && N >= kVjpCellOrderMin) {
        const double* xo;
        const float* go;
        if ((rc = cell_order_f32(ctx, x, (const float*)gbar, N, &xo, &go, stream))) return rc;
        return run_vjp(ctx, theta, H, xo, N, go, true, grad, stream);
    }
    return run_vjp(ctx, theta, H, x, N, gbar, prec == BEM_PREC_MIXED, grad, stream);
}

int bem_jtj(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N, const void* resid, double* JtJ,
            double* Jtr, bem_gram gram, bem_prec prec, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, x, N);
    if (rc) return rc;
    if (N > 0 && !resid) return set_error(ctx, BEM_EINVAL, "resid is null");
    if (H > 0 && (!JtJ || !Jtr)) return set_error(ctx, BEM_EINVAL, "JtJ / Jtr is null");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return set_error(ctx, BEM_EINVAL, "bad precision %d", (int)prec);
    if (gram != BEM_GRAM_FP64 && gram != BEM_GRAM_FP32_MFMA && gram != BEM_GRAM_BF16X3_MFMA && gram != BEM_GRAM_FP64_VALU)
        return set_error(ctx, BEM_EINVAL, "bad gram mode %d", (int)gram);
    return run_jtj(ctx, theta, H, x, N, resid, prec == BEM_PREC_MIXED, (int)gram, JtJ, Jtr, stream);
}

int lm_step(bem_ctx* ctx, double* theta, int32_t H, const double* x, int64_t N, const double* target,
            bem_lm_state* state, bem_gram gram, bem_prec prec, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, x, N);
    if (rc) return rc;
    if (!state) return set_error(ctx, BEM_EINVAL, "state is null");
    if (N > 0 && !target) return set_error(ctx, BEM_EINVAL, "target is null");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return set_error(ctx, BEM_EINVAL, "bad precision %d", (int)prec);
    if (gram != BEM_GRAM_FP64 && gram != BEM_GRAM_FP32_MFMA && gram != BEM_GRAM_BF16X3_MFMA && gram != BEM_GRAM_FP64_VALU)
        return set_error(ctx, BEM_EINVAL, "bad gram mode %d", (int)gram);
    if (state->mean_rule != 0 && state->mean_rule != 1) return set_error(ctx, BEM_EINVAL, "bad mean_rule");
    if (state->compat != 0 && state->compat != 1) return set_error(ctx, BEM_EINVAL, "bad compat flag");
    if (!(state->lambda > 0.0) || !std::isfinite(state->lambda)) return set_error(ctx, BEM_EINVAL, "lambda must be > 0");
    state->lambda = std::fmin(std::fmax(state->lambda, 1e-12), 1e12);
    rc = run_lm_step(ctx, theta, H, x, N, target, state, (int)gram, prec == BEM_PREC_MIXED, stream);
    if (rc && ctx->err.empty()) set_error(ctx, rc, "lm_step failed");
    return rc;
}

int bem_jacobian(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N, double* J, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, x, N);
    if (rc) return rc;
    if (N > 0 && H > 0 && !J) return set_error(ctx, BEM_EINVAL, "J is null");
    if (N > (1 << 20)) return set_error(ctx, BEM_EINVAL, "bem_jacobian is meant for small N (<= 2^20)");
    return run_jacobian(ctx, theta, H, x, N, J, stream);
}

int bem_set_regularization(bem_ctx* ctx, const bem_reg* reg)
{
    if (!ctx) return BEM_EINVAL;
    ctx->err.clear();
    if (!reg) {
        ctx->reg = bem_reg{};
        return BEM_OK;
    }
    char why[160];
    if (check_reg(*reg, why, sizeof(why))) return set_error(ctx, BEM_EINVAL, "%s", why);
    ctx->reg = *reg;
    return BEM_OK;
}

int bem_regularization(bem_ctx* ctx, const double* theta, int32_t H, double* value, double* grad, double* hess,
                       int32_t* pairs, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, nullptr, 0);
    if (rc) return rc;
    if (!value) return set_error(ctx, BEM_EINVAL, "value is null");
    if ((grad == nullptr) != (hess == nullptr)) return set_error(ctx, BEM_EINVAL, "give both grad and hess or neither");
    const int64_t P = (int64_t)ctx->npar * H;
    if (grad && P > 0) {
        if ((rc = fill_f64(ctx, grad, P, 0.0, stream))) return rc;
        if ((rc = fill_f64(ctx, hess, P * P, 0.0, stream))) return rc;
    }
    int np = 0;
    if ((rc = reg_terms(ctx, theta, H, true, grad, hess, value, &np, stream))) return rc;
    if (pairs) *pairs = np;
    return BEM_OK;
}

int bem_prune(bem_ctx* ctx, double* theta, int32_t H, double threshold, int32_t* H_out, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, nullptr, 0);
    if (rc) return rc;
    if (!H_out) return set_error(ctx, BEM_EINVAL, "H_out is null");
    if (!(threshold >= 0.0) || !std::isfinite(threshold)) return set_error(ctx, BEM_EINVAL, "threshold must be >= 0");
    int kept = 0;
    if ((rc = run_prune(ctx, theta, H, threshold, &kept, stream))) return rc;
    *H_out = kept;
    return BEM_OK;
}

int bem_partition_samples(bem_ctx* ctx, const int32_t* labels, int64_t N, int32_t D, const double* x, const double* T,
                          double* x_out, double* T_out, int64_t* offsets, hipStream_t stream)
{
    if (!ctx) return BEM_EINVAL;
    ctx->err.clear();
    if (!offsets) return set_error(ctx, BEM_EINVAL, "offsets is null");
    if (N < 0 || N > ((int64_t)1 << 31)) return set_error(ctx, BEM_EINVAL, "N = %lld out of range", (long long)N);
    if (N > 0 && (!labels || !x || !x_out || (T && !T_out)))
        return set_error(ctx, BEM_EINVAL, "null labels, x, x_out or T_out");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, BEM_EHIP, "hipSetDevice(%d)", ctx->device);
    return run_partition(ctx, labels, N, D, x, T, x_out, T_out, offsets, stream);
}

int bem_boundary_solve(bem_ctx* ctx, const double* theta, int32_t H, double* F, double* U, hipStream_t stream)
{
    int rc = check_common(ctx, theta, H, nullptr, 0);
    if (rc) return rc;
    if ((rc = prepare_forward(ctx, theta, H, false, stream))) return rc;
    const size_t bytes = (size_t)ctx->M * 3 * sizeof(double);
    if (F && hipMemcpyAsync(F, ctx->F.ptr, bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "copy F");
    if (U && hipMemcpyAsync(U, ctx->U.ptr, bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "copy U");
    return BEM_OK;
}

int bem_get_matrix(bem_ctx* ctx, int32_t which, double* out, hipStream_t stream)
{
    if (!ctx) return BEM_EINVAL;
    ctx->err.clear();
    if (!out) return set_error(ctx, BEM_EINVAL, "out is null");
    if (which != 0 && which != 1) return set_error(ctx, BEM_EINVAL, "which must be 0 or 1");
    if (ctx->state < 1 + which) return set_error(ctx, BEM_ESTATE, "matrix not available yet");
    const DevBuf& b = which ? ctx->Apinv : ctx->A;
    if (hipMemcpyAsync(out, b.ptr, (size_t)ctx->M * ctx->M * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "copy matrix");
    return BEM_OK;
}

int32_t bem_num_elements(const bem_ctx* ctx) { return ctx ? ctx->M : 0; }

int32_t bem_near_capacity(const bem_ctx* ctx) { return ctx ? ctx->near_slots : 0; }

int bem_profile(bem_ctx* ctx, int32_t enable)
{
    if (!ctx) return BEM_EINVAL;
    prof_resolve(ctx);
    for (int t = 0; t < PT_COUNT; ++t) {
        ctx->prof.total_ms[t] = 0.0;
        ctx->prof.launches[t] = 0;
    }
    ctx->prof.on = enable != 0;
    return BEM_OK;
}

int bem_profile_read(bem_ctx* ctx, int32_t tag, double* total_ms, int64_t* launches)
{
    if (!ctx || tag < 0 || tag >= PT_COUNT) return BEM_EINVAL;
    prof_resolve(ctx);
    if (total_ms) *total_ms = ctx->prof.total_ms[tag];
    if (launches) *launches = ctx->prof.launches[tag];
    return BEM_OK;
}

const char* bem_profile_name(int32_t tag)
{
    static const char* names[PT_COUNT] = {"sweep_f64", "sweep_mixed", "vjp_segments", "vjp_elements", "features",
                                          "beta_rows", "gram_f64", "gram_mfma", "xr", "cholesky", "boundary",
                                          "near_pairs"};
    return (tag >= 0 && tag < PT_COUNT) ? names[tag] : "";
}

int bem_factor_info(const bem_ctx* ctx, double* sigma_n, double* shift)
{
    if (!ctx || ctx->state < 2) return BEM_ESTATE;
    if (sigma_n) *sigma_n = ctx->sigma_n;
    if (shift) *shift = ctx->shift;
    return BEM_OK;
}

void bem_destroy(bem_ctx* ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    DevBuf* bufs[] = {&ctx->A, &ctx->Apinv, &ctx->LU, &ctx->piv, &ctx->un, &ctx->vn, &ctx->flag, &ctx->scal,
                      &ctx->seg64, &ctx->seg32, &ctx->F, &ctx->U, &ctx->elem64, &ctx->elem32, &ctx->red,
                      &ctx->tmp0, &ctx->tmp1, &ctx->tmp2, &ctx->tmp3, &ctx->tmp4, &ctx->tmp5, &ctx->lmw,
                      &ctx->nearw, &ctx->nearv, &ctx->nearf, &ctx->regw, &ctx->egeo, &ctx->cholw, &ctx->sortw, &ctx->boxw,
                      &ctx->tilew};
    for (DevBuf* b : bufs) release(*b);
    for (hipEvent_t e : ctx->ev)
        if (e) hipEventDestroy(e);
    if (ctx->s2) hipStreamDestroy(ctx->s2);
    prof_resolve(ctx);
    for (hipEvent_t e : ctx->prof.pool) hipEventDestroy(e);
    delete ctx;
}

const char* bem_last_error(const bem_ctx* ctx)
{
    if (!ctx) return g_build_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"
