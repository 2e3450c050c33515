// reg.hip - regularisation terms of the LM step (Sec. 4.4: handle length, end point
// snapping, sparsity) with their analytic gradients and positive semi-definite Hessians,
// and handle pruning.  Everything here is float64 and O(H) (snapping: O(H^2) end point
// pairs), so a thread owns a handle or an end point and writes only that one's rows and
// columns of the gradient and Hessian.
#include <cmath>

#include "common.hpp"

namespace bem {

namespace {

// Columns of one handle's parameters: first and last end point (x; y follows), jump vectors.
struct HandleCols {
    int Q, e0, e1, nwd, wd[2], nwc, wc[2];
};

__host__ __device__ inline HandleCols handle_cols(int model)
{
    if (model == 1) return HandleCols{10, 0, 2, 1, {4, 0}, 1, {7, 0}};
    return HandleCols{20, 0, 6, 2, {8, 11}, 2, {14, 17}};
}

// column of coordinate 0 of end point e = 2h + j
__device__ inline int64_t endpoint_col(const HandleCols& L, int e)
{
    return (int64_t)(e >> 1) * L.Q + ((e & 1) ? L.e1 : L.e0);
}

// Hessian block update: Hm[r0 + a][c0 + b] += s * B[a][b], a, b < n
__device__ inline void add_block(double* Hm, int64_t P, int64_t r0, int64_t c0, int n, const double* B, double s)
{
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) Hm[(r0 + a) * P + c0 + b] += s * B[a * n + b];
}

// Thread per handle: length and sparsity terms.  vals[h] = the handle's value; with grad,
// g and Hm (P x P) are accumulated on the handle's own columns.
__global__ void k_reg_handles(const double* __restrict__ theta, int H, int model, bem_reg r, int grad,
                              double* __restrict__ g, double* __restrict__ Hm, int64_t P, double* __restrict__ vals)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    const HandleCols L = handle_cols(model);
    const double* th = theta + (size_t)h * L.Q;
    const int64_t base = (int64_t)h * L.Q;
    double v = 0.0;
    if (r.length_weight > 0.0) {
        const double dx = th[L.e1] - th[L.e0], dy = th[L.e1 + 1] - th[L.e0 + 1];
        const double ln = sqrt(dx * dx + dy * dy);
        if (ln > r.length_max) {
            const double ex = ln - r.length_max;
            v += r.length_weight * ex * ex;
            if (grad) {
                const double tx = dx / ln, ty = dy / ln;
                const double gs = 2.0 * r.length_weight * ex;
                const int64_t c0 = base + L.e0, c1 = base + L.e1;
                g[c1] += gs * tx;
                g[c1 + 1] += gs * ty;
                g[c0] -= gs * tx;
                g[c0 + 1] -= gs * ty;
                // 2 mu (tau tau^T + ex / l (I - tau tau^T)) on (E1, E1), (E0, E0); minus on the cross blocks
                const double q = ex / ln;
                const double B[4] = {tx * tx + q * (1.0 - tx * tx), tx * ty - q * tx * ty,
                                     tx * ty - q * tx * ty, ty * ty + q * (1.0 - ty * ty)};
                const double s2 = 2.0 * r.length_weight;
                add_block(Hm, P, c1, c1, 2, B, s2);
                add_block(Hm, P, c0, c0, 2, B, s2);
                add_block(Hm, P, c0, c1, 2, B, -s2);
                add_block(Hm, P, c1, c0, 2, B, -s2);
            }
        }
    }
    for (int kind = 0; kind < 2; ++kind) {
        const double lam = kind == 0 ? r.sparse_wd : r.sparse_wc;
        if (!(lam > 0.0)) continue;
        const int n = kind == 0 ? L.nwd : L.nwc;
        for (int m = 0; m < n; ++m) {
            const int c = kind == 0 ? L.wd[m] : L.wc[m];
            const double w0 = th[c], w1 = th[c + 1], w2 = th[c + 2];
            const double s = sqrt(w0 * w0 + w1 * w1 + w2 * w2 + r.sparse_eps * r.sparse_eps);
            const double tt = tanh(s / r.sparse_t);
            v += lam * r.sparse_t * tt;
            if (!grad || s == 0.0) continue;
            const double f1 = lam * (1.0 - tt * tt);          // d/ds of lam t tanh(s/t)
            const double u[3] = {w0 / s, w1 / s, w2 / s};
            double B[9];
            for (int a = 0; a < 3; ++a) {
                g[base + c + a] += f1 * u[a];
                for (int b = 0; b < 3; ++b) B[3 * a + b] = (a == b ? 1.0 : 0.0) - u[a] * u[b];
            }
            add_block(Hm, P, base + c, base + c, 3, B, f1 / s);
        }
    }
    vals[h] = v;
}

// Unit direction of handle h's chord E1 - E0 (0 for a zero-length handle).
__device__ inline void chord_dir(const double* theta, const HandleCols& L, int h, double& tx, double& ty)
{
#pragma clang fp contract(off)
    const double* th = theta + (size_t)h * L.Q;
    const double dx = th[L.e1] - th[L.e0], dy = th[L.e1 + 1] - th[L.e0 + 1];
    const double ln = sqrt(dx * dx + dy * dy);
    tx = ln > 0.0 ? dx / ln : 0.0;
    ty = ln > 0.0 ? dy / ln : 0.0;
}

// Thread per end point i: best[i] = the end point j of another handle, closer than dist,
// with the lowest snapping score (the first one on ties), or -1.  The score's arithmetic is
// kept in separately rounded operations (no contraction) so that the decision is the one
// the plain formula takes.
__global__ void k_snap_best(const double* __restrict__ theta, int H, int model, double dist, double mix,
                            int* __restrict__ best)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 2 * H;
    if (i >= n) return;
    const HandleCols L = handle_cols(model);
    const double* ei = theta + endpoint_col(L, i);
    const double xi = ei[0], yi = ei[1];
    double ti_x, ti_y;
    chord_dir(theta, L, i >> 1, ti_x, ti_y);
    double bs = INFINITY;
    int b = -1;
    for (int j = 0; j < n; ++j) {
        if ((j >> 1) == (i >> 1)) continue;
        const double* ej = theta + endpoint_col(L, j);
        const double dx = xi - ej[0], dy = yi - ej[1];
        const double d = sqrt(dx * dx + dy * dy);
        if (!(d < dist)) continue;
        double tj_x, tj_y;
        chord_dir(theta, L, j >> 1, tj_x, tj_y);
        const double dot = fabs(ti_x * tj_x + ti_y * tj_y);
        const double s = mix * (d / dist) + (1.0 - mix) * (1.0 - dot);
        if (s < bs) {
            bs = s;
            b = j;
        }
    }
    best[i] = b;
}

// Thread per end point i: if i and best[i] = j > i are each other's best, the pair's value
// mu |e_i - e_j|^2 goes to vals[i] (and with grad its gradient and Hessian into the two
// end points' columns); cnt[i] = 1 for a pair.
__global__ void k_snap_apply(const double* __restrict__ theta, int H, int model, double mu,
                             const int* __restrict__ best, int grad, double* __restrict__ g, double* __restrict__ Hm,
                             int64_t P, double* __restrict__ vals, int* __restrict__ cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * H) return;
    const int j = best[i];
    double v = 0.0;
    int c = 0;
    if (j > i && best[j] == i) {
        const HandleCols L = handle_cols(model);
        const int64_t ci = endpoint_col(L, i), cj = endpoint_col(L, j);
        const double dx = theta[ci] - theta[cj], dy = theta[ci + 1] - theta[cj + 1];
        v = mu * (dx * dx + dy * dy);
        c = 1;
        if (grad) {
            g[ci] += 2.0 * mu * dx;
            g[ci + 1] += 2.0 * mu * dy;
            g[cj] -= 2.0 * mu * dx;
            g[cj + 1] -= 2.0 * mu * dy;
            const double I2[4] = {1.0, 0.0, 0.0, 1.0};
            add_block(Hm, P, ci, ci, 2, I2, 2.0 * mu);
            add_block(Hm, P, cj, cj, 2, I2, 2.0 * mu);
            add_block(Hm, P, ci, cj, 2, I2, -2.0 * mu);
            add_block(Hm, P, cj, ci, 2, I2, -2.0 * mu);
        }
    }
    vals[i] = v;
    cnt[i] = c;
}

// One block: out[0] = sum of vals[0 .. n), out[1] = sum of cnt[0 .. m) (fixed order).
__global__ void __launch_bounds__(256) k_reg_sum(const double* __restrict__ vals, int64_t n,
                                                 const int* __restrict__ cnt, int64_t m, double* __restrict__ out)
{
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) a += vals[i];
    for (int64_t i = threadIdx.x; i < m; i += 256) b += (double)cnt[i];
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

// keep[h] = 1 if the handle's wd norm or wc norm (largest over its ends) is >= threshold
__global__ void k_prune_flags(const double* __restrict__ theta, int H, int model, double thr, int* __restrict__ keep)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    const HandleCols L = handle_cols(model);
    const double* th = theta + (size_t)h * L.Q;
    bool k = false;
    for (int kind = 0; kind < 2; ++kind) {
        const int n = kind == 0 ? L.nwd : L.nwc;
        double nm = 0.0;
        bool nan = false;
        for (int m = 0; m < n; ++m) {
            const int c = kind == 0 ? L.wd[m] : L.wc[m];
            const double v = sqrt(th[c] * th[c] + th[c + 1] * th[c + 1] + th[c + 2] * th[c + 2]);
            nan = nan || isnan(v);
            nm = fmax(nm, v);
        }
        if (!nan && nm >= thr) k = true;
    }
    keep[h] = k ? 1 : 0;
}

// One block of 1024 threads: stable compaction of the kept handles' rows into out;
// count[0] = the number kept.  Thread t scans the contiguous chunk [t c, (t + 1) c).
__global__ void __launch_bounds__(1024) k_prune_compact(const double* __restrict__ theta, int H, int Q,
                                                        const int* __restrict__ keep, double* __restrict__ out,
                                                        int* __restrict__ count)
{
    __shared__ int pre[1024];
    const int t = threadIdx.x;
    const int chunk = (H + 1023) / 1024;
    const int lo = t * chunk < H ? t * chunk : H, hi = lo + chunk < H ? lo + chunk : H;
    int c = 0;
    for (int h = lo; h < hi; ++h) c += keep[h];
    pre[t] = c;
    __syncthreads();
    for (int s = 1; s < 1024; s <<= 1) {       // inclusive scan (Hillis-Steele)
        const int v = t >= s ? pre[t - s] : 0;
        __syncthreads();
        pre[t] += v;
        __syncthreads();
    }
    int o = pre[t] - c;
    for (int h = lo; h < hi; ++h)
        if (keep[h]) {
            for (int q = 0; q < Q; ++q) out[(size_t)o * Q + q] = theta[(size_t)h * Q + q];
            ++o;
        }
    if (t == 1023) count[0] = pre[1023];
}

}  // namespace

bool reg_active(const bem_ctx* ctx)
{
    const bem_reg& r = ctx->reg;
    return r.length_weight > 0.0 || r.snap_weight > 0.0 || r.sparse_wd > 0.0 || r.sparse_wc > 0.0;
}

int check_reg(const bem_reg& r, char* why, size_t n)
{
    const double w[] = {r.length_weight, r.length_max, r.snap_weight, r.sparse_wd, r.sparse_wc};
    for (double v : w)
        if (!(v >= 0.0) || !std::isfinite(v)) {
            snprintf(why, n, "regularisation weights and length_max must be finite and >= 0");
            return BEM_EINVAL;
        }
    if (r.snap_weight > 0.0 && (!(r.snap_dist > 0.0) || !std::isfinite(r.snap_dist) || !(r.snap_mix >= 0.0) ||
                                !(r.snap_mix <= 1.0))) {
        snprintf(why, n, "snapping needs snap_dist > 0 and snap_mix in [0, 1]");
        return BEM_EINVAL;
    }
    if ((r.sparse_wd > 0.0 || r.sparse_wc > 0.0) &&
        (!(r.sparse_t > 0.0) || !std::isfinite(r.sparse_t) || !(r.sparse_eps >= 0.0) || !std::isfinite(r.sparse_eps))) {
        snprintf(why, n, "sparsity needs sparse_t > 0 and sparse_eps >= 0");
        return BEM_EINVAL;
    }
    return BEM_OK;
}

// Regularisation terms at theta.  choose: pick the snapping pairs at theta (else keep the
// ones of the last call).  With g and Hm (both or neither) their gradient and Hessian are
// added into them.  *value (host) = the terms' sum, *pairs (host, may be null) = snapped
// pairs.  Synchronises.
int reg_terms(bem_ctx* ctx, const double* theta, int H, bool choose, double* g, double* Hm, double* value, int* pairs,
              hipStream_t s)
{
    int rc;
    const bem_reg& r = ctx->reg;
    const int model = ctx->model;
    const int64_t P = (int64_t)ctx->npar * H;
    const bool snap = r.snap_weight > 0.0;
    if (snap && H > 65536) return set_error(ctx, BEM_EINVAL, "end point snapping is limited to H <= 65536");
    const int n = H > 0 ? H : 1;
    // regw: vals [3H] | out [2] | best [2H] int | cnt [2H] int
    const size_t bytes = ((size_t)3 * n + 2) * sizeof(double) + (size_t)4 * n * sizeof(int) + 64;
    if ((rc = ensure(ctx, ctx->regw, bytes, s))) return rc;
    double* vals = (double*)ctx->regw.ptr;
    double* out = vals + (size_t)3 * n;
    int* best = (int*)(out + 2);
    int* cnt = best + 2 * n;
    const int grad = g != nullptr;
    if (H > 0) {
        hipLaunchKernelGGL(k_reg_handles, dim3(blocks_for(H, 128)), dim3(128), 0, s, theta, H, model, r, grad, g, Hm,
                           P, vals);
        if (snap) {
            if (choose)
                hipLaunchKernelGGL(k_snap_best, dim3(blocks_for(2 * H, 128)), dim3(128), 0, s, theta, H, model,
                                   r.snap_dist, r.snap_mix, best);
            hipLaunchKernelGGL(k_snap_apply, dim3(blocks_for(2 * H, 128)), dim3(128), 0, s, theta, H, model,
                               r.snap_weight, (const int*)best, grad, g, Hm, P, vals + H, cnt);
        }
    }
    const int64_t nv = H > 0 ? (snap ? 3 * (int64_t)H : H) : 0;
    const int64_t nc = H > 0 && snap ? 2 * (int64_t)H : 0;
    hipLaunchKernelGGL(k_reg_sum, dim3(1), dim3(256), 0, s, (const double*)vals, nv, (const int*)cnt, nc, out);
    if ((rc = check_launch(ctx, "regularisation"))) return rc;
    double host[2];
    if (hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "regularisation readback");
    *value = host[0];
    if (pairs) *pairs = (int)host[1];
    return BEM_OK;
}

int run_prune(bem_ctx* ctx, double* theta, int H, double thr, int* H_out, hipStream_t s)
{
    int rc;
    const int Q = ctx->npar;
    if (H == 0) {
        *H_out = 0;
        return BEM_OK;
    }
    // tmp0: the compacted rows; regw: keep [H] and the count
    if ((rc = ensure(ctx, ctx->tmp0, (size_t)H * Q * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->regw, ((size_t)H + 16) * sizeof(int), s))) return rc;
    int* keep = (int*)ctx->regw.ptr;
    int* count = keep + H;
    double* out = (double*)ctx->tmp0.ptr;
    hipLaunchKernelGGL(k_prune_flags, dim3(blocks_for(H, 256)), dim3(256), 0, s, (const double*)theta, H, ctx->model,
                       thr, keep);
    hipLaunchKernelGGL(k_prune_compact, dim3(1), dim3(1024), 0, s, (const double*)theta, H, Q, (const int*)keep, out,
                       count);
    if ((rc = check_launch(ctx, "prune"))) return rc;
    int kept = 0;
    if (hipMemcpyAsync(&kept, count, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "prune readback");
    if (kept > 0 && hipMemcpyAsync(theta, out, (size_t)kept * Q * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "prune copy");
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, BEM_EHIP, "prune sync");
    *H_out = kept;
    return BEM_OK;
}

}  // namespace bem
