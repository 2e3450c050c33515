// forward.hip - the forward path of one evaluation (Sec. 3.1.3):
//   expand     theta -> straight segment table (float64 and float32 copies)
//   bnd_rhs    F_i = 3-point Gauss integral of f over outer element i
//   solve      U = A+ F  (and the transposed product for the adjoint)
//   pack       outer element table with the solved values U
//   sweep      u(x) = cbar + sum_j beta_j(x) U_j + f(x) for every sample
#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr double kGaussNode = 0.77459666924148337703585307995647992;   // sqrt(3/5)
constexpr double kGaussW0 = 5.0 / 9.0, kGaussW1 = 8.0 / 9.0;

// One thread per segment: vertices at t = j/S and j+1/S of the handle (cubic Bezier, or the
// segment A -> B of a straight handle, model 1); cubic jumps linear in t between the handle's
// two ends, straight jumps constant.
__global__ void k_expand(const double* __restrict__ theta, int H, int S, int model, double* __restrict__ seg64,
                         float* __restrict__ seg32)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= H * S) return;
    const int h = k / S, j = k % S;
    const bool straight = model == 1;
    const double* th = theta + (size_t)h * (straight ? 10 : 20);
    const double ta = (double)j / (double)S, tb = (double)(j + 1) / (double)S;
    double wa[4], wb[4];
    vertex_weights(model, ta, wa);
    vertex_weights(model, tb, wb);
    double ax = 0, ay = 0, bx = 0, by = 0;
    for (int c = 0; c < (straight ? 2 : 4); ++c) {
        ax += wa[c] * th[2 * c]; ay += wa[c] * th[2 * c + 1];
        bx += wb[c] * th[2 * c]; by += wb[c] * th[2 * c + 1];
    }
    const double vx = bx - ax, vy = by - ay;
    // a segment no longer than kDegenerateLength carries no integral and no derivative
    const bool live = vx * vx + vy * vy > kDegenerateLength * kDegenerateLength;
    const double L2 = live ? vx * vx + vy * vy : 0.0;
    const double kd = live ? 1.0 / (4.0 * kPi * L2) : 0.0;
    const double ks = live ? 1.0 / (8.0 * kPi * L2 * sqrt(L2)) : 0.0;
    double rec[kSegStride];
    rec[0] = ax; rec[1] = ay; rec[2] = bx; rec[3] = by; rec[4] = vx; rec[5] = vy;
    rec[6] = L2; rec[7] = kd; rec[8] = ks;
    for (int c = 0; c < 3; ++c) {
        if (straight) {
            rec[kWdA + c] = rec[kWdB + c] = th[4 + c];
            rec[kWcA + c] = rec[kWcB + c] = th[7 + c];
        } else {
            rec[kWdA + c] = (1.0 - ta) * th[8 + c] + ta * th[11 + c];
            rec[kWdB + c] = (1.0 - tb) * th[8 + c] + tb * th[11 + c];
            rec[kWcA + c] = (1.0 - ta) * th[14 + c] + ta * th[17 + c];
            rec[kWcB + c] = (1.0 - tb) * th[14 + c] + tb * th[17 + c];
        }
    }
    rec[kIL2] = live ? 1.0 / L2 : 0.0;
    rec[22] = rec[23] = 0.0;
    double* o = seg64 + (size_t)k * kSegStride;
    float* o32 = seg32 + (size_t)k * kSegStride;
    for (int c = 0; c < kSegStride; ++c) { o[c] = rec[c]; o32[c] = (float)rec[c]; }
    if (!live) {
        // float32 record of a degenerate segment: a point far outside the domain with
        // v = 0 and kd = ks = 0, whose moments evaluate to exactly 0 without special cases
        // in the forward sweeps (the derivative sweeps skip it by its L2 = 0)
        o32[0] = o32[2] = 1.0e6f;
        o32[1] = o32[3] = 1.0e6f;
        o32[4] = o32[5] = 0.0f;
    }
}

__device__ inline double block_reduce(double v, double* red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}


// F[i, c] = sum_q w_q |G_i|/2 f_c(x_iq): one block per element, threads over segments.
__global__ void k_boundary_rhs(const double* __restrict__ seg, int K, const double* __restrict__ eg, double eps2,
                               double* __restrict__ F)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    double ax, ay, bx, by;
    load_element(eg, i, ax, ay, bx, by);
    const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by), hx = 0.5 * (bx - ax), hy = 0.5 * (by - ay);
    const double half = sqrt(hx * hx + hy * hy);
    const double node[3] = {-kGaussNode, 0.0, kGaussNode};
    const double w[3] = {kGaussW0 * half, kGaussW1 * half, kGaussW0 * half};
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double* s = seg + (size_t)k * kSegStride;
        const SegGeom<double> g = load_geom(s);
        for (int q = 0; q < 3; ++q) {
            const Moments<double> mo = seg_moments<double, DevF64>(g, mx + node[q] * hx, my + node[q] * hy, eps2);
            for (int c = 0; c < 3; ++c)
                acc[c] += w[q] * (mo.da * s[kWdA + c] + mo.db * s[kWdB + c] + mo.sa * s[kWcA + c] + mo.sb * s[kWcB + c]);
        }
    }
    for (int c = 0; c < 3; ++c) {
        const double r = block_reduce(acc[c], red);
        if (threadIdx.x == 0) F[(size_t)i * 3 + c] = r;
    }
}

// Mixed-precision boundary right-hand side: as k_boundary_rhs, with the pairs of a Gauss
// point and a segment in float32 from the float32 tables unless they are near (the sweeps'
// predicate), then in float64; sums in float64.
__global__ void k_boundary_rhs_mixed(const double* __restrict__ seg, const float* __restrict__ seg32, int K,
                                     const double* __restrict__ eg, double eps2, float near2, double* __restrict__ F)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    double ax, ay, bx, by;
    load_element(eg, i, ax, ay, bx, by);
    const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by), hx = 0.5 * (bx - ax), hy = 0.5 * (by - ay);
    const double half = sqrt(hx * hx + hy * hy);
    const double node[3] = {-kGaussNode, 0.0, kGaussNode};
    const double w[3] = {kGaussW0 * half, kGaussW1 * half, kGaussW0 * half};
    double px[3], py[3];
    float pxf[3], pyf[3];
    for (int q = 0; q < 3; ++q) {
        px[q] = mx + node[q] * hx;
        py[q] = my + node[q] * hy;
        pxf[q] = (float)px[q];
        pyf[q] = (float)py[q];
    }
    const float eps2f = (float)eps2;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float* s32 = seg32 + (size_t)k * kSegStride;
        const SegGeom<float> gf = load_geom(s32);
        for (int q = 0; q < 3; ++q) {
            if (near_segment(gf.ax, gf.ay, gf.bx, gf.by, gf.L2, pxf[q], pyf[q], near2)) {
                const double* s = seg + (size_t)k * kSegStride;
                const Moments<double> mo = seg_moments<double, DevF64>(load_geom(s), px[q], py[q], eps2);
                for (int c = 0; c < 3; ++c)
                    acc[c] += w[q] * (mo.da * s[kWdA + c] + mo.db * s[kWdB + c] + mo.sa * s[kWcA + c] + mo.sb * s[kWcB + c]);
            } else {
                const Moments<float> mo = seg_moments<float, DevF32, false>(gf, pxf[q], pyf[q], eps2f);
                for (int c = 0; c < 3; ++c)
                    acc[c] += w[q] * (double)(mo.da * s32[kWdA + c] + mo.db * s32[kWdB + c] + mo.sa * s32[kWcA + c] +
                                              mo.sb * s32[kWcB + c]);
            }
        }
    }
    for (int c = 0; c < 3; ++c) {
        const double r = block_reduce(acc[c], red);
        if (threadIdx.x == 0) F[(size_t)i * 3 + c] = r;
    }
}

// out[i, c] = sum_j A+[i, j] in[j, c]   (transpose: sum_j A+[j, i] in[j, c])
__global__ void k_apply_pinv(const double* __restrict__ Ap, int M, const double* __restrict__ in, double* __restrict__ out,
                             int transpose)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double a = transpose ? Ap[(size_t)j * M + i] : Ap[(size_t)i * M + j];
        for (int c = 0; c < 3; ++c) acc[c] += a * in[(size_t)j * 3 + c];
    }
    for (int c = 0; c < 3; ++c) {
        const double r = block_reduce(acc[c], red);
        if (threadIdx.x == 0) out[(size_t)i * 3 + c] = r;
    }
}

__global__ void k_pack_elements(const double* __restrict__ U, int M, const double* __restrict__ eg,
                                double* __restrict__ e64, float* __restrict__ e32)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double ax, ay, bx, by;
    load_element(eg, i, ax, ay, bx, by);
    const double rec[kElemStride] = {ax, ay, bx - ax, by - ay, U[3 * i], U[3 * i + 1], U[3 * i + 2], 0.0};
    for (int c = 0; c < kElemStride; ++c) {
        e64[(size_t)i * kElemStride + c] = rec[c];
        e32[(size_t)i * kElemStride + c] = (float)rec[c];
    }
}

// FP64 sweep: one thread per sample, every wavefront walks the whole segment
// and element tables (wave-uniform addresses: scalar loads).
__global__ void __launch_bounds__(256) k_sweep_f64(const double* __restrict__ x, int64_t N, const double* __restrict__ seg,
                                                   int K, const double* __restrict__ el, int M, double eps2,
                                                   double c0, double c1, double c2, double* __restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double X = x[2 * i], Y = x[2 * i + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < K; ++k) {
        const double* s = seg + (size_t)k * kSegStride;
        const SegGeom<double> g = load_geom(s);
        const Moments<double> m = seg_moments<double, DevF64>(g, X, Y, eps2);
        a0 += m.da * s[kWdA + 0] + m.db * s[kWdB + 0] + m.sa * s[kWcA + 0] + m.sb * s[kWcB + 0];
        a1 += m.da * s[kWdA + 1] + m.db * s[kWdB + 1] + m.sa * s[kWcA + 1] + m.sb * s[kWcB + 1];
        a2 += m.da * s[kWdA + 2] + m.db * s[kWdB + 2] + m.sa * s[kWcA + 2] + m.sb * s[kWcB + 2];
    }
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int j = 0; j < M; ++j) {
        const double* e = el + (size_t)j * kElemStride;
        const double beta = element_beta<double, DevF64>(e[0], e[1], e[2], e[3], X, Y);
        b0 += beta * e[4]; b1 += beta * e[5]; b2 += beta * e[6];
    }
    u[3 * i + 0] = c0 + b0 + a0;
    u[3 * i + 1] = c1 + b1 + a1;
    u[3 * i + 2] = c2 + b2 + a2;
}

}  // namespace

int launch_expand(bem_ctx* ctx, const double* theta, int H, hipStream_t s)
{
    const int K = H * ctx->opts.segs_per_handle;
    int rc;
    const size_t n = (size_t)(K > 0 ? K : 1) * kSegStride;
    if ((rc = ensure(ctx, ctx->seg64, n * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->seg32, n * sizeof(float), s))) return rc;
    return launch_expand_into(ctx, theta, H, (double*)ctx->seg64.ptr, (float*)ctx->seg32.ptr, s);
}

int launch_expand_into(bem_ctx* ctx, const double* theta, int H, double* seg64, float* seg32, hipStream_t s)
{
    const int S = ctx->opts.segs_per_handle;
    const int K = H * S;
    if (K == 0) return BEM_OK;
    hipLaunchKernelGGL(k_expand, dim3(blocks_for(K, 256)), dim3(256), 0, s, theta, H, S, ctx->model, seg64, seg32);
    return check_launch(ctx, "expand");
}

int launch_boundary_rhs(bem_ctx* ctx, int K, double* F, bool mixed, hipStream_t s)
{
    const double eps2 = ctx->opts.eps * ctx->opts.eps;
    {
        ProfScope ps_(ctx, PT_BOUNDARY, s);
        if (mixed) {
            const double nf = near_radius(ctx->opts.near_factor);
            hipLaunchKernelGGL(k_boundary_rhs_mixed, dim3(ctx->M), dim3(256), 0, s, (const double*)ctx->seg64.ptr,
                               (const float*)ctx->seg32.ptr, K, (const double*)ctx->egeo.ptr, eps2, (float)(nf * nf), F);
        } else {
            hipLaunchKernelGGL(k_boundary_rhs, dim3(ctx->M), dim3(256), 0, s, (const double*)ctx->seg64.ptr, K,
                               (const double*)ctx->egeo.ptr, eps2, F);
        }
    }
    return check_launch(ctx, "boundary_rhs");
}

int launch_boundary_solve(bem_ctx* ctx, const double* F, double* U, bool transpose, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply_pinv, dim3(ctx->M), dim3(256), 0, s, (const double*)ctx->Apinv.ptr, ctx->M, F, U,
                       transpose ? 1 : 0);
    return check_launch(ctx, "boundary_solve");
}

int launch_pack_elements(bem_ctx* ctx, const double* U, hipStream_t s)
{
    int rc;
    if ((rc = ensure(ctx, ctx->elem64, (size_t)ctx->M * kElemStride * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->elem32, (size_t)ctx->M * kElemStride * sizeof(float), s))) return rc;
    return launch_pack_elements_into(ctx, U, (double*)ctx->elem64.ptr, (float*)ctx->elem32.ptr, s);
}

int launch_pack_elements_into(bem_ctx* ctx, const double* U, double* el64, float* el32, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_elements, dim3(blocks_for(ctx->M, 256)), dim3(256), 0, s, U, ctx->M, (const double*)ctx->egeo.ptr,
                       el64, el32);
    return check_launch(ctx, "pack_elements");
}

int launch_sweep_f64(bem_ctx* ctx, const double* x, int64_t N, int K, const double* cbar, double* u, hipStream_t s)
{
    if (N == 0) return BEM_OK;
    const double eps2 = ctx->opts.eps * ctx->opts.eps;
    {
        ProfScope ps_(ctx, PT_SWEEP_F64, s);
        hipLaunchKernelGGL(k_sweep_f64, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, (const double*)ctx->seg64.ptr, K,
                           (const double*)ctx->elem64.ptr, ctx->M, eps2, cbar[0], cbar[1], cbar[2], u);
    }
    return check_launch(ctx, "sweep_f64");
}

}  // namespace bem
