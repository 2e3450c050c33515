// sweep_mixed.hip - mixed-precision forward sweep (Sec. 3.1.3 evaluation of
// u(x) at every sample).  Far pairs run in float32 from the float32 copies of
// the segment and element tables; a pair whose two end points both lie within
// 2*near_factor*L of the sample (a set containing every sample closer than
// near_factor*L to the segment) is evaluated in float64 from the float64
// tables and the float64 sample.  Far and near sums are kept apart and added
// in float64 at the end.
#include "common.hpp"

namespace bem {

namespace {

__global__ void __launch_bounds__(256) k_sweep_mixed(const double* __restrict__ x, int64_t N,
                                                     const float* __restrict__ seg32, const double* __restrict__ seg64,
                                                     int K, const float* __restrict__ el32, const double* __restrict__ el64,
                                                     int M, float eps2f, double eps2, float near2, double c0, double c1,
                                                     double c2, float* __restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double X = x[2 * i], Y = x[2 * i + 1];
    const float Xf = (float)X, Yf = (float)Y;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    double n0 = 0.0, n1 = 0.0, n2 = 0.0;
    for (int k = 0; k < K; ++k) {
        const float* s = seg32 + (size_t)k * kSegStride;
        const SegGeom<float> g = load_geom(s);
        if (g.L2 == 0.0f) continue;                    // degenerate segment (wave-uniform branch)
        const float dx = g.ax - Xf, dy = g.ay - Yf, ex = g.bx - Xf, ey = g.by - Yf;
        const float lim = near2 * g.L2;
        const bool near = (dx * dx + dy * dy < lim) && (ex * ex + ey * ey < lim);
        if (near) {
            const double* s64 = seg64 + (size_t)k * kSegStride;
            const SegGeom<double> g64 = load_geom(s64);
            const Moments<double> m = seg_moments<double, DevF64>(g64, X, Y, eps2);
            n0 += m.da * s64[kWdA + 0] + m.db * s64[kWdB + 0] + m.sa * s64[kWcA + 0] + m.sb * s64[kWcB + 0];
            n1 += m.da * s64[kWdA + 1] + m.db * s64[kWdB + 1] + m.sa * s64[kWcA + 1] + m.sb * s64[kWcB + 1];
            n2 += m.da * s64[kWdA + 2] + m.db * s64[kWdB + 2] + m.sa * s64[kWcA + 2] + m.sb * s64[kWcB + 2];
        } else {
            const Moments<float> m = seg_moments<float, DevF32, false>(g, Xf, Yf, eps2f);
            f0 += m.da * s[kWdA + 0] + m.db * s[kWdB + 0] + m.sa * s[kWcA + 0] + m.sb * s[kWcB + 0];
            f1 += m.da * s[kWdA + 1] + m.db * s[kWdB + 1] + m.sa * s[kWcA + 1] + m.sb * s[kWcB + 1];
            f2 += m.da * s[kWdA + 2] + m.db * s[kWdB + 2] + m.sa * s[kWcA + 2] + m.sb * s[kWcB + 2];
        }
    }
    float b0 = 0.f, b1 = 0.f, b2 = 0.f;
    for (int j = 0; j < M; ++j) {
        const float* e = el32 + (size_t)j * kElemStride;
        const float dx = e[0] - Xf, dy = e[1] - Yf;
        const float ex = dx + e[2], ey = dy + e[3];
        const float lim = near2 * (e[2] * e[2] + e[3] * e[3]);
        if ((dx * dx + dy * dy < lim) && (ex * ex + ey * ey < lim)) {
            const double* e64 = el64 + (size_t)j * kElemStride;
            const double beta = element_beta<double, DevF64>(e64[0], e64[1], e64[2], e64[3], X, Y);
            n0 += beta * e64[4]; n1 += beta * e64[5]; n2 += beta * e64[6];
        } else {
            const float beta = element_beta<float, DevF32>(e[0], e[1], e[2], e[3], Xf, Yf);
            b0 += beta * e[4]; b1 += beta * e[5]; b2 += beta * e[6];
        }
    }
    u[3 * i + 0] = (float)(c0 + ((double)b0 + (double)f0 + n0));
    u[3 * i + 1] = (float)(c1 + ((double)b1 + (double)f1 + n1));
    u[3 * i + 2] = (float)(c2 + ((double)b2 + (double)f2 + n2));
}

}  // namespace

int launch_sweep_mixed(bem_ctx* ctx, const double* x, int64_t N, int K, const double* cbar, float* u, hipStream_t s)
{
    if (N == 0) return BEM_OK;
    const double eps2 = ctx->opts.eps * ctx->opts.eps;
    const double nf = 2.0 * ctx->opts.near_factor;
    {
        ProfScope ps_(ctx, PT_SWEEP_MIXED, s);
        hipLaunchKernelGGL(k_sweep_mixed, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, (const float*)ctx->seg32.ptr,
                           (const double*)ctx->seg64.ptr, K, (const float*)ctx->elem32.ptr, (const double*)ctx->elem64.ptr,
                           ctx->M, (float)eps2, eps2, (float)(nf * nf), cbar[0], cbar[1], cbar[2], u);
    }
    return check_launch(ctx, "sweep_mixed");
}

}  // namespace bem
