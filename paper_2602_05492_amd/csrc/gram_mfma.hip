// gram_mfma.hip - the normal-equation contraction on the matrix cores (Eq.
// losshessian): G += X X^T over one sample tile, X the feature-major tile
// [W rows x n samples], only the needed 128x128 output tiles.
//
//   FP32_MFMA   : v_mfma_f32_32x32x2_f32 on float rows
//   BF16X3_MFMA : rows split x = hi + lo (bfloat16); hi*hi + hi*lo + lo*hi on
//                 v_mfma_f32_32x32x16_bf16 (the lo*lo term is below float32
//                 rounding of the product)
// Accumulation is float32 over the tile's samples and float64 across tiles
// (the epilogue adds into the float64 Gram).  A block of 4 wavefronts owns a
// 128x128 tile; each wavefront a 64x64 quarter as 2x2 MFMA 32x32 tiles.  The
// A and B operands of every MFMA come from rows of the same matrix with the
// same lane -> (row, k-slot) assignment, so each k of the slab is summed once.
#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ inline bf16x8 load_bf16x8(const uint16_t* __restrict__ p, int64_t k, int64_t n)
{
    u16x8 v;
    if (k + 8 <= n) {
        v = *(const u16x8*)(p + k);
    } else {
        for (int e = 0; e < 8; ++e) v[e] = (k + e < n) ? p[k + e] : (uint16_t)0;
    }
    return __builtin_bit_cast(bf16x8, v);
}

__device__ inline floatx4 load_f32x4(const float* __restrict__ p, int64_t k, int64_t n)
{
    floatx4 v;
    if (k + 4 <= n) {
        v = *(const floatx4*)(p + k);
    } else {
        for (int e = 0; e < 4; ++e) v[e] = (k + e < n) ? p[k + e] : 0.0f;
    }
    return v;
}

__device__ inline void epilogue(const floatx16 (&acc)[2][2], int64_t rbase, int64_t cbase, int W, double* __restrict__ G)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 31, lk = lane >> 5;
    for (int mi = 0; mi < 2; ++mi)
        for (int nj = 0; nj < 2; ++nj)
            for (int r = 0; r < 16; ++r) {
                const int64_t i = rbase + 32 * mi + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int64_t j = cbase + 32 * nj + li;
                if (i < W && j < W) G[i * W + j] += (double)acc[mi][nj][r];
            }
}

__global__ void __launch_bounds__(256) k_gram_bf16x3(const uint16_t* __restrict__ Xh, const uint16_t* __restrict__ Xl,
                                                     int64_t ld, int W, int64_t n, const int* __restrict__ tiles,
                                                     double* __restrict__ G)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t rbase = (int64_t)tiles[2 * blockIdx.x] * 128 + 64 * (wave >> 1);
    const int64_t cbase = (int64_t)tiles[2 * blockIdx.x + 1] * 128 + 64 * (wave & 1);
    floatx16 acc[2][2];
    for (int mi = 0; mi < 2; ++mi)
        for (int nj = 0; nj < 2; ++nj)
            for (int r = 0; r < 16; ++r) acc[mi][nj][r] = 0.0f;
    const uint16_t* ah[2];
    const uint16_t* al[2];
    const uint16_t* bh[2];
    const uint16_t* bl[2];
    bool arow[2], bcol[2];
    for (int q = 0; q < 2; ++q) {
        const int64_t ra = rbase + 32 * q + li, cb = cbase + 32 * q + li;
        arow[q] = ra < W;
        bcol[q] = cb < W;
        ah[q] = Xh + (arow[q] ? ra : 0) * ld;
        al[q] = Xl + (arow[q] ? ra : 0) * ld;
        bh[q] = Xh + (bcol[q] ? cb : 0) * ld;
        bl[q] = Xl + (bcol[q] ? cb : 0) * ld;
    }
    const bf16x8 zero = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    for (int64_t k0 = 0; k0 < n; k0 += 16) {
        const int64_t k = k0 + 8 * lk;
        bf16x8 a_hi[2], a_lo[2], b_hi[2], b_lo[2];
        for (int q = 0; q < 2; ++q) {
            a_hi[q] = arow[q] ? load_bf16x8(ah[q], k, n) : zero;
            a_lo[q] = arow[q] ? load_bf16x8(al[q], k, n) : zero;
            b_hi[q] = bcol[q] ? load_bf16x8(bh[q], k, n) : zero;
            b_lo[q] = bcol[q] ? load_bf16x8(bl[q], k, n) : zero;
        }
        for (int mi = 0; mi < 2; ++mi)
            for (int nj = 0; nj < 2; ++nj) {
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[mi], b_hi[nj], acc[mi][nj], 0, 0, 0);
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[mi], b_lo[nj], acc[mi][nj], 0, 0, 0);
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lo[mi], b_hi[nj], acc[mi][nj], 0, 0, 0);
            }
    }
    epilogue(acc, rbase, cbase, W, G);
}

__global__ void __launch_bounds__(256) k_gram_f32(const float* __restrict__ X, int64_t ld, int W, int64_t n,
                                                  const int* __restrict__ tiles, double* __restrict__ G)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t rbase = (int64_t)tiles[2 * blockIdx.x] * 128 + 64 * (wave >> 1);
    const int64_t cbase = (int64_t)tiles[2 * blockIdx.x + 1] * 128 + 64 * (wave & 1);
    floatx16 acc[2][2];
    for (int mi = 0; mi < 2; ++mi)
        for (int nj = 0; nj < 2; ++nj)
            for (int r = 0; r < 16; ++r) acc[mi][nj][r] = 0.0f;
    const float* ap[2];
    const float* bp[2];
    bool arow[2], bcol[2];
    for (int q = 0; q < 2; ++q) {
        const int64_t ra = rbase + 32 * q + li, cb = cbase + 32 * q + li;
        arow[q] = ra < W;
        bcol[q] = cb < W;
        ap[q] = X + (arow[q] ? ra : 0) * ld;
        bp[q] = X + (bcol[q] ? cb : 0) * ld;
    }
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = 0; k0 < n; k0 += 8) {
        const int64_t k = k0 + 4 * lk;
        floatx4 a[2], b[2];
        for (int q = 0; q < 2; ++q) {
            a[q] = arow[q] ? load_f32x4(ap[q], k, n) : zero;
            b[q] = bcol[q] ? load_f32x4(bp[q], k, n) : zero;
        }
        for (int s = 0; s < 4; ++s)
            for (int mi = 0; mi < 2; ++mi)
                for (int nj = 0; nj < 2; ++nj)
                    acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mi][s], b[nj][s], acc[mi][nj], 0, 0, 0);
    }
    epilogue(acc, rbase, cbase, W, G);
}

// R[f][c] += sum_t X[f][t] r[t][c]  (float64 sums; X float or bf16 hi + lo)
template <bool Bf16>
__global__ void __launch_bounds__(256) k_xr(const void* __restrict__ Xhi, const uint16_t* __restrict__ Xlo, int64_t ld,
                                            int64_t n, const double* __restrict__ r, double* __restrict__ R)
{
    __shared__ double red[3][256];
    const int64_t f = blockIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        double v;
        if (Bf16) {
            const uint16_t h = ((const uint16_t*)Xhi)[f * ld + t], l = Xlo[f * ld + t];
            v = (double)__uint_as_float((uint32_t)h << 16) + (double)__uint_as_float((uint32_t)l << 16);
        } else {
            v = (double)((const float*)Xhi)[f * ld + t];
        }
        s0 += v * r[3 * t]; s1 += v * r[3 * t + 1]; s2 += v * r[3 * t + 2];
    }
    red[0][threadIdx.x] = s0; red[1][threadIdx.x] = s1; red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) R[f * 3 + c] += red[c][0];
}

}  // namespace

int launch_gram_mfma(bem_ctx* ctx, int gram, const void* Xhi, const uint16_t* Xlo, int64_t ld, int W, int64_t n,
                     const int* tiles128, int ntiles, double* G, hipStream_t s)
{
    if (n <= 0 || ntiles <= 0) return BEM_OK;
    if (gram == BEM_GRAM_BF16X3_MFMA)
        {
            ProfScope ps_(ctx, PT_GRAM_MFMA, s);
            hipLaunchKernelGGL(k_gram_bf16x3, dim3(ntiles), dim3(256), 0, s, (const uint16_t*)Xhi, Xlo, ld, W, n, tiles128, G);
        }
    else
        {
            ProfScope ps_(ctx, PT_GRAM_MFMA, s);
            hipLaunchKernelGGL(k_gram_f32, dim3(ntiles), dim3(256), 0, s, (const float*)Xhi, ld, W, n, tiles128, G);
        }
    return check_launch(ctx, "gram_mfma");
}

int launch_xr(bem_ctx* ctx, int gram, const void* Xhi, const uint16_t* Xlo, int64_t ld, int W, int64_t n,
              const double* r, double* R, hipStream_t s)
{
    if (n <= 0) return BEM_OK;
    if (gram == BEM_GRAM_BF16X3_MFMA)
        {
            ProfScope ps_(ctx, PT_XR, s);
            hipLaunchKernelGGL(k_xr<true>, dim3(W), dim3(256), 0, s, Xhi, Xlo, ld, n, r, R);
        }
    else
        {
            ProfScope ps_(ctx, PT_XR, s);
            hipLaunchKernelGGL(k_xr<false>, dim3(W), dim3(256), 0, s, Xhi, Xlo, ld, n, r, R);
        }
    return check_launch(ctx, "xr");
}

}  // namespace bem
