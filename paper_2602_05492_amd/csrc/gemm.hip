// gemm.hip - float64 dense products used around the normal equations:
//   C = alpha op(A) op(B) + beta C   (row-major, op = identity or transpose)
// Plain products of more than 2^22 multiply-adds go to rocBLAS dgemm (FP64 MFMA;
// atomics off, so results are reproducible); the rest, and every launch restricted
// to a list of output tiles (the upper-triangle FP64 Gram), run in k_gemm_f64:
// 64x64 output tiles, 16-deep k slabs staged through LDS, 4x4 outputs per thread.
#include <rocblas/rocblas.h>

#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

__global__ void __launch_bounds__(256) k_gemm_f64(int m, int n, int k, double alpha, const double* __restrict__ A,
                                                  int64_t lda, int ta, const double* __restrict__ B, int64_t ldb, int tb,
                                                  double beta, double* __restrict__ C, int64_t ldc,
                                                  const int* __restrict__ tiles)
{
    __shared__ double As[TK][TM + 1];
    __shared__ double Bs[TK][TN + 1];
    int bm, bn;
    if (tiles) {
        bm = tiles[2 * blockIdx.x];
        bn = tiles[2 * blockIdx.x + 1];
    } else {
        bm = blockIdx.y;
        bn = blockIdx.x;
    }
    const int row0 = bm * TM, col0 = bn * TN;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < k; k0 += TK) {
        // load a TM x TK slab of op(A) and a TK x TN slab of op(B)
        for (int e = threadIdx.x; e < TM * TK; e += 256) {
            int r, kk;
            if (ta) { r = e % TM; kk = e / TM; }
            else { kk = e % TK; r = e / TK; }
            const int gr = row0 + r, gk = k0 + kk;
            double v = 0.0;
            if (gr < m && gk < k) v = ta ? A[(size_t)gk * lda + gr] : A[(size_t)gr * lda + gk];
            As[kk][r] = v;
        }
        for (int e = threadIdx.x; e < TK * TN; e += 256) {
            int c, kk;
            if (tb) { kk = e % TK; c = e / TK; }
            else { c = e % TN; kk = e / TN; }
            const int gc = col0 + c, gk = k0 + kk;
            double v = 0.0;
            if (gc < n && gk < k) v = tb ? B[(size_t)gc * ldb + gk] : B[(size_t)gk * ldb + gc];
            Bs[kk][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            double a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i) {
        const int r = row0 + ty + 16 * i;
        if (r >= m) continue;
        for (int j = 0; j < 4; ++j) {
            const int c = col0 + tx + 16 * j;
            if (c >= n) continue;
            double* o = C + (size_t)r * ldc + c;
            *o = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * *o);
        }
    }
}

}  // namespace

// The context's rocBLAS handle on stream s (created on first use).
static rocblas_handle blas(bem_ctx* ctx, hipStream_t s)
{
    if (!ctx->blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
        rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed);
        ctx->blas = h;
    }
    rocblas_handle h = (rocblas_handle)ctx->blas;
    if (rocblas_set_stream(h, s) != rocblas_status_success) return nullptr;
    return h;
}

int gemm_f64(bem_ctx* ctx, int m, int n, int k, double alpha, const double* A, int64_t lda, bool ta, const double* B,
             int64_t ldb, bool tb, double beta, double* C, int64_t ldc, hipStream_t s, const int* tiles, int ntiles)
{
    if (m <= 0 || n <= 0) return BEM_OK;
    if (!tiles && k > 0 && (double)m * n * k > (double)(1 << 22)) {
        // row-major C = op(A) op(B) is column-major C^T = op(B)^T op(A)^T on the same memory
        rocblas_handle h = blas(ctx, s);
        if (!h) return set_error(ctx, BEM_EHIP, "rocBLAS handle");
        const rocblas_status st =
            rocblas_dgemm(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                          ta ? rocblas_operation_transpose : rocblas_operation_none, n, m, k, &alpha, B, (int)ldb, A,
                          (int)lda, &beta, C, (int)ldc);
        if (st != rocblas_status_success) return set_error(ctx, BEM_EHIP, "rocblas_dgemm: status %d", (int)st);
        return BEM_OK;
    }
    if (tiles) {
        if (ntiles <= 0) return BEM_OK;
        hipLaunchKernelGGL(k_gemm_f64, dim3(ntiles), dim3(256), 0, s, m, n, k, alpha, A, lda, ta ? 1 : 0, B, ldb,
                           tb ? 1 : 0, beta, C, ldc, tiles);
    } else {
        hipLaunchKernelGGL(k_gemm_f64, dim3(blocks_for(n, TN), blocks_for(m, TM)), dim3(256), 0, s, m, n, k, alpha, A,
                           lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, C, ldc, (const int*)nullptr);
    }
    return check_launch(ctx, "gemm_f64");
}

}  // namespace bem
