// gemm.hip - float64 dense products used around the normal equations:
//   C = alpha op(A) op(B) + beta C   (row-major, op = identity or transpose)
// k_gemm_f64_mfma: 128 x 128 (or 64 x 64) output tiles on float64 MFMA (v_mfma_f64_16x16x4f64), 16-deep
//   k slabs staged through LDS (double buffered, the next slab prefetched into registers while
//   the current one is multiplied); also the float64 Gram restricted to a list of output tiles.
// k_gemm_skinny: products with at most 4 columns (J^T r of the float64 Gram path): a wavefront
//   per output row streaming the row of A, a wavefront reduction at the end.
// k_gemm_f64: the plain VALU product (64 x 64 tiles, 4 x 4 outputs per thread), kept for the
//   float64 VALU Gram mode.
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


// ---- float64 MFMA product ------------------------------------------------------------------
// Block tile kMB x kMB, 4 wavefronts as 2 x 2, each wavefront 64 x 64 as 4 x 4 tiles of
// v_mfma_f64_16x16x4f64.  Operand lane layout of that instruction: lane l holds A[l mod 16][l / 16]
// of its 16 x 4 slice and B[l / 16][l mod 16] of its 4 x 16 slice; accumulator element q of lane l
// is row 4 q + l / 16, column l mod 16 of the 16 x 16 tile.  Both operand slabs are stored in LDS
// k-major ([k][row] and [k][col]) so that each operand is one ds_read_b64 per lane.
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kMB = 128, kMK = 16;

// element e of a BM x kMK slab of op(X) starting at (r0, k0): its slab coordinates and value
// (0 outside the m x k operand).  Non-transposed X is row-major [row][k] (16 consecutive
// threads read one row's 16 k values); transposed X is stored [k][row].
template <int BM>
__device__ inline double slab_load(const double* __restrict__ X, int64_t ldx, int tx, int r0, int k0, int rows, int kd,
                                   int e, int& sr, int& sk)
{
    if (tx) { sk = e / BM; sr = e % BM; }
    else { sr = e / kMK; sk = e % kMK; }
    const int gr = r0 + sr, gk = k0 + sk;
    const bool in = gr < rows && gk < kd;
    const int64_t off = tx ? (int64_t)(in ? gk : 0) * ldx + (in ? gr : 0) : (int64_t)(in ? gr : 0) * ldx + (in ? gk : 0);
    const double v = X[off];                       // always a valid address; replaced when outside
    return in ? v : 0.0;
}

// BM x BM output tile per block (BM = 128: each wavefront 64 x 64 as 4 x 4 MFMA tiles; BM = 64:
// 32 x 32 as 2 x 2, for products whose 128-tile grid would leave most CUs idle).
template <int BM>
__global__ void __launch_bounds__(256, BM == 128 ? 2 : 4) k_gemm_f64_mfma(int m, int n, int k, double alpha,
                                                                        const double* __restrict__ A, int64_t lda, int ta,
                                                                        const double* __restrict__ B, int64_t ldb, int tb,
                                                                        double beta, double* __restrict__ C, int64_t ldc,
                                                                        const int* __restrict__ tiles)
{
    constexpr int LD = BM + 4;                  // LDS row stride (doubles)
    constexpr int NL = BM * kMK / 256;          // slab elements per thread and operand
    constexpr int TI = BM / 32;                 // 16 x 16 MFMA tiles per wavefront and dimension
    __shared__ double As[2][kMK][LD];
    __shared__ double Bs[2][kMK][LD];
    int bm, bn;
    if (tiles) {
        bm = tiles[2 * blockIdx.x];
        bn = tiles[2 * blockIdx.x + 1];
    } else {
        bm = blockIdx.y;
        bn = blockIdx.x;
    }
    const int row0 = bm * BM, col0 = bn * BM;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    // B as a (k x n) operand: op(B) row-major [k][col] unless transposed ([col][k]); slab_load takes
    // the "row" index as the column of op(B), so its transposition flag is the opposite one
    const int tbB = tb ? 0 : 1;
    double pa[NL], pb[NL];
    int ar[NL], ak[NL], br[NL], bk[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        pa[i] = slab_load<BM>(A, lda, ta, row0, 0, m, k, tid + 256 * i, ar[i], ak[i]);
        pb[i] = slab_load<BM>(B, ldb, tbB, col0, 0, n, k, tid + 256 * i, br[i], bk[i]);
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        As[0][ak[i]][ar[i]] = pa[i];
        Bs[0][bk[i]][br[i]] = pb[i];
    }
    __syncthreads();
    d4_t acc[TI][TI];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TI; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int nk = (k + kMK - 1) / kMK;
    for (int s = 0; s < nk; ++s) {
        const int cur = s & 1;
        const bool more = s + 1 < nk;
        if (more) {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                pa[i] = slab_load<BM>(A, lda, ta, row0, (s + 1) * kMK, m, k, tid + 256 * i, ar[i], ak[i]);
                pb[i] = slab_load<BM>(B, ldb, tbB, col0, (s + 1) * kMK, n, k, tid + 256 * i, br[i], bk[i]);
            }
        }
#pragma unroll
        for (int ks = 0; ks < kMK; ks += 4) {
            const int kk = ks + (l >> 4), rr = l & 15;
            double a[TI], b[TI];
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = As[cur][kk][(BM / 2) * wr + 16 * i + rr];
#pragma unroll
            for (int j = 0; j < TI; ++j) b[j] = Bs[cur][kk][(BM / 2) * wc + 16 * j + rr];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TI; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                As[cur ^ 1][ak[i]][ar[i]] = pa[i];
                Bs[cur ^ 1][bk[i]][br[i]] = pb[i];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TI; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = row0 + (BM / 2) * wr + 16 * i + 4 * q + (l >> 4);
                const int c = col0 + (BM / 2) * wc + 16 * j + (l & 15);
                if (r < m && c < n) {
                    double* o = C + (size_t)r * ldc + c;
                    *o = alpha * acc[i][j][q] + (beta == 0.0 ? 0.0 : beta * *o);
                }
            }
}

// ---- products with at most kSkinnyMaxN columns ---------------------------------------------
// C[r][j] = alpha sum_t A[r][t] op(B)[t][j] + beta C[r][j]: a wavefront per row r (4 per block),
// lanes striding over t, then a wavefront reduction (fixed order, reproducible).
constexpr int kSkinnyMaxN = 4;
__global__ void __launch_bounds__(256) k_gemm_skinny(int m, int n, int k, double alpha, const double* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ B, int64_t ldb, int tb,
                                                     double beta, double* __restrict__ C, int64_t ldc)
{
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    if (r >= m) return;
    double acc[kSkinnyMaxN] = {0.0, 0.0, 0.0, 0.0};
    const double* a = A + (size_t)r * lda;
    for (int t = l; t < k; t += 64) {
        const double v = a[t];
#pragma unroll
        for (int j = 0; j < kSkinnyMaxN; ++j)
            if (j < n) acc[j] += v * (tb ? B[(size_t)j * ldb + t] : B[(size_t)t * ldb + j]);
    }
#pragma unroll
    for (int j = 0; j < kSkinnyMaxN; ++j)
        for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
    if (l < n) {
        double v = acc[0];
#pragma unroll
        for (int j = 1; j < kSkinnyMaxN; ++j)
            if (l == j) v = acc[j];
        double* o = C + (size_t)r * ldc + l;
        *o = alpha * v + (beta == 0.0 ? 0.0 : beta * *o);
    }
}

}  // namespace

int gemm_f64(bem_ctx* ctx, int m, int n, int k, double alpha, const double* A, int64_t lda, bool ta, const double* B,
             int64_t ldb, bool tb, double beta, double* C, int64_t ldc, hipStream_t s, const int* tiles, int ntiles,
             bool valu)
{
    if (m <= 0 || n <= 0) return BEM_OK;
    if (tiles) {
        if (ntiles <= 0) return BEM_OK;
        if (valu)
            hipLaunchKernelGGL(k_gemm_f64, dim3(ntiles), dim3(256), 0, s, m, n, k, alpha, A, lda, ta ? 1 : 0, B, ldb,
                               tb ? 1 : 0, beta, C, ldc, tiles);
        else
            hipLaunchKernelGGL(k_gemm_f64_mfma<kMB>, dim3(ntiles), dim3(256), 0, s, m, n, k, alpha, A, lda, ta ? 1 : 0,
                               B, ldb, tb ? 1 : 0, beta, C, ldc, tiles);
        return check_launch(ctx, "gemm_f64");
    }
    if (valu) {
        hipLaunchKernelGGL(k_gemm_f64, dim3(blocks_for(n, TN), blocks_for(m, TM)), dim3(256), 0, s, m, n, k, alpha, A,
                           lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, C, ldc, (const int*)nullptr);
    } else if (n <= kSkinnyMaxN && !ta) {
        hipLaunchKernelGGL(k_gemm_skinny, dim3(blocks_for(m, 4)), dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb,
                           tb ? 1 : 0, beta, C, ldc);
    } else if ((int64_t)blocks_for(n, kMB) * blocks_for(m, kMB) >= 1024) {
        hipLaunchKernelGGL(k_gemm_f64_mfma<kMB>, dim3(blocks_for(n, kMB), blocks_for(m, kMB)), dim3(256), 0, s, m, n, k,
                           alpha, A, lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, C, ldc, (const int*)nullptr);
    } else {
        // fewer than two rounds of 128-tiles over the CUs: 64-tiles, 4x the blocks
        hipLaunchKernelGGL(k_gemm_f64_mfma<64>, dim3(blocks_for(n, 64), blocks_for(m, 64)), dim3(256), 0, s, m, n, k,
                           alpha, A, lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, C, ldc, (const int*)nullptr);
    }
    return check_launch(ctx, "gemm_f64");
}

}  // namespace bem
