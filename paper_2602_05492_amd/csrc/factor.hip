// factor.hip - one-time float64 outer-boundary system (Sec. 3.1.3):
// Galerkin assembly of Eq. bie_galerkin, pivoted LU, smallest singular
// triplet by inverse iteration, deflation and the explicit truncated
// pseudo-inverse A+ = B^{-1} - v_n u_n^T / s, B = A + (s - sigma_n) u_n v_n^T.
#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr double kGaussNode = 0.77459666924148337703585307995647992;   // sqrt(3/5)
constexpr double kGaussW0 = 5.0 / 9.0, kGaussW1 = 8.0 / 9.0;


// Element table of the counter-clockwise unit square with m elements per side.
__global__ void k_square_elements(int M, int m, double* __restrict__ eg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    square_element(i, m, eg[4 * i], eg[4 * i + 1], eg[4 * i + 2], eg[4 * i + 3]);
}

// A_ij = delta_ij |G_i|/2 + sum_{q,q'} w_q w_q' dG/dn_y(x_iq, y_jq'), the coincident term zero.
__global__ void k_assemble(double* __restrict__ A, int M, const double* __restrict__ eg)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= M) return;
    double ax, ay, bx, by, cx, cy, dx, dy;
    load_element(eg, i, ax, ay, bx, by);
    load_element(eg, j, cx, cy, dx, dy);
    const double li = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
    const double lj = sqrt((dx - cx) * (dx - cx) + (dy - cy) * (dy - cy));
    double val = 0.0;
    if (i == j) {
        val = 0.5 * li;
    } else {
        const double nx = (dy - cy) / lj, ny = -(dx - cx) / lj;     // outward normal of element j
        const double node[3] = {-kGaussNode, 0.0, kGaussNode};
        const double w[3] = {kGaussW0, kGaussW1, kGaussW0};
        const double mix = 0.5 * (ax + bx), miy = 0.5 * (ay + by), hix = 0.5 * (bx - ax), hiy = 0.5 * (by - ay);
        const double mjx = 0.5 * (cx + dx), mjy = 0.5 * (cy + dy), hjx = 0.5 * (dx - cx), hjy = 0.5 * (dy - cy);
        for (int q = 0; q < 3; ++q) {
            const double px = mix + node[q] * hix, py = miy + node[q] * hiy;
            double s = 0.0;
            for (int r = 0; r < 3; ++r) {
                const double yx = mjx + node[r] * hjx - px, yy = mjy + node[r] * hjy - py;
                s += w[r] * (nx * yx + ny * yy) / (yx * yx + yy * yy);
            }
            val += w[q] * s;
        }
        val *= -(0.5 * li) * (0.5 * lj) * kInv2Pi;
    }
    A[(size_t)i * M + j] = val;
}

// ---- pivoted LU, right-looking, one column per step ----------------------------
__global__ void k_lu_pivot(double* __restrict__ A, int n, int k, int* __restrict__ piv, int* __restrict__ flag)
{
    __shared__ double sv[1024];
    __shared__ int si[1024];
    const int t = threadIdx.x;
    double best = -1.0;
    int bi = n;
    for (int i = k + t; i < n; i += blockDim.x) {
        const double a = fabs(A[(size_t)i * n + k]);
        if (a > best) { best = a; bi = i; }
    }
    sv[t] = best; si[t] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
            const double o = sv[t + s];
            const int oi = si[t + s];
            if (o > sv[t] || (o == sv[t] && oi < si[t])) { sv[t] = o; si[t] = oi; }
        }
        __syncthreads();
    }
    const int p = si[0] < n ? si[0] : k;      // a column of NaNs picks no row: keep k and flag it
    if (t == 0) {
        piv[k] = p;
        if (!(sv[0] > 0.0)) flag[0] = 1;
    }
    if (p != k) {
        for (int j = t; j < n; j += blockDim.x) {
            const double a = A[(size_t)k * n + j];
            A[(size_t)k * n + j] = A[(size_t)p * n + j];
            A[(size_t)p * n + j] = a;
        }
    }
}

__global__ void k_lu_update(double* __restrict__ A, int n, int k)
{
    const int i = k + 1 + blockIdx.x;
    const double akk = A[(size_t)k * n + k];
    const double aik = A[(size_t)i * n + k];
    __syncthreads();
    const double l = aik / akk;
    if (threadIdx.x == 0) A[(size_t)i * n + k] = l;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x)
        A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
}

// ---- single-block triangular solves with the LU factors (x in shared memory) -----
// Solve A x = b (trans = 0) or A^T x = b (trans = 1) for PA = LU; b is overwritten.
// LUt is the transpose of LU, so that every sweep reads contiguous rows.
__device__ void lu_solve_block(const double* __restrict__ LU, const double* __restrict__ LUt,
                               const int* __restrict__ piv, int n, double* x, bool trans)
{
    const int t = threadIdx.x, nt = blockDim.x;
    if (!trans) {
        if (t == 0)
            for (int k = 0; k < n; ++k) { const int p = piv[k]; const double a = x[k]; x[k] = x[p]; x[p] = a; }
        __syncthreads();
        for (int j = 0; j < n; ++j) {                       // L y = P b, unit diagonal
            const double yj = x[j];
            for (int i = j + 1 + t; i < n; i += nt) x[i] -= LUt[(size_t)j * n + i] * yj;
            __syncthreads();
        }
        for (int j = n - 1; j >= 0; --j) {                  // U x = y
            if (t == 0) x[j] /= LU[(size_t)j * n + j];
            __syncthreads();
            const double xj = x[j];
            for (int i = t; i < j; i += nt) x[i] -= LUt[(size_t)j * n + i] * xj;
            __syncthreads();
        }
    } else {
        for (int j = 0; j < n; ++j) {                       // U^T z = b
            if (t == 0) x[j] /= LU[(size_t)j * n + j];
            __syncthreads();
            const double zj = x[j];
            for (int i = j + 1 + t; i < n; i += nt) x[i] -= LU[(size_t)j * n + i] * zj;
            __syncthreads();
        }
        for (int j = n - 1; j >= 0; --j) {                  // L^T w = z, unit diagonal
            const double wj = x[j];
            for (int i = t; i < j; i += nt) x[i] -= LU[(size_t)j * n + i] * wj;
            __syncthreads();
        }
        if (t == 0)
            for (int k = n - 1; k >= 0; --k) { const int p = piv[k]; const double a = x[k]; x[k] = x[p]; x[p] = a; }
        __syncthreads();
    }
}

__device__ double block_sum(double v, double* red)
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

// Smallest singular triplet by inverse iteration on A^T A with the LU of A:
// u <- A^{-T} v / |.|, x = A^{-1} u, sigma = 1/|x|, v = sigma x  (so A v = sigma u),
// until v changes by less than 1e-14 (at most iters rounds).  Each round shrinks the error
// by (sigma_n / sigma_{n-1})^2: a closed boundary's constant null space converges in a few
// rounds, an open boundary's smallest singular value, less separated, in tens.
__global__ void k_smallest_triplet(const double* __restrict__ LU, const double* __restrict__ LUt,
                                   const int* __restrict__ piv, int n, int iters,
                                   double* __restrict__ u_out, double* __restrict__ v_out, double* __restrict__ sig)
{
    extern __shared__ double sh[];
    double* x = sh;               // n
    double* red = sh + n;         // blockDim.x
    const int t = threadIdx.x, nt = blockDim.x;
    const double v0 = 1.0 / sqrt((double)n);
    for (int i = t; i < n; i += nt) x[i] = v0;
    __syncthreads();
    double sigma = 0.0;
    for (int it = 0; it < iters; ++it) {
        lu_solve_block(LU, LUt, piv, n, x, true);
        double s = 0.0;
        for (int i = t; i < n; i += nt) s += x[i] * x[i];
        const double nrm = sqrt(block_sum(s, red));
        for (int i = t; i < n; i += nt) { x[i] /= nrm; u_out[i] = x[i]; }
        __syncthreads();
        lu_solve_block(LU, LUt, piv, n, x, false);
        s = 0.0;
        for (int i = t; i < n; i += nt) s += x[i] * x[i];
        const double nx = sqrt(block_sum(s, red));
        sigma = 1.0 / nx;
        double d = 0.0;
        for (int i = t; i < n; i += nt) {
            x[i] *= sigma;
            if (it > 0) d += (x[i] - v_out[i]) * (x[i] - v_out[i]);
            v_out[i] = x[i];
        }
        const double change = sqrt(block_sum(d, red));
        if (it > 0 && change < 1e-14) break;
    }
    if (t == 0) sig[0] = sigma;
}

__global__ void k_frobenius(const double* __restrict__ A, int64_t nn, double* __restrict__ out)
{
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nn; i += blockDim.x) s += A[i] * A[i];
    const double r = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = r;
}

// B = A + (s - sigma) u v^T
__global__ void k_deflate(const double* __restrict__ A, double* __restrict__ B, int n, const double* __restrict__ u,
                          const double* __restrict__ v, const double* __restrict__ scal)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    const double c = scal[1] - scal[2];       // shift - sigma_n
    B[(size_t)i * n + j] = A[(size_t)i * n + j] + c * u[i] * v[j];
}

// Column j of B^{-1}: one block per column.
__global__ void k_inverse_columns(const double* __restrict__ LU, const double* __restrict__ LUt,
                                  const int* __restrict__ piv, int n, double* __restrict__ X)
{
    extern __shared__ double x[];
    const int j = blockIdx.x;
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
    lu_solve_block(LU, LUt, piv, n, x, false);
    for (int i = threadIdx.x; i < n; i += blockDim.x) X[(size_t)i * n + j] = x[i];
}

// A+ = B^{-1} - v u^T / s
__global__ void k_pinv_finish(double* __restrict__ X, int n, const double* __restrict__ u, const double* __restrict__ v,
                              const double* __restrict__ scal)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    X[(size_t)i * n + j] -= v[i] * u[j] / scal[1];
}

__global__ void k_transpose(const double* __restrict__ src, double* __restrict__ dst, int n)
{
    __shared__ double tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;     // 32 x 8 threads
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        if (i < n && j < n) tile[r][tx] = src[(size_t)i * n + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + r, j = by + tx;
        if (i < n && j < n) dst[(size_t)i * n + j] = tile[tx][r];
    }
}

__global__ void k_set_shift(double* scal, int n)
{
    // scal[0] = |A|_F^2 (input), scal[1] = shift s = |A|_F / sqrt(n), scal[2] = sigma_n (set by the triplet kernel)
    scal[1] = sqrt(scal[0] / (double)n);
}

}  // namespace

int launch_square_elements(bem_ctx* ctx, hipStream_t s)
{
    hipLaunchKernelGGL(k_square_elements, dim3(blocks_for(ctx->M, 256)), dim3(256), 0, s, ctx->M, ctx->per_side,
                       (double*)ctx->egeo.ptr);
    return check_launch(ctx, "square elements");
}

int launch_assemble(bem_ctx* ctx, hipStream_t s)
{
    const int M = ctx->M;
    dim3 grid(blocks_for(M, 256), M);
    hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, (double*)ctx->A.ptr, M, (const double*)ctx->egeo.ptr);
    return check_launch(ctx, "assemble");
}

static int lu_factor(bem_ctx* ctx, double* A, int n, int* piv, int* flag, hipStream_t s)
{
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(1024), 0, s, A, n, k, piv, flag);
        if (k + 1 < n)
            hipLaunchKernelGGL(k_lu_update, dim3(n - k - 1), dim3(256), 0, s, A, n, k);
    }
    return check_launch(ctx, "lu");
}

int launch_factor(bem_ctx* ctx, hipStream_t s)
{
    const int n = ctx->M;
    const size_t nn = (size_t)n * n;
    int rc;
    if ((rc = ensure(ctx, ctx->LU, nn * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->Apinv, nn * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->piv, (size_t)n * sizeof(int), s))) return rc;
    if ((rc = ensure(ctx, ctx->un, (size_t)n * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->vn, (size_t)n * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->flag, 16, s))) return rc;
    if ((rc = ensure(ctx, ctx->scal, 8 * sizeof(double), s))) return rc;
    double* A = (double*)ctx->A.ptr;
    double* LU = (double*)ctx->LU.ptr;
    double* X = (double*)ctx->Apinv.ptr;
    int* piv = (int*)ctx->piv.ptr;
    int* flag = (int*)ctx->flag.ptr;
    double* u = (double*)ctx->un.ptr;
    double* v = (double*)ctx->vn.ptr;
    double* scal = (double*)ctx->scal.ptr;
    if (hipMemsetAsync(flag, 0, 16, s) != hipSuccess) return set_error(ctx, BEM_EHIP, "memset flag");
    if (hipMemcpyAsync(LU, A, nn * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "copy A");
    if ((rc = lu_factor(ctx, LU, n, piv, flag, s))) return rc;
    const int nt = 1024;
    const size_t shm = ((size_t)n + nt) * sizeof(double);
    double* LUt = X;      // the pseudo-inverse buffer holds the transposed factors until the end
    dim3 tgrid(blocks_for(n, 32), blocks_for(n, 32));
    hipLaunchKernelGGL(k_transpose, tgrid, dim3(32, 8), 0, s, LU, LUt, n);
    hipLaunchKernelGGL(k_smallest_triplet, dim3(1), dim3(nt), shm, s, LU, LUt, piv, n, 1000, u, v, scal + 2);
    hipLaunchKernelGGL(k_frobenius, dim3(1), dim3(1024), 0, s, A, (int64_t)nn, scal);
    hipLaunchKernelGGL(k_set_shift, dim3(1), dim3(1), 0, s, scal, n);
    dim3 grid(blocks_for(n, 256), n);
    hipLaunchKernelGGL(k_deflate, grid, dim3(256), 0, s, A, LU, n, u, v, scal);
    if ((rc = check_launch(ctx, "triplet/deflate"))) return rc;
    if ((rc = lu_factor(ctx, LU, n, piv, flag, s))) return rc;
    // B^{-1} column by column; the transposed factors move to the A buffer's twin
    if ((rc = ensure(ctx, ctx->tmp0, nn * sizeof(double), s))) return rc;
    double* LUt2 = (double*)ctx->tmp0.ptr;
    hipLaunchKernelGGL(k_transpose, tgrid, dim3(32, 8), 0, s, LU, LUt2, n);
    hipLaunchKernelGGL(k_inverse_columns, dim3(n), dim3(256), (size_t)n * sizeof(double), s, LU, LUt2, piv, n, X);
    hipLaunchKernelGGL(k_pinv_finish, grid, dim3(256), 0, s, X, n, u, v, scal);
    if ((rc = check_launch(ctx, "inverse"))) return rc;
    int hflag[4] = {0, 0, 0, 0};
    double hs[3];
    if (hipMemcpyAsync(hflag, flag, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hs, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "factor readback");
    if (hflag[0]) return set_error(ctx, BEM_ENUMERIC, "zero pivot in the LU of the boundary matrix");
    ctx->shift = hs[1];
    ctx->sigma_n = hs[2];
    if (!(hs[2] > 0.0) || !(hs[1] > 0.0)) return set_error(ctx, BEM_ENUMERIC, "bad singular triplet");
    return BEM_OK;
}

}  // namespace bem
