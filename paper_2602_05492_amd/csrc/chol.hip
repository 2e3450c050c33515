// chol.hip - float64 Cholesky of the damped approximate Hessian
// lambda D + J^T J (Eq. optimstep: positive definite, solved by Cholesky,
// Sec. 4.3) and the two triangular solves for the LM step.
// Blocked right-looking factorisation with 64-column panels: diagonal block
// in LDS, panel rows by per-row forward substitution, trailing update by the
// float64 GEMM.  A non-positive or non-finite pivot raises a device flag.
#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr int NB = 64;

// dmax[0] = max_i H_ii (one block)
__global__ void k_diag_max(const double* __restrict__ H, int64_t P, double* __restrict__ dmax)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < P; i += blockDim.x) m = fmax(m, H[i * P + i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dmax[0] = red[0];
}

// A = H + lam * diag(max(H_ii, 1e-12 * max_j H_jj))
__global__ void k_damp(const double* __restrict__ H, int64_t P, double lam, const double* __restrict__ dmax,
                       double* __restrict__ A)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= P) return;
    double v = H[i * P + j];
    if (i == j) v += lam * fmax(v, 1e-12 * dmax[0]);
    A[i * P + j] = v;
}

__device__ inline double readlane_f64(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Factor the diagonal block kb in place (lower triangle).  One wavefront, lane i
// holds row i in registers; column j's pivot and entries come from the owning
// lanes by readlane (the loops are unrolled, so every lane index is a constant).
// Rows / columns past the matrix are an identity block.
__global__ void __launch_bounds__(64) k_potrf_diag(double* __restrict__ A, int64_t P, int kb, int* __restrict__ flag)
{
    const int64_t o = (int64_t)kb * NB;
    const int nb = (int)(P - o < NB ? P - o : NB);
    const int i = threadIdx.x;
    double a[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        a[k] = (i < nb && k < nb) ? (k <= i ? A[(o + i) * P + o + k] : 0.0) : (i == k ? 1.0 : 0.0);
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const double d = readlane_f64(a[j], j);
        const bool ok = d > 0.0 && isfinite(d);
        bad |= !ok;
        const double sj = ok ? sqrt(d) : 1.0;
        a[j] = i == j ? sj : a[j] / sj;
        // entries above the diagonal of a row are never read back, so all lanes update
#pragma unroll
        for (int k = j + 1; k < NB; ++k) a[k] -= a[j] * readlane_f64(a[j], k);
    }
    if (bad && i == 0) flag[0] = 1;
    if (i < nb)
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (k <= i && k < nb) A[(o + i) * P + o + k] = a[k];
}

// Panel rows below diagonal block kb: row <- row L_kk^{-T}.  A block of 64 threads
// stages 64 rows and L_kk in LDS with coalesced loads; thread r then substitutes row r.
__global__ void __launch_bounds__(64) k_trsm_panel(double* __restrict__ A, int64_t P, int kb)
{
    __shared__ double L[NB][NB + 1];
    __shared__ double R[NB][NB + 1];
    const int64_t o = (int64_t)kb * NB;
    const int64_t r0 = o + NB + (int64_t)blockIdx.x * NB;
    const int nr = (int)(P - r0 < NB ? P - r0 : NB);
    const int t = threadIdx.x;
    for (int i = 0; i < NB; ++i) {
        L[i][t] = t <= i ? A[(o + i) * P + o + t] : 0.0;
        R[i][t] = i < nr ? A[(r0 + i) * P + o + t] : 0.0;
    }
    __syncthreads();
    if (t < nr) {
        for (int j = 0; j < NB; ++j) {
            double sum = R[t][j];
            for (int l = 0; l < j; ++l) sum -= R[t][l] * L[j][l];
            R[t][j] = sum / L[j][j];
        }
    }
    __syncthreads();
    for (int i = 0; i < nr; ++i) A[(r0 + i) * P + o + t] = R[i][t];
}

// Triangular solve of diagonal block kb on the nrhs columns of B [P][nrhs] (in place):
// L y = b (trans 0) or L^T y = b (trans 1).  One wavefront; thread t owns row t.
constexpr int kMaxRhs = 4;
__global__ void __launch_bounds__(64) k_trsv_diag(const double* __restrict__ A, int64_t P, int kb,
                                                  double* __restrict__ B, int nrhs, int trans)
{
    __shared__ double x[NB][kMaxRhs];
    const int64_t o = (int64_t)kb * NB;
    const int nb = (int)(P - o < NB ? P - o : NB);
    const int t = threadIdx.x;
    if (t < nb)
        for (int c = 0; c < nrhs; ++c) x[t][c] = B[(o + t) * nrhs + c];
    __syncthreads();
    if (!trans) {
        for (int j = 0; j < nb; ++j) {
            if (t < nrhs) x[j][t] /= A[(o + j) * P + o + j];
            __syncthreads();
            if (t > j && t < nb) {
                const double l = A[(o + t) * P + o + j];
                for (int c = 0; c < nrhs; ++c) x[t][c] -= l * x[j][c];
            }
            __syncthreads();
        }
    } else {
        for (int j = nb - 1; j >= 0; --j) {
            if (t < nrhs) x[j][t] /= A[(o + j) * P + o + j];
            __syncthreads();
            if (t < j) {
                const double l = A[(o + j) * P + o + t];
                for (int c = 0; c < nrhs; ++c) x[t][c] -= l * x[j][c];
            }
            __syncthreads();
        }
    }
    if (t < nb)
        for (int c = 0; c < nrhs; ++c) B[(o + t) * nrhs + c] = x[t][c];
}

}  // namespace

// Damp, factor and check: returns BEM_ENOTPD when a pivot fails (host sync).
int chol_factor(bem_ctx* ctx, const double* H, int64_t P, double lam, double* A, int* dflag, double* dscal,
                hipStream_t s)
{
    int rc;
    hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(256), 0, s, H, P, dscal);
    hipLaunchKernelGGL(k_damp, dim3(blocks_for(P, 256), P), dim3(256), 0, s, H, P, lam, dscal, A);
    if ((rc = fill_i32(ctx, dflag, 1, 0, s))) return rc;
    const int nblk = (int)((P + NB - 1) / NB);
    ProfScope ps_(ctx, PT_CHOLESKY, s);
    for (int kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(64), 0, s, A, P, kb, dflag);
        const int64_t rem = P - (int64_t)(kb + 1) * NB;
        if (rem > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3(blocks_for(rem, NB)), dim3(NB), 0, s, A, P, kb);
            double* panel = A + (int64_t)(kb + 1) * NB * P + (int64_t)kb * NB;
            double* trail = A + (int64_t)(kb + 1) * NB * P + (int64_t)(kb + 1) * NB;
            if ((rc = gemm_f64(ctx, (int)rem, (int)rem, NB, -1.0, panel, P, false, panel, P, true, 1.0, trail, P, s,
                               nullptr, 0)))
                return rc;
        }
    }
    if ((rc = check_launch(ctx, "cholesky"))) return rc;
    int hflag = 0;
    if (hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "cholesky flag readback");
    return hflag ? BEM_ENOTPD : BEM_OK;
}

// B <- (L L^T)^{-1} B with the factor in A; B [P][nrhs] row-major, nrhs <= 4.
int chol_solve(bem_ctx* ctx, const double* A, int64_t P, double* B, int nrhs, hipStream_t s)
{
    int rc;
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(ctx, BEM_EINVAL, "chol_solve: 1..4 right-hand sides");
    ProfScope ps_(ctx, PT_CHOLESKY, s);
    const int nblk = (int)((P + NB - 1) / NB);
    for (int kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(NB), 0, s, A, P, kb, B, nrhs, 0);
        const int64_t rem = P - (int64_t)(kb + 1) * NB;
        if (rem > 0 &&
            (rc = gemm_f64(ctx, (int)rem, nrhs, NB, -1.0, A + (int64_t)(kb + 1) * NB * P + (int64_t)kb * NB, P, false,
                           B + (int64_t)kb * NB * nrhs, nrhs, false, 1.0, B + (int64_t)(kb + 1) * NB * nrhs, nrhs, s,
                           nullptr, 0)))
            return rc;
    }
    for (int kb = nblk - 1; kb >= 0; --kb) {
        hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(NB), 0, s, A, P, kb, B, nrhs, 1);
        const int64_t o = (int64_t)kb * NB;
        const int nb = (int)(P - o < NB ? P - o : NB);
        if (o > 0 && (rc = gemm_f64(ctx, (int)o, nrhs, nb, -1.0, A + o * P, P, true, B + o * nrhs, nrhs, false, 1.0, B,
                                    nrhs, s, nullptr, 0)))
            return rc;
    }
    return check_launch(ctx, "cholesky solve");
}

}  // namespace bem
