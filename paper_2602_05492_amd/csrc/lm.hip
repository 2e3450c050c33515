// lm.hip - one Levenberg-Marquardt step (Eq. optimstep, Sec. 4.3) on the
// samples of the call: mean colour, residual and loss, gradient by the
// adjoint, approximate Hessian by the normal equations, damped Cholesky
// solve, trial evaluation on the same samples, accept / reject and damping
// update (lambda / 10 on a decrease of the loss, * 10 otherwise).
#include <cmath>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr int kRedBlocks = 512;

__global__ void k_fill_i32(int* __restrict__ p, int64_t n, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// partial[b] = sums over a strided share of rows: mode 0: sum_c (u - T)^2 and r = u - T written;
// mode 1: per-channel sums of T (3 partials); mode 2: per-channel sums of T - u.
template <class UT>
__global__ void __launch_bounds__(256) k_rowsum(const UT* __restrict__ u, const double* __restrict__ T, int64_t N,
                                                int mode, UT* __restrict__ r, double* __restrict__ partial)
{
    __shared__ double red[3][256];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const double t0 = T[3 * i], t1 = T[3 * i + 1], t2 = T[3 * i + 2];
        if (mode == 1) {
            a0 += t0; a1 += t1; a2 += t2;
            continue;
        }
        const double u0 = (double)u[3 * i], u1 = (double)u[3 * i + 1], u2 = (double)u[3 * i + 2];
        if (mode == 2) {
            a0 += t0 - u0; a1 += t1 - u1; a2 += t2 - u2;
            continue;
        }
        const double r0 = u0 - t0, r1 = u1 - t1, r2 = u2 - t2;
        if (r) { r[3 * i] = (UT)r0; r[3 * i + 1] = (UT)r1; r[3 * i + 2] = (UT)r2; }
        a0 += r0 * r0 + r1 * r1 + r2 * r2;
    }
    red[0][threadIdx.x] = a0; red[1][threadIdx.x] = a1; red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) partial[3 * blockIdx.x + c] = red[c][0];
}

// ---- compatibility condition (Sec. 3.1.2) and its enforcement (Sec. 4.3) -------------------
// A [3][P]: a_c . theta = int over the handles of w_c for fixed end points.  A segment's jump is
// linear between its end values, so per cubic handle alpha_h = sum_k L_k (2 - t_k - t_{k+1}) / 2
// at wc0_{h,c} and beta_h = sum_k L_k (t_k + t_{k+1}) / 2 at wc1_{h,c}; a straight handle's
// constant wc_{h,c} has the coefficient alpha_h + beta_h = sum_k L_k (model 1).  Thread per
// handle, from the float64 segment table (degenerate segments have L2 = 0 there).  A must be
// zero beforehand.
__global__ void k_compat_vectors(const double* __restrict__ seg64, int H, int S, int model, int64_t P,
                                 double* __restrict__ A)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    double alpha = 0.0, beta = 0.0;
    for (int k = 0; k < S; ++k) {
        const double L = sqrt(seg64[((size_t)h * S + k) * kSegStride + 6]);
        const double ta = (double)k / (double)S, tb = (double)(k + 1) / (double)S;
        alpha += L * (2.0 - ta - tb) / 2.0;
        beta += L * (ta + tb) / 2.0;
    }
    for (int c = 0; c < 3; ++c) {
        if (model == 1) {
            A[(size_t)c * P + (size_t)h * 10 + 7 + c] = alpha + beta;
        } else {
            A[(size_t)c * P + (size_t)h * 20 + 14 + c] = alpha;
            A[(size_t)c * P + (size_t)h * 20 + 17 + c] = beta;
        }
    }
}

__device__ inline void block_sum(double* v, int n, double (*red)[256])
{
    for (int i = 0; i < n; ++i) red[i][threadIdx.x] = v[i];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int i = 0; i < n; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
        __syncthreads();
    }
    for (int i = 0; i < n; ++i) v[i] = red[i][0];
    __syncthreads();
}

// Right-hand sides of the constrained step: R [P][4] = [g | a_0 | a_1 | a_2].
__global__ void k_pack_rhs(const double* __restrict__ g, const double* __restrict__ A, int64_t P, double* __restrict__ R)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    R[4 * p] = g[p];
    for (int c = 0; c < 3; ++c) R[4 * p + 1 + c] = A[(size_t)c * P + p];
}

// Constrained damped step (one block): R [P][4] holds delta0 = Hd^{-1} g and X_c = Hd^{-1} a_c;
// solve (A^T X) nu = A^T delta0 over the channels with a nonzero a_c (Gaussian elimination with
// partial pivoting) and write delta = delta0 - X nu, so that A^T delta = 0.
__global__ void __launch_bounds__(256) k_compat_solve(const double* __restrict__ A, const double* __restrict__ R,
                                                      int64_t P, double* __restrict__ delta)
{
    __shared__ double red[12][256];
    __shared__ double nu[3];
    double v[12];
    for (int i = 0; i < 12; ++i) v[i] = 0.0;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        for (int i = 0; i < 3; ++i) {
            const double a = A[(size_t)i * P + p];
            for (int j = 0; j < 3; ++j) v[3 * i + j] += a * R[4 * p + 1 + j];
            v[9 + i] += a * R[4 * p];
        }
    }
    block_sum(v, 12, red);
    if (threadIdx.x == 0) {
        int idx[3], n = 0;
        for (int c = 0; c < 3; ++c)
            if (v[4 * c] > 0.0) idx[n++] = c;             // a_c = 0: no constraint on that channel
        double M[3][4];
        for (int r = 0; r < n; ++r) {
            for (int q = 0; q < n; ++q) M[r][q] = v[3 * idx[r] + idx[q]];
            M[r][n] = v[9 + idx[r]];
        }
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int r = col + 1; r < n; ++r)
                if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
            for (int q = 0; q <= n; ++q) { const double tmp = M[col][q]; M[col][q] = M[piv][q]; M[piv][q] = tmp; }
            for (int r = col + 1; r < n; ++r) {
                const double f = M[r][col] / M[col][col];
                for (int q = col; q <= n; ++q) M[r][q] -= f * M[col][q];
            }
        }
        double sol[3] = {0.0, 0.0, 0.0};
        for (int r = n - 1; r >= 0; --r) {
            double s = M[r][n];
            for (int q = r + 1; q < n; ++q) s -= M[r][q] * sol[q];
            sol[r] = s / M[r][r];
        }
        for (int c = 0; c < 3; ++c) nu[c] = 0.0;
        for (int r = 0; r < n; ++r) nu[idx[r]] = sol[r];
    }
    __syncthreads();
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x)
        delta[p] = R[4 * p] - (R[4 * p + 1] * nu[0] + R[4 * p + 2] * nu[1] + R[4 * p + 3] * nu[2]);
}

// Re-projection of the wc parameters of theta onto a_c . theta = 0 with a_c taken at theta's own
// end points (one block; the three a_c have disjoint supports); out[0] = the largest remaining
// |a_c . theta| relative to sum_p |a_c[p] theta[p]|.
__global__ void __launch_bounds__(256) k_reproject(const double* __restrict__ A, int64_t P, double* __restrict__ theta,
                                                   double* __restrict__ out)
{
    __shared__ double red[6][256];
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x)
        for (int c = 0; c < 3; ++c) {
            const double a = A[(size_t)c * P + p];
            v[c] += a * theta[p];
            v[3 + c] += a * a;
        }
    block_sum(v, 6, red);
    double f[3];
    for (int c = 0; c < 3; ++c) f[c] = v[3 + c] > 0.0 ? v[c] / v[3 + c] : 0.0;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x)
        theta[p] -= A[p] * f[0] + A[(size_t)P + p] * f[1] + A[2 * (size_t)P + p] * f[2];
    __syncthreads();
    for (int c = 0; c < 6; ++c) v[c] = 0.0;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x)
        for (int c = 0; c < 3; ++c) {
            const double a = A[(size_t)c * P + p];
            v[c] += a * theta[p];
            v[3 + c] += fabs(a * theta[p]);
        }
    block_sum(v, 6, red);
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int c = 0; c < 3; ++c)
            if (v[3 + c] > 0.0) m = fmax(m, fabs(v[c]) / v[3 + c]);
        out[0] = m;
    }
}

__global__ void k_finish_sum(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partial[3 * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

__global__ void k_scale(double* __restrict__ v, int64_t n, double s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] *= s;
}

__global__ void k_axpy_to(const double* __restrict__ a, const double* __restrict__ d, int64_t n, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - d[i];
}

__global__ void k_finite(const double* __restrict__ v, int64_t n, int* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i])) flag[0] = 1;
}

}  // namespace

int fill_i32(bem_ctx* ctx, int* p, int64_t n, int v, hipStream_t s)
{
    if (n <= 0) return BEM_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return check_launch(ctx, "fill_i32");
}

// Three-component sums over the N rows (mode as k_rowsum) into host out[3]; synchronises.
static int row_sums(bem_ctx* ctx, const void* u, bool f32, const double* T, int64_t N, int mode, void* r, double* out,
                    double* dpart, hipStream_t s)
{
    const int nb = N > 0 ? (int)((N + 255) / 256 < kRedBlocks ? (N + 255) / 256 : kRedBlocks) : 1;
    if (N > 0) {
        if (f32)
            hipLaunchKernelGGL(k_rowsum<float>, dim3(nb), dim3(256), 0, s, (const float*)u, T, N, mode, (float*)r, dpart);
        else
            hipLaunchKernelGGL(k_rowsum<double>, dim3(nb), dim3(256), 0, s, (const double*)u, T, N, mode, (double*)r, dpart);
        hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(64), 0, s, dpart, nb, dpart + 3 * kRedBlocks);
    } else {
        fill_f64(ctx, dpart + 3 * kRedBlocks, 3, 0.0, s);
    }
    int rc = check_launch(ctx, "row sums");
    if (rc) return rc;
    if (hipMemcpyAsync(out, dpart + 3 * kRedBlocks, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "row sums readback");
    return BEM_OK;
}

// Morton index of each sample's cell in a kCellSide x kCellSide grid over the outer boundary's
// bounding box (coordinates clamped into it).  The mixed LM step visits the samples cell by cell,
// so that the 64 samples of a wavefront are neighbours: a segment near one of them is then near
// many, the near pairs of a wavefront fall into long runs of equal segments, and the adjoint
// adds one set of sums per run instead of one per pair.
constexpr int kCellBits = 5, kCellSide = 1 << kCellBits, kCells = kCellSide * kCellSide;
__global__ void k_cell_labels(const double* __restrict__ x, int64_t N, double x0, double y0, double sx, double sy,
                              int32_t* __restrict__ lab)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    // fmax first, so that a NaN coordinate lands in cell 0
    const int cx = (int)fmin(fmax((x[2 * i] - x0) * sx, 0.0), (double)(kCellSide - 1));
    const int cy = (int)fmin(fmax((x[2 * i + 1] - y0) * sy, 0.0), (double)(kCellSide - 1));
    int m = 0;
    for (int b = 0; b < kCellBits; ++b) m |= (((cx >> b) & 1) << (2 * b)) | (((cy >> b) & 1) << (2 * b + 1));
    lab[i] = m;
}

// Deal the cell-ordered 64-sample chunks out in a stride permutation: full chunk c goes to
// chunk (c * stride) mod nchunk (stride coprime to nchunk), the samples of a short last chunk stay
// in place.  Each wavefront keeps its 64 neighbours, while consecutive wavefronts come from
// distant cells, so that float32 sums over consecutive samples (the Gram's accumulation within a
// sample tile) see them in effectively random order: in cell order their partial sums wander
// further and the LM step moved up to 2.7x further from the float64 step.
__global__ void k_deal_chunks(const double* __restrict__ x, const double* __restrict__ T, int64_t N, int64_t nchunk,
                              int64_t stride, double* __restrict__ xo, double* __restrict__ To)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t c = i >> 6;
    const int64_t j = c < nchunk ? ((c * stride) % nchunk) * 64 + (i & 63) : i;
    xo[2 * j] = x[2 * i];
    xo[2 * j + 1] = x[2 * i + 1];
    To[3 * j] = T[3 * i];
    To[3 * j + 1] = T[3 * i + 1];
    To[3 * j + 2] = T[3 * i + 2];
}

__global__ void k_widen3(const float* __restrict__ g, int64_t n, double* __restrict__ o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = (double)g[i];
}

__global__ void k_narrow3(const double* __restrict__ g, int64_t n, float* __restrict__ o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = (float)g[i];
}

// Largest overflowing near-pair count of a wavefront in a mixed sweep (0: no slice overflowed).
static int read_need(bem_ctx* ctx, const int* dneed, hipStream_t s, int* need)
{
    *need = 0;
    if (!dneed) return BEM_OK;
    if (hipMemcpyAsync(need, dneed, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "near-pair count readback");
    return BEM_OK;
}

// Raise the context's near-pair capacity to hold wavefronts of `need` pairs with a quarter of
// headroom (a fresh batch of samples seldom packs more than that into one wavefront, and each
// overflow costs a repeated sweep); true if that is more than the slots per wavefront of the
// list that overflowed.
static bool raise_near_slots(bem_ctx* ctx, int need, int64_t nwaves, int slots)
{
    if (need <= slots) return false;
    const int want = near_slots_for(need + need / 4, nwaves);
    if (want > ctx->near_slots) ctx->near_slots = want;
    return want > slots;
}

// Samples and their float32 cotangents reordered cell by cell (the order of lm_step's sweeps) into
// the context's sort workspace, without a host synchronisation; *xo and *go point into it.
int cell_order_f32(bem_ctx* ctx, const double* x, const float* g, int64_t N, const double** xo, const float** go,
                   hipStream_t s)
{
    int rc;
    const size_t lb = ((size_t)N * sizeof(int32_t) + 255) / 256 * 256;
    const size_t gb = ((size_t)N * 3 * sizeof(float) + 255) / 256 * 256;
    if ((rc = ensure(ctx, ctx->sortw, lb + gb + (size_t)N * 8 * sizeof(double), s))) return rc;
    int32_t* lab = (int32_t*)ctx->sortw.ptr;
    float* g32 = (float*)((char*)ctx->sortw.ptr + lb);
    double* xc = (double*)((char*)ctx->sortw.ptr + lb + gb);
    double* gw = xc + 2 * N;                      // cotangents widened, input order
    double* gc = gw + 3 * N;                      // cell order
    const double bw = ctx->bbox[2] - ctx->bbox[0], bh = ctx->bbox[3] - ctx->bbox[1];
    hipLaunchKernelGGL(k_cell_labels, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, ctx->bbox[0], ctx->bbox[1],
                       bw > 0.0 ? kCellSide / bw : 0.0, bh > 0.0 ? kCellSide / bh : 0.0, lab);
    hipLaunchKernelGGL(k_widen3, dim3(blocks_for(3 * N, 256)), dim3(256), 0, s, g, 3 * N, gw);
    // every label is a cell index in [0, kCells), so every sample is kept
    if ((rc = run_partition(ctx, lab, N, kCells, x, gw, xc, gc, nullptr, s))) return rc;
    hipLaunchKernelGGL(k_narrow3, dim3(blocks_for(3 * N, 256)), dim3(256), 0, s, (const double*)gc, 3 * N, g32);
    if ((rc = check_launch(ctx, "sample reordering"))) return rc;
    *xo = xc;
    *go = g32;
    return BEM_OK;
}

int run_lm_step(bem_ctx* ctx, double* theta, int H, const double* x, int64_t N, const double* T, bem_lm_state* st,
                int gram, bool mixed, hipStream_t s)
{
    int rc;
    const int64_t P = (int64_t)ctx->npar * H;
    const size_t ue = mixed ? sizeof(float) : sizeof(double);
    const int64_t n3 = 3 * (N > 0 ? N : 1);
    // lm workspace layout (ctx->lmw): u | r | g | JtJ | (spare P) | A | delta | theta' | partials | flag |
    // compatibility vectors [3][P] | right-hand sides [P][4] | violation
    const size_t bytes = 2 * (size_t)n3 * ue + ((size_t)P + 2 * (size_t)P * P + 2 * (size_t)P + (size_t)P +
                                                 3 * (size_t)kRedBlocks + 8 + 7 * (size_t)P + 8) * sizeof(double) + 64;
    if ((rc = ensure(ctx, ctx->lmw, bytes, s))) return rc;
    char* base = (char*)ctx->lmw.ptr;
    void* u = base;
    void* r = base + (size_t)n3 * ue;
    double* g = (double*)(base + 2 * (size_t)n3 * ue);
    double* JtJ = g + P;
    double* A = JtJ + (size_t)P * P + P;
    double* delta = A + (size_t)P * P;
    double* th1 = delta + P;
    double* dpart = th1 + (size_t)P;
    int* dflag = (int*)(dpart + 3 * kRedBlocks + 4);
    double* cA = dpart + 3 * kRedBlocks + 8;
    double* cX = cA + 3 * (size_t)P;          // [P][4]: gradient and the three a_c, solved in place
    double* cviol = cX + 4 * (size_t)P;
    if (st->data_count < 0 || (st->data_count > 0 && st->data_count < N))
        return set_error(ctx, BEM_EINVAL, "data_count %lld must be 0 or at least N = %lld", (long long)st->data_count,
                         (long long)N);
    // the data terms divide by the samples drawn over the whole image (a subdomain's step sums
    // only its own)
    const double nd = st->data_count > 0 ? (double)st->data_count : (double)N;
    st->compat_violation = 0.0;
    st->reg_value = 0.0;
    st->snap_pairs = 0;
    const bem_prec prec = mixed ? BEM_PREC_MIXED : BEM_PREC_FP64;
    st->accepted = 0;
    st->chol_retries = 0;
    // mixed precision: samples and targets reordered into a workspace, cell by cell and then with
    // the cell-ordered wavefronts dealt out (the step's results depend on the order only through
    // rounding)
    if (mixed && N > 0) {
        const size_t lb = ((size_t)N * sizeof(int32_t) + 255) / 256 * 256;
        if ((rc = ensure(ctx, ctx->sortw, lb + (size_t)N * 10 * sizeof(double), s))) return rc;
        int32_t* lab = (int32_t*)ctx->sortw.ptr;
        double* xc = (double*)((char*)ctx->sortw.ptr + lb);     // cell order
        double* Tc = xc + 2 * N;
        double* xs = Tc + 3 * N;                                 // chunks dealt out
        double* Ts = xs + 2 * N;
        const double bw = ctx->bbox[2] - ctx->bbox[0], bh = ctx->bbox[3] - ctx->bbox[1];
        hipLaunchKernelGGL(k_cell_labels, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, ctx->bbox[0], ctx->bbox[1],
                           bw > 0.0 ? kCellSide / bw : 0.0, bh > 0.0 ? kCellSide / bh : 0.0, lab);
        std::vector<int64_t> off(kCells + 1);
        if ((rc = run_partition(ctx, lab, N, kCells, x, T, xc, Tc, off.data(), s))) return rc;
        if (off[kCells] != N) return set_error(ctx, BEM_EHIP, "sample reordering kept %lld of %lld samples",
                                               (long long)off[kCells], (long long)N);
        const int64_t nchunk = N / 64;
        int64_t stride = nchunk > 1 ? ((int64_t)(0.382 * (double)nchunk) | 1) : 1;
        while (nchunk > 1 && std::gcd(stride, nchunk) != 1) stride += 2;
        hipLaunchKernelGGL(k_deal_chunks, dim3(blocks_for(N, 256)), dim3(256), 0, s, (const double*)xc, (const double*)Tc, N,
                           nchunk, stride, xs, Ts);
        if ((rc = check_launch(ctx, "sample reordering"))) return rc;
        x = xs;
        T = Ts;
    }
    // mean colour
    double sums[3];
    if (st->mean_rule == 0) {
        if ((rc = row_sums(ctx, nullptr, false, T, N, 1, nullptr, sums, dpart, s))) return rc;
        for (int c = 0; c < 3; ++c) st->cbar_sum[c] += sums[c];
        st->cbar_count += N;
        for (int c = 0; c < 3; ++c) st->cbar[c] = st->cbar_count > 0 ? st->cbar_sum[c] / (double)st->cbar_count : 0.0;
    } else {
        const double zero[3] = {0.0, 0.0, 0.0};
        if ((rc = bem_eval(ctx, theta, H, x, N, zero, u, prec, s))) return rc;
        if ((rc = row_sums(ctx, u, mixed, T, N, 2, nullptr, sums, dpart, s))) return rc;
        for (int c = 0; c < 3; ++c) st->cbar[c] = N > 0 ? sums[c] / (double)N : 0.0;
    }
    // residual and loss at theta; the mixed sweep's near-pair list serves the adjoint and the
    // normal equations below (same samples, same parameters).  Should the list overflow, its
    // capacity is raised and the sweep repeated, so that they find every near pair in it.
    NearList nl{};
    if (mixed) {
        if ((rc = prepare_forward(ctx, theta, H, true, s))) return rc;
        for (int pass = 0;; ++pass) {
            if ((rc = launch_sweep_mixed(ctx, x, N, H * ctx->opts.segs_per_handle, st->cbar, (float*)u, s, &nl)))
                return rc;
            if ((rc = row_sums(ctx, u, mixed, T, N, 0, r, sums, dpart, s))) return rc;
            int need = 0;
            if ((rc = read_need(ctx, nl.need, s, &need))) return rc;
            nl.overflowed = need > 0;        // without overflow the flagged-sample kernels are skipped
            if (pass > 0 || !raise_near_slots(ctx, need, nl.nwaves, nl.slots)) break;
        }
    } else {
        if ((rc = bem_eval(ctx, theta, H, x, N, st->cbar, u, prec, s))) return rc;
        if ((rc = row_sums(ctx, u, mixed, T, N, 0, r, sums, dpart, s))) return rc;
    }
    const double L0 = N > 0 ? 0.5 * sums[0] / nd : 0.0;
    st->loss_before = L0;
    st->loss_after = L0;
    if (!std::isfinite(L0)) return set_error(ctx, BEM_ENUMERIC, "non-finite loss at the current parameters");
    if (H == 0 || N == 0) return BEM_OK;
    // gradient g = (1/m) J^T r and Hessian H = (1/m) J^T J.  Mixed precision with an MFMA Gram and
    // handles of several segments: g is formed with the J tiles (the handle rows' J^T r summed in the
    // feature kernel, the beta rows' read back from the tile), so no separate adjoint sweep runs
    // (LM workload, S = 32: 512 -> 445 ms per step, A/B on one box).  With one segment per handle
    // the in-kernel sums cost more than the adjoint (paper-native workload: 26.5 -> 26.0 ms with
    // the adjoint), so there, and otherwise, g comes from the adjoint (bem_vjp's kernels) and the
    // normal equations form J^T J only.
    const bool g_from_tiles = mixed && (gram == BEM_GRAM_FP32_MFMA || gram == BEM_GRAM_BF16X3_MFMA) &&
                              ctx->opts.segs_per_handle >= 2;
    if (g_from_tiles) {
        if ((rc = run_jtj(ctx, theta, H, x, N, r, mixed, gram, JtJ, g, s, &nl, nd))) return rc;
    } else {
        if ((rc = run_vjp(ctx, theta, H, x, N, r, mixed, g, s, mixed ? &nl : nullptr))) return rc;
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(P, 256)), dim3(256), 0, s, g, P, 1.0 / nd);
        if ((rc = run_jtj(ctx, theta, H, x, N, r, mixed, gram, JtJ, nullptr, s, mixed ? &nl : nullptr, nd))) return rc;
    }
    // regularisation terms (Sec. 4.4): gradient and Hessian into g and J^T J, value into the loss;
    // the snapping pairs chosen here are kept for the trial point
    const bool reg = reg_active(ctx);
    double R0 = 0.0;
    if (reg) {
        int np = 0;
        if ((rc = reg_terms(ctx, theta, H, true, g, JtJ, &R0, &np, s))) return rc;
        st->reg_value = R0;
        st->snap_pairs = np;
        st->loss_before = L0 + R0;
        st->loss_after = L0 + R0;
    }
    // damped Cholesky, raising lambda until it factors
    double lam = st->lambda;
    for (int attempt = 0;; ++attempt) {
        rc = chol_factor(ctx, JtJ, P, lam, A, dflag, dpart, s);
        if (rc == BEM_OK) break;
        if (rc != BEM_ENOTPD) return rc;
        if (attempt >= 10) {
            st->lambda = lam;
            return set_error(ctx, BEM_ENOTPD, "damped normal matrix not positive definite after %d retries", attempt);
        }
        lam = std::fmin(lam * 10.0, 1e12);
        st->chol_retries++;
    }
    st->lambda = lam;
    const int S = ctx->opts.segs_per_handle;
    if (!st->compat) {
        if (hipMemcpyAsync(delta, g, P * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "copy gradient");
        if ((rc = chol_solve(ctx, A, P, delta, 1, s))) return rc;
    } else {
        // the step restricted to A^T delta = 0 (A at the current end points, whose segment table
        // the normal equations left in place): one solve of Hd [delta0 | X] = [g | A], then the
        // 3x3 Schur complement
        if ((rc = fill_f64(ctx, cA, 3 * P, 0.0, s))) return rc;
        hipLaunchKernelGGL(k_compat_vectors, dim3(blocks_for(H, 64)), dim3(64), 0, s, (const double*)ctx->seg64.ptr, H,
                           S, ctx->model, P, cA);
        hipLaunchKernelGGL(k_pack_rhs, dim3(blocks_for(P, 256)), dim3(256), 0, s, (const double*)g,
                           (const double*)cA, P, cX);
        if ((rc = chol_solve(ctx, A, P, cX, 4, s))) return rc;
        hipLaunchKernelGGL(k_compat_solve, dim3(1), dim3(256), 0, s, (const double*)cA, (const double*)cX, P, delta);
    }
    if ((rc = fill_i32(ctx, dflag, 1, 0, s))) return rc;
    hipLaunchKernelGGL(k_finite, dim3(blocks_for(P, 256)), dim3(256), 0, s, delta, P, dflag);
    hipLaunchKernelGGL(k_axpy_to, dim3(blocks_for(P, 256)), dim3(256), 0, s, theta, delta, P, th1);
    if ((rc = check_launch(ctx, "update"))) return rc;
    if (st->compat) {
        // re-projection of w_c at the new end points
        if ((rc = launch_expand(ctx, th1, H, s))) return rc;
        if ((rc = fill_f64(ctx, cA, 3 * P, 0.0, s))) return rc;
        hipLaunchKernelGGL(k_compat_vectors, dim3(blocks_for(H, 64)), dim3(64), 0, s, (const double*)ctx->seg64.ptr, H,
                           S, ctx->model, P, cA);
        hipLaunchKernelGGL(k_reproject, dim3(1), dim3(256), 0, s, (const double*)cA, P, th1, cviol);
        hipLaunchKernelGGL(k_finite, dim3(blocks_for(P, 256)), dim3(256), 0, s, th1, P, dflag);
        if ((rc = check_launch(ctx, "compatibility"))) return rc;
        if (hipMemcpyAsync(&st->compat_violation, cviol, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "violation readback");
    }
    // trial loss on the same samples and mean colour (an overflow of its near-pair list raises the
    // capacity for later calls)
    if ((rc = bem_eval(ctx, th1, H, x, N, st->cbar, u, prec, s))) return rc;
    if ((rc = row_sums(ctx, u, mixed, T, N, 0, nullptr, sums, dpart, s))) return rc;
    if (mixed) {
        int need = 0;
        const int64_t nw = (int64_t)blocks_for(N, 256) * 4;
        if ((rc = read_need(ctx, ctx->sweep_need, s, &need))) return rc;
        raise_near_slots(ctx, need, nw, near_slots_for(ctx->near_slots, nw));
    }
    int hflag = 0;
    if (hipMemcpy(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "flag readback");
    double L1 = 0.5 * sums[0] / nd;
    if (reg) {
        double R1 = 0.0;
        if ((rc = reg_terms(ctx, th1, H, false, nullptr, nullptr, &R1, nullptr, s))) return rc;
        L1 += R1;
    }
    st->loss_after = L1;
    if (!hflag && std::isfinite(L1) && L1 < st->loss_before) {
        if (hipMemcpyAsync(theta, th1, P * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "accept copy");
        st->accepted = 1;
        st->lambda = std::fmax(lam / 10.0, 1e-12);
    } else {
        st->lambda = std::fmin(lam * 10.0, 1e12);
    }
    return BEM_OK;
}

}  // namespace bem
