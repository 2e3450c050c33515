// chol.hip - float64 Cholesky of the damped approximate Hessian
// lambda D + J^T J (Eq. optimstep: positive definite, solved by Cholesky,
// Sec. 4.3) and the two triangular solves for the LM step.
// Blocked right-looking factorisation with 64-column panels: the diagonal block
// in one wavefront's registers, inverted in the same kernel; the panel as a GEMM
// with that inverse; the trailing update as a rank-64 symmetric update.  The solves
// use the inverted diagonal blocks too: one launch per block and direction.  A
// non-positive or non-finite pivot raises a device flag.
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

// Factor the diagonal block kb in place (lower triangle) and write its inverse to
// Linv [64][64] (row-major).  256 threads, the block in LDS, factored by 16-column
// sub-blocks p = 0..3: wavefront 0 factors the 16 x 16 diagonal sub-block in registers
// (lane i < 16 holds row i; pivot and column entries by readlane, loops unrolled so every
// lane index is a constant; a reciprocal square root per pivot, no divisions) and inverts it (lane j forms column j by forward
// substitution); all threads then form the sub-panel below it (rows times the
// sub-block's inverse transposed) and apply the rank-16 update to the trailing lower
// triangle.  The inverse of the whole block follows by block rows:
// X_ij = -D_i^{-1} sum_{k=j}^{i-1} L_ik X_kj for j < i, X_ii = D_i^{-1}.  Rows / columns
// past the matrix are an identity block.
constexpr int DB = 16;                  // sub-block of the diagonal-block factorization
__global__ void __launch_bounds__(256) k_potrf_diag(double* __restrict__ A, int64_t P, int kb, int* __restrict__ flag,
                                                    double* __restrict__ Linv)
{
    __shared__ double S[NB][NB + 1];    // the block, factored in place (lower triangle)
    __shared__ double X[NB][NB + 1];    // its inverse (lower triangle; zero above)
    const int64_t o = (int64_t)kb * NB;
    const int nb = (int)(P - o < NB ? P - o : NB);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // all 16 loads of a thread in flight at once: entries outside the lower triangle load the
    // block's first element (always in bounds) and are then replaced
    double g[NB * NB / 256];
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
        const int e = tid + 256 * q, r = e >> 6, c = e & 63;
        const bool in = r < nb && c <= r;
        g[q] = A[(o + (in ? r : 0)) * P + o + (in ? c : 0)];
    }
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
        const int e = tid + 256 * q, r = e >> 6, c = e & 63;
        S[r][c] = (r < nb && c <= r) ? g[q] : ((r == c && r >= nb) ? 1.0 : 0.0);
        X[r][c] = 0.0;
    }
    __syncthreads();
    bool bad = false;
    for (int p = 0; p < NB / DB; ++p) {
        const int d0 = p * DB;
        if (w == 0) {
            double a[DB];
#pragma unroll
            for (int k = 0; k < DB; ++k) a[k] = (lane < DB && k <= lane) ? S[d0 + lane][d0 + k] : 0.0;
            double ri[DB];                  // 1 / L_jj (the pivots' reciprocal square roots)
#pragma unroll
            for (int j = 0; j < DB; ++j) {
                const double dj = readlane_f64(a[j], j);
                const bool ok = dj > 0.0 && isfinite(dj);
                bad |= !ok;
                ri[j] = ok ? rsqrt(dj) : 1.0;
                a[j] = lane == j ? (ok ? dj * ri[j] : 1.0) : a[j] * ri[j];
                // entries above the diagonal of a row are never read back, so all lanes update
#pragma unroll
                for (int k = j + 1; k < DB; ++k) a[k] -= a[j] * readlane_f64(a[j], k);
            }
            if (lane < DB) {
#pragma unroll
                for (int k = 0; k < DB; ++k)
                    if (k <= lane) S[d0 + lane][d0 + k] = a[k];
            }
            __threadfence_block();          // the stores complete before the broadcast reads below
            // column `lane` of the sub-block's inverse: x_k = (delta_k,lane - sum_{m<k} L_km x_m) / L_kk,
            // L_km read back from LDS by broadcast (the wavefront's own stores above, in order)
            double x[DB];
#pragma unroll
            for (int k = 0; k < DB; ++k) {
                double acc = lane == k ? 1.0 : 0.0;
#pragma unroll
                for (int m = 0; m < k; ++m) acc -= S[d0 + k][d0 + m] * x[m];
                x[k] = acc * ri[k];
            }
            if (lane < DB) {
#pragma unroll
                for (int k = 0; k < DB; ++k)
                    if (k >= lane) X[d0 + k][d0 + lane] = x[k];
            }
        }
        __syncthreads();
        // sub-panel: rows r >= d0 + 16, columns d0 .. d0 + 15: S[r][d0 + j] = sum_{m<=j} S[r][d0 + m] X[d0 + j][d0 + m]
        const int nr = NB - d0 - DB;
        double v[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int e = tid + 256 * q;
            v[q] = 0.0;
            if (e < nr * DB) {
                const int r = d0 + DB + e / DB, j = e % DB;
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < DB; ++m) acc += S[r][d0 + m] * X[d0 + j][d0 + m];
                v[q] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int e = tid + 256 * q;
            if (e < nr * DB) S[d0 + DB + e / DB][d0 + e % DB] = v[q];
        }
        __syncthreads();
        // trailing lower triangle: S[r][c] -= sum_m S[r][d0 + m] S[c][d0 + m], d0 + 16 <= c <= r
        for (int e = tid; e < nr * nr; e += 256) {
            const int r = d0 + DB + e / nr, c = d0 + DB + e % nr;
            if (c > r) continue;
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < DB; ++m) acc += S[r][d0 + m] * S[c][d0 + m];
            S[r][c] -= acc;
        }
        __syncthreads();
    }
    // off-diagonal blocks of the inverse, block row by block row
    for (int i = 1; i < NB / DB; ++i) {
        const int n = i * DB * DB;       // entries of the blocks (i, j), j < i
        double v[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {    // T_ij = sum_{k=j}^{i-1} L_ik X_kj
            const int e = tid + 256 * q;
            v[q] = 0.0;
            if (e < n) {
                // X[k][col] is zero for k below col's block, so the sum may start at 0
                const int a = e / (i * DB), col = e % (i * DB);
                double acc = 0.0;
                for (int kq = 0; kq < i; ++kq) {
#pragma unroll
                    for (int m = 0; m < DB; ++m) acc += S[i * DB + a][kq * DB + m] * X[kq * DB + m][col];
                }
                v[q] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int e = tid + 256 * q;
            if (e < n) X[i * DB + e / (i * DB)][e % (i * DB)] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {    // X_ij = -D_i^{-1} T_ij
            const int e = tid + 256 * q;
            v[q] = 0.0;
            if (e < n) {
                const int a = e / (i * DB), col = e % (i * DB);
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < DB; ++m) acc += X[i * DB + a][i * DB + m] * X[i * DB + m][col];
                v[q] = -acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int e = tid + 256 * q;
            if (e < n) X[i * DB + e / (i * DB)][e % (i * DB)] = v[q];
        }
        __syncthreads();
    }
    if (tid == 0 && bad) flag[0] = 1;
#pragma unroll
    for (int e = tid; e < NB * NB; e += 256) {
        const int r = e >> 6, c = e & 63;
        if (r < nb && c <= r) A[(o + r) * P + o + c] = S[r][c];
        Linv[e] = X[r][c];
    }
}

// Panel rows below diagonal block kb, in place: row <- row Linv_kk^T (= row L_kk^{-T}), with
// Linv pointing at block kb's inverse [64][64].
// 256 threads; the block stages its 64 rows and Linv_kk in LDS with coalesced loads and
// thread (w, t) forms column t of rows w, w + 4, ...
// skip: row blocks below the diagonal block left out (the first one may come from k_next_diag).
__global__ void __launch_bounds__(256) k_panel(double* __restrict__ A, int64_t P, int kb,
                                               const double* __restrict__ Linv, int skip)
{
    __shared__ double R[NB][NB];        // rows (read by broadcast)
    __shared__ double LiT[NB][NB];      // LiT[k][j] = Linv[j][k]
    const int64_t o = (int64_t)kb * NB;
    const int64_t r0 = o + NB + (int64_t)(blockIdx.x + skip) * NB;
    const int nr = (int)(P - r0 < NB ? P - r0 : NB);
    const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
    // loads first (all in flight; rows past the matrix read row r0 and are then zeroed)
    double gr[NB / 4], gl[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const int i = w + 4 * q;
        gr[q] = A[(r0 + (i < nr ? i : 0)) * P + o + t];
        gl[q] = Linv[(size_t)i * NB + t];
    }
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const int i = w + 4 * q;
        R[i][t] = i < nr ? gr[q] : 0.0;
        LiT[t][i] = gl[q];
    }
    __syncthreads();
    double out[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) out[q] = 0.0;
#pragma unroll 4
    for (int k = 0; k < NB; ++k) {
        const double l = LiT[k][t];                   // (Linv^T)[k][t]
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) out[q] += R[w + 4 * q][k] * l;
    }
#pragma unroll
    for (int q = 0; q < NB / 4; ++q)
        if (w + 4 * q < nr) A[(r0 + w + 4 * q) * P + o + t] = out[q];
}

// Trailing update of step kb on float64 MFMA: C -= L21 L21^T on the lower triangle of the
// trailing matrix C = A[o2:, o2:], o2 = 64 (kb + 1), with the panel L21 = A[o2:, o:o+64].
// One block per 64 x 64 tile (I, J), I >= J (linear block index -> (I, J)); 4 waves, each a
// 32 x 32 quarter as 2 x 2 tiles of v_mfma_f64_16x16x4f64.  The two 64-row panel slices are
// staged in LDS transposed ([k][row], all 64 k in one pass, every global load of the block
// issued before the first wait) so that an MFMA operand (lane l: row l mod 16, k l / 16, the
// same pattern for both operands) is one ds_read per lane.
// Accumulator element q of lane l is row 4 q + l / 16, column l mod 16 of its 16 x 16 tile.
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kSyrkLd = 72;              // LDS row stride (doubles) of the transposed slices
// mode 0: every tile; 1: every tile but the first diagonal one (I = J = 0, updated by k_next_diag).
__global__ void __launch_bounds__(256) k_syrk64(double* __restrict__ A, int64_t P, int kb, int nt, int mode)
{
    __shared__ double SI[NB][kSyrkLd];   // [k][row] of the panel rows of tile row I
    __shared__ double SJ[NB][kSyrkLd];   // and of tile column J
    const int64_t o = (int64_t)kb * NB, o2 = o + NB;
    const int64_t rem = P - o2;
    // tile (I, J), I >= J, from the linear index b = I (I + 1) / 2 + J
    const int b = blockIdx.x;
    if (mode == 1 && b == 0) return;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    if (I >= nt) return;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t rI = (int64_t)I * NB, rJ = (int64_t)J * NB;
    // every global load first, all in flight: the 16 entries of C this thread updates and the two
    // 64-row x 64-k panel slices (entries past the matrix read an in-bounds one and are then
    // replaced)
    double c[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gr = rI + 32 * wr + 16 * i + 4 * q + (l >> 4);
                const int64_t gc = rJ + 32 * wc + 16 * j + (l & 15);
                const bool in = gr < rem && gc <= gr;
                c[i][j][q] = A[(o2 + (in ? gr : 0)) * P + o2 + (in ? gc : 0)];
            }
    double vi[NB * NB / 256], vj[NB * NB / 256];
#pragma unroll
    for (int m = 0; m < NB * NB / 256; ++m) {
        const int e = tid + 256 * m, r = e >> 6, k = e & 63;
        const int64_t gi = rI + r, gj = rJ + r;
        vi[m] = A[(o2 + (gi < rem ? gi : 0)) * P + o + k];
        vj[m] = A[(o2 + (gj < rem ? gj : 0)) * P + o + k];
    }
#pragma unroll
    for (int m = 0; m < NB * NB / 256; ++m) {
        const int e = tid + 256 * m, r = e >> 6, k = e & 63;
        SI[k][r] = rI + r < rem ? vi[m] : 0.0;
        SJ[k][r] = rJ + r < rem ? vj[m] : 0.0;
    }
    __syncthreads();
    d4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NB; ks += 4) {
        const int kk = ks + (l >> 4), rr = l & 15;
        const double a0 = SI[kk][32 * wr + rr], a1 = SI[kk][32 * wr + 16 + rr];
        const double b0 = SJ[kk][32 * wc + rr], b1 = SJ[kk][32 * wc + 16 + rr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gr = rI + 32 * wr + 16 * i + 4 * q + (l >> 4);
                const int64_t gc = rJ + 32 * wc + 16 * j + (l & 15);
                if (gr < rem && gc <= gr) A[(o2 + gr) * P + o2 + gc] = c[i][j][q] - acc[i][j][q];
            }
}

// Look-ahead of step kb (one block): the first row block of the panel,
// L1 = A[o2:o2+64, o:o+64] Linv_kb^T, written in place, and the next diagonal block's update
// A[o2:o2+64, o2:o2+64] -= L1 L1^T on its lower triangle, o2 = 64 (kb + 1).  Both products on
// float64 MFMA with the operand and accumulator layout of k_syrk64; the rows of L1 past the
// matrix are zero (their rows of A are neither read nor written).  Requires P > o2.
__global__ void __launch_bounds__(256) k_next_diag(double* __restrict__ A, int64_t P, int kb,
                                                   const double* __restrict__ Linv)
{
    __shared__ double SI[NB][kSyrkLd];   // [k][row]: A's row block, then L1
    __shared__ double SJ[NB][kSyrkLd];   // [k][j] = Linv_kb[j][k]
    const int64_t o = (int64_t)kb * NB, o2 = o + NB;
    const int nr = (int)(P - o2 < NB ? P - o2 : NB);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    // every global load first (entries past the matrix or above the diagonal read an in-bounds
    // one and are then replaced): this thread's 16 entries of the diagonal block, the row block
    // and the inverse
    double c[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gr = 32 * wr + 16 * i + 4 * q + (l >> 4), gc = 32 * wc + 16 * j + (l & 15);
                const bool in = gr < nr && gc <= gr;
                c[i][j][q] = A[(o2 + (in ? gr : 0)) * P + o2 + (in ? gc : 0)];
            }
    double va[NB * NB / 256], vl[NB * NB / 256];
#pragma unroll
    for (int m = 0; m < NB * NB / 256; ++m) {
        const int e = tid + 256 * m, r = e >> 6, k = e & 63;
        va[m] = A[(o2 + (r < nr ? r : 0)) * P + o + k];
        vl[m] = Linv[(size_t)r * NB + k];
    }
#pragma unroll
    for (int m = 0; m < NB * NB / 256; ++m) {
        const int e = tid + 256 * m, r = e >> 6, k = e & 63;
        SI[k][r] = r < nr ? va[m] : 0.0;
        SJ[k][r] = vl[m];
    }
    __syncthreads();
    d4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NB; ks += 4) {
        const int kk = ks + (l >> 4), rr = l & 15;
        const double a0 = SI[kk][32 * wr + rr], a1 = SI[kk][32 * wr + 16 + rr];
        const double b0 = SJ[kk][32 * wc + rr], b1 = SJ[kk][32 * wc + 16 + rr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();                    // every wave is done reading SI
    // L1 to A and, transposed ([k = column][row]), back into SI
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gr = 32 * wr + 16 * i + 4 * q + (l >> 4), gc = 32 * wc + 16 * j + (l & 15);
                SI[gc][gr] = acc[i][j][q];
                if (gr < nr) A[(o2 + gr) * P + o + gc] = acc[i][j][q];
            }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NB; ks += 4) {
        const int kk = ks + (l >> 4), rr = l & 15;
        const double a0 = SI[kk][32 * wr + rr], a1 = SI[kk][32 * wr + 16 + rr];
        const double b0 = SI[kk][32 * wc + rr], b1 = SI[kk][32 * wc + 16 + rr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gr = 32 * wr + 16 * i + 4 * q + (l >> 4), gc = 32 * wc + 16 * j + (l & 15);
                if (gr < nr && gc <= gr) A[(o2 + gr) * P + o2 + gc] = c[i][j][q] - acc[i][j][q];
            }
}

// Forward step kb of L y = b with the inverted diagonal blocks, B [P][nrhs]: every block
// forms y_kb = Linv_kb b_kb; block 0 writes it to Y, block t >= 1 subtracts L y_kb from the
// 64 rows starting at o + 64 t (B rows of block kb itself are not modified in this step).
// 256 threads: operand tiles are staged in LDS, each wave loading 16 rows, and the products
// are split over the 4 waves by k and summed in LDS.
constexpr int kMaxRhs = 4;
// the four waves' partial sums of row t
__device__ inline void solve_sum(const double (*part)[NB][kMaxRhs], int t, int nrhs, double* out)
{
    for (int c = 0; c < nrhs; ++c) out[c] = part[0][t][c] + part[1][t][c] + part[2][t][c] + part[3][t][c];
}

template <int nrhs>
__global__ void __launch_bounds__(256) k_fwd_step(const double* __restrict__ A, int64_t P, int kb,
                                                  const double* __restrict__ Linv, double* __restrict__ B,
                                                  double* __restrict__ Y)
{
    __shared__ double T[NB][NB + 1];
    __shared__ double At[NB][NB + 1];   // the block's rows of L (loaded with T: it does not depend on y)
    __shared__ double bk[NB][kMaxRhs];
    __shared__ double y[NB][kMaxRhs];
    __shared__ double part[4][NB][kMaxRhs];
    const int64_t o = (int64_t)kb * NB;
    const int nb = (int)(P - o < NB ? P - o : NB);
    const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double* L0 = Linv + (size_t)kb * NB * NB;
    const int64_t r0 = o + (int64_t)blockIdx.x * NB;
    const int nr = blockIdx.x == 0 ? 0 : (int)(P - r0 < NB ? P - r0 : NB);
    // loads first (all in flight; entries past the matrix read an in-bounds one and are then zeroed)
    double gl[NB / 4], ga[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const int r = w + 4 * q;
        gl[q] = L0[(size_t)r * NB + t];
        ga[q] = blockIdx.x != 0 ? A[(r0 + (r < nr ? r : 0)) * P + o + (t < nb ? t : 0)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const int r = w + 4 * q;
        T[r][t] = gl[q];
        At[r][t] = (r < nr && t < nb) ? ga[q] : 0.0;
    }
    if (w == 0)
        for (int c = 0; c < nrhs; ++c) bk[t][c] = t < nb ? B[(o + t) * nrhs + c] : 0.0;
    __syncthreads();
    {
        double acc[nrhs] = {};
        for (int k = 16 * w; k < 16 * w + 16; ++k) {
            const double l = T[t][k];
            for (int c = 0; c < nrhs; ++c) acc[c] += l * bk[k][c];
        }
        for (int c = 0; c < nrhs; ++c) part[w][t][c] = acc[c];
    }
    __syncthreads();
    if (w == 0) {
        double v[nrhs];
        solve_sum(part, t, nrhs, v);
        for (int c = 0; c < nrhs; ++c) y[t][c] = v[c];
        if (blockIdx.x == 0 && t < nb)
            for (int c = 0; c < nrhs; ++c) Y[(o + t) * nrhs + c] = v[c];
    }
    if (blockIdx.x == 0) return;
    __syncthreads();
    {
        double acc[nrhs] = {};
        for (int k = 16 * w; k < 16 * w + 16; ++k) {
            const double l = At[t][k];
            for (int c = 0; c < nrhs; ++c) acc[c] += l * y[k][c];
        }
        for (int c = 0; c < nrhs; ++c) part[w][t][c] = acc[c];
    }
    __syncthreads();
    if (w == 0 && t < nr) {
        double v[nrhs];
        solve_sum(part, t, nrhs, v);
        for (int c = 0; c < nrhs; ++c) B[(r0 + t) * nrhs + c] -= v[c];
    }
}

// Backward step kb of L^T x = y: every block forms x_kb = Linv_kb^T y_kb; block 0 writes it
// to X, block t >= 1 subtracts L[block kb rows, c]^T x_kb from the 64 entries of Y starting
// at column c = 64 (t - 1) (only columns before block kb; Y rows of block kb are only read).
template <int nrhs>
__global__ void __launch_bounds__(256) k_bwd_step(const double* __restrict__ A, int64_t P, int kb,
                                                  const double* __restrict__ Linv, double* __restrict__ Y,
                                                  double* __restrict__ X)
{
    __shared__ double T[NB][NB + 1];
    __shared__ double At[NB][NB + 1];   // block kb's rows of L at this block's columns (loaded with T)
    __shared__ double yk[NB][kMaxRhs];
    __shared__ double x[NB][kMaxRhs];
    __shared__ double part[4][NB][kMaxRhs];
    const int64_t o = (int64_t)kb * NB;
    const int nb = (int)(P - o < NB ? P - o : NB);
    const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double* L0 = Linv + (size_t)kb * NB * NB;
    const int64_t col = (int64_t)(blockIdx.x - 1) * NB + t;
    // loads first (all in flight; entries past the matrix read an in-bounds one and are then zeroed)
    double gl[NB / 4], ga[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const int r = w + 4 * q;
        gl[q] = L0[(size_t)r * NB + t];
        ga[q] = blockIdx.x != 0 ? A[(o + (r < nb ? r : 0)) * P + (col < o ? col : 0)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const int r = w + 4 * q;
        T[r][t] = gl[q];
        At[r][t] = (r < nb && col < o) ? ga[q] : 0.0;
    }
    if (w == 0)
        for (int c = 0; c < nrhs; ++c) yk[t][c] = t < nb ? Y[(o + t) * nrhs + c] : 0.0;
    __syncthreads();
    {
        double acc[nrhs] = {};
        for (int k = 16 * w; k < 16 * w + 16; ++k) {
            const double l = T[k][t];                  // (Linv^T)[t][k]
            for (int c = 0; c < nrhs; ++c) acc[c] += l * yk[k][c];
        }
        for (int c = 0; c < nrhs; ++c) part[w][t][c] = acc[c];
    }
    __syncthreads();
    if (w == 0) {
        double v[nrhs];
        solve_sum(part, t, nrhs, v);
        for (int c = 0; c < nrhs; ++c) x[t][c] = v[c];
        if (blockIdx.x == 0 && t < nb)
            for (int c = 0; c < nrhs; ++c) X[(o + t) * nrhs + c] = v[c];
    }
    if (blockIdx.x == 0) return;
    __syncthreads();
    {
        double acc[nrhs] = {};
        for (int r = 16 * w; r < 16 * w + 16; ++r) {
            const double l = At[r][t];
            for (int c = 0; c < nrhs; ++c) acc[c] += l * x[r][c];
        }
        for (int c = 0; c < nrhs; ++c) part[w][t][c] = acc[c];
    }
    __syncthreads();
    if (w == 0 && col < o) {
        double v[nrhs];
        solve_sum(part, t, nrhs, v);
        for (int c = 0; c < nrhs; ++c) Y[col * nrhs + c] -= v[c];
    }
}

}  // namespace

// Damp, factor and check: returns BEM_ENOTPD when a pivot fails (host sync).  Blocked
// right-looking with 64-column panels: the diagonal block and its inverse by k_potrf_diag,
// the panel as A21 Linv^T (in place; its first row block by k_next_diag), the trailing
// lower triangle by a rank-64 update.  The inverted diagonal blocks stay in the context
// for chol_solve.
int chol_factor(bem_ctx* ctx, const double* H, int64_t P, double lam, double* A, int* dflag, double* dscal,
                hipStream_t s)
{
    int rc;
    const int nblk = (int)((P + NB - 1) / NB);
    // cholw: inverted diagonal blocks [nblk][64][64] | solve vector [P][4]
    if ((rc = ensure(ctx, ctx->cholw, ((size_t)nblk * NB * NB + (size_t)P * kMaxRhs) * sizeof(double), s))) return rc;
    double* linv = (double*)ctx->cholw.ptr;
    hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(256), 0, s, H, P, dscal);
    hipLaunchKernelGGL(k_damp, dim3(blocks_for(P, 256), P), dim3(256), 0, s, H, P, lam, dscal, A);
    if ((rc = fill_i32(ctx, dflag, 1, 0, s))) return rc;
    ProfScope ps_(ctx, PT_CHOLESKY, s);
    // Look-ahead: only the next diagonal block's inputs stay on the caller's stream (k_next_diag:
    // the panel's first row block and that block's update, then its factor); the rest of the
    // panel and the trailing update run on the second stream.  Step kb's trailing update waits
    // for k_next_diag(kb) (it reads the first row block), and k_next_diag(kb + 1) waits for that
    // update (it reads the tiles it wrote).  The two streams touch disjoint tiles meanwhile.
    hipStream_t s2 = s;
    const bool ahead = nblk > 2;
    if (ahead && (rc = aux_stream(ctx, &s2))) return rc;
    hipEvent_t evP = ctx->ev[0], evN = ctx->ev[1], evS = ctx->ev[6];
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, A, P, 0, dflag, linv);
    for (int kb = 0; kb < nblk; ++kb) {
        double* Li = linv + (size_t)kb * NB * NB;
        const int64_t rem = P - (int64_t)(kb + 1) * NB;
        if (rem <= 0) break;
        const int nt = blocks_for(rem, NB);
        if (!ahead) {
            hipLaunchKernelGGL(k_panel, dim3(nt), dim3(256), 0, s, A, P, kb, (const double*)Li, 0);
            hipLaunchKernelGGL(k_syrk64, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, A, P, kb, nt, 0);
            hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, A, P, kb + 1, dflag, Li + NB * NB);
            continue;
        }
        // second stream: the panel below the next diagonal block, once block kb is factored
        if (hipEventRecord(evP, s) != hipSuccess || hipStreamWaitEvent(s2, evP, 0) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "cholesky event");
        if (nt > 1) hipLaunchKernelGGL(k_panel, dim3(nt - 1), dim3(256), 0, s2, A, P, kb, (const double*)Li, 1);
        // caller's stream: the next diagonal block, once the previous trailing update is done
        if (kb > 0 && hipStreamWaitEvent(s, evS, 0) != hipSuccess) return set_error(ctx, BEM_EHIP, "cholesky wait");
        hipLaunchKernelGGL(k_next_diag, dim3(1), dim3(256), 0, s, A, P, kb, (const double*)Li);
        if (nt > 1) {
            if (hipEventRecord(evN, s) != hipSuccess || hipStreamWaitEvent(s2, evN, 0) != hipSuccess)
                return set_error(ctx, BEM_EHIP, "cholesky event");
            hipLaunchKernelGGL(k_syrk64, dim3(nt * (nt + 1) / 2), dim3(256), 0, s2, A, P, kb, nt, 1);
            if (hipEventRecord(evS, s2) != hipSuccess) return set_error(ctx, BEM_EHIP, "cholesky event");
        }
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, A, P, kb + 1, dflag, Li + NB * NB);
    }
    if (ahead && hipStreamWaitEvent(s, evS, 0) != hipSuccess) return set_error(ctx, BEM_EHIP, "cholesky join");
    if ((rc = check_launch(ctx, "cholesky"))) return rc;
    ctx->chol_P = P;
    int hflag = 0;
    if (hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "cholesky flag readback");
    return hflag ? BEM_ENOTPD : BEM_OK;
}

// B <- (L L^T)^{-1} B with the factor in A and the inverted diagonal blocks of the last
// chol_factor; B [P][nrhs] row-major, nrhs <= 4.  One launch per block and direction.
// Forward then backward block steps for nrhs right-hand sides (B [P][nrhs] in, solution out; Y [P][nrhs] scratch).
template <int nrhs>
static void solve_steps(const double* A, int64_t P, int nblk, const double* linv, double* B, double* Y, hipStream_t s)
{
    for (int kb = 0; kb < nblk; ++kb) {
        const int64_t rem = P - (int64_t)(kb + 1) * NB;
        const int nbk = 1 + (rem > 0 ? blocks_for(rem, NB) : 0);
        hipLaunchKernelGGL(k_fwd_step<nrhs>, dim3(nbk), dim3(256), 0, s, A, P, kb, linv, B, Y);
    }
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int64_t o = (int64_t)kb * NB;
        const int nbk = 1 + (o > 0 ? blocks_for(o, NB) : 0);
        hipLaunchKernelGGL(k_bwd_step<nrhs>, dim3(nbk), dim3(256), 0, s, A, P, kb, linv, Y, B);
    }
}

int chol_solve(bem_ctx* ctx, const double* A, int64_t P, double* B, int nrhs, hipStream_t s)
{
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(ctx, BEM_EINVAL, "chol_solve: 1..4 right-hand sides");
    if (ctx->chol_P != P) return set_error(ctx, BEM_ESTATE, "chol_solve without a matching chol_factor");
    ProfScope ps_(ctx, PT_CHOLESKY, s);
    const int nblk = (int)((P + NB - 1) / NB);
    const double* linv = (const double*)ctx->cholw.ptr;
    double* Y = (double*)ctx->cholw.ptr + (size_t)nblk * NB * NB;
    switch (nrhs) {
    case 1: solve_steps<1>(A, P, nblk, linv, B, Y, s); break;
    case 2: solve_steps<2>(A, P, nblk, linv, B, Y, s); break;
    case 3: solve_steps<3>(A, P, nblk, linv, B, Y, s); break;
    default: solve_steps<4>(A, P, nblk, linv, B, Y, s); break;
    }
    return check_launch(ctx, "cholesky solve");
}

}  // namespace bem
