// gram_mfma.hip - the normal-equation contraction on the matrix cores (Eq.
// losshessian): G += X X^T over one sample tile, X the feature-major tile
// [W rows x n samples], only the needed output tiles (256x256 split-BF16,
// 128x128 FP32).
//
//   FP32_MFMA   : v_mfma_f32_32x32x2_f32 on float rows
//   BF16X3_MFMA : rows split x = hi + lo (bfloat16); hi*hi + hi*lo + lo*hi on
//                 v_mfma_f32_32x32x16_bf16 (the lo*lo term is below float32
//                 rounding of the product)
// Accumulation is float32 over one part of the tile's samples and float64
// across tiles and parts (the epilogue adds into the float64 Gram of the part).
// The A and B operands of every MFMA come from rows of the same matrix with the
// same lane -> (row, k-slot) assignment, so each k of the slab is summed once.
#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

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

// Zero output tile [row0, row0 + ts) x [col0, col0 + ts) of G (clipped to W): the part of a work entry
// that holds no samples, when the Gram writes rather than accumulates.
__device__ inline void zero_tile(double* __restrict__ G, int64_t row0, int64_t col0, int ts, int W)
{
    for (int e = threadIdx.x; e < ts * ts; e += blockDim.x) {
        const int64_t i = row0 + e / ts, j = col0 + e % ts;
        if (i < W && j < W) G[i * W + j] = 0.0;
    }
}

__device__ inline void epilogue(const floatx16 (&acc)[2][2], int64_t rbase, int64_t cbase, int W, int accumulate,
                                double* __restrict__ G)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 31, lk = lane >> 5;
    for (int mi = 0; mi < 2; ++mi)
        for (int nj = 0; nj < 2; ++nj)
            for (int r = 0; r < 16; ++r) {
                const int64_t i = rbase + 32 * mi + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int64_t j = cbase + 32 * nj + li;
                if (i < W && j < W) G[i * W + j] = (accumulate ? G[i * W + j] : 0.0) + (double)acc[mi][nj][r];
            }
}

// Block -> work entry: blocks are handed to the 8 XCDs round-robin (block b runs
// on XCD b mod 8), so XCD x is given the contiguous run of entries
// [x * per, (x + 1) * per) of the work list; entries ordered by super-tiles keep
// the operand panels of the blocks running together on one XCD few, and they
// are then served from that XCD's L2.
__device__ inline int work_index(int nwork)
{
    const int per = (nwork + 7) >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

__global__ void __launch_bounds__(256) k_gram_f32(const float* __restrict__ X, int64_t ld, int W, int64_t n_all,
                                                  const int* __restrict__ work, int nwork, int64_t kchunk,
                                                  double* __restrict__ G, int64_t gstride, int accumulate)
{
    const int wi = work_index(nwork);
    if (wi >= nwork) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t rbase = (int64_t)work[3 * wi] * 128 + 64 * (wave >> 1);
    const int64_t cbase = (int64_t)work[3 * wi + 1] * 128 + 64 * (wave & 1);
    const int64_t kb = (int64_t)work[3 * wi + 2] * kchunk;
    const int64_t n = kb + kchunk < n_all ? kb + kchunk : n_all;
    G += (int64_t)work[3 * wi + 2] * gstride;
    if (kb >= n) {
        if (!accumulate) zero_tile(G, (int64_t)work[3 * wi] * 128, (int64_t)work[3 * wi + 1] * 128, 128, W);
        return;
    }
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
    for (int64_t k0 = kb; k0 < n; k0 += 8) {
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
    epilogue(acc, rbase, cbase, W, accumulate, G);
}

// Split-bfloat16 Gram with LDS staging: a block of 8 wavefronts owns a 256x256
// output tile (wavefront w: rows 64*(w/2).., cols 128*(w%2).., 2x4 MFMA tiles of
// 32x32).  The tile is in 32-sample blocks ([t / 32][row][t % 32], zero beyond
// the last sample), so one 32-sample stage of a 256-row operand slab (A hi/lo,
// B hi/lo) is a contiguous 16 KiB run and every 128-byte line fetched is used
// whole.  Stages go from global memory straight into LDS (global_load_lds, 16
// bytes per lane, no staging registers) and are double buffered (2 x 64 KiB):
// stage k+1 is in flight while stage k is multiplied, one barrier per stage.
// LDS rows are 64 bytes (4 chunks of 8 samples); chunk c of row r sits at
// position c ^ swz(r), swz(r) = ((r >> 1) ^ (r >> 2)) & 3, so that the 16-byte
// operand reads of 16 consecutive rows fall in distinct banks.  A wavefront's
// load instruction fills 1 KiB of LDS (16 rows) in lane order, so each lane
// fetches the global chunk whose swizzled position is its own.
constexpr int G2_T = 256, G2_BK = 32;

__device__ inline int g2_lds(int r, int c)   // element offset of chunk c of row r in one slab
{
    return (r << 5) + ((c ^ (((r >> 1) ^ (r >> 2)) & 3)) << 3);
}

__global__ void __launch_bounds__(512) k_gram_bf16x3_lds(const uint16_t* __restrict__ Xh, const uint16_t* __restrict__ Xl,
                                                         int W, int n_all, const int* __restrict__ work,
                                                         int nwork, int kchunk, double* __restrict__ G,
                                                         int64_t gstride, int accumulate)
{
    __shared__ __attribute__((aligned(16))) uint16_t sm0[4][G2_T * G2_BK];   // [A hi, A lo, B hi, B lo]
    __shared__ __attribute__((aligned(16))) uint16_t sm1[4][G2_T * G2_BK];
    const int wi = work_index(nwork);
    if (wi >= nwork) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 31, lk = lane >> 5;
    const int row0 = work[3 * wi] * G2_T;
    const int col0 = work[3 * wi + 1] * G2_T;
    // samples [kb, n) of this entry's part; partial Gram of the part
    const int kb = work[3 * wi + 2] * kchunk;
    const int n = kb + kchunk < n_all ? kb + kchunk : n_all;
    G += (int64_t)work[3 * wi + 2] * gstride;
    if (kb >= n) {                                         // part beyond a ragged last tile
        if (!accumulate) zero_tile(G, row0, col0, G2_T, W);
        return;
    }
    const int wr = wave >> 1, wc = wave & 1;
    const int W32 = W << 5;    // elements per 32-sample block of the tile
    // direct loads: this wavefront fills row blocks wave and wave + 8 (16 rows each) of each slab;
    // lane l writes row rb*16 + l/4, position l%4, i.e. global chunk (l%4) ^ swz(row)
    const int lr = lane >> 2;
    const int lc = (lane & 3) ^ (((lr >> 1) ^ (lr >> 2)) & 3);   // swz of the row (depends on lr only)
    int gsrc[2][2];            // [A/B][block j] element offset of this lane's chunk within a 32-sample block
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int r = (wave + 8 * j) * 16 + lr;
        const int ra = row0 + r < W ? row0 + r : W - 1;   // rows past the matrix: any valid row (their
        const int rb = col0 + r < W ? col0 + r : W - 1;   // products land outside G and are dropped)
        gsrc[0][j] = (ra << 5) + (lc << 3);
        gsrc[1][j] = (rb << 5) + (lc << 3);
    }
#define G2_LOAD_STAGE(SM, K0)                                                                  \
    {                                                                                          \
        const int kb_ = ((K0) >> 5) * W32;                                                     \
        _Pragma("unroll") for (int ab = 0; ab < 2; ++ab)                                       \
        _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                        \
            const int d_ = (wave + 8 * j) * 16 * 32;                                           \
            __builtin_amdgcn_global_load_lds((const void*)(Xh + kb_ + gsrc[ab][j]),            \
                                             (void*)&SM[2 * ab][d_], 16, 0, 0);                \
            __builtin_amdgcn_global_load_lds((const void*)(Xl + kb_ + gsrc[ab][j]),            \
                                             (void*)&SM[2 * ab + 1][d_], 16, 0, 0);            \
        }                                                                                      \
    }
    // operand read offsets: rows of this lane, chunk 2 * h + lk for half h of the stage.  Rows 32 m
    // further on sit 1024 m elements further (the swizzle depends on row bits 1..3 only), so one
    // offset per half and operand serves every 32-row tile with an immediate displacement.
    int aoff[2], boff[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        aoff[h] = g2_lds(wr * 64 + li, 2 * h + lk);
        boff[h] = g2_lds(wc * 128 + li, 2 * h + lk);
    }
// multiply the stage in LDS buffer SM: 8 steps (half h = step / 4, column tile nj = step % 4);
// the B operands of the next step (and the A operands of the second half) are read from LDS
// while the current step's MFMAs run
#define G2_A(SM, h, ah, al)                                                                   \
    _Pragma("unroll") for (int mi = 0; mi < 2; ++mi) {                                        \
        ah[mi] = __builtin_bit_cast(bf16x8, *(const u16x8*)&SM[0][aoff[h] + 1024 * mi]);      \
        al[mi] = __builtin_bit_cast(bf16x8, *(const u16x8*)&SM[1][aoff[h] + 1024 * mi]);      \
    }
#define G2_B(SM, h, nj, bh, bl)                                                               \
    bh = __builtin_bit_cast(bf16x8, *(const u16x8*)&SM[2][boff[h] + 1024 * (nj)]);            \
    bl = __builtin_bit_cast(bf16x8, *(const u16x8*)&SM[3][boff[h] + 1024 * (nj)]);
#define G2_STEP(ah, al, bh, bl, nj)                                                           \
    _Pragma("unroll") for (int mi = 0; mi < 2; ++mi) {                                        \
        acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mi], bh, acc[mi][nj], 0, 0, 0); \
        acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mi], bl, acc[mi][nj], 0, 0, 0); \
        acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[mi], bh, acc[mi][nj], 0, 0, 0); \
    }
// order inside a step: its LDS reads (for the next step) first, then its 6 MFMAs; no
// instruction crosses a step boundary
#define G2_ORDER(nreads)                                                                      \
    __builtin_amdgcn_sched_group_barrier(0x100, nreads, 0);                                   \
    __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);                                        \
    __builtin_amdgcn_sched_barrier(0);
// operands of a stage's first step (A of the first half, B of column tile 0)
#define G2_HEAD(SM)                                                                           \
    G2_A(SM, 0, a0h, a0l)                                                                     \
    G2_B(SM, 0, 0, b0h, b0l)
// steps 0..6 of the stage in SM (its first operands already requested); the operands of step 7
// are in registers at the end, and no LDS read of SM is left in flight once lgkmcnt is 0
#define G2_BODY(SM)                                                                           \
    G2_B(SM, 0, 1, b1h, b1l)  G2_STEP(a0h, a0l, b0h, b0l, 0)  G2_ORDER(2)                     \
    G2_B(SM, 0, 2, b0h, b0l)  G2_STEP(a0h, a0l, b1h, b1l, 1)  G2_ORDER(2)                     \
    G2_B(SM, 0, 3, b1h, b1l)  G2_STEP(a0h, a0l, b0h, b0l, 2)  G2_ORDER(2)                     \
    G2_A(SM, 1, a1h, a1l)                                                                     \
    G2_B(SM, 1, 0, b0h, b0l)  G2_STEP(a0h, a0l, b1h, b1l, 3)  G2_ORDER(6)                     \
    G2_B(SM, 1, 1, b1h, b1l)  G2_STEP(a1h, a1l, b0h, b0l, 0)  G2_ORDER(2)                     \
    G2_B(SM, 1, 2, b0h, b0l)  G2_STEP(a1h, a1l, b1h, b1l, 1)  G2_ORDER(2)                     \
    G2_B(SM, 1, 3, b1h, b1l)  G2_STEP(a1h, a1l, b0h, b0l, 2)  G2_ORDER(2)
// end of the stage in CUR at sample k0, the other buffer NXT holding stage k0 + 32 (if any):
// every wavefront has read CUR and written its share of NXT -> barrier; CUR is refilled with stage
// k0 + 64; the first operands of NXT are requested (unused past the last stage; the reads stay
// inside the buffer) and the step-7 MFMAs of CUR, whose operands are in registers, cover their
// latency and the barrier's LDS burst
#define G2_TURN(CUR, NXT, k0)                                                                 \
    __builtin_amdgcn_s_waitcnt(0x3f70);               /* vmcnt(0): this wavefront's loads of NXT */ \
    __syncthreads();                                                                          \
    if ((k0) + 2 * G2_BK < n) G2_LOAD_STAGE(CUR, (k0) + 2 * G2_BK)                            \
    G2_HEAD(NXT)                                                                              \
    __builtin_amdgcn_sched_barrier(0);                                                        \
    G2_STEP(a1h, a1l, b1h, b1l, 3)                                                            \
    __builtin_amdgcn_sched_barrier(0);
    floatx16 acc[2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 4; ++nj)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][nj][r] = 0.0f;
    bf16x8 a0h[2], a0l[2], a1h[2], a1l[2], b0h, b0l, b1h, b1l;
    G2_LOAD_STAGE(sm0, kb)
    __builtin_amdgcn_s_waitcnt(0x3f70);
    __syncthreads();
    if (kb + G2_BK < n) G2_LOAD_STAGE(sm1, kb + G2_BK)
    G2_HEAD(sm0)
    for (int k0 = kb;; k0 += 2 * G2_BK) {
        // stage k0 in sm0, stage k0 + 32 (if any) arriving in sm1
        G2_BODY(sm0)
        G2_TURN(sm0, sm1, k0)
        if (k0 + G2_BK >= n) break;
        G2_BODY(sm1)
        G2_TURN(sm1, sm0, k0 + G2_BK)
        if (k0 + 2 * G2_BK >= n) break;
    }
#undef G2_LOAD_STAGE
#undef G2_A
#undef G2_B
#undef G2_STEP
#undef G2_ORDER
#undef G2_HEAD
#undef G2_BODY
#undef G2_TURN
    // epilogue: G += acc (G = acc for the first sample tile).  A tile inside the matrix reads its 16
    // values of an MFMA tile in one batch (one wait instead of 16); tiles at the matrix edge go
    // element by element.
    const bool inside = row0 + G2_T <= W && col0 + G2_T <= W;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 4; ++nj) {
            const int ib = row0 + wr * 64 + 32 * mi + 4 * lk;
            const int j = col0 + wc * 128 + 32 * nj + li;
            if (inside) {
                double* g = G + (int64_t)ib * W + j;
                double v[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = accumulate ? g[(int64_t)(8 * (r >> 2) + (r & 3)) * W] : 0.0;
#pragma unroll
                for (int r = 0; r < 16; ++r) g[(int64_t)(8 * (r >> 2) + (r & 3)) * W] = v[r] + (double)acc[mi][nj][r];
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = ib + 8 * (r >> 2) + (r & 3);
                    if (i < W && j < W)
                        G[(int64_t)i * W + j] = (accumulate ? G[(int64_t)i * W + j] : 0.0) + (double)acc[mi][nj][r];
                }
            }
        }
}

// R[f][c] += sum_t X[f][t] r[t][c]  (float64 sums; float rows of stride ld)
__global__ void __launch_bounds__(256) k_xr_f32(const float* __restrict__ X, int64_t ld, int64_t n,
                                                const double* __restrict__ r, double* __restrict__ R, int f0)
{
    __shared__ double red[3][256];
    const int64_t f = f0 + (int64_t)blockIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        const double v = (double)X[f * ld + t];
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

// Blocked split-bfloat16 tile: partial sums over sample-block group g,
// Rp[g][f][c] = sum over the group's samples of (hi + lo)[f][t] r[t][c].  A
// wavefront reads 16 rows x 4 chunks of 8 samples of one 32-sample block (1 KiB
// contiguous); the 4 chunk lanes of a row are summed by shuffles.
constexpr int kXrGroups = kXrPartials;

__global__ void __launch_bounds__(256) k_xr_bf16(const uint16_t* __restrict__ Xh, const uint16_t* __restrict__ Xl, int W,
                                                 int64_t n, int64_t blocks_per_group, const double* __restrict__ r,
                                                 double* __restrict__ Rp, int f0)
{
    const int lane = threadIdx.x & 63;
    const int f = f0 + blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + (lane >> 2);
    const int cq = lane & 3;
    const int64_t nb = (n + 31) / 32;
    const int64_t b0 = (int64_t)blockIdx.y * blocks_per_group;
    const int64_t b1 = b0 + blocks_per_group < nb ? b0 + blocks_per_group : nb;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (f < W) {
        for (int64_t b = b0; b < b1; ++b) {
            const size_t i = (size_t)b * ((size_t)W << 5) + ((size_t)f << 5) + (size_t)(cq << 3);
            const u16x8 h = *(const u16x8*)(Xh + i);
            const u16x8 l = *(const u16x8*)(Xl + i);
            const int64_t t0 = b * 32 + cq * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t t = t0 + e;
                if (t < n) {
                    const double v = (double)__uint_as_float((uint32_t)h[e] << 16) +
                                     (double)__uint_as_float((uint32_t)l[e] << 16);
                    s0 += v * r[3 * t]; s1 += v * r[3 * t + 1]; s2 += v * r[3 * t + 2];
                }
            }
        }
    }
    s0 += __shfl_xor(s0, 1); s1 += __shfl_xor(s1, 1); s2 += __shfl_xor(s2, 1);
    s0 += __shfl_xor(s0, 2); s1 += __shfl_xor(s1, 2); s2 += __shfl_xor(s2, 2);
    if (cq == 0 && f < W) {
        double* o = Rp + ((size_t)blockIdx.y * W + f) * 3;
        o[0] = s0; o[1] = s1; o[2] = s2;
    }
}

// R[f][c] += sum_g Rp[g][f][c] (fixed order), rows f >= f0
__global__ void k_xr_finish(const double* __restrict__ Rp, int W, int groups, double* __restrict__ R, int f0)
{
    const int i = 3 * f0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * W) return;
    double v = 0.0;
    for (int g = 0; g < groups; ++g) v += Rp[(size_t)g * 3 * W + i];
    R[i] += v;
}

}  // namespace

// G[part] += X X^T over the work entries (row tile, column tile, part): part p covers
// samples [p * kchunk, (p + 1) * kchunk) of the tile and adds into G + p * gstride (accumulate = 0:
// writes, for the first sample tile; entries outside the work list are not touched).
int launch_gram_mfma(bem_ctx* ctx, int gram, const void* Xhi, const uint16_t* Xlo, int64_t ld, int W, int64_t n,
                     const int* work, int nwork, int64_t kchunk, double* G, int64_t gstride, bool accumulate,
                     hipStream_t s)
{
    if (n <= 0 || nwork <= 0) return BEM_OK;
    const int grid = 8 * ((nwork + 7) / 8);
    if (gram == BEM_GRAM_BF16X3_MFMA)
        {
            ProfScope ps_(ctx, PT_GRAM_MFMA, s);
            // blocked tile (ld unused); element offsets inside one operand array are 32-bit
            // (W * tile rows < 2^31 is checked by the caller)
            hipLaunchKernelGGL(k_gram_bf16x3_lds, dim3(grid), dim3(512), 0, s, (const uint16_t*)Xhi, Xlo, W, (int)n,
                               work, nwork, (int)kchunk, G, gstride, accumulate ? 1 : 0);
        }
    else
        {
            ProfScope ps_(ctx, PT_GRAM_MFMA, s);
            hipLaunchKernelGGL(k_gram_f32, dim3(grid), dim3(256), 0, s, (const float*)Xhi, ld, W, n, work, nwork, kchunk,
                               G, gstride, accumulate ? 1 : 0);
        }
    return check_launch(ctx, "gram_mfma");
}

// R += X r over one sample tile for the rows [f0, W); Rp is a workspace of kXrGroups * W * 3 doubles
// (split-BF16 only).
int launch_xr(bem_ctx* ctx, int gram, const void* Xhi, const uint16_t* Xlo, int64_t ld, int W, int64_t n,
              const double* r, double* R, double* Rp, hipStream_t s, int f0)
{
    if (n <= 0 || f0 >= W) return BEM_OK;
    ProfScope ps_(ctx, PT_XR, s);
    const int rows = W - f0;
    if (gram == BEM_GRAM_BF16X3_MFMA) {
        const int64_t nb = (n + 31) / 32;
        const int64_t per = (nb + kXrGroups - 1) / kXrGroups;
        hipLaunchKernelGGL(k_xr_bf16, dim3((rows + 63) / 64, kXrGroups), dim3(256), 0, s, (const uint16_t*)Xhi, Xlo, W,
                           n, per, r, Rp, f0);
        hipLaunchKernelGGL(k_xr_finish, dim3((3 * rows + 255) / 256), dim3(256), 0, s, (const double*)Rp, W, kXrGroups,
                           R, f0);
    } else {
        hipLaunchKernelGGL(k_xr_f32, dim3(rows), dim3(256), 0, s, (const float*)Xhi, ld, n, r, R, f0);
    }
    return check_launch(ctx, "xr");
}

}  // namespace bem
