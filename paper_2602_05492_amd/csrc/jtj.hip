// jtj.hip - Monte Carlo normal equations (Eq. losshessian, Eq. lossjacobian)
// with the Jacobian of the differential BIE (Eq. diffbie, Sec. 3.2):
//
//   J_c(x) = df_c/dtheta(x) + sum_i beta_i(x) Z_c[i, :],   Z = A+ dF/dtheta.
//
// Per sample x and channel c the augmented row a_c(x) = [g_c(x) | e(x) | beta(x)]
// holds the G*H geometry derivatives of f_c, the C*H channel-independent colour
// coefficients and the M outer-element weights, so that J_c(x) = a_c(x) S_c with
// S_c = [E_c ; Z_c'] (E_c a column selection).  Cubic handles: G = 8 (control
// points), C = 4 (wd and wc at both ends); straight handles: G = 4 (end points),
// C = 2 (the constant wd and wc).
// Sample tiles of feature rows Xt = [g_1 | g_2 | g_3 | e | beta] (feature-major,
// W = (3G + C)H + M rows) are formed by the feature kernels and contracted into the
// Gram G = sum_x Xt Xt^T (only the blocks the three channels need), and into
// R = sum_x Xt r.  Afterwards, per channel,
//   J^T J += E_c^T A_c E_c + sym(E_c^T B_c Z_c') + Z_c'^T D Z_c'
// with A_c, B_c, D the channel's blocks of G, and J^T r likewise.
#include <algorithm>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <vector>

#include <cstring>

#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr double kGaussNode = 0.77459666924148337703585307995647992;
constexpr double kGaussW0 = 5.0 / 9.0, kGaussW1 = 8.0 / 9.0;

// ---- output element types of the feature kernels ------------------------------
__device__ inline uint16_t bf16_bits(float v)
{
    // round to nearest even (inputs are finite)
    const uint32_t u = __float_as_uint(v);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Feature element (f, t) of a tile.  float64 / float32 tiles are row-major with
// row stride ld; the split-bfloat16 tile is stored in blocks of 32 samples,
// [t / 32][f][t % 32] with ld = the number of rows, so that one 32-sample stage
// of consecutive rows is one contiguous run of memory for the Gram kernel.
template <class OutT> struct Store;
template <> struct Store<double> {
    __device__ static void put(double* hi, uint16_t*, int64_t f, int64_t t, int64_t ld, double v) { hi[f * ld + t] = v; }
};
template <> struct Store<float> {
    __device__ static void put(float* hi, uint16_t*, int64_t f, int64_t t, int64_t ld, double v)
    {
        hi[f * ld + t] = (float)v;
    }
};
// hi + lo bfloat16 split of the float value
template <> struct Store<uint16_t> {
    __device__ static void put(uint16_t* hi, uint16_t* lo, int64_t f, int64_t t, int64_t ld, double v)
    {
        const size_t i = (size_t)(t >> 5) * (size_t)(ld << 5) + (size_t)(f << 5) + (size_t)(t & 31);
        const float x = (float)v;
        const uint16_t h = bf16_bits(x);
        hi[i] = h;
        lo[i] = bf16_bits(x - bf16_value(h));
    }
};

// Feature rows of one (point, handle): the chained gradients geo[c][q] on the four weights of
// vertex_weights and the coefficients col[m] of wd0, wd1, wc0, wc1 (jumps at t = 0 and t = 1).
// Channel c's geometry rows start at c * gp, gp = G H rounded up to a multiple of 256 (the
// Gram's tile), so that no Gram tile mixes two channels; the colour rows start at 3 gp.
// Cubic handles (model 0, G = 8): rows c gp + 8h + q and 3 gp + 4h + m.  Straight handles
// (model 1, G = 4): the end-point gradients are geo[c][0..3], rows c gp + 4h + q, and the
// constant jumps take the sum of their two end coefficients, rows 3 gp + 2h + {0: wd, 1: wc}.
template <class OutT, class A>
__device__ inline void store_handle_rows(int model, OutT* Xt, uint16_t* Xlo, int H, int h, int64_t t, int64_t ld,
                                         int64_t gp, const A (&geo)[3][8], const A (&col)[4])
{
    if (model == 1) {
        for (int c = 0; c < 3; ++c)
            for (int q = 0; q < 4; ++q)
                Store<OutT>::put(Xt, Xlo, (int64_t)c * gp + 4 * h + q, t, ld, (double)geo[c][q]);
        Store<OutT>::put(Xt, Xlo, 3 * gp + 2 * h, t, ld, (double)col[0] + (double)col[1]);
        Store<OutT>::put(Xt, Xlo, 3 * gp + 2 * h + 1, t, ld, (double)col[2] + (double)col[3]);
        return;
    }
    for (int c = 0; c < 3; ++c)
        for (int q = 0; q < 8; ++q)
            Store<OutT>::put(Xt, Xlo, (int64_t)c * gp + 8 * h + q, t, ld, (double)geo[c][q]);
    for (int q = 0; q < 4; ++q) Store<OutT>::put(Xt, Xlo, 3 * gp + 4 * h + q, t, ld, (double)col[q]);
}

// Padding rows [c gp + G H, (c + 1) gp) of the three geometry blocks are zero in every tile.
template <class OutT>
__global__ void k_zero_pad(OutT* __restrict__ Xt, uint16_t* __restrict__ Xlo, int64_t ld, int64_t gp, int64_t gh,
                           int64_t npts)
{
    const int64_t pad = gp - gh;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * pad * npts) return;
    const int64_t r = i / npts, t = i % npts;
    Store<OutT>::put(Xt, Xlo, (r / pad) * gp + gh + r % pad, t, ld, 0.0);
}

// ---- J^T r of the handle rows, formed with the features -------------------------------
// Per (sample, handle) the products of its feature rows with the sample's residuals:
// v[8 c + q] = geo[c][q] r_c (the channel-c geometry rows), v[24 + 3 m + c] = col[m] r_c (the
// channel-shared colour rows against each channel's residual): 36 values, summed over the 256
// samples of a block in float32 (wavefront reduction, then the 4 wavefronts through LDS) and
// stored per block; k_jtr_handles adds the blocks in float64.
constexpr int kJtrVals = 36;

// Sum of v over the 64 lanes of a wavefront for v[0..31] by recursive halving (after the steps
// with offsets 32, 16, 8, 4, 2 lane l holds the sum over its half-wavefront of v[(l >> 1) & 31],
// the offset-1 step completes it), and for v[32..35] by butterflies; the 4 wavefronts' sums are
// then added through LDS and written to out[0..35].
template <class A>
__device__ inline void handle_jtr_block(const A (&geo)[3][8], const A (&col)[4], float r0, float r1, float r2,
                                        float (*red)[kJtrVals], float* __restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float v[32];
    float e[4];
    const float r[3] = {r0, r1, r2};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < 8; ++q) v[8 * c + q] = (float)geo[c][q] * r[c];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = 24 + 3 * m + c;
            const float p = (float)col[m] * r[c];
            if (i < 32) v[i] = p;
            else e[i - 32] = p;
        }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int half = 16 >> k, o = 32 >> k;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < half) {
                const float keep = up ? v[i + half] : v[i];
                const float send = up ? v[i] : v[i + half];
                v[i] = keep + __shfl_xor(send, o, 64);
            }
        }
    }
    v[0] += __shfl_xor(v[0], 1, 64);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 6; ++k) e[i] += __shfl_xor(e[i], 32 >> k, 64);
    if ((lane & 1) == 0) red[wave][(lane >> 1) & 31] = v[0];
    if (lane < 4) red[wave][32 + lane] = e[lane];
    __syncthreads();
    if (threadIdx.x < kJtrVals)
        out[threadIdx.x] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// Feature row of product v of handle h (cubic: rows as store_handle_rows; straight: geometry q < 4,
// the colour products of m = 0, 1 (wd) and m = 2, 3 (wc) go to the one constant-jump row) and its
// channel; -1 for a product that has no row (straight geometry q >= 4).
__host__ __device__ inline int64_t jtr_row(int model, int v, int h, int64_t gp, int* c)
{
    if (v < 24) {
        const int cc = v / 8, q = v % 8;
        *c = cc;
        if (model == 1) return q < 4 ? (int64_t)cc * gp + 4 * h + q : -1;
        return (int64_t)cc * gp + 8 * h + q;
    }
    const int m = (v - 24) / 3;
    *c = (v - 24) % 3;
    if (model == 1) return 3 * gp + 2 * h + (m >> 1);
    return 3 * gp + 4 * h + m;
}

// R[row][c] += sum over the tile's blocks of rpart[block][h][v] (float64, fixed order): a block per
// handle h, lane v of each wavefront a product, the 4 wavefronts splitting the blocks (b = w mod 4)
// and adding their partial sums in a fixed order through LDS.  For straight handles the two
// products that share a row are added by the lane of the first (m even) of them.
__global__ void __launch_bounds__(256) k_jtr_handles(const float* __restrict__ rpart, int nblocks, int H, int model,
                                                     int64_t gp, double* __restrict__ R)
{
    __shared__ double part[4][kJtrVals];
    const int h = blockIdx.x;
    const int v = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc = 0.0;
    if (v < kJtrVals)
        for (int b = wave; b < nblocks; b += 4) acc += (double)rpart[((size_t)b * H + h) * kJtrVals + v];
    if (v < kJtrVals) part[wave][v] = acc;
    __syncthreads();
    if (wave != 0 || v >= kJtrVals) return;
    int c;
    const int64_t row = jtr_row(model, v, h, gp, &c);
    if (row < 0) return;
    const bool pair = model == 1 && v >= 24 && (((v - 24) / 3) & 1) == 0;   // m even: also take m + 1
    if (model == 1 && v >= 24 && !pair) return;
    double tot = (part[0][v] + part[1][v]) + (part[2][v] + part[3][v]);
    if (pair) tot += (part[0][v + 3] + part[1][v + 3]) + (part[2][v + 3] + part[3][v + 3]);
    R[row * 3 + c] += tot;
}

// J^T r of one flagged sample's handle rows (the inline kernel): float64 atomics into R.
template <class A>
__device__ inline void handle_jtr_atomic(int model, int h, int64_t gp, const A (&geo)[3][8], const A (&col)[4],
                                         const float* rr, double* __restrict__ R)
{
#pragma unroll
    for (int v = 0; v < kJtrVals; ++v) {
        int c;
        const int64_t row = jtr_row(model, v, h, gp, &c);
        if (row < 0) continue;
        const double f = v < 24 ? (double)geo[v / 8][v % 8] : (double)col[(v - 24) / 3];
        atomicAdd(R + row * 3 + c, f * (double)rr[c]);
    }
}

// Handle features of one point and one handle (thread per (point, handle)):
//   rows c*8H + 8h + 2j + d : d f_c / d P_{h,j,d}      (c = 0..2, j = 0..3, d = x, y)
//   rows 24H + 4h + m       : coefficient of wd0, wd1, wc0, wc1 of handle h (any channel)
// The vertex gradient of the polyline is chained to control points with the
// Bernstein weights of the vertex parameter t_k = k/S (straight handles: to the end
// points with 1 - t_k, t_k; rows as store_handle_rows).
//
// Float64 (Mixed = false), or mixed with near pairs inline in float64: the latter
// runs only for the samples flagged in `only` (their near-pair list overflowed).
template <bool Mixed, class OutT>
__global__ void __launch_bounds__(256) k_features(const double* __restrict__ x, int64_t npts,
                                                  const double* __restrict__ seg64, const float* __restrict__ seg32,
                                                  int H, int S, int model, int64_t gp, double eps2, float eps2f,
                                                  float near2, const uint8_t* __restrict__ only,
                                                  OutT* __restrict__ Xt, uint16_t* __restrict__ Xlo, int64_t ld,
                                                  const float* __restrict__ rr = nullptr, double* __restrict__ R = nullptr)
{
    using A = typename std::conditional<Mixed, float, double>::type;
    const int h = blockIdx.y;
    // all points: one per thread; only the flagged ones (only != null): a few blocks stride
    // over the tile, so that a tile with few or no flagged samples costs a small launch
    const int64_t stride = only ? (int64_t)gridDim.x * blockDim.x : npts;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npts; t += stride) {
        if (only && !only[t]) continue;
        const double X = x[2 * t], Y = x[2 * t + 1];
        const float Xf = (float)X, Yf = (float)Y;
        A geo[3][8];
        A col[4];
        A pv[3][2];   // gradient carried to the next vertex (from the previous segment's b end)
        for (int c = 0; c < 3; ++c) {
            for (int q = 0; q < 8; ++q) geo[c][q] = A(0);
            pv[c][0] = pv[c][1] = A(0);
        }
        for (int q = 0; q < 4; ++q) col[q] = A(0);
        for (int j = 0; j <= S; ++j) {
            // contributions to vertex j: a end of segment j (if j < S) + b end of segment j-1 (carried)
            A va[3][2] = {{A(0), A(0)}, {A(0), A(0)}, {A(0), A(0)}};
            A vb[3][2] = {{A(0), A(0)}, {A(0), A(0)}, {A(0), A(0)}};
            if (j < S) {
                const int k = h * S + j;
                const double* s64 = seg64 + (size_t)k * kSegStride;
                const double ta = (double)j / (double)S, tb = (double)(j + 1) / (double)S;
                Moments<A> m{A(0), A(0), A(0), A(0)};
                bool done = false;
                if (s64[6] == 0.0) done = true;                  // degenerate segment: nothing
                if (!done && Mixed) {
                    const float* s32 = seg32 + (size_t)k * kSegStride;
                    const SegGeom<float> gf = load_geom(s32);
                    if (!near_segment(gf.ax, gf.ay, gf.bx, gf.by, gf.L2, Xf, Yf, near2)) {
                        const PairState<float> st = pair_forward<float, DevF32, false>(gf, Xf, Yf, eps2f);
                        const Moments<float> mf = pair_moments(gf, st);
                        m = Moments<A>{(A)mf.da, (A)mf.db, (A)mf.sa, (A)mf.sb};
                        for (int c = 0; c < 3; ++c) {
                            const Grad4<float> gr = pair_backward(gf, st, eps2f, s32[kWdA + c], s32[kWdB + c],
                                                                  s32[kWcA + c], s32[kWcB + c]);
                            va[c][0] = gr.ax; va[c][1] = gr.ay; vb[c][0] = gr.bx; vb[c][1] = gr.by;
                        }
                        done = true;
                    }
                }
                if (!done) {
                    const SegGeom<double> g = load_geom(s64);
                    const PairState<double> st = pair_forward<double, DevF64, true>(g, X, Y, eps2);
                    const Moments<double> md = pair_moments(g, st);
                    m = Moments<A>{(A)md.da, (A)md.db, (A)md.sa, (A)md.sb};
                    for (int c = 0; c < 3; ++c) {
                        const Grad4<double> gr = pair_backward(g, st, eps2, s64[kWdA + c], s64[kWdB + c], s64[kWcA + c],
                                                               s64[kWcB + c]);
                        va[c][0] = (A)gr.ax; va[c][1] = (A)gr.ay; vb[c][0] = (A)gr.bx; vb[c][1] = (A)gr.by;
                    }
                }
                col[0] += m.da * (A)(1.0 - ta) + m.db * (A)(1.0 - tb);
                col[1] += m.da * (A)ta + m.db * (A)tb;
                col[2] += m.sa * (A)(1.0 - ta) + m.sb * (A)(1.0 - tb);
                col[3] += m.sa * (A)ta + m.sb * (A)tb;
            }
            double B[4];
            vertex_weights(model, (double)j / (double)S, B);
            for (int c = 0; c < 3; ++c) {
                const A gx = va[c][0] + pv[c][0], gy = va[c][1] + pv[c][1];
                for (int q = 0; q < 4; ++q) {
                    geo[c][2 * q] += (A)B[q] * gx;
                    geo[c][2 * q + 1] += (A)B[q] * gy;
                }
                pv[c][0] = vb[c][0];
                pv[c][1] = vb[c][1];
            }
        }
        store_handle_rows(model, Xt, Xlo, H, h, t, ld, gp, geo, col);
        if (rr) handle_jtr_atomic(model, h, gp, geo, col, rr + 3 * t, R);     // J^T r of a flagged sample
    }
}

// One (sample, segment) pair of the mixed feature kernel: its moments and its end-point gradient
// matrix, chained into col and geo (V: the vertex table at the segment's a end).  With Test the
// values are masked to zero where the pair is near or the segment degenerate (every lane takes the
// same path, with no branch-local copies of the loop-carried sums).  Without Test (a group of
// segments whose box is out of the wavefront's reach: every pair far) a degenerate segment still
// gives zeros: its float32 record is a far point with v = 0 and kd = ks = 0.
__device__ __forceinline__ void feature_pair(const float* __restrict__ s32, const float* __restrict__ V, float Xf,
                                             float Yf, float eps2f, float near2, bool Test, float (&geo)[3][8],
                                             float (&col)[4], float (&pv)[3][2])
{
    const SegGeom<float> gf = load_geom(s32);
    const PairState<float> st = pair_forward<float, DevF32, false>(gf, Xf, Yf, eps2f);
    Moments<float> m = pair_moments(gf, st);
    // the end-point gradient is linear in the channel's end densities: one matrix per pair serves
    // the three channels
    GradMatrix<float> G = pair_grad_matrix(gf, st, eps2f);
    if (Test) {
        const bool far = gf.L2 != 0.0f && !near_segment(gf.ax, gf.ay, gf.bx, gf.by, gf.L2, Xf, Yf, near2);
        m.da = far ? m.da : 0.f;
        m.db = far ? m.db : 0.f;
        m.sa = far ? m.sa : 0.f;
        m.sb = far ? m.sb : 0.f;
        for (int r = 0; r < 4; ++r)
            for (int k = 0; k < 4; ++k) G.g[r][k] = far ? G.g[r][k] : 0.f;
    }
    const float ta = V[4], sa_ = V[5];
    const float tb = V[12], sb_ = V[13];
    col[0] += m.da * sa_ + m.db * sb_;
    col[1] += m.da * ta + m.db * tb;
    col[2] += m.sa * sa_ + m.sb * sb_;
    col[3] += m.sa * ta + m.sb * tb;
    for (int c = 0; c < 3; ++c) {
        const Grad4<float> gr = grad_apply(G, s32[kWdA + c], s32[kWdB + c], s32[kWcA + c], s32[kWcB + c]);
        const float gx = gr.ax + pv[c][0], gy = gr.ay + pv[c][1];
        for (int q = 0; q < 4; ++q) {
            geo[c][2 * q] += V[q] * gx;
            geo[c][2 * q + 1] += V[q] * gy;
        }
        pv[c][0] = gr.bx;
        pv[c][1] = gr.by;
    }
}

constexpr int kFeatVals = 28;   // chained contributions of one pair: geo[3][8] and col[4]

// Mixed handle features: float32 pairs, near pairs skipped (same predicate as the
// classification), then the float64 contributions of this sample's listed near pairs
// with this handle's segments are added.  runs (k_near_runs) gives the range of the
// handle's entries in the wavefront's slice; the wavefront walks it with uniform
// (scalar) loads and each lane takes the entries of its own sample.  x points at the
// tile's first sample, whose global index is t0 (a multiple of 64); flagged samples
// are rewritten afterwards by k_features<true>.
template <class OutT>
__global__ void __launch_bounds__(256, 6) k_features_far(const double* __restrict__ x, int64_t npts, int64_t t0,
                                                      const float* __restrict__ seg32, int H, int S, int model,
                                                      int64_t gp, float eps2f,
                                                      float near2, const NearPair* __restrict__ list, int slots,
                                                      const int2* __restrict__ runs,
                                                      const uint8_t* __restrict__ flag, const float* __restrict__ corr,
                                                      const float* __restrict__ vtab, const float4* __restrict__ box,
                                                      OutT* __restrict__ Xt, uint16_t* __restrict__ Xlo, int64_t ld,
                                                      const float* __restrict__ rr, float* __restrict__ rpart)
{
    __shared__ float jtr_red[4][kJtrVals];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int h = blockIdx.y;
    const bool valid = t < npts;
    float geo[3][8];
    float col[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < 3; ++c)
        for (int q = 0; q < 8; ++q) geo[c][q] = 0.f;
    bool take = false;
    // the wavefront's sample box (every lane takes part in the reductions, so before the branch on
    // valid): groups of segments farther than their near radius take the loop without near tests
    // (handles of few segments keep every near test: there a box lookup per pair and the box itself
    // would cost more than they save; paper-native handles, S = 1: +0.25 ms per LM step)
    const bool cull = S >= 8;
    const float Xv = valid ? (float)x[2 * t] : 0.f, Yv = valid ? (float)x[2 * t + 1] : 0.f;
    float wx0 = 0.f, wx1 = 0.f, wy0 = 0.f, wy1 = 0.f;
    if (cull) {
        wx0 = uniform_f32(wave_min(valid ? Xv : INFINITY));
        wx1 = uniform_f32(wave_max(valid ? Xv : -INFINITY));
        wy0 = uniform_f32(wave_min(valid ? Yv : INFINITY));
        wy1 = uniform_f32(wave_max(valid ? Yv : -INFINITY));
    }
    if (valid) {
        const float Xf = Xv, Yf = Yv;
        // pv[c]: the b-end gradient of segment j - 1, carried to vertex j; each channel's a-end
        // gradient is chained into geo as soon as it is formed, so that only one channel's
        // end-point gradients are live at a time
        float pv[3][2];
        for (int c = 0; c < 3; ++c) pv[c][0] = pv[c][1] = 0.f;
        // test: whether the pairs need the near test (false once the segment's group of kBoxGroup
        // segments is out of the wavefront's reach; wave-uniform, looked up at each group's start)
        bool test = true;
#pragma unroll 1
        for (int j = 0; j < S; ++j) {
            const int k = h * S + j;
            if (cull && (j == 0 || k % kBoxGroup == 0)) test = !box_culled(box, k / kBoxGroup, wx0, wy0, wx1, wy1);
            feature_pair(seg32 + (size_t)k * kSegStride, vtab + 8 * j, Xf, Yf, eps2f, near2, test, geo, col, pv);
        }
        {
            const float* B = vtab + 8 * S;                  // the last vertex takes the carried b end
            for (int c = 0; c < 3; ++c)
                for (int q = 0; q < 4; ++q) {
                    geo[c][2 * q] += B[q] * pv[c][0];
                    geo[c][2 * q + 1] += B[q] * pv[c][1];
                }
        }
        const int64_t i = t0 + t;
        take = !flag[i];
        // the wavefront's index within the tile (the same for all its lanes, as t0 is a multiple of 64)
        const int wl = __builtin_amdgcn_readfirstlane((int)(t >> 6));
        const int2 run = runs[(size_t)wl * H + h];
        const NearPair* sl = list + ((t0 >> 6) + wl) * (int64_t)slots;
        const float* cw = corr + (size_t)wl * slots * kFeatVals;
        for (int e = run.x; e < run.y; ++e) {
            const NearPair p = sl[e];
            if (!take || p.sample != (int32_t)i) continue;
            const float* cr = cw + (size_t)e * kFeatVals;
            for (int c = 0; c < 3; ++c)
                for (int q = 0; q < 8; ++q) geo[c][q] += cr[8 * c + q];
            for (int q = 0; q < 4; ++q) col[q] += cr[24 + q];
        }
        store_handle_rows(model, Xt, Xlo, H, h, t, ld, gp, geo, col);
    }
    // with rr (the tile's residuals) the block also forms its part of J^T r over its samples and
    // this handle's rows; every thread joins the reduction (samples past the tile and flagged
    // samples, whose rows and J^T r the inline kernel rewrites, with zero residual)
    if (rr) {
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if (valid && take) {
            r0 = rr[3 * t];
            r1 = rr[3 * t + 1];
            r2 = rr[3 * t + 2];
        }
        handle_jtr_block(geo, col, r0, r1, r2, jtr_red, rpart + ((size_t)blockIdx.x * H + h) * kJtrVals);
    }
}

// Ranges of each handle's entries in the near-pair slices of a tile's wavefronts
// w0 .. w0 + nw - 1 (entries sorted by segment; element entries come last):
// runs[(w - w0) H + h] = [first entry with seg >= h S, first entry with seg >= (h + 1) S).
__global__ void __launch_bounds__(256) k_near_runs(const NearPair* __restrict__ list, int slots,
                                                   const int* __restrict__ wave_count, int64_t w0, int64_t nw, int H,
                                                   int S, int2* __restrict__ runs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nw * H) return;
    const int64_t w = w0 + t / H;
    const int h = (int)(t % H);
    const NearPair* sl = list + w * slots;
    const int cnt = wave_count[w];
    int b[2];
    for (int k = 0; k < 2; ++k) {
        const int key = (h + k) * S;
        int lo = 0, hi = cnt;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sl[mid].seg < key) lo = mid + 1;
            else hi = mid;
        }
        b[k] = lo;
    }
    runs[t] = make_int2(b[0], b[1]);
}

// Zero the samples [n, n rounded up to 32) of every row of a blocked split-bfloat16
// tile: the Gram kernel reads whole 32-sample blocks.
__global__ void k_zero_tail(uint16_t* __restrict__ Xh, uint16_t* __restrict__ Xl, int64_t W, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tail = ((n + 31) & ~(int64_t)31) - n;
    if (i >= W * tail) return;
    const int64_t f = i / tail, t = n + i % tail;
    const size_t e = (size_t)(t >> 5) * (size_t)(W << 5) + (size_t)(f << 5) + (size_t)(t & 31);
    Xh[e] = 0;
    Xl[e] = 0;
}

// Vertex table of the float32 feature kernel: vtab[8 j + q] = the vertex weights at t_j
// (vertex_weights), vtab[8 j + 4] = t_j, vtab[8 j + 5] = 1 - t_j, t_j = j / S.
__global__ void k_vertex_table(int S, int model, float* __restrict__ vtab)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > S) return;
    const double t = (double)j / (double)S;
    double B[4];
    vertex_weights(model, t, B);
    for (int q = 0; q < 4; ++q) vtab[8 * j + q] = (float)B[q];
    vtab[8 * j + 4] = (float)t;
    vtab[8 * j + 5] = (float)(1.0 - t);
    vtab[8 * j + 6] = vtab[8 * j + 7] = 0.0f;
}

// Float64 contributions of one listed near (sample, segment) pair to its handle's
// features: o[28] = geo[3][8] and col[4] as in store_handle_rows (geometry already
// chained with the vertex weights); k_features_near stores them at the pair's slot
// of the tile (wavefronts w0 .. w0 + nw - 1), corr[slot][28].
__device__ inline void features_near_pair(const NearPair p, const double* __restrict__ x,
                                          const double* __restrict__ seg64, int S, int model, double eps2,
                                          float* __restrict__ o)
{
    const double X = x[2 * (int64_t)p.sample], Y = x[2 * (int64_t)p.sample + 1];
    const double* s64 = seg64 + (size_t)p.seg * kSegStride;
    const SegGeom<double> g = load_geom(s64);
    const int j = p.seg % S;
    const double ta = (double)j / (double)S, tb = (double)(j + 1) / (double)S;
    double Ba[4], Bb[4];
    vertex_weights(model, ta, Ba);
    vertex_weights(model, tb, Bb);
    const PairState<double> st = pair_forward<double, DevF64, true>(g, X, Y, eps2);
    const Moments<double> m = pair_moments(g, st);
    for (int c = 0; c < 3; ++c) {
        const Grad4<double> gr = pair_backward(g, st, eps2, s64[kWdA + c], s64[kWdB + c], s64[kWcA + c], s64[kWcB + c]);
        for (int q = 0; q < 4; ++q) {
            o[8 * c + 2 * q] = (float)(Ba[q] * gr.ax + Bb[q] * gr.bx);
            o[8 * c + 2 * q + 1] = (float)(Ba[q] * gr.ay + Bb[q] * gr.by);
        }
    }
    o[24] = (float)(m.da * (1.0 - ta) + m.db * (1.0 - tb));
    o[25] = (float)(m.da * ta + m.db * tb);
    o[26] = (float)(m.sa * (1.0 - ta) + m.sb * (1.0 - tb));
    o[27] = (float)(m.sa * ta + m.sb * tb);
}

// block per wavefront slice w0 + blockIdx.x, its threads looping over the slice's entries
__global__ void __launch_bounds__(256) k_features_near(const NearPair* __restrict__ list, int slots,
                                                       const int* __restrict__ wave_count,
                                                       const uint8_t* __restrict__ flag, int64_t w0,
                                                       const double* __restrict__ x, const double* __restrict__ seg64,
                                                       int K, int S, int model, double eps2,
                                                       float* __restrict__ corr)
{
    const int64_t w = w0 + blockIdx.x;
    const int cnt = wave_count[w];
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const NearPair p = list[w * slots + e];
        if (p.seg >= K || flag[p.sample]) continue;
        features_near_pair(p, x, seg64, S, model, eps2, corr + ((size_t)blockIdx.x * slots + e) * kFeatVals);
    }
}

// beta rows: Xt[row0 + j][t] = beta_j(x_t); thread per point, each block row of the grid a
// run of kBetaRun elements (element data by uniform loads), so that a launch has few, long
// blocks rather than one short block per element.
constexpr int kBetaRun = 32;
template <bool Mixed, class OutT>
__global__ void __launch_bounds__(256) k_beta_rows(const double* __restrict__ x, int64_t npts,
                                                   const double* __restrict__ el64, const float* __restrict__ el32,
                                                   int M, float near2, OutT* __restrict__ Xt, uint16_t* __restrict__ Xlo,
                                                   int64_t ld, int64_t row0)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    const double X = x[2 * t], Y = x[2 * t + 1];
    const float Xf = (float)X, Yf = (float)Y;
    const int j0 = blockIdx.y * kBetaRun, j1 = j0 + kBetaRun < M ? j0 + kBetaRun : M;
    for (int j = j0; j < j1; ++j) {
        const double* e = el64 + (size_t)j * kElemStride;
        double b;
        if (Mixed) {
            const float* f = el32 + (size_t)j * kElemStride;
            if (near_element(f[0], f[1], f[2], f[3], Xf, Yf, near2))
                b = element_beta<double, DevF64>(e[0], e[1], e[2], e[3], X, Y);
            else
                b = (double)element_beta<float, DevF32>(f[0], f[1], f[2], f[3], Xf, Yf);
        } else {
            b = element_beta<double, DevF64>(e[0], e[1], e[2], e[3], X, Y);
        }
        Store<OutT>::put(Xt, Xlo, row0 + j, t, ld, b);
    }
}

// beta rows into a split-bfloat16 tile in the blocked layout [t / 32][row][t % 32]: the block
// computes its 256 samples x kBetaRunBlocked elements into LDS, then writes whole runs: the
// kBetaRunBlocked rows of one 32-sample block are one contiguous 1 KiB run (hi, and another for
// lo), written with 16-byte stores.  (Written lane by lane, each store instruction of a
// wavefront covered two 64-byte halves of cache lines; beside the Gram that took 1.5-2.4 ms
// per 32,768-sample tile against 0.05 ms alone.)  LDS rows hold their 8-sample chunks in
// XOR-swizzled order (chunk q of row r at q ^ (r & 7)), so that the 16-byte reads of 16 rows
// at one chunk fall in different banks; 16 KiB, so that a block fits beside a Gram block.
// Samples past npts in a written block are zeros.
constexpr int kBetaRunBlocked = 16;
constexpr int kBetaJtrVals = 3 * kBetaRunBlocked;   // 16 beta rows x 3 residual channels

// J^T r of a block's beta rows: value 3 jj + c = sum over the block's 256 samples of
// beta[jj] r_c, in float32.  Values 0..31 by recursive halving over the wavefront (lane l ends
// with value (l >> 1) & 31 summed over its lane pair, the offset-1 step completes it), values
// 32..47 likewise with four halving steps (lane l: value 32 + ((l >> 2) & 15)) and two
// butterflies; the 4 wavefronts are added through LDS and values 0 .. nv-1 written to out.
__device__ inline void beta_jtr_block(const float (&bv)[kBetaRunBlocked], float r0, float r1, float r2,
                                      float (*red)[kBetaJtrVals], float* __restrict__ out, int nv)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float r[3] = {r0, r1, r2};
    float v[32], e[16];
#pragma unroll
    for (int i = 0; i < kBetaJtrVals; ++i) {
        const float p = bv[i / 3] * r[i % 3];
        if (i < 32) v[i] = p;
        else e[i - 32] = p;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int half = 16 >> k, o = 32 >> k;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < half) {
                const float keep = up ? v[i + half] : v[i];
                const float send = up ? v[i] : v[i + half];
                v[i] = keep + __shfl_xor(send, o, 64);
            }
        }
    }
    v[0] += __shfl_xor(v[0], 1, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int half = 8 >> k, o = 32 >> k;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < half) {
                const float keep = up ? e[i + half] : e[i];
                const float send = up ? e[i] : e[i + half];
                e[i] = keep + __shfl_xor(send, o, 64);
            }
        }
    }
    e[0] += __shfl_xor(e[0], 2, 64);
    e[0] += __shfl_xor(e[0], 1, 64);
    if ((lane & 1) == 0) red[wave][(lane >> 1) & 31] = v[0];
    if ((lane & 3) == 0) red[wave][32 + ((lane >> 2) & 15)] = e[0];
    __syncthreads();
    if (threadIdx.x < nv)
        out[threadIdx.x] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// R[row0 + j][c] += sum over the tile's sample blocks b of bpart[b][j][c] (float64, fixed order):
// a thread per (j, c).
__global__ void __launch_bounds__(256) k_jtr_beta(const float* __restrict__ bpart, int nblocks, int M, int64_t row0,
                                                  double* __restrict__ R)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * M) return;
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) acc += (double)bpart[(size_t)b * 3 * M + i];
    R[row0 * 3 + i] += acc;
}
template <bool Mixed>
__global__ void __launch_bounds__(256) k_beta_rows_blocked(const double* __restrict__ x, int64_t npts,
                                                           const double* __restrict__ el64,
                                                           const float* __restrict__ el32, int M, float near2,
                                                           uint16_t* __restrict__ Xh, uint16_t* __restrict__ Xl,
                                                           int64_t ld, int64_t row0, const float* __restrict__ rr,
                                                           float* __restrict__ bpart)
{
    constexpr int R = kBetaRunBlocked;
    __shared__ __attribute__((aligned(16))) uint16_t sh[2][R][256];
    __shared__ float jtr_red[4][kBetaJtrVals];
    const int64_t t0 = (int64_t)blockIdx.x * 256;
    const int64_t t = t0 + threadIdx.x;
    const int j0 = blockIdx.y * R, nj = M - j0 < R ? M - j0 : R;
    const bool live = t < npts;
    const double X = live ? x[2 * t] : 0.0, Y = live ? x[2 * t + 1] : 0.0;
    const float Xf = (float)X, Yf = (float)Y;
    float bv[R];                                      // this sample's beta values (the J^T r products)
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        bv[jj] = 0.0f;
        if (jj >= nj) continue;
        const int j = j0 + jj;
        const double* e = el64 + (size_t)j * kElemStride;
        double b = 0.0;
        if (live) {
            if (Mixed) {
                const float* f = el32 + (size_t)j * kElemStride;
                if (near_element(f[0], f[1], f[2], f[3], Xf, Yf, near2))
                    b = element_beta<double, DevF64>(e[0], e[1], e[2], e[3], X, Y);
                else
                    b = (double)element_beta<float, DevF32>(f[0], f[1], f[2], f[3], Xf, Yf);
            } else {
                b = element_beta<double, DevF64>(e[0], e[1], e[2], e[3], X, Y);
            }
        }
        const float v = (float)b;
        bv[jj] = v;
        const uint16_t h = bf16_bits(v);
        const int col = threadIdx.x ^ ((jj & 7) << 3);
        sh[0][jj][col] = h;
        sh[1][jj][col] = bf16_bits(v - bf16_value(h));
    }
    __syncthreads();
    // hi and lo x 8 sample blocks x R rows x 4 chunks of 8 samples; a wavefront writes the R rows of
    // one sample block (R x 64 bytes, contiguous)
    constexpr int per = 8 * R * 4;
    for (int e = threadIdx.x; e < 2 * per; e += 256) {
        const int which = e / per, r = e % per;
        const int sb = r / (R * 4), jj = (r >> 2) % R, c = r & 3;
        // sample blocks wholly past npts are not written: the tile holds npts rounded up to 32
        // (64) samples, which need not reach the block's 256
        if (jj >= nj || t0 + sb * 32 >= npts) continue;
        const int q = (sb * 4 + c) ^ (jj & 7);          // swizzled 8-sample chunk of this row
        const uint4 v = *reinterpret_cast<const uint4*>(&sh[which][jj][q * 8]);
        uint16_t* dst = (which ? Xl : Xh) + (size_t)((t0 >> 5) + sb) * (size_t)(ld << 5) +
                        (size_t)((row0 + j0 + jj) << 5) + c * 8;
        *reinterpret_cast<uint4*>(dst) = v;
    }
    // with residuals (mixed J^T r): the block's sums of beta r over its samples, rows j0 .. j0+nj-1
    if (rr) {
        const float r0 = live ? rr[3 * t] : 0.0f, r1 = live ? rr[3 * t + 1] : 0.0f, r2 = live ? rr[3 * t + 2] : 0.0f;
        beta_jtr_block(bv, r0, r1, r2, jtr_red, bpart + ((size_t)blockIdx.x * M + j0) * 3, 3 * nj);
    }
}

__global__ void k_gauss_points(int M, const double* __restrict__ eg, double* __restrict__ gx)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * M) return;
    const int i = t / 3, q = t % 3;
    double ax, ay, bx, by;
    load_element(eg, i, ax, ay, bx, by);
    const double node = q == 0 ? -kGaussNode : (q == 1 ? 0.0 : kGaussNode);
    gx[2 * t] = 0.5 * (ax + bx) + node * 0.5 * (bx - ax);
    gx[2 * t + 1] = 0.5 * (ay + by) + node * 0.5 * (by - ay);
}

// dF[i][f] = sum_q w_q |G_i|/2 Xg[f][3i + q]
__global__ void k_boundary_features(const double* __restrict__ Xg, int nf, int M, const double* __restrict__ eg,
                                    double* __restrict__ dF)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (f >= nf) return;
    double ax, ay, bx, by;
    load_element(eg, i, ax, ay, bx, by);
    const double half = 0.5 * sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
    const double* r = Xg + (size_t)f * 3 * M + 3 * i;
    dF[(size_t)i * nf + f] = half * (kGaussW0 * r[0] + kGaussW1 * r[1] + kGaussW0 * r[2]);
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

template <class T>
__global__ void k_to_f64(const T* __restrict__ in, int64_t n, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

// Feature layout of the normal equations: G geometry rows per handle and channel, C
// channel-shared colour rows per handle, H handles (the rows of Xt are
// [g_0 (GH) | g_1 | g_2 | e (CH) | beta (M)]).
struct Layout {
    int G, C, H;
    int64_t Gp;     // rows of one channel's geometry block in Xt (G H rounded up to the Gram tile)
    __host__ __device__ int64_t geo() const { return (int64_t)G * H; }
    __host__ __device__ int64_t handle_rows() const { return 3 * Gp + (int64_t)C * H; }
    __host__ __device__ int compact() const { return (G + C) * H; }
    __host__ __device__ int params() const { return G + 3 * C; }
    // row of Xt of compact index a of channel c ([g_c | e | beta])
    __host__ __device__ int64_t row(int a, int c) const
    {
        return a < geo() ? (int64_t)c * Gp + a : 3 * Gp + (a - geo());
    }
};

// Channel-c augmented Gram in compact order [g_c (GH) | e (CH) | beta (M)],
// symmetric fill from the upper triangle of G.  The compact-to-row map is increasing, so
// entry (a, b) comes from G[row(a)][row(b)] for a <= b and from G[row(b)][row(a)] below the
// diagonal.  A block owns a 32 x 32 tile of (a, b); a tile below the diagonal reads its
// mirror tile along a (coalesced) and transposes it through LDS.
__global__ void __launch_bounds__(256) k_gather_gram(const double* __restrict__ G, int64_t W, Layout L, int c, int Wc,
                                                     double* __restrict__ Gc)
{
    __shared__ double T[32][33];
    const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    if (b0 + 31 < a0) {                  // wholly below the diagonal: T[b][a] = G[row(b)][row(a)]
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int bb = b0 + ty + 8 * k, aa = a0 + tx;
            if (aa < Wc) T[ty + 8 * k][tx] = G[(size_t)L.row(bb, c) * W + L.row(aa, c)];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int a = a0 + ty + 8 * k, b = b0 + tx;
            if (a < Wc) Gc[(size_t)a * Wc + b] = T[tx][ty + 8 * k];
        }
        return;
    }
    const int b = b0 + tx;
    if (b >= Wc) return;
    const int64_t ib = L.row(b, c);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = a0 + ty + 8 * k;
        if (a >= Wc) break;
        const int64_t ia = L.row(a, c);
        // the upper triangle holds every needed entry (diagonal tiles are computed whole)
        Gc[(size_t)a * Wc + b] = ia <= ib ? G[(size_t)ia * W + ib] : G[(size_t)ib * W + ia];
    }
}

// Zc[i][a] = Z[i][row(a)] for the handle part of the compact order (a < (G + C)H)
__global__ void k_gather_z(const double* __restrict__ Z, Layout L, int M, int c, double* __restrict__ Zc)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int n = L.compact();
    if (a >= n) return;
    Zc[(size_t)i * n + a] = Z[(size_t)i * L.handle_rows() + L.row(a, c)];
}

// theta column of compact index a of channel c: geometry (G per handle, shared by the
// channels) first, then the colour parameters, 3 per colour coefficient (RGB)
__device__ inline int64_t param_col(int a, Layout L, int c)
{
    if (a < L.geo()) return (int64_t)L.params() * (a / L.G) + (a % L.G);
    const int b = a - (int)L.geo();
    return (int64_t)L.params() * (b / L.C) + L.G + 3 * (b % L.C) + c;
}

// Every entry of J^T J from the three channels' blocks v_c(a, b) = Gc_c[a][b] + (S_c[a][b] +
// S_c[b][a]) (compact indices a, b < n12), written once (no fill, no read-modify-write):
// geometry x geometry entries are shared by the channels and take v_0 + v_1 + v_2; an entry
// with a colour parameter of channel c takes v_c; colour entries of two different channels
// are zero.  A block owns a 32 x 32 tile of (a, b) and reads S_c[b][a] through LDS, so both
// reads of S are coalesced; v_c(a, b) = v_c(b, a) bit for bit, so J^T J is exactly symmetric.
__global__ void __launch_bounds__(256) k_scatter_jtj(const double* __restrict__ Gc, int64_t gcs, int Wc,
                                                     const double* __restrict__ S, int64_t ss, Layout L, double s,
                                                     double* __restrict__ JtJ, int64_t P)
{
    __shared__ double T[3][32][33];
    const int n = L.compact();
    const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int bb = b0 + ty + 8 * k, aa = a0 + tx;   // S_c[bb][aa], aa contiguous
            T[c][ty + 8 * k][tx] = (bb < n && aa < n) ? S[c * ss + (size_t)bb * n + aa] : 0.0;
        }
    __syncthreads();
    const int b = b0 + tx;
    if (b >= n) return;
    const int64_t geo = L.geo();
    const int Q = L.params();
    const bool gb = b < geo;
    const int64_t cb = gb ? (int64_t)Q * (b / L.G) + b % L.G
                          : (int64_t)Q * ((b - geo) / L.C) + L.G + 3 * ((b - geo) % L.C);   // + channel
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = a0 + ty + 8 * k;
        if (a >= n) break;
        double v[3];
        for (int c = 0; c < 3; ++c)
            v[c] = Gc[c * gcs + (size_t)a * Wc + b] + (S[c * ss + (size_t)a * n + b] + T[c][tx][ty + 8 * k]);
        const bool ga = a < geo;
        const int64_t ca = ga ? (int64_t)Q * (a / L.G) + a % L.G
                              : (int64_t)Q * ((a - geo) / L.C) + L.G + 3 * ((a - geo) % L.C);
        if (ga && gb) {
            JtJ[ca * P + cb] = s * ((v[0] + v[1]) + v[2]);
        } else if (ga) {
            for (int c = 0; c < 3; ++c) JtJ[ca * P + cb + c] = s * v[c];
        } else if (gb) {
            for (int c = 0; c < 3; ++c) JtJ[(ca + c) * P + cb] = s * v[c];
        } else {
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) JtJ[(ca + c) * P + cb + d] = c == d ? s * v[c] : 0.0;
        }
    }
}

// Jtr[col(a)] += s * (R[row(a)][c] + sum_i Zc[i][a] R[beta row i][c]): a block per 64 compact
// indices a, its 4 wavefronts splitting the M beta rows (coalesced reads of Zc along a), the four
// partial sums added in a fixed order through LDS.
__global__ void __launch_bounds__(256) k_scatter_g(const double* __restrict__ R, const double* __restrict__ Zc,
                                                   Layout L, int M, int c, double s, double* __restrict__ Jtr)
{
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int a = blockIdx.x * 64 + lane;
    const int n = L.compact();
    const int64_t rb = L.handle_rows();
    double v = 0.0;
    if (a < n)
        for (int i = wave; i < M; i += 4) v += Zc[(size_t)i * n + a] * R[(rb + i) * 3 + c];
    part[wave][lane] = v;
    __syncthreads();
    if (wave == 0 && a < n)
        Jtr[param_col(a, L, c)] += s * (R[(size_t)L.row(a, c) * 3 + c] + ((part[0][lane] + part[1][lane]) +
                                                                            (part[2][lane] + part[3][lane])));
}

// J[n][c][p] assembly for the explicit Jacobian: features + beta . Z
__global__ void k_assemble_jacobian(const double* __restrict__ Xt, int64_t ld, const double* __restrict__ BZ, Layout L,
                                    int64_t npts, double* __restrict__ J)
{
    const int64_t t = blockIdx.y;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int Q = L.params();
    const int P = Q * L.H;
    const int64_t nf = L.handle_rows();
    if (p >= P || t >= npts) return;
    const int h = p / Q, q = p % Q;
    for (int c = 0; c < 3; ++c) {
        double v;
        if (q < L.G) {
            const int64_t f = (int64_t)c * L.Gp + (int64_t)L.G * h + q;
            v = Xt[(size_t)f * ld + t] + BZ[(size_t)t * nf + f];
        } else {
            const int m = (q - L.G) / 3, cc = (q - L.G) % 3;
            const int64_t f = 3 * L.Gp + (int64_t)L.C * h + m;
            v = cc == c ? Xt[(size_t)f * ld + t] + BZ[(size_t)t * nf + f] : 0.0;
        }
        J[((size_t)t * 3 + c) * P + p] = v;
    }
}

}  // namespace

int fill_f64(bem_ctx* ctx, double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return BEM_OK;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n, v);
    return check_launch(ctx, "fill");
}

constexpr int64_t kGeoAlign = 256;   // the split-BF16 Gram's tile
static Layout layout_of(const bem_ctx* ctx, int H)
{
    const int64_t gh = (int64_t)ctx->ngeo * H;
    return Layout{ctx->ngeo, ctx->ncol, H, (gh + kGeoAlign - 1) / kGeoAlign * kGeoAlign};
}

// Feature rows of npts points into Xt (ld: row stride of float64 / float32 tiles,
// row count of the blocked bfloat16 tile); rows 0..(3G + C)H - 1 handle
// features, the next M rows beta when with_beta.  OutT: double, float or uint16_t (bf16 hi, lo in Xlo).
// Mixed precision needs the near-pair list of the whole sample set (nl), the tile's
// first global sample index t0 (a multiple of 64), the global samples xg and a
// correction buffer of ceil(npts / 64) * nl->slots * 28 floats and a run table of
// ceil(npts / 64) * H entries.
// With rr (float residuals of the npts samples, mixed only) J^T r of the handle rows is added into
// R [W][3] as the features are formed (block partial sums in rpart, ceil(npts / 256) * H * 36 floats).
template <class OutT>
static int launch_features(bem_ctx* ctx, const double* x, int64_t npts, int H, bool mixed, bool with_beta, OutT* Xt,
                           uint16_t* Xlo, int64_t ld, hipStream_t s, const NearList* nl = nullptr, int64_t t0 = 0,
                           const double* xg = nullptr, float* corr = nullptr, const float* vtab = nullptr,
                           int2* runs = nullptr, const float* rr = nullptr, float* rpart = nullptr, double* R = nullptr,
                           const float4* box = nullptr, float* bpart = nullptr)
{
    if (npts == 0) return BEM_OK;
    const int S = ctx->opts.segs_per_handle;
    const int model = ctx->model;
    const double eps2 = ctx->opts.eps * ctx->opts.eps;
    const double nf = near_radius(ctx->opts.near_factor);
    const float near2 = (float)(nf * nf);
    const Layout L = layout_of(ctx, H);
    const int64_t beta_row0 = L.handle_rows();
    const int64_t gp = L.Gp;
    const dim3 grid(blocks_for(npts, 256), H);
    if (mixed && (!nl || !xg || !corr || !vtab || !runs || !box || (t0 & 63)))
        return set_error(ctx, BEM_EINVAL, "mixed features need the near-pair list (internal)");
    if (H > 0) {
        if (mixed) {
            const int64_t nw = (npts + 63) / 64;
            {
                ProfScope ps_(ctx, PT_NEAR, s);
                hipLaunchKernelGGL(k_features_near, dim3(nw), dim3(256), 0, s, nl->list, nl->slots, nl->count, nl->flag,
                                   t0 >> 6, xg, (const double*)ctx->seg64.ptr, H * S, S, model, eps2, corr);
                hipLaunchKernelGGL(k_near_runs, dim3(blocks_for(nw * H, 256)), dim3(256), 0, s, nl->list, nl->slots,
                                   nl->count, t0 >> 6, nw, H, S, runs);
            }
            ProfScope ps_(ctx, PT_FEATURES, s);
            hipLaunchKernelGGL((k_features_far<OutT>), grid, dim3(256), 0, s, x, npts, t0, (const float*)ctx->seg32.ptr,
                               H, S, model, gp, (float)eps2, near2, nl->list, nl->slots, (const int2*)runs, nl->flag, corr,
                               vtab, box, Xt, Xlo, ld, rr, rpart);
            if (rr)
                hipLaunchKernelGGL(k_jtr_handles, dim3(H), dim3(256), 0, s, (const float*)rpart, (int)grid.x, H, model,
                                   gp, R);
            const int fb = blocks_for(npts, 256) < 16 ? blocks_for(npts, 256) : 16;
            if (nl->overflowed)
                hipLaunchKernelGGL((k_features<true, OutT>), dim3(fb, H), dim3(256), 0, s, x, npts, (const double*)ctx->seg64.ptr,
                               (const float*)ctx->seg32.ptr, H, S, model, gp, eps2, (float)eps2, near2, nl->flag + t0,
                               Xt, Xlo, ld, rr, R);
        } else {
            ProfScope ps_(ctx, PT_FEATURES, s);
            hipLaunchKernelGGL((k_features<false, OutT>), grid, dim3(256), 0, s, x, npts, (const double*)ctx->seg64.ptr,
                               (const float*)ctx->seg32.ptr, H, S, model, gp, eps2, (float)eps2, near2,
                               (const uint8_t*)nullptr, Xt, Xlo, ld);
        }
    }
    if (H > 0 && gp > L.geo()) {
        const int64_t nz = 3 * (gp - L.geo()) * npts;
        hipLaunchKernelGGL((k_zero_pad<OutT>), dim3(blocks_for(nz, 256)), dim3(256), 0, s, Xt, Xlo, ld, gp, L.geo(), npts);
    }
    if (with_beta && std::is_same<OutT, uint16_t>::value) {
        const dim3 gb(blocks_for(npts, 256), blocks_for(ctx->M, kBetaRunBlocked));
        ProfScope ps_(ctx, PT_BETA_ROWS, s);
        // with residuals and a partials buffer (mixed J^T r) the beta rows' J^T r is summed here as well
        const float* brr = mixed && rr && bpart && R ? rr : nullptr;
        if (mixed)
            hipLaunchKernelGGL((k_beta_rows_blocked<true>), gb, dim3(256), 0, s, x, npts, (const double*)ctx->elem64.ptr,
                               (const float*)ctx->elem32.ptr, ctx->M, near2, (uint16_t*)Xt, Xlo, ld, beta_row0, brr,
                               bpart);
        else
            hipLaunchKernelGGL((k_beta_rows_blocked<false>), gb, dim3(256), 0, s, x, npts, (const double*)ctx->elem64.ptr,
                               (const float*)ctx->elem32.ptr, ctx->M, near2, (uint16_t*)Xt, Xlo, ld, beta_row0,
                               (const float*)nullptr, (float*)nullptr);
        if (brr)
            hipLaunchKernelGGL(k_jtr_beta, dim3(blocks_for(3 * (int64_t)ctx->M, 256)), dim3(256), 0, s, (const float*)bpart,
                               (int)gb.x, ctx->M, beta_row0, R);
    } else if (with_beta) {
        const dim3 gb(blocks_for(npts, 256), blocks_for(ctx->M, kBetaRun));
        if (mixed)
            {
                ProfScope ps_(ctx, PT_BETA_ROWS, s);
                hipLaunchKernelGGL((k_beta_rows<true, OutT>), gb, dim3(256), 0, s, x, npts, (const double*)ctx->elem64.ptr,
                                   (const float*)ctx->elem32.ptr, ctx->M, near2, Xt, Xlo, ld, beta_row0);
            }
        else
            {
                ProfScope ps_(ctx, PT_BETA_ROWS, s);
                hipLaunchKernelGGL((k_beta_rows<false, OutT>), gb, dim3(256), 0, s, x, npts, (const double*)ctx->elem64.ptr,
                                   (const float*)ctx->elem32.ptr, ctx->M, near2, Xt, Xlo, ld, beta_row0);
            }
    }
    return check_launch(ctx, "features");
}

// Z = A+ dF/dtheta in feature columns [M][(3G + C)H] -> ctx->tmp4 (also leaves Gauss features in tmp3)
int boundary_derivatives(bem_ctx* ctx, int H, hipStream_t s, double** Zout)
{
    int rc;
    const int M = ctx->M;
    const int nf = (int)layout_of(ctx, H).handle_rows();
    const size_t gxs = (size_t)3 * M * 2;
    if ((rc = ensure(ctx, ctx->tmp3, (gxs + (size_t)nf * 3 * M) * sizeof(double), s))) return rc;
    if ((rc = ensure(ctx, ctx->tmp4, (size_t)2 * M * nf * sizeof(double), s))) return rc;
    double* gx = (double*)ctx->tmp3.ptr;
    double* Xg = gx + gxs;
    double* dF = (double*)ctx->tmp4.ptr;
    double* Z = dF + (size_t)M * nf;
    hipLaunchKernelGGL(k_gauss_points, dim3(blocks_for(3 * M, 256)), dim3(256), 0, s, M, (const double*)ctx->egeo.ptr, gx);
    if ((rc = launch_features<double>(ctx, gx, 3 * (int64_t)M, H, false, false, Xg, nullptr, 3 * (int64_t)M, s))) return rc;
    hipLaunchKernelGGL(k_boundary_features, dim3(blocks_for(nf, 256), M), dim3(256), 0, s, Xg, nf, M,
                       (const double*)ctx->egeo.ptr, dF);
    if ((rc = check_launch(ctx, "boundary features"))) return rc;
    if ((rc = gemm_f64(ctx, M, nf, M, 1.0, (const double*)ctx->Apinv.ptr, M, false, dF, nf, false, 0.0, Z, nf, s,
                       nullptr, 0)))
        return rc;
    *Zout = Z;
    return BEM_OK;
}

static std::vector<int> gram_tiles(const Layout& L, int W, int ts)
{
    // upper-triangle ts x ts tiles, skipping pairs of tiles that lie inside two
    // different channels' geometry blocks (those products never enter J^T J)
    const int nt = (W + ts - 1) / ts;
    const int64_t g = L.Gp;
    auto region = [&](int t) {
        const int64_t lo = (int64_t)t * ts, hi = lo + ts - 1;
        if (lo >= 3 * g) return -1;                              // colour coefficients / beta: shared
        if (hi >= 3 * g) return -2;                              // straddles geometry and shared rows
        const int64_t c0 = lo / g, c1 = hi / g;
        return c0 == c1 ? (int)c0 : -2;
    };
    std::vector<int> t;
    for (int i = 0; i < nt; ++i)
        for (int j = i; j < nt; ++j) {
            const int ri = region(i), rj = region(j);
            if (ri >= 0 && rj >= 0 && ri != rj) continue;
            t.push_back(i);
            t.push_back(j);
        }
    return t;
}

// Work list of the MFMA Grams: (row tile, column tile, sample part) for every
// needed tile and part, part-major, then by super-tiles of 4 x 8 output tiles,
// then row and column.  Consecutive entries share operand panels (the Gram
// kernels give each XCD a contiguous run of entries).
static std::vector<int> gram_work(const std::vector<int>& tiles, int parts)
{
    const int nt = (int)tiles.size() / 2;
    std::vector<int> order(nt);
    for (int t = 0; t < nt; ++t) order[t] = t;
    auto key = [&](int t) {
        const int i = tiles[2 * t], j = tiles[2 * t + 1];
        return std::make_tuple(i / 4, j / 8, i, j);
    };
    std::sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<int> w;
    w.reserve((size_t)3 * nt * parts);
    for (int p = 0; p < parts; ++p)
        for (int t : order) {
            w.push_back(tiles[2 * t]);
            w.push_back(tiles[2 * t + 1]);
            w.push_back(p);
        }
    return w;
}

namespace {
// G[0] += G[1] + ... + G[parts - 1] (fixed order) over the ts x ts output tile of work entry
// blockIdx.x, rows split over gridDim.y blocks (blockDim.x = ts, a thread per column)
__global__ void __launch_bounds__(256) k_sum_parts(double* __restrict__ G, int parts, int64_t W,
                                                   const int* __restrict__ work, int ts)
{
    const int64_t c0 = (int64_t)work[3 * blockIdx.x + 1] * ts;
    const int64_t rt = (int64_t)work[3 * blockIdx.x] * ts;   // the tile's first row
    const int rows = (ts + gridDim.y - 1) / gridDim.y;
    const int64_t r0 = rt + (int64_t)blockIdx.y * rows;
    const int64_t r1 = rt + ts < r0 + rows ? rt + ts : r0 + rows;
    const int64_t c = c0 + threadIdx.x % ts;
    for (int64_t r = r0 + threadIdx.x / ts; r < r1; r += blockDim.x / ts) {
        if (r >= W || c >= W) continue;
        const size_t e = (size_t)r * W + c;
        double v = G[e];
        for (int p = 1; p < parts; ++p) v += G[(size_t)p * W * W + e];
        G[e] = v;
    }
}
}  // namespace

int run_jtj(bem_ctx* ctx, const double* theta, int H, const double* x, int64_t N, const void* resid, bool mixed,
            int gram, double* JtJ, double* Jtr, hipStream_t s, const NearList* pre, double norm)
{
    int rc;
    const int M = ctx->M;
    const Layout L = layout_of(ctx, H);
    const int64_t P = (int64_t)L.params() * H;
    const int64_t W = L.handle_rows() + M;
    const int n12 = L.compact();          // handle part of one channel's compact order
    const int Wc = n12 + M;
    if (H == 0) return BEM_OK;
    if ((rc = prepare_forward_tables(ctx, theta, H, s))) return rc;
    double* Z = nullptr;
    if ((rc = boundary_derivatives(ctx, H, s, &Z))) return rc;
    // sample tiles
    // sample tile: large for the float64 Gram; for the MFMA Grams small enough that the tile of
    // feature rows (W x T, 4 bytes per entry) stays resident in the last-level cache while every
    // output tile re-reads it
    // sample tile: 32,768 for the split-BF16 Gram (1 GB of blocked bf16 pairs at the LM workload; 3
    // parts of 10,944 samples per launch)
    // float64 Gram on MFMA (BEM_GRAM_FP64) or on the VALU (BEM_GRAM_FP64_VALU): float64 tiles
    const bool f64 = gram == BEM_GRAM_FP64 || gram == BEM_GRAM_FP64_VALU;
    int64_t T = ctx->opts.tile_rows > 0 ? ctx->opts.tile_rows
                                        : (gram == BEM_GRAM_FP32_MFMA ? 8192 : (f64 ? 16384 : 32768));
    const size_t elem = f64 ? 8 : 4;
    while (T > 1024 && (size_t)W * T * elem > ((size_t)3 << 30)) T /= 2;
    if (T > N) T = N > 0 ? N : 1;
    T = (T + 63) / 64 * 64;
    if (gram == BEM_GRAM_BF16X3_MFMA)
        while (T > 64 && W * T >= ((int64_t)1 << 31)) T = (T / 2 + 63) / 64 * 64;   // 32-bit offsets in the Gram
    // default tile size: a short last tile (at most a quarter of a tile) is spread over the others,
    // since it would cost a Gram launch of its own (the launch's partial-Gram traffic does not
    // shrink with the samples)
    if (ctx->opts.tile_rows <= 0 && N > T) {
        const int64_t nt = N / T, tail = N - nt * T;
        const int64_t T2 = ((N + nt - 1) / nt + 63) / 64 * 64;
        if (tail > 0 && tail <= T / 4 && (size_t)W * T2 * elem <= ((size_t)3 << 30) &&
            (gram != BEM_GRAM_BF16X3_MFMA || W * T2 < ((int64_t)1 << 31)))
            T = T2;
    }
    // MFMA Grams with several sample tiles: the Gram of tile t runs on a second stream while tile t+1's
    // feature rows are formed on the caller's stream (two tile buffers), so the VALU-bound feature
    // kernels and the MFMA-bound Gram share the chip.  Sharing slows a Gram launch by about a third
    // and short launches beside it several-fold (measured), so it pays only when the feature work
    // (handle segment pairs per sample, H S) is a sizeable share of the Gram's (its distinct output
    // area): from about a third of the Gram's time, H S >= area / 8000.
    const int64_t gram_area = (int64_t)(gram_tiles(L, (int)W, 256).size() / 2) * 256 * 256;
    const bool shares = !f64 && (int64_t)H * ctx->opts.segs_per_handle * 8000 >= gram_area;
    // default split-BF16 tile when the Gram runs alone: the fewest tiles the tile buffer holds,
    // balanced (fewer Gram launches and partial-Gram read-modify-writes: paper-native step -0.2 ms
    // with 2 tiles of 50,048 samples against 3 of 33,344)
    if (ctx->opts.tile_rows <= 0 && gram == BEM_GRAM_BF16X3_MFMA && !shares && N > T) {
        int64_t Tmax = (int64_t)(((size_t)3 << 30) / ((size_t)W * elem)) / 64 * 64;
        const int64_t Toff = (((int64_t)1 << 31) - 1) / W / 64 * 64;          // 32-bit offsets in the Gram
        if (Toff < Tmax) Tmax = Toff;
        if (Tmax > T) {
            const int64_t nt = (N + Tmax - 1) / Tmax;
            const int64_t T2 = ((N + nt - 1) / nt + 63) / 64 * 64;
            if (T2 > T) T = T2;
        }
    }
    // split-BF16 Gram: the sample tile is split into 3 parts with partial Grams of their own,
    // so that a launch has 3x the blocks (fewer idle CUs in its last round) and stays
    // deterministic (no atomics)
    const int parts = gram == BEM_GRAM_BF16X3_MFMA ? 3 : 1;
    const int64_t kchunk = ((T + parts - 1) / parts + 31) / 32 * 32;
    const bool overlap = shares && N > T;
    const size_t tile_bytes = ((size_t)W * T * elem + 255) / 256 * 256;
    hipStream_t sg = s;
    if (overlap && (rc = aux_stream(ctx, &sg))) return rc;
    // tmp0: feature tile(s); tmp1: R [W][3] + G [parts][W][W] + X r partials; tmp2: residual in f64
    if ((rc = ensure(ctx, ctx->tmp0, tile_bytes * (overlap ? 2 : 1), s))) return rc;
    if ((rc = ensure(ctx, ctx->tmp1,
                     ((size_t)parts * W * W + (size_t)W * 3 + (size_t)kXrPartials * W * 3) * sizeof(double), s)))
        return rc;
    if ((rc = ensure(ctx, ctx->tmp2, (size_t)(N > 0 ? N : 1) * 3 * sizeof(double), s))) return rc;
    double* R = (double*)ctx->tmp1.ptr;
    double* G = R + (size_t)W * 3;
    double* Rp = G + (size_t)parts * W * W;
    double* r64 = (double*)ctx->tmp2.ptr;
    // the first sample tile's Gram writes G (every entry of its tile list, in every part), so only
    // J^T r's partials (and G itself without samples) start from zero
    if ((rc = fill_f64(ctx, R, N > 0 ? W * 3 : (int64_t)parts * W * W + W * 3, 0.0, s))) return rc;
    // Jtr == nullptr: J^T J only (the LM step takes its gradient from the adjoint)
    const bool want_r = Jtr != nullptr;
    if (N > 0 && want_r) {
        if (mixed)
            hipLaunchKernelGGL(k_to_f64<float>, dim3(blocks_for(3 * N, 256)), dim3(256), 0, s, (const float*)resid, 3 * N, r64);
        else
            hipLaunchKernelGGL(k_to_f64<double>, dim3(blocks_for(3 * N, 256)), dim3(256), 0, s, (const double*)resid, 3 * N, r64);
    }
    const int ts = gram == BEM_GRAM_FP64_VALU ? 64 : (gram == BEM_GRAM_BF16X3_MFMA ? 256 : 128);
    const std::vector<int> tiles = f64 ? gram_tiles(L, (int)W, ts) : gram_work(gram_tiles(L, (int)W, ts), parts);
    const int ntiles = f64 ? (int)tiles.size() / 2 : (int)tiles.size() / 3;
    // the work list lives on the device (tilew); it is uploaded when its configuration changes, the
    // only host synchronisation of this call apart from workspace growth
    const int64_t key[4] = {W, H, ctx->model, gram};
    if (std::memcmp(key, ctx->tiles_key, sizeof(key)) != 0) {
        ctx->tiles_key[0] = -1;
        if ((rc = ensure(ctx, ctx->tilew, tiles.size() * sizeof(int), s))) return rc;
        if (hipMemcpyAsync(ctx->tilew.ptr, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)       // the host copy goes out of scope below
            return set_error(ctx, BEM_EHIP, "tile list upload");
        std::memcpy(ctx->tiles_key, key, sizeof(key));
    }
    const int* dtiles = (const int*)ctx->tilew.ptr;
    // tmp5: the vertex table, then the near-pair corrections and run table of one sample tile
    const int S = ctx->opts.segs_per_handle;
    const size_t vtab_bytes = ((size_t)(S + 1) * 8 * sizeof(float) + 255) / 256 * 256;
    NearList nl{};
    if (mixed && N > 0) {
        if (pre) nl = *pre;
        else if ((rc = near_classify(ctx, ctx->nearf, x, N, H * ctx->opts.segs_per_handle, 0, &nl, s))) return rc;
    }
    const size_t corr_bytes = mixed ? ((size_t)((T + 63) / 64) * nl.slots * kFeatVals * sizeof(float) + 255) / 256 * 256 : 0;
    const size_t runs_bytes = mixed ? ((size_t)((T + 63) / 64) * H * sizeof(int2) + 255) / 256 * 256 : 0;
    // mixed tiles for an MFMA Gram: J^T r of the handle rows is summed as the features are formed
    // (float32 per 256-sample block, float64 across blocks); only the beta rows are read back
    const bool fused_r = want_r && mixed && !f64;
    const size_t rpart_bytes = fused_r ? (size_t)blocks_for(T, 256) * H * kJtrVals * sizeof(float) : 0;
    // the split-BF16 tile's beta rows sum their J^T r in the beta-row kernel too (no read-back pass)
    const bool fused_beta = fused_r && gram == BEM_GRAM_BF16X3_MFMA;
    const size_t bpart_bytes = fused_beta ? ((size_t)blocks_for(T, 256) * M * 3 * sizeof(float) + 255) / 256 * 256 : 0;
    if ((rc = ensure(ctx, ctx->tmp5, vtab_bytes + corr_bytes + runs_bytes + rpart_bytes + bpart_bytes + 256, s)))
        return rc;
    float* vtab = (float*)ctx->tmp5.ptr;
    float* corr = mixed ? (float*)((char*)ctx->tmp5.ptr + vtab_bytes) : nullptr;
    int2* runs = mixed ? (int2*)((char*)ctx->tmp5.ptr + vtab_bytes + corr_bytes) : nullptr;
    float* rpart = fused_r ? (float*)((char*)ctx->tmp5.ptr + vtab_bytes + corr_bytes + runs_bytes) : nullptr;
    float* bpart = fused_beta ? (float*)((char*)ctx->tmp5.ptr + vtab_bytes + corr_bytes + runs_bytes + rpart_bytes)
                              : nullptr;
    const float* rr = fused_r ? (const float*)resid : nullptr;
    const int xr_row0 = fused_r ? (int)L.handle_rows() : 0;
    hipLaunchKernelGGL(k_vertex_table, dim3(blocks_for(S + 1, 64)), dim3(64), 0, s, S, ctx->model, vtab);
    const float4* box = nullptr;        // culling boxes of the segment groups (mixed feature kernel)
    if (mixed && (rc = near_boxes(ctx, H * S, 0, &box, s))) return rc;
    hipEvent_t* evF = ctx->ev;          // features of the tile in buffer b done
    hipEvent_t* evG = ctx->ev + 2;      // Gram of the tile in buffer b done
    if (overlap) {                      // the Gram stream starts after everything queued so far
        if (hipEventRecord(ctx->ev[4], s) != hipSuccess || hipStreamWaitEvent(sg, ctx->ev[4], 0) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "stream fork");
    }
    int it = 0;
    for (int64_t t0 = 0; t0 < N; t0 += T, ++it) {
        const int64_t n = N - t0 < T ? N - t0 : T;
        const double* xt = x + 2 * t0;
        const int buf = overlap ? (it & 1) : 0;
        void* tile = (char*)ctx->tmp0.ptr + (size_t)buf * tile_bytes;
        if (overlap && it >= 2 && hipStreamWaitEvent(s, evG[buf], 0) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "stream wait");
        if (f64) {
            double* Xt = (double*)tile;
            if ((rc = launch_features<double>(ctx, xt, n, H, mixed, true, Xt, nullptr, T, s, &nl, t0, x, corr, vtab, runs,
                                              nullptr, nullptr, nullptr, box)))
                return rc;
            {
                ProfScope ps_(ctx, PT_GRAM_F64, s);
                rc = gemm_f64(ctx, (int)W, (int)W, (int)n, 1.0, Xt, T, false, Xt, T, true, it > 0 ? 1.0 : 0.0, G, W, s,
                              dtiles, ntiles, gram == BEM_GRAM_FP64_VALU);
            }
            if (rc) return rc;
            if (want_r &&
                (rc = gemm_f64(ctx, (int)W, 3, (int)n, 1.0, Xt, T, false, r64 + 3 * t0, 3, false, 1.0, R, 3, s, nullptr, 0)))
                return rc;
        } else if (gram == BEM_GRAM_FP32_MFMA) {
            float* Xt = (float*)tile;
            if ((rc = launch_features<float>(ctx, xt, n, H, mixed, true, Xt, nullptr, T, s, &nl, t0, x, corr, vtab, runs,
                                             rr ? rr + 3 * t0 : nullptr, rpart, R, box)))
                return rc;
            if (overlap && (hipEventRecord(evF[buf], s) != hipSuccess || hipStreamWaitEvent(sg, evF[buf], 0) != hipSuccess))
                return set_error(ctx, BEM_EHIP, "stream wait");
            if ((rc = launch_gram_mfma(ctx, gram, Xt, nullptr, T, (int)W, n, dtiles, ntiles, kchunk, G, W * W, it > 0, sg)))
                return rc;
            if (want_r && (rc = launch_xr(ctx, gram, Xt, nullptr, T, (int)W, n, r64 + 3 * t0, R, Rp, sg, xr_row0)))
                return rc;
        } else {
            uint16_t* Xh = (uint16_t*)tile;
            uint16_t* Xl = Xh + (size_t)W * T;
            // blocked layout: ld is the row count
            if ((rc = launch_features<uint16_t>(ctx, xt, n, H, mixed, true, Xh, Xl, W, s, &nl, t0, x, corr, vtab, runs,
                                                rr ? rr + 3 * t0 : nullptr, rpart, R, box, bpart)))
                return rc;
            if (n & 31)
                hipLaunchKernelGGL(k_zero_tail, dim3(blocks_for(W * (32 - (n & 31)), 256)), dim3(256), 0, s, Xh, Xl, W, n);
            if (overlap && (hipEventRecord(evF[buf], s) != hipSuccess || hipStreamWaitEvent(sg, evF[buf], 0) != hipSuccess))
                return set_error(ctx, BEM_EHIP, "stream wait");
            if ((rc = launch_gram_mfma(ctx, gram, Xh, Xl, T, (int)W, n, dtiles, ntiles, kchunk, G, W * W, it > 0, sg)))
                return rc;
            if (want_r && !fused_beta &&
                (rc = launch_xr(ctx, gram, Xh, Xl, T, (int)W, n, r64 + 3 * t0, R, Rp, sg, xr_row0)))
                return rc;
        }
        if (overlap && hipEventRecord(evG[buf], sg) != hipSuccess) return set_error(ctx, BEM_EHIP, "stream event");
    }
    if (overlap) {                      // join: the caller's stream continues after the last Gram
        if (hipEventRecord(ctx->ev[5], sg) != hipSuccess || hipStreamWaitEvent(s, ctx->ev[5], 0) != hipSuccess)
            return set_error(ctx, BEM_EHIP, "stream join");
    }
    if (parts > 1 && N > 0) {
        // the first ntiles / parts work entries are part 0's, one per tile of the list
        hipLaunchKernelGGL(k_sum_parts, dim3(ntiles / parts, 8), dim3(256), 0, s, G, parts, W, dtiles, ts);
        if ((rc = check_launch(ctx, "gram parts"))) return rc;
    }
    // contraction: per channel the compact Gram and S, then every entry of J^T J in one pass
    // (1/N) sum over the samples, or (1/norm): the samples drawn over the whole image
    const double sc = N > 0 ? 1.0 / (norm > 0.0 ? norm : (double)N) : 0.0;
    if (want_r && (rc = fill_f64(ctx, Jtr, P, 0.0, s))) return rc;
    const size_t wc2 = (size_t)Wc * Wc;
    const size_t szc = (size_t)M * n12;
    const size_t sn = (size_t)n12 * n12;
    if ((rc = ensure(ctx, ctx->tmp2, (3 * wc2 + szc + 3 * sn + (size_t)(N > 0 ? N : 1) * 3) * sizeof(double), s)))
        return rc;
    double* Gc3 = (double*)ctx->tmp2.ptr + (size_t)(N > 0 ? N : 1) * 3;   // after r64 (no longer needed)
    double* Zc = Gc3 + 3 * wc2;
    double* S3 = Zc + szc;
    for (int c = 0; c < 3; ++c) {
        double* Gc = Gc3 + c * wc2;
        double* S1 = S3 + c * sn;
        hipLaunchKernelGGL(k_gather_gram, dim3(blocks_for(Wc, 32), blocks_for(Wc, 32)), dim3(256), 0, s, G, W, L, c,
                           Wc, Gc);
        hipLaunchKernelGGL(k_gather_z, dim3(blocks_for(n12, 256), M), dim3(256), 0, s, Z, L, M, c, Zc);
        if ((rc = check_launch(ctx, "gather"))) return rc;
        // The channel's block of J^T J is G + B Zc + (B Zc)^T + Zc^T D Zc with B = Gc[0:n12, n12:Wc]
        // and D = Gc[n12:, n12:] (symmetric), which equals G + S + S^T with S = Y Zc and
        // Y = B + (1/2) Zc^T D: two products instead of three.  Y overwrites B in Gc.
        if ((rc = gemm_f64(ctx, n12, M, M, 0.5, Zc, n12, true, Gc + (size_t)n12 * Wc + n12, Wc, false, 1.0, Gc + n12, Wc, s,
                           nullptr, 0)))
            return rc;
        if ((rc = gemm_f64(ctx, n12, n12, M, 1.0, Gc + n12, Wc, false, Zc, n12, false, 0.0, S1, n12, s, nullptr, 0))) return rc;
        if (want_r) {
            hipLaunchKernelGGL(k_scatter_g, dim3(blocks_for(n12, 64)), dim3(256), 0, s, R, Zc, L, M, c, sc, Jtr);
            if ((rc = check_launch(ctx, "scatter"))) return rc;
        }
    }
    if (n12 > 0) {
        hipLaunchKernelGGL(k_scatter_jtj, dim3(blocks_for(n12, 32), blocks_for(n12, 32)), dim3(256), 0, s, Gc3,
                           (int64_t)wc2, Wc, S3, (int64_t)sn, L, sc, JtJ, P);
        if ((rc = check_launch(ctx, "scatter"))) return rc;
    }
    return BEM_OK;
}

int run_jacobian(bem_ctx* ctx, const double* theta, int H, const double* x, int64_t N, double* J, hipStream_t s)
{
    int rc;
    const int M = ctx->M;
    const Layout L = layout_of(ctx, H);
    const int nf = (int)L.handle_rows();
    const int64_t W = nf + M;
    if (H == 0 || N == 0) return BEM_OK;
    if ((rc = prepare_forward_tables(ctx, theta, H, s))) return rc;
    double* Z = nullptr;
    if ((rc = boundary_derivatives(ctx, H, s, &Z))) return rc;
    const int64_t ld = N;
    if ((rc = ensure(ctx, ctx->tmp0, ((size_t)W * N + (size_t)N * nf) * sizeof(double), s))) return rc;
    double* Xt = (double*)ctx->tmp0.ptr;
    double* BZ = Xt + (size_t)W * N;
    if ((rc = launch_features<double>(ctx, x, N, H, false, true, Xt, nullptr, ld, s))) return rc;
    // BZ[t][f] = sum_i beta_i(t) Z[i][f]  (beta rows of Xt transposed)
    if ((rc = gemm_f64(ctx, (int)N, nf, M, 1.0, Xt + (size_t)nf * ld, ld, true, Z, nf, false, 0.0, BZ, nf, s, nullptr,
                       0)))
        return rc;
    hipLaunchKernelGGL(k_assemble_jacobian, dim3(blocks_for((int64_t)L.params() * H, 256), N), dim3(256), 0, s, Xt, ld,
                       BZ, L, N, J);
    return check_launch(ctx, "jacobian");
}

}  // namespace bem
