// vjp.hip - reverse mode of the forward path (Eq. diffbie, Sec. 3.2), as a
// vector-Jacobian product with cotangents gbar(x) of u(x):
//
//   segments  per handle segment, sums over samples of the pair adjoint:
//             d/da, d/db of sum_c gbar_c f_c   and  sum gbar_c M_m  (16 sums)
//   psi       psi_j = sum_x gbar(x) beta_j(x) for every outer element
//   mu        mu = A+^T psi  (the transposed boundary solve)
//   boundary  the same segment adjoint at the 3M boundary Gauss points with
//             cotangent mu_i w_q |G_i|/2 (F_i = sum_q w_q |G_i|/2 f(x_iq))
//   chain     segment end points -> Bezier control points (Bernstein weights),
//             end densities -> handle-end jumps (1 - t, t)
//
// Sweep mapping: the 64 lanes of a wavefront own 64 consecutive segments (or
// outer elements) and keep their sums in registers; the wavefront walks a
// chunk of samples whose positions and cotangents are wave-uniform (scalar
// loads).  Four wavefronts of a block split the chunk and are summed through
// LDS; chunks are summed by a separate fixed-order pass, so results do not
// depend on scheduling.
#include <mutex>

#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {

constexpr int kV = kSegVjpVals;   // 16 sums per segment
constexpr int kNearCopies = 16;   // partial rows the listed near pairs add into
constexpr double kGaussNode = 0.77459666924148337703585307995647992;
constexpr double kGaussW0 = 5.0 / 9.0, kGaussW1 = 8.0 / 9.0;

template <class GT>
__device__ inline void load_cot(const GT* __restrict__ gbar, int64_t s, double& g0, double& g1, double& g2)
{
    g0 = (double)gbar[3 * s]; g1 = (double)gbar[3 * s + 1]; g2 = (double)gbar[3 * s + 2];
}

template <class T>
__device__ inline void add_pair(T* acc, const Grad4<T>& gr, const Moments<T>& m, T g0, T g1, T g2)
{
    acc[0] += gr.ax; acc[1] += gr.ay; acc[2] += gr.bx; acc[3] += gr.by;
    acc[4] += m.da * g0; acc[5] += m.da * g1; acc[6] += m.da * g2;
    acc[7] += m.db * g0; acc[8] += m.db * g1; acc[9] += m.db * g2;
    acc[10] += m.sa * g0; acc[11] += m.sa * g1; acc[12] += m.sa * g2;
    acc[13] += m.sb * g0; acc[14] += m.sb * g1; acc[15] += m.sb * g2;
}

template <bool Mixed, class GT>
__global__ void __launch_bounds__(256) k_vjp_segments(const double* __restrict__ x, const GT* __restrict__ gbar,
                                                      int64_t N, int64_t chunk, const double* __restrict__ seg64,
                                                      const float* __restrict__ seg32, int K, double eps2, float eps2f,
                                                      float near2, double* __restrict__ partial)
{
    __shared__ double red[3][64][kV + 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k = blockIdx.x * 64 + lane;
    const int64_t n0 = (int64_t)blockIdx.y * chunk;
    const int64_t n1 = n0 + chunk < N ? n0 + chunk : N;
    double acc[kV];
    for (int v = 0; v < kV; ++v) acc[v] = 0.0;
    if (k < K) {
        const double* s64 = seg64 + (size_t)k * kSegStride;
        const SegGeom<double> g = load_geom(s64);
        if (g.L2 > 0.0) {
            double w[12];
            for (int c = 0; c < 12; ++c) w[c] = s64[kWdA + c];
            if (!Mixed) {
                for (int64_t s = n0 + wave; s < n1; s += 4) {
                    const double X = x[2 * s], Y = x[2 * s + 1];
                    double g0, g1, g2;
                    load_cot(gbar, s, g0, g1, g2);
                    const double wa = g0 * w[0] + g1 * w[1] + g2 * w[2];
                    const double wb = g0 * w[3] + g1 * w[4] + g2 * w[5];
                    const double sa = g0 * w[6] + g1 * w[7] + g2 * w[8];
                    const double sb = g0 * w[9] + g1 * w[10] + g2 * w[11];
                    const PairState<double> st = pair_forward<double, DevF64, true>(g, X, Y, eps2);
                    add_pair(acc, pair_backward(g, st, eps2, wa, wb, sa, sb), pair_moments(g, st), g0, g1, g2);
                }
            } else {
                // float32 far pairs; near pairs are evaluated in float64 by k_vjp_near
                // (listed pairs) and k_vjp_flagged (samples whose list slice overflowed)
                const float* s32 = seg32 + (size_t)k * kSegStride;
                const SegGeom<float> gf = load_geom(s32);
                float wf[12];
                for (int c = 0; c < 12; ++c) wf[c] = s32[kWdA + c];
                for (int64_t s0 = n0 + wave; s0 < n1; s0 += 4 * 64) {
                    // float sums over at most 64 samples, then folded into the float64 sums
                    float af[kV];
                    for (int v = 0; v < kV; ++v) af[v] = 0.0f;
                    const int64_t s1 = s0 + 4 * 64 < n1 ? s0 + 4 * 64 : n1;
                    for (int64_t s = s0; s < s1; s += 4) {
                        const float Xf = (float)x[2 * s], Yf = (float)x[2 * s + 1];
                        const float f0 = (float)gbar[3 * s], f1 = (float)gbar[3 * s + 1], f2 = (float)gbar[3 * s + 2];
                        const bool skip = near_segment(gf.ax, gf.ay, gf.bx, gf.by, gf.L2, Xf, Yf, near2);
                        const float wa = f0 * wf[0] + f1 * wf[1] + f2 * wf[2];
                        const float wb = f0 * wf[3] + f1 * wf[4] + f2 * wf[5];
                        const float sa = f0 * wf[6] + f1 * wf[7] + f2 * wf[8];
                        const float sb = f0 * wf[9] + f1 * wf[10] + f2 * wf[11];
                        const PairState<float> st = pair_forward<float, DevF32, false>(gf, Xf, Yf, eps2f);
                        const float on = skip ? 0.0f : 1.0f;
                        add_pair(af, pair_backward(gf, st, eps2f, on * wa, on * wb, on * sa, on * sb),
                                 pair_moments(gf, st), on * f0, on * f1, on * f2);
                    }
                    for (int v = 0; v < kV; ++v) acc[v] += (double)af[v];
                }
            }
        }
    }
    if (wave > 0)
        for (int v = 0; v < kV; ++v) red[wave - 1][lane][v] = acc[v];
    __syncthreads();
    if (wave == 0 && k < K) {
        double* o = partial + ((size_t)blockIdx.y * K + k) * kV;
        for (int v = 0; v < kV; ++v) o[v] = ((acc[v] + red[0][lane][v]) + red[1][lane][v]) + red[2][lane][v];
    }
}

// psi_j = sum_x gbar(x) beta_j(x): lanes own outer elements.
template <bool Mixed, class GT>
__global__ void __launch_bounds__(256) k_vjp_elements(const double* __restrict__ x, const GT* __restrict__ gbar,
                                                      int64_t N, int64_t chunk, const double* __restrict__ el64,
                                                      const float* __restrict__ el32, int M, float near2,
                                                      double* __restrict__ partial)
{
    __shared__ double red[3][64][3];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = blockIdx.x * 64 + lane;
    const int64_t n0 = (int64_t)blockIdx.y * chunk;
    const int64_t n1 = n0 + chunk < N ? n0 + chunk : N;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (j < M) {
        const double* e = el64 + (size_t)j * kElemStride;
        const double ax = e[0], ay = e[1], vx = e[2], vy = e[3];
        if (!Mixed) {
            for (int64_t s = n0 + wave; s < n1; s += 4) {
                double g0, g1, g2;
                load_cot(gbar, s, g0, g1, g2);
                const double b = element_beta<double, DevF64>(ax, ay, vx, vy, x[2 * s], x[2 * s + 1]);
                a0 += b * g0; a1 += b * g1; a2 += b * g2;
            }
        } else {
            const float* ef = el32 + (size_t)j * kElemStride;
            const float fax = ef[0], fay = ef[1], fvx = ef[2], fvy = ef[3];
            for (int64_t s0 = n0 + wave; s0 < n1; s0 += 4 * 64) {
                float b0 = 0.f, b1 = 0.f, b2 = 0.f;
                const int64_t s1 = s0 + 4 * 64 < n1 ? s0 + 4 * 64 : n1;
                for (int64_t s = s0; s < s1; s += 4) {
                    const float Xf = (float)x[2 * s], Yf = (float)x[2 * s + 1];
                    const bool skip = near_element(fax, fay, fvx, fvy, Xf, Yf, near2);
                    const float b = skip ? 0.0f : element_beta<float, DevF32>(fax, fay, fvx, fvy, Xf, Yf);
                    b0 += b * (float)gbar[3 * s]; b1 += b * (float)gbar[3 * s + 1]; b2 += b * (float)gbar[3 * s + 2];
                }
                a0 += (double)b0; a1 += (double)b1; a2 += (double)b2;
            }
        }
    }
    if (wave > 0) { red[wave - 1][lane][0] = a0; red[wave - 1][lane][1] = a1; red[wave - 1][lane][2] = a2; }
    __syncthreads();
    if (wave == 0 && j < M) {
        double* o = partial + ((size_t)blockIdx.y * M + j) * 3;
        o[0] = ((a0 + red[0][lane][0]) + red[1][lane][0]) + red[2][lane][0];
        o[1] = ((a1 + red[0][lane][1]) + red[1][lane][1]) + red[2][lane][1];
        o[2] = ((a2 + red[0][lane][2]) + red[1][lane][2]) + red[2][lane][2];
    }
}

// Float64 adjoint of one near (sample, segment) pair: the 16 per-segment sums of the pair in a[].
__device__ inline void near_segment_values(const double* __restrict__ s, double X, double Y, double g0, double g1,
                                           double g2, double eps2, double* __restrict__ a)
{
    for (int v = 0; v < kV; ++v) a[v] = 0.0;
    const SegGeom<double> g = load_geom(s);
    if (g.L2 == 0.0) return;
    const double wa = g0 * s[kWdA] + g1 * s[kWdA + 1] + g2 * s[kWdA + 2];
    const double wb = g0 * s[kWdB] + g1 * s[kWdB + 1] + g2 * s[kWdB + 2];
    const double sa = g0 * s[kWcA] + g1 * s[kWcA + 1] + g2 * s[kWcA + 2];
    const double sb = g0 * s[kWcB] + g1 * s[kWcB + 1] + g2 * s[kWcB + 2];
    const PairState<double> st = pair_forward<double, DevF64, true>(g, X, Y, eps2);
    add_pair(a, pair_backward(g, st, eps2, wa, wb, sa, sb), pair_moments(g, st), g0, g1, g2);
}

// Same, added into segsum[seg][16] (atomics).
__device__ inline void near_segment_adjoint(const double* __restrict__ s, double X, double Y, double g0, double g1,
                                            double g2, double eps2, double* __restrict__ o)
{
    double a[kV];
    near_segment_values(s, X, Y, g0, g1, g2, eps2, a);
    for (int v = 0; v < kV; ++v) atomicAdd(o + v, a[v]);
}

// Float64 beta of one near (sample, outer element) pair times the cotangent, added into psisum[j][3].
__device__ inline void near_element_adjoint(const double* __restrict__ e, double X, double Y, double g0, double g1,
                                            double g2, double* __restrict__ o)
{
    const double b = element_beta<double, DevF64>(e[0], e[1], e[2], e[3], X, Y);
    atomicAdd(o + 0, b * g0);
    atomicAdd(o + 1, b * g1);
    atomicAdd(o + 2, b * g2);
}

// Listed near pairs of the mixed adjoint: block per wavefront slice, a wavefront
// taking 64 consecutive entries at a time.  Entries of a slice are sorted by segment,
// so the wavefront first sums equal segments by a segmented scan over its lanes, and
// one lane per run adds the sums with atomics into kNearCopies extra partial rows of
// each fixed-order reduction: value c into row (slice + c) mod kNearCopies, so that
// the 16 atomics of a run (most runs hold one pair) go to 16 cache lines and slices
// near the same segment to different rows, rather than queueing on one line.  Pairs
// of flagged samples are left to k_vjp_flagged (into the first row), which redoes all
// near pairs of such a sample.
__global__ void __launch_bounds__(256) k_vjp_near(const NearPair* __restrict__ list, int slots,
                                                  const int* __restrict__ wave_count,
                                                  const uint8_t* __restrict__ flag,
                                                  const double* __restrict__ x, const float* __restrict__ gbar,
                                                  const double* __restrict__ seg64, int K,
                                                  const double* __restrict__ el64, int M, double eps2,
                                                  double* __restrict__ segsum, double* __restrict__ psisum)
{
    // block per wavefront slice; wavefront q of the block takes the slice's 64-entry chunks q, q + 4, ...
    const int64_t wv = blockIdx.x;
    const int cnt = wave_count[wv];
    const NearPair* sl = list + wv * slots;
    const int lane = threadIdx.x & 63;
    constexpr int kNone = 0x7fffffff;                 // key of an empty slot: after every entry
    for (int c0 = (threadIdx.x >> 6) * 64; c0 < cnt; c0 += 256) {
        const int e = c0 + lane;
        double v[kV];
        for (int c = 0; c < kV; ++c) v[c] = 0.0;
        int key = kNone;
        if (e < cnt) {
            const NearPair p = sl[e];
            key = p.seg;
            const int64_t i = p.sample;
            if (!flag[i]) {
                const double X = x[2 * i], Y = x[2 * i + 1];
                const double g0 = gbar[3 * i], g1 = gbar[3 * i + 1], g2 = gbar[3 * i + 2];
                if (p.seg < K) {
                    near_segment_values(seg64 + (size_t)p.seg * kSegStride, X, Y, g0, g1, g2, eps2, v);
                } else {
                    const double* el = el64 + (size_t)(p.seg - K) * kElemStride;
                    const double b = element_beta<double, DevF64>(el[0], el[1], el[2], el[3], X, Y);
                    v[0] = b * g0; v[1] = b * g1; v[2] = b * g2;
                }
            }
        }
        // inclusive segmented scan: after the step with offset o, v holds the sum over the lanes
        // (l - 2o, l] with the same key (keys ascend along the lanes)
        for (int o = 1; o < 64; o <<= 1) {
            const int ko = __shfl_up(key, o);
            const bool take = lane >= o && ko == key;
            for (int c = 0; c < kV; ++c) {
                const double w = __shfl_up(v[c], o);
                if (take) v[c] += w;
            }
        }
        // value c of a run goes to partial row (slice + c) mod kNearCopies
        const int kn = __shfl_down(key, 1);
        if ((lane == 63 || kn != key) && key != kNone) {
            if (key < K) {
                for (int c = 0; c < kV; ++c)
                    atomicAdd(segsum + (size_t)((wv + c) % kNearCopies) * K * kV + (size_t)key * kV + c, v[c]);
            } else {
                for (int c = 0; c < 3; ++c)
                    atomicAdd(psisum + (size_t)((wv + c) % kNearCopies) * M * 3 + 3 * (size_t)(key - K) + c, v[c]);
            }
        }
    }
}

// Every near pair of each flagged sample (thread per sample; flagged samples are rare).
__global__ void __launch_bounds__(256) k_vjp_flagged(const uint8_t* __restrict__ flag, int64_t N,
                                                     const double* __restrict__ x, const float* __restrict__ gbar,
                                                     const float* __restrict__ seg32, const double* __restrict__ seg64,
                                                     int K, const float* __restrict__ el32,
                                                     const double* __restrict__ el64, int M, double eps2, float near2,
                                                     double* __restrict__ segsum, double* __restrict__ psisum)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !flag[i]) return;
    const double X = x[2 * i], Y = x[2 * i + 1];
    const float Xf = (float)X, Yf = (float)Y;
    const double g0 = gbar[3 * i], g1 = gbar[3 * i + 1], g2 = gbar[3 * i + 2];
    for (int k = 0; k < K; ++k) {
        const float* s = seg32 + (size_t)k * kSegStride;
        if (near_segment(s[0], s[1], s[2], s[3], s[6], Xf, Yf, near2))
            near_segment_adjoint(seg64 + (size_t)k * kSegStride, X, Y, g0, g1, g2, eps2, segsum + (size_t)k * kV);
    }
    for (int j = 0; j < M; ++j) {
        const float* e = el32 + (size_t)j * kElemStride;
        if (near_element(e[0], e[1], e[2], e[3], Xf, Yf, near2))
            near_element_adjoint(el64 + (size_t)j * kElemStride, X, Y, g0, g1, g2, psisum + 3 * (size_t)j);
    }
}

// out[i] = sum_p partial[p * len + i], fixed order.
__global__ void k_reduce_parts(const double* __restrict__ partial, int nparts, int64_t len, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += partial[(size_t)p * len + i];
    out[i] = s;
}

// Gauss points of the outer elements and their cotangents mu_i w_q |G_i|/2.
__global__ void k_gauss_cotangent(const double* __restrict__ mu, int M, const double* __restrict__ eg, double* __restrict__ gx,
                                  double* __restrict__ gc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * M) return;
    const int i = t / 3, q = t % 3;
    double ax, ay, bx, by;
    load_element(eg, i, ax, ay, bx, by);
    const double hx = 0.5 * (bx - ax), hy = 0.5 * (by - ay);
    const double node = q == 0 ? -kGaussNode : (q == 1 ? 0.0 : kGaussNode);
    const double w = (q == 1 ? kGaussW1 : kGaussW0) * sqrt(hx * hx + hy * hy);
    gx[2 * t] = 0.5 * (ax + bx) + node * hx;
    gx[2 * t + 1] = 0.5 * (ay + by) + node * hy;
    for (int c = 0; c < 3; ++c) gc[3 * t + c] = mu[3 * i + c] * w;
}

// Segment sums -> theta gradient: one thread per handle.  Cubic handles chain the vertex
// gradients to the control points with Bernstein weights and the end jumps with (1 - t, t);
// straight handles (model 1) chain them to the end points with (1 - t, t) and sum the jumps.
__global__ void k_chain_theta(const double* __restrict__ sg, int H, int S, int model, double* __restrict__ grad)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    double out[20];
    for (int p = 0; p < 20; ++p) out[p] = 0.0;
    const bool straight = model == 1;
    for (int j = 0; j < S; ++j) {
        const double* v = sg + ((size_t)h * S + j) * kV;
        const double ta = (double)j / (double)S, tb = (double)(j + 1) / (double)S;
        double Ba[4], Bb[4];
        vertex_weights(model, ta, Ba);
        vertex_weights(model, tb, Bb);
        for (int c = 0; c < 4; ++c) {
            out[2 * c] += Ba[c] * v[0] + Bb[c] * v[2];
            out[2 * c + 1] += Ba[c] * v[1] + Bb[c] * v[3];
        }
        if (straight) {
            for (int c = 0; c < 3; ++c) {
                out[4 + c] += v[4 + c] + v[7 + c];       // wd
                out[7 + c] += v[10 + c] + v[13 + c];     // wc
            }
            continue;
        }
        for (int c = 0; c < 3; ++c) {
            out[8 + c] += (1.0 - ta) * v[4 + c] + (1.0 - tb) * v[7 + c];     // wd at end 0
            out[11 + c] += ta * v[4 + c] + tb * v[7 + c];                    // wd at end 1
            out[14 + c] += (1.0 - ta) * v[10 + c] + (1.0 - tb) * v[13 + c];  // wc at end 0
            out[17 + c] += ta * v[10 + c] + tb * v[13 + c];                  // wc at end 1
        }
    }
    const int q = straight ? 10 : 20;
    for (int p = 0; p < q; ++p) grad[(size_t)h * q + p] = out[p];
}

int chunks_for(int64_t N, int groups, int64_t& chunk)
{
    int64_t nch = (4096 + groups - 1) / groups;
    const int64_t cap = (N + 255) / 256;
    if (nch > cap) nch = cap;
    if (nch < 1) nch = 1;
    chunk = (N + nch - 1) / nch;
    if (chunk < 1) chunk = 1;
    nch = (N + chunk - 1) / chunk;
    if (nch < 1) nch = 1;
    return (int)nch;
}

}  // namespace

// Bytes of device workspace the float64 adjoint carves for K segments, M elements and N samples
// (tables, partial sums, psi, mu, boundary Gauss points, segment sums), each piece 256-aligned.
static size_t carve_round(size_t b) { return (b + 255) / 256 * 256; }

size_t vjp_f64_workspace_bytes(int K, int M, int64_t N)
{
    const int kgroups = (K + 63) / 64, mgroups = (M + 63) / 64;
    int64_t c = 1;
    const int ns = N > 0 ? chunks_for(N, kgroups, c) : 0;
    const int ng = chunks_for(3 * (int64_t)M, kgroups, c);
    const int ne = N > 0 ? chunks_for(N, mgroups, c) : 0;
    const size_t k1 = (size_t)(K > 0 ? K : 1);
    return carve_round(k1 * kSegStride * sizeof(double)) + carve_round(k1 * kSegStride * sizeof(float)) +
           carve_round((size_t)M * kElemStride * sizeof(double)) + carve_round((size_t)M * kElemStride * sizeof(float)) +
           carve_round((size_t)M * 3 * sizeof(double)) + carve_round((size_t)(ns + ng) * k1 * kV * sizeof(double)) +
           carve_round(((size_t)(ne > 0 ? ne : 1) * M * 3 + 2 * (size_t)M * 3) * sizeof(double)) +
           carve_round((size_t)3 * M * 5 * sizeof(double)) + carve_round(k1 * kV * sizeof(double));
}

int run_vjp(bem_ctx* ctx, const double* theta, int H, const double* x, int64_t N, const void* gbar, bool mixed,
            double* grad, hipStream_t s, const NearList* pre, const Carve* carve)
{
    int rc;
    const int S = ctx->opts.segs_per_handle;
    const int K = H * S;
    const int M = ctx->M;
    const double eps2 = ctx->opts.eps * ctx->opts.eps;
    const double nf = near_radius(ctx->opts.near_factor);
    const float near2 = (float)(nf * nf);
    if (H == 0) return BEM_OK;
    if (carve && mixed) return set_error(ctx, BEM_EINVAL, "the carved adjoint is float64 only (internal)");
    const int kgroups = (K + 63) / 64, mgroups = (M + 63) / 64;
    int64_t chunk_s = 1, chunk_g = 1, chunk_e = 1;
    const int ns = N > 0 ? chunks_for(N, kgroups, chunk_s) : 0;
    const int ng = chunks_for(3 * (int64_t)M, kgroups, chunk_g);
    const int ne = N > 0 ? chunks_for(N, mgroups, chunk_e) : 0;
    const int extra = mixed && N > 0 ? kNearCopies : 0; // partial rows for the float64 near pairs
    const size_t seg_part = (size_t)(ns + ng + extra) * K * kV;
    const size_t el_rows = (size_t)(ne > 0 ? ne : 1) + extra;
    const size_t seg_n = (size_t)(K > 0 ? K : 1) * kSegStride;
    double *seg64w, *el64w, *Uw, *part, *epart, *gx, *redw;
    float *seg32w, *el32w;
    if (carve) {
        // every workspace from the caller's device memory, in the order vjp_f64_workspace_bytes counts
        if (vjp_f64_workspace_bytes(K, M, N) > carve->bytes)
            return set_error(ctx, BEM_EINVAL, "%zu bytes of workspace for K = %d, M = %d, N = %lld exceed the %zu "
                             "available", vjp_f64_workspace_bytes(K, M, N), K, M, (long long)N, carve->bytes);
        char* p = carve->base;
        auto take = [&](size_t b) { char* q = p; p += carve_round(b); return q; };
        seg64w = (double*)take(seg_n * sizeof(double));
        seg32w = (float*)take(seg_n * sizeof(float));
        el64w = (double*)take((size_t)M * kElemStride * sizeof(double));
        el32w = (float*)take((size_t)M * kElemStride * sizeof(float));
        Uw = (double*)take((size_t)M * 3 * sizeof(double));
        part = (double*)take(seg_part * sizeof(double));
        epart = (double*)take((el_rows * M * 3 + 2 * (size_t)M * 3) * sizeof(double));
        gx = (double*)take((size_t)3 * M * 5 * sizeof(double));
        redw = (double*)take((size_t)K * kV * sizeof(double));
    } else {
        // workspaces: tmp1 segment partials, tmp2 element partials + psi + mu, tmp3 Gauss points, red segment sums
        if ((rc = ensure(ctx, ctx->seg64, seg_n * sizeof(double), s))) return rc;
        if ((rc = ensure(ctx, ctx->seg32, seg_n * sizeof(float), s))) return rc;
        if ((rc = ensure(ctx, ctx->U, (size_t)M * 3 * sizeof(double), s))) return rc;
        if ((rc = ensure(ctx, ctx->elem64, (size_t)M * kElemStride * sizeof(double), s))) return rc;
        if ((rc = ensure(ctx, ctx->elem32, (size_t)M * kElemStride * sizeof(float), s))) return rc;
        if ((rc = ensure(ctx, ctx->tmp1, seg_part * sizeof(double), s))) return rc;
        if ((rc = ensure(ctx, ctx->tmp2, (el_rows * M * 3 + 2 * (size_t)M * 3) * sizeof(double), s))) return rc;
        if ((rc = ensure(ctx, ctx->tmp3, (size_t)3 * M * 5 * sizeof(double), s))) return rc;
        if ((rc = ensure(ctx, ctx->red, (size_t)K * kV * sizeof(double), s))) return rc;
        seg64w = (double*)ctx->seg64.ptr;
        seg32w = (float*)ctx->seg32.ptr;
        Uw = (double*)ctx->U.ptr;
        el64w = (double*)ctx->elem64.ptr;
        el32w = (float*)ctx->elem32.ptr;
        part = (double*)ctx->tmp1.ptr;
        epart = (double*)ctx->tmp2.ptr;
        gx = (double*)ctx->tmp3.ptr;
        redw = (double*)ctx->red.ptr;
    }
    if ((rc = launch_expand_into(ctx, theta, H, seg64w, seg32w, s))) return rc;
    if ((rc = launch_pack_elements_into(ctx, Uw, el64w, el32w, s))) return rc;   // element geometry only
    double* psi = epart + el_rows * M * 3;
    double* mu = psi + (size_t)M * 3;
    double* gc = gx + (size_t)3 * M * 2;
    const double* seg64 = seg64w;
    const float* seg32 = seg32w;
    const double* el64 = el64w;
    const float* el32 = el32w;
    if (N > 0) {
        if (!mixed) {
            {
                ProfScope ps_(ctx, PT_VJP_SEGMENTS, s);
                hipLaunchKernelGGL((k_vjp_segments<false, double>), dim3(kgroups, ns), dim3(256), 0, s, x,
                                   (const double*)gbar, N, chunk_s, seg64, seg32, K, eps2, (float)eps2, near2, part);
            }
            {
                ProfScope ps_(ctx, PT_VJP_ELEMENTS, s);
                hipLaunchKernelGGL((k_vjp_elements<false, double>), dim3(mgroups, ne), dim3(256), 0, s, x,
                                   (const double*)gbar, N, chunk_e, el64, el32, M, near2, epart);
            }
        } else {
            double* segnear = part + (size_t)(ns + ng) * K * kV;
            double* psinear = epart + (size_t)ne * M * 3;
            NearList nl;
            if (pre) nl = *pre;
            else if ((rc = near_classify(ctx, ctx->nearv, x, N, K, M, &nl, s))) return rc;
            if ((rc = fill_f64(ctx, segnear, (int64_t)kNearCopies * K * kV, 0.0, s))) return rc;
            if ((rc = fill_f64(ctx, psinear, (int64_t)kNearCopies * M * 3, 0.0, s))) return rc;
            {
                ProfScope ps_(ctx, PT_VJP_SEGMENTS, s);
                hipLaunchKernelGGL((k_vjp_segments<true, float>), dim3(kgroups, ns), dim3(256), 0, s, x,
                                   (const float*)gbar, N, chunk_s, seg64, seg32, K, eps2, (float)eps2, near2, part);
            }
            {
                ProfScope ps_(ctx, PT_VJP_ELEMENTS, s);
                hipLaunchKernelGGL((k_vjp_elements<true, float>), dim3(mgroups, ne), dim3(256), 0, s, x,
                                   (const float*)gbar, N, chunk_e, el64, el32, M, near2, epart);
            }
            {
                ProfScope ps_(ctx, PT_NEAR, s);
                hipLaunchKernelGGL(k_vjp_near, dim3(nl.nwaves), dim3(256), 0, s, nl.list, nl.slots, nl.count, nl.flag, x,
                                   (const float*)gbar, seg64, K, el64, M, eps2, segnear, psinear);
                if (nl.overflowed)
                    hipLaunchKernelGGL(k_vjp_flagged, dim3(blocks_for(N, 256)), dim3(256), 0, s, nl.flag, N, x,
                                   (const float*)gbar, seg32, seg64, K, el32, el64, M, eps2, near2, segnear, psinear);
            }
        }
        hipLaunchKernelGGL(k_reduce_parts, dim3(blocks_for((int64_t)M * 3, 256)), dim3(256), 0, s, epart, ne + extra,
                           (int64_t)M * 3, psi);
        if ((rc = check_launch(ctx, "vjp sweeps"))) return rc;
        if ((rc = launch_boundary_solve(ctx, psi, mu, true, s))) return rc;
        hipLaunchKernelGGL(k_gauss_cotangent, dim3(blocks_for(3 * M, 256)), dim3(256), 0, s, mu, M,
                           (const double*)ctx->egeo.ptr, gx, gc);
        {
            ProfScope ps_(ctx, PT_VJP_SEGMENTS, s);
            hipLaunchKernelGGL((k_vjp_segments<false, double>), dim3(kgroups, ng), dim3(256), 0, s, gx, gc,
                               (int64_t)3 * M, chunk_g, seg64, seg32, K, eps2, (float)eps2, near2,
                               part + (size_t)ns * K * kV);
        }
        hipLaunchKernelGGL(k_reduce_parts, dim3(blocks_for((int64_t)K * kV, 256)), dim3(256), 0, s, part,
                           ns + ng + extra, (int64_t)K * kV, redw);
    } else {
        hipLaunchKernelGGL(k_reduce_parts, dim3(blocks_for((int64_t)K * kV, 256)), dim3(256), 0, s, part, 0,
                           (int64_t)K * kV, redw);
    }
    hipLaunchKernelGGL(k_chain_theta, dim3(blocks_for(H, 64)), dim3(64), 0, s, (const double*)redw, H, S,
                       ctx->model, grad);
    return check_launch(ctx, "vjp");
}

}  // namespace bem

// ---- allocation-free float64 adjoint ----------------------------------------------------------
// Every workspace of bem_vjp_noalloc (segment and element tables, partial sums, psi, mu, boundary
// Gauss points, segment sums) is carved from this array; each device that runs the library holds
// its own copy for the life of the process.  Host code never passes the array's name to a kernel:
// its device address, found once per device with hipGetSymbolAddress, is kept in g_scratch.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch[kScratchDevices] = {};

// device address of this device's scratch array (the context's device is current)
int scratch_address(bem_ctx* ctx, char** out)
{
    const int dev = ctx->device;
    if (dev < 0 || dev >= kScratchDevices)
        return bem::set_error(ctx, BEM_EINVAL, "device %d beyond the %d the scratch table covers", dev, kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return bem::set_error(ctx, BEM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                  hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = (char*)g_scratch[dev];
    return BEM_OK;
}
}  // namespace

extern "C" int bem_vjp_noalloc(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N,
                               const double* gbar, double* grad, hipStream_t stream)
{
    using namespace bem;
    int rc = check_common(ctx, theta, H, x, N);
    if (rc) return rc;
    if (N > 0 && !gbar) return set_error(ctx, BEM_EINVAL, "gbar is null");
    if (H > 0 && !grad) return set_error(ctx, BEM_EINVAL, "grad is null");
    const int K = H * ctx->opts.segs_per_handle;
    const size_t need = vjp_f64_workspace_bytes(K, ctx->M, N);
    if (need > kScratchBytes)
        return set_error(ctx, BEM_EINVAL, "bem_vjp_noalloc: %zu bytes of workspace for K = %d segments, M = %d "
                         "elements, N = %lld samples exceed its %zu-byte scratch", need, K, ctx->M, (long long)N,
                         kScratchBytes);
    char* base = nullptr;
    if ((rc = scratch_address(ctx, &base))) return rc;
    // no profiling events for this call (recording them may allocate)
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    const Carve carve{base, kScratchBytes};
    rc = run_vjp(ctx, theta, H, x, N, gbar, false, grad, stream, nullptr, &carve);
    ctx->prof.on = prof;
    return rc;
}

