// sweep_mixed.hip - mixed-precision forward sweep (Sec. 3.1.3 evaluation of
// u(x) at every sample).
//
// Far pairs run in float32 from the float32 copies of the segment and element
// tables.  A pair whose two end points both lie within max(2 nf, nf + 1)*L of the
// sample, nf = near_factor (a set containing every sample closer than nf*L to
// the segment) is not evaluated there: the wavefront appends (sample, segment) to its
// own slice of a list, and a second kernel evaluates the listed
// pairs in float64 from the float64 tables and the float64 sample, adding into
// float64 per-sample sums.  Keeping float64 code out of the float32 sweep keeps
// its register count (and occupancy) at that of the float32 arithmetic.
// Should a wavefront's slice overflow, the samples whose pairs did not fit are
// flagged and recomputed by a sweep that evaluates near pairs inline.
#include "common.hpp"
#include "sweep_common.hpp"

namespace bem {

namespace {


// Appending needs no atomics: each wavefront owns a slice and counts its entries
// in a wave-uniform register.

__device__ inline void append_near(bool near, int32_t sample, int32_t seg, NearPair* __restrict__ slice, int slots,
                                   int& used, bool& overflow)
{
    const uint64_t mask = __ballot(near);
    if (mask == 0) return;
    const int lane = threadIdx.x & 63;
    if (near) {
        const int slot = used + __popcll(mask & ((1ull << lane) - 1ull));
        if (slot < slots) slice[slot] = NearPair{sample, seg};
        else overflow = true;
    }
    used += __popcll(mask);
}

// The segment records are staged through LDS in chunks: the block copies a chunk with
// coalesced 16-byte loads, then every wavefront reads each record by broadcast LDS reads.
// Measured on one MI355X against the alternatives (LM workload, sweep time per step):
// wave-uniform scalar loads of each record 81 ms, scalar loads issued one record ahead
// 86 ms, LDS staging 72 ms.  The outer-element records (32 KB in all) stay on scalar
// loads: staging them as well was no faster.
constexpr int kStageSegs = 256;                                 // segment records per chunk
constexpr int kSweepStage = kStageSegs * (kSegStride / 4);      // float4 slots (24 KB)
static_assert(kSegStride % 4 == 0, "segment records are whole float4s");
static_assert(kStageSegs % kBoxGroup == 0, "box groups lie within a chunk");

// Copies n float4s of records into the block's stage; every thread of the block calls it.
__device__ inline void stage_records(float4* __restrict__ stage, const float* __restrict__ src, int n)
{
    __syncthreads();                              // the previous chunk has been read by all
    const float4* s4 = reinterpret_cast<const float4*>(src);
    for (int e = threadIdx.x; e < n; e += blockDim.x) stage[e] = s4[e];
    __syncthreads();
}

// The float32 record of a degenerate segment evaluates to exactly zero and is
// never near (its L2 is 0), so the segment loop needs no branch for it.
__global__ void __launch_bounds__(256) k_sweep_far(const double* __restrict__ x, int64_t N,
                                                   const float* __restrict__ seg32, int K,
                                                   const float* __restrict__ el32, int M, float eps2f, float near2,
                                                   const float4* __restrict__ box,
                                                   float* __restrict__ u, NearPair* __restrict__ list, int slots,
                                                   int* __restrict__ wave_count, uint8_t* __restrict__ flag,
                                                   int* __restrict__ need)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t wave = i >> 6;
    NearPair* slice = list + wave * slots;
    const bool live = i < N;                       // the tail wave keeps its idle lanes for the ballots
    const float Xf = live ? (float)x[2 * i] : 0.0f, Yf = live ? (float)x[2 * i + 1] : 0.0f;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    bool overflow = false;
    int used = 0;
    // the wavefront's sample box: groups of segments farther than their near radius take the
    // loop without near tests (every pair in them is far; the result is the same)
    const float wx0 = uniform_f32(wave_min(live ? Xf : INFINITY)), wx1 = uniform_f32(wave_max(live ? Xf : -INFINITY));
    const float wy0 = uniform_f32(wave_min(live ? Yf : INFINITY)), wy1 = uniform_f32(wave_max(live ? Yf : -INFINITY));
    __shared__ float4 stage[kSweepStage];
    for (int k0 = 0; k0 < K; k0 += kStageSegs) {
        const int nk = K - k0 < kStageSegs ? K - k0 : kStageSegs;
        stage_records(stage, seg32 + (size_t)k0 * kSegStride, nk * (kSegStride / 4));
        for (int q0 = 0; q0 < nk; q0 += kBoxGroup) {
            const int q1 = q0 + kBoxGroup < nk ? q0 + kBoxGroup : nk;
            if (box_culled(box, (k0 + q0) / kBoxGroup, wx0, wy0, wx1, wy1)) {
                for (int kk = q0; kk < q1; ++kk) {
                    const float* s = reinterpret_cast<const float*>(stage + kk * (kSegStride / 4));
                    const SegGeom<float> g = load_geom(s);
                    const Moments<float> m = seg_moments<float, DevF32, false>(g, Xf, Yf, eps2f);
                    f0 += m.da * s[kWdA] + m.db * s[kWdB] + m.sa * s[kWcA] + m.sb * s[kWcB];
                    f1 += m.da * s[kWdA + 1] + m.db * s[kWdB + 1] + m.sa * s[kWcA + 1] + m.sb * s[kWcB + 1];
                    f2 += m.da * s[kWdA + 2] + m.db * s[kWdB + 2] + m.sa * s[kWcA + 2] + m.sb * s[kWcB + 2];
                }
                continue;
            }
            for (int kk = q0; kk < q1; ++kk) {
                const float* s = reinterpret_cast<const float*>(stage + kk * (kSegStride / 4));
                const SegGeom<float> g = load_geom(s);
                float w[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) w[c] = s[kWdA + c];
                const bool near = live & near_segment(g.ax, g.ay, g.bx, g.by, g.L2, Xf, Yf, near2);
                append_near(near, (int32_t)i, k0 + kk, slice, slots, used, overflow);
                const Moments<float> m = seg_moments<float, DevF32, false>(g, Xf, Yf, eps2f);
                const float on = near ? 0.0f : 1.0f;
                f0 += on * (m.da * w[0] + m.db * w[3] + m.sa * w[6] + m.sb * w[9]);
                f1 += on * (m.da * w[1] + m.db * w[4] + m.sa * w[7] + m.sb * w[10]);
                f2 += on * (m.da * w[2] + m.db * w[5] + m.sa * w[8] + m.sb * w[11]);
            }
        }
    }
    float b0 = 0.f, b1 = 0.f, b2 = 0.f;
    const int nsg = (K + kBoxGroup - 1) / kBoxGroup;     // element groups' boxes follow the segments'
    for (int j0 = 0; j0 < M; j0 += kBoxGroup) {
        const int j1 = j0 + kBoxGroup < M ? j0 + kBoxGroup : M;
        if (box_culled(box, nsg + j0 / kBoxGroup, wx0, wy0, wx1, wy1)) {
            for (int j = j0; j < j1; ++j) {
                const float* e = el32 + (size_t)j * kElemStride;
                const float beta = element_beta<float, DevF32>(e[0], e[1], e[2], e[3], Xf, Yf);
                b0 += beta * e[4]; b1 += beta * e[5]; b2 += beta * e[6];
            }
            continue;
        }
        for (int j = j0; j < j1; ++j) {
            const float* e = el32 + (size_t)j * kElemStride;
            const bool near = live & near_element(e[0], e[1], e[2], e[3], Xf, Yf, near2);
            append_near(near, (int32_t)i, K + j, slice, slots, used, overflow);
            const float beta = near ? 0.0f : element_beta<float, DevF32>(e[0], e[1], e[2], e[3], Xf, Yf);
            b0 += beta * e[4]; b1 += beta * e[5]; b2 += beta * e[6];
        }
    }
    if ((threadIdx.x & 63) == 0) {
        wave_count[wave] = used < slots ? used : slots;
        if (used > slots) atomicMax(need, used);
    }
    if (!live) return;
    u[3 * i + 0] = b0 + f0;
    u[3 * i + 1] = b1 + f1;
    u[3 * i + 2] = b2 + f2;
    flag[i] = overflow ? 1 : 0;
}

// Bounding boxes for culling near-pair tests per wavefront: box g (g < ceil(K / kBoxGroup): segments
// [kBoxGroup g, kBoxGroup (g + 1)); after those, group g - nsg of kBoxGroup outer elements) = the end
// points' extent (xmin, ymin, xmax, ymax) and the largest near radius sqrt(near2 L2) of its members.
// Degenerate segments (L2 = 0) are never near and are left out; a box with no member is empty
// (min > max) and culls everything.
__global__ void k_near_boxes(const float* __restrict__ seg32, int K, const float* __restrict__ el32, int M,
                             float near2, float4* __restrict__ box)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int nsg = (K + kBoxGroup - 1) / kBoxGroup;
    if (g >= nsg + (M + kBoxGroup - 1) / kBoxGroup) return;
    float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY, r = 0.0f;
    if (g < nsg) {
        const int k1 = (g + 1) * kBoxGroup < K ? (g + 1) * kBoxGroup : K;
        for (int k = g * kBoxGroup; k < k1; ++k) {
            const float* sg = seg32 + (size_t)k * kSegStride;
            if (sg[6] == 0.0f) continue;
            x0 = fminf(x0, fminf(sg[0], sg[2])); x1 = fmaxf(x1, fmaxf(sg[0], sg[2]));
            y0 = fminf(y0, fminf(sg[1], sg[3])); y1 = fmaxf(y1, fmaxf(sg[1], sg[3]));
            r = fmaxf(r, sqrtf(near2 * sg[6]));
        }
    } else {
        const int j0 = (g - nsg) * kBoxGroup, j1 = j0 + kBoxGroup < M ? j0 + kBoxGroup : M;
        for (int j = j0; j < j1; ++j) {
            const float* e = el32 + (size_t)j * kElemStride;
            const float bx = e[0] + e[2], by = e[1] + e[3];
            x0 = fminf(x0, fminf(e[0], bx)); x1 = fmaxf(x1, fmaxf(e[0], bx));
            y0 = fminf(y0, fminf(e[1], by)); y1 = fmaxf(y1, fmaxf(e[1], by));
            r = fmaxf(r, sqrtf(near2 * (e[2] * e[2] + e[3] * e[3])));
        }
    }
    box[2 * g] = make_float4(x0, y0, x1, y1);
    box[2 * g + 1] = make_float4(r, 0.0f, 0.0f, 0.0f);
}

// Near-pair classification only (for the adjoint and the J tiles): the same wavefront slices and
// predicate as the float32 forward sweep.  Each wavefront first bounds its samples and skips every
// group of kBoxGroup segments (and of outer elements) whose box is farther than its near radius;
// the exact test runs for the others, in segment order.  With samples visited cell by cell a
// wavefront's box is small and most groups are skipped.
__global__ void __launch_bounds__(256) k_classify(const double* __restrict__ x, int64_t N,
                                                  const float* __restrict__ seg32, int K,
                                                  const float* __restrict__ el32, int M, float near2,
                                                  const float4* __restrict__ box,
                                                  NearPair* __restrict__ list, int slots, int* __restrict__ wave_count,
                                                  uint8_t* __restrict__ flag, int* __restrict__ need)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t wave = i >> 6;
    NearPair* slice = list + wave * slots;
    const bool live = i < N;
    const float Xf = live ? (float)x[2 * i] : 0.0f, Yf = live ? (float)x[2 * i + 1] : 0.0f;
    const float wx0 = uniform_f32(wave_min(live ? Xf : INFINITY)), wx1 = uniform_f32(wave_max(live ? Xf : -INFINITY));
    const float wy0 = uniform_f32(wave_min(live ? Yf : INFINITY)), wy1 = uniform_f32(wave_max(live ? Yf : -INFINITY));
    bool overflow = false;
    int used = 0;
    const int nsg = (K + kBoxGroup - 1) / kBoxGroup;
    for (int g = 0; g < nsg; ++g) {
        if (box_culled(box, g, wx0, wy0, wx1, wy1)) continue;
        const int k1 = (g + 1) * kBoxGroup < K ? (g + 1) * kBoxGroup : K;
        for (int k = g * kBoxGroup; k < k1; ++k) {
            const float* s = seg32 + (size_t)k * kSegStride;
            const bool near = live & near_segment(s[0], s[1], s[2], s[3], s[6], Xf, Yf, near2);
            append_near(near, (int32_t)i, k, slice, slots, used, overflow);
        }
    }
    for (int g = 0; g * kBoxGroup < M; ++g) {
        if (box_culled(box, nsg + g, wx0, wy0, wx1, wy1)) continue;
        const int j1 = (g + 1) * kBoxGroup < M ? (g + 1) * kBoxGroup : M;
        for (int j = g * kBoxGroup; j < j1; ++j) {
            const float* e = el32 + (size_t)j * kElemStride;
            const bool near = live & near_element(e[0], e[1], e[2], e[3], Xf, Yf, near2);
            append_near(near, (int32_t)i, K + j, slice, slots, used, overflow);
        }
    }
    if ((threadIdx.x & 63) == 0) {
        wave_count[wave] = used < slots ? used : slots;
        if (used > slots) atomicMax(need, used);
    }
    if (live) flag[i] = overflow ? 1 : 0;
}

// Listed near pairs in float64: block per wavefront slice (its threads loop over the
// slice's entries only), the sums of the slice's 64 samples in LDS, then stored to
// acc[3 * sample + c] (every sample belongs to exactly one slice, so no global atomics).
__global__ void __launch_bounds__(256) k_near_pairs(const NearPair* __restrict__ list,
                                                    const int* __restrict__ wave_count, int slots, int64_t N,
                                                    const double* __restrict__ x, const double* __restrict__ seg64,
                                                    int K, const double* __restrict__ el64, double eps2,
                                                    double* __restrict__ acc)
{
    __shared__ double sacc[64 * 3];
    const int64_t w = blockIdx.x;
    const int cnt = wave_count[w];
    if (threadIdx.x < 64 * 3) sacc[threadIdx.x] = 0.0;
    __syncthreads();
    const NearPair* sl = list + w * slots;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const NearPair p = sl[e];
        const double X = x[2 * (int64_t)p.sample], Y = x[2 * (int64_t)p.sample + 1];
        double v0, v1, v2;
        if (p.seg < K) {
            const double* s = seg64 + (size_t)p.seg * kSegStride;
            const SegGeom<double> g = load_geom(s);
            const Moments<double> m = seg_moments<double, DevF64>(g, X, Y, eps2);
            v0 = m.da * s[kWdA + 0] + m.db * s[kWdB + 0] + m.sa * s[kWcA + 0] + m.sb * s[kWcB + 0];
            v1 = m.da * s[kWdA + 1] + m.db * s[kWdB + 1] + m.sa * s[kWcA + 1] + m.sb * s[kWcB + 1];
            v2 = m.da * s[kWdA + 2] + m.db * s[kWdB + 2] + m.sa * s[kWcA + 2] + m.sb * s[kWcB + 2];
        } else {
            const double* el = el64 + (size_t)(p.seg - K) * kElemStride;
            const double beta = element_beta<double, DevF64>(el[0], el[1], el[2], el[3], X, Y);
            v0 = beta * el[4]; v1 = beta * el[5]; v2 = beta * el[6];
        }
        const int ls = p.sample - (int)(w * 64);     // the slice lists its own wavefront's samples
        atomicAdd(&sacc[3 * ls + 0], v0);
        atomicAdd(&sacc[3 * ls + 1], v1);
        atomicAdd(&sacc[3 * ls + 2], v2);
    }
    __syncthreads();
    if (threadIdx.x < 64 * 3) {
        const int64_t gi = w * 64 * 3 + threadIdx.x;
        if (gi < 3 * N) acc[gi] = sacc[threadIdx.x];
    }
}

__global__ void k_combine(float* __restrict__ u, const double* __restrict__ acc, int64_t N, double c0, double c1,
                          double c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    u[3 * i + 0] = (float)(c0 + ((double)u[3 * i + 0] + acc[3 * i + 0]));
    u[3 * i + 1] = (float)(c1 + ((double)u[3 * i + 1] + acc[3 * i + 1]));
    u[3 * i + 2] = (float)(c2 + ((double)u[3 * i + 2] + acc[3 * i + 2]));
}

// Whole-sample mixed evaluation with near pairs inline, for flagged samples only
// (the list overflowed for them).
__global__ void __launch_bounds__(256) k_sweep_inline(const double* __restrict__ x, int64_t N,
                                                      const uint8_t* __restrict__ flag,
                                                      const float* __restrict__ seg32, const double* __restrict__ seg64,
                                                      int K, const float* __restrict__ el32,
                                                      const double* __restrict__ el64, int M, float eps2f, double eps2,
                                                      float near2, double c0, double c1, double c2,
                                                      float* __restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !flag[i]) return;
    const double X = x[2 * i], Y = x[2 * i + 1];
    const float Xf = (float)X, Yf = (float)Y;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    double n0 = 0.0, n1 = 0.0, n2 = 0.0;
    for (int k = 0; k < K; ++k) {
        const float* s = seg32 + (size_t)k * kSegStride;
        const SegGeom<float> g = load_geom(s);
        if (near_segment(g.ax, g.ay, g.bx, g.by, g.L2, Xf, Yf, near2)) {
            const double* s64 = seg64 + (size_t)k * kSegStride;
            const SegGeom<double> g64 = load_geom(s64);
            const Moments<double> m = seg_moments<double, DevF64>(g64, X, Y, eps2);
            n0 += m.da * s64[kWdA + 0] + m.db * s64[kWdB + 0] + m.sa * s64[kWcA + 0] + m.sb * s64[kWcB + 0];
            n1 += m.da * s64[kWdA + 1] + m.db * s64[kWdB + 1] + m.sa * s64[kWcA + 1] + m.sb * s64[kWcB + 1];
            n2 += m.da * s64[kWdA + 2] + m.db * s64[kWdB + 2] + m.sa * s64[kWcA + 2] + m.sb * s64[kWcB + 2];
        } else {
            const Moments<float> m = seg_moments<float, DevF32, false>(g, Xf, Yf, eps2f);
            f0 += m.da * s[kWdA + 0] + m.db * s[kWdB + 0] + m.sa * s[kWcA + 0] + m.sb * s[kWcB + 0];
            f1 += m.da * s[kWdA + 1] + m.db * s[kWdB + 1] + m.sa * s[kWcA + 1] + m.sb * s[kWcB + 1];
            f2 += m.da * s[kWdA + 2] + m.db * s[kWdB + 2] + m.sa * s[kWcA + 2] + m.sb * s[kWcB + 2];
        }
    }
    float b0 = 0.f, b1 = 0.f, b2 = 0.f;
    for (int j = 0; j < M; ++j) {
        const float* e = el32 + (size_t)j * kElemStride;
        if (near_element(e[0], e[1], e[2], e[3], Xf, Yf, near2)) {
            const double* e64 = el64 + (size_t)j * kElemStride;
            const double beta = element_beta<double, DevF64>(e64[0], e64[1], e64[2], e64[3], X, Y);
            n0 += beta * e64[4]; n1 += beta * e64[5]; n2 += beta * e64[6];
        } else {
            const float beta = element_beta<float, DevF32>(e[0], e[1], e[2], e[3], Xf, Yf);
            b0 += beta * e[4]; b1 += beta * e[5]; b2 += beta * e[6];
        }
    }
    u[3 * i + 0] = (float)(c0 + ((double)b0 + (double)f0 + n0));
    u[3 * i + 1] = (float)(c1 + ((double)b1 + (double)f1 + n1));
    u[3 * i + 2] = (float)(c2 + ((double)b2 + (double)f2 + n2));
}

}  // namespace

int near_boxes(bem_ctx* ctx, int K, int M, const float4** box, hipStream_t s)
{
    int rc;
    const int nbox = (K + kBoxGroup - 1) / kBoxGroup + (M + kBoxGroup - 1) / kBoxGroup;
    if ((rc = ensure(ctx, ctx->boxw, (size_t)(nbox > 0 ? nbox : 1) * 2 * sizeof(float4), s))) return rc;
    const double nf = near_radius(ctx->opts.near_factor);
    if (nbox > 0)
        hipLaunchKernelGGL(k_near_boxes, dim3(blocks_for(nbox, 256)), dim3(256), 0, s, (const float*)ctx->seg32.ptr, K,
                           (const float*)ctx->elem32.ptr, M, (float)(nf * nf), (float4*)ctx->boxw.ptr);
    *box = (const float4*)ctx->boxw.ptr;
    return check_launch(ctx, "near boxes");
}

// Classify the near pairs of samples x[0..N) (segments, and outer elements when M > 0) into buf.
int near_classify(bem_ctx* ctx, DevBuf& buf, const double* x, int64_t N, int K, int M, NearList* out, hipStream_t s)
{
    int rc;
    const double nf = near_radius(ctx->opts.near_factor);
    const int64_t nwaves = N > 0 ? (int64_t)blocks_for(N, 256) * 4 : 0;
    const int slots = near_slots_for(ctx->near_slots, nwaves);
    // list [nwaves][slots] | counts [nwaves] | overflow count (256 bytes) | flags [N]
    const size_t list_bytes = ((size_t)nwaves * slots * sizeof(NearPair) + 255) / 256 * 256;
    const size_t cnt_bytes = ((size_t)nwaves * sizeof(int) + 255) / 256 * 256;
    if ((rc = ensure(ctx, buf, list_bytes + cnt_bytes + 256 + (size_t)N + 256, s))) return rc;
    char* base = (char*)buf.ptr;
    out->list = (NearPair*)base;
    out->count = (int*)(base + list_bytes);
    out->need = (int*)(base + list_bytes + cnt_bytes);
    out->flag = (uint8_t*)(base + list_bytes + cnt_bytes + 256);
    out->nwaves = nwaves;
    out->slots = slots;
    if ((rc = fill_i32(ctx, out->need, 1, 0, s))) return rc;
    if (N == 0) return BEM_OK;
    ProfScope ps_(ctx, PT_NEAR, s);
    const float4* box;
    if ((rc = near_boxes(ctx, K, M, &box, s))) return rc;
    hipLaunchKernelGGL(k_classify, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, (const float*)ctx->seg32.ptr, K,
                       (const float*)ctx->elem32.ptr, M, (float)(nf * nf), box, out->list, slots,
                       out->count, out->flag, out->need);
    return check_launch(ctx, "classify");
}

int launch_sweep_mixed(bem_ctx* ctx, const double* x, int64_t N, int K, const double* cbar, float* u, hipStream_t s,
                       NearList* out)
{
    if (out) *out = NearList{};
    ctx->sweep_need = nullptr;
    if (N == 0) return BEM_OK;
    int rc;
    const double eps2 = ctx->opts.eps * ctx->opts.eps;
    const double nf = near_radius(ctx->opts.near_factor);
    const float near2 = (float)(nf * nf);
    // per-wavefront near-pair slices, their counts, float64 sums, overflow flags
    const int64_t nwaves = (int64_t)blocks_for(N, 256) * 4;     // every launched wavefront, idle tail ones too
    const int slots = near_slots_for(ctx->near_slots, nwaves);
    const int64_t nslots = nwaves * slots;
    // list [nwaves][slots] | float64 sums [N][3] | counts [nwaves] | overflow count (256 bytes) | flags [N]
    const size_t list_bytes = (size_t)nslots * sizeof(NearPair);
    const size_t acc_bytes = (size_t)N * 3 * sizeof(double);
    const size_t cnt_bytes = ((size_t)nwaves * sizeof(int) + 255) / 256 * 256;
    if ((rc = ensure(ctx, ctx->nearw, list_bytes + acc_bytes + cnt_bytes + 256 + (size_t)N + 256, s))) return rc;
    char* base = (char*)ctx->nearw.ptr;
    NearPair* list = (NearPair*)base;
    double* acc = (double*)(base + list_bytes);
    int* wave_count = (int*)(base + list_bytes + acc_bytes);
    int* need = (int*)(base + list_bytes + acc_bytes + cnt_bytes);
    uint8_t* flag = (uint8_t*)(base + list_bytes + acc_bytes + cnt_bytes + 256);
    ctx->sweep_need = need;
    if ((rc = fill_i32(ctx, need, 1, 0, s))) return rc;
    if (out) *out = NearList{list, wave_count, flag, need, nwaves, slots, true};
    const float4* box;
    if ((rc = near_boxes(ctx, K, ctx->M, &box, s))) return rc;
    {
        ProfScope ps_(ctx, PT_SWEEP_MIXED, s);
        hipLaunchKernelGGL(k_sweep_far, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, (const float*)ctx->seg32.ptr,
                           K, (const float*)ctx->elem32.ptr, ctx->M, (float)eps2, near2, box, u, list, slots,
                           wave_count, flag, need);
    }
    {
        ProfScope ps_(ctx, PT_NEAR, s);
        hipLaunchKernelGGL(k_near_pairs, dim3(nwaves), dim3(256), 0, s, list, wave_count, slots, N, x,
                           (const double*)ctx->seg64.ptr, K, (const double*)ctx->elem64.ptr, eps2, acc);
    }
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(N, 256)), dim3(256), 0, s, u, acc, N, cbar[0], cbar[1], cbar[2]);
    hipLaunchKernelGGL(k_sweep_inline, dim3(blocks_for(N, 256)), dim3(256), 0, s, x, N, flag,
                       (const float*)ctx->seg32.ptr, (const double*)ctx->seg64.ptr, K, (const float*)ctx->elem32.ptr,
                       (const double*)ctx->elem64.ptr, ctx->M, (float)eps2, eps2, near2, cbar[0], cbar[1], cbar[2], u);
    return check_launch(ctx, "sweep_mixed");
}

}  // namespace bem
