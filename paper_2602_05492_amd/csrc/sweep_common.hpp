// sweep_common.hpp - geometry of the outer boundary and layout constants
// shared by the kernels of the forward, adjoint and normal-equation paths.
#pragma once

#include "common.hpp"

namespace bem {

// Sums kept per handle segment by the adjoint: d/da (2), d/db (2) of the
// cotangent-weighted handle term, and sum_x gbar_c M_m for the four moments
// m = Md_a, Md_b, Ms_a, Ms_b and three channels c (12).
constexpr int kSegVjpVals = 16;

// Element i of the counter-clockwise unit square with m elements per side.
__device__ inline void square_element(int i, int m, double& ax, double& ay, double& bx, double& by)
{
    const int side = i / m, k = i % m;
    const double t0 = (double)k / (double)m, t1 = (double)(k + 1) / (double)m;
    const double cx0 = (side == 1 || side == 2) ? 1.0 : 0.0;
    const double cy0 = (side >= 2) ? 1.0 : 0.0;
    const double dx = side == 0 ? 1.0 : (side == 2 ? -1.0 : 0.0);
    const double dy = side == 1 ? 1.0 : (side == 3 ? -1.0 : 0.0);
    ax = cx0 + t0 * dx; ay = cy0 + t0 * dy;
    bx = cx0 + t1 * dx; by = cy0 + t1 * dy;
}

// Outer element i of the element table eg [M][4] (a x, a y, b x, b y).
__device__ inline void load_element(const double* eg, int i, double& ax, double& ay, double& bx, double& by)
{
    const double* e = eg + 4 * (size_t)i;
    ax = e[0];
    ay = e[1];
    bx = e[2];
    by = e[3];
}

// ---- near-singular pairs of the mixed-precision sweeps ---------------------------
// A pair is near when both end points of the segment lie within rho*L of the
// sample, rho = near_radius(near_factor).  A sample at distance d < nf*L from the
// segment is within d + L < (nf + 1)*L of either end point, so rho = max(2 nf,
// nf + 1) makes the near set contain every sample closer than nf*L to the
// segment (for nf >= 1 the radius is 2 nf*L).  The test is written with explicit
// roundings so that every kernel that classifies a pair takes the same decision.
inline double near_radius(double nf) { return nf >= 1.0 ? 2.0 * nf : nf + 1.0; }

__device__ inline bool near_segment(float ax, float ay, float bx, float by, float L2, float X, float Y, float near2)
{
    const float dx = __fsub_rn(ax, X), dy = __fsub_rn(ay, Y), ex = __fsub_rn(bx, X), ey = __fsub_rn(by, Y);
    const float lim = __fmul_rn(near2, L2);
    const float dd = __fmaf_rn(dx, dx, __fmul_rn(dy, dy));
    const float ee = __fmaf_rn(ex, ex, __fmul_rn(ey, ey));
    return (dd < lim) & (ee < lim);
}
// Outer element stored as start point a and direction v.
__device__ inline bool near_element(float ax, float ay, float vx, float vy, float X, float Y, float near2)
{
    const float dx = __fsub_rn(ax, X), dy = __fsub_rn(ay, Y);
    const float ex = __fadd_rn(dx, vx), ey = __fadd_rn(dy, vy);
    const float lim = __fmul_rn(near2, __fmaf_rn(vx, vx, __fmul_rn(vy, vy)));
    const float dd = __fmaf_rn(dx, dx, __fmul_rn(dy, dy));
    const float ee = __fmaf_rn(ex, ex, __fmul_rn(ey, ey));
    return (dd < lim) & (ee < lim);
}

// Culling of near-pair tests: a box per group of kBoxGroup consecutive segments (and of outer
// elements), k_near_boxes.  A wavefront whose samples all lie farther from a group's box than the
// group's largest near radius can skip the group's near tests: no pair in it is near.
constexpr int kBoxGroup = 32;

// True when no sample of the wavefront's box [wx0, wx1] x [wy0, wy1] can be near a member of box g:
// the boxes' distance exceeds the members' largest near radius by a margin far above the float32
// rounding of the exact test (a pair is near only if both of its end points lie within the radius).
__device__ inline bool box_culled(const float4* __restrict__ box, int g, float wx0, float wy0, float wx1, float wy1)
{
    const float4 b = box[2 * g];
    const float r = box[2 * g + 1].x * 1.001f + 1e-6f;
    const float dx = fmaxf(0.0f, fmaxf(b.x - wx1, wx0 - b.z));
    const float dy = fmaxf(0.0f, fmaxf(b.y - wy1, wy0 - b.w));
    return !(b.x <= b.z) || dx * dx + dy * dy > r * r;      // empty box, or too far
}

__device__ inline float wave_min(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
// a value equal in every lane of the wavefront, held in a scalar register
__device__ inline float uniform_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

struct NearPair {
    int32_t sample;   // index within the launch's sample range
    int32_t seg;      // < K: handle segment, else outer element seg - K
};

// Each wavefront of 64 consecutive samples owns a slice of `slots` list slots (a
// multiple of 256; the context's capacity, bem_ctx::near_slots); entries are
// appended in increasing segment order, so the entries of one handle form a
// contiguous run of a slice.  A wavefront whose near pairs do not fit records its
// count in *need (atomic maximum), from which lm_step raises the capacity.
constexpr int kWaveSlotsMin = 16 * 64;
constexpr int kWaveSlotsMax = 256 * 64;
constexpr size_t kNearListMaxBytes = (size_t)1 << 32;

// Workspace of one classification: slices, per-wavefront counts, per-sample
// overflow flags, the largest overflowing count.
struct NearList {
    NearPair* list = nullptr;
    int* count = nullptr;
    uint8_t* flag = nullptr;
    int* need = nullptr;
    int64_t nwaves = 0;
    int slots = kWaveSlotsMin;
    bool overflowed = true;     // false only once a readback of *need has shown that no slice overflowed
};

// Capacity for wavefronts of `need` near pairs over nwaves wavefronts: need rounded up to
// 256, within [kWaveSlotsMin, kWaveSlotsMax] and a list of at most kNearListMaxBytes.
inline int near_slots_for(int need, int64_t nwaves)
{
    int64_t cap = nwaves > 0 ? (int64_t)(kNearListMaxBytes / ((size_t)nwaves * sizeof(NearPair))) : kWaveSlotsMax;
    cap = cap < kWaveSlotsMax ? cap & ~(int64_t)255 : kWaveSlotsMax;
    if (cap < kWaveSlotsMin) cap = kWaveSlotsMin;
    const int64_t want = ((int64_t)need + 255) / 256 * 256;
    return (int)(want < cap ? (want > kWaveSlotsMin ? want : kWaveSlotsMin) : cap);
}

}  // namespace bem
