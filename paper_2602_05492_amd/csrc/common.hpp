// common.hpp - context, workspaces and launch helpers shared by the library's
// translation units.  Not part of the public ABI (see include/bem.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/bem.h"
#include "seg_math.hpp"

namespace bem {

// ---- device math policies ---------------------------------------------------
struct DevF64 {
    __device__ static double log(double x) { return ::log(x); }
    __device__ static double log1p(double x) { return ::log1p(x); }
    __device__ static double sqrt(double x) { return ::sqrt(x); }
    __device__ static double rcp(double x) { return 1.0 / x; }
    __device__ static double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    __device__ static double atan2(double y, double x) { return ::atan2(y, x); }
};

// Segments no longer than this (domain-width units) are degenerate: their
// integral is below ~1e-11 for the regularised kernels and the derivative
// with respect to their end points has no limit as the length goes to 0, so
// they contribute nothing (an expansion of a zero-length handle carries
// rounding-level lengths of ~1e-16).
constexpr double kDegenerateLength = 1e-12;

// ---- layouts ----------------------------------------------------------------
// Segment record: SegGeom (9 values) + wd_a, wd_b, wc_a, wc_b RGB (12) + 1/L2 = 22, padded.
constexpr int kSegStride = 24;
// Element record: ax, ay, vx, vy, U0, U1, U2, pad.
constexpr int kElemStride = 8;

// density offsets inside a segment record, and the slot of 1/L2
constexpr int kWdA = 9, kWdB = 12, kWcA = 15, kWcB = 18, kIL2 = 21;

template <class T>
__device__ inline SegGeom<T> load_geom(const T* __restrict__ s)
{
    SegGeom<T> g;
    g.ax = s[0]; g.ay = s[1]; g.bx = s[2]; g.by = s[3];
    g.vx = s[4]; g.vy = s[5]; g.L2 = s[6]; g.kd = s[7]; g.ks = s[8]; g.iL2 = s[kIL2];
    return g;
}

// ---- device buffers -----------------------------------------------------------
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace bem

namespace bem {
// Kernel families timed with HIP events when profiling is on (bem_profile).
enum ProfTag {
    PT_SWEEP_F64 = 0, PT_SWEEP_MIXED, PT_VJP_SEGMENTS, PT_VJP_ELEMENTS, PT_FEATURES, PT_BETA_ROWS, PT_GRAM_F64,
    PT_GRAM_MFMA, PT_XR, PT_CHOLESKY, PT_BOUNDARY, PT_NEAR, PT_COUNT
};
struct ProfState {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> tags;
    std::vector<hipEvent_t> starts, stops;
    double total_ms[PT_COUNT] = {};
    int64_t launches[PT_COUNT] = {};
};
}  // namespace bem

struct bem_ctx {
    bem_opts opts{};
    int M = 0;               // outer elements
    int per_side = 0;
    int state = 0;           // 0 empty, 1 built, 2 factored
    int device = 0;
    // handle parametrisation: parameters per handle, and per handle in a feature row of the
    // normal equations the geometry columns of one channel and the channel-shared colour columns
    int model = 0, npar = 20, ngeo = 8, ncol = 4;
    bem_reg reg{};           // regularisation terms of lm_step (all off by default)
    int64_t chol_P = -1;     // order of the last Cholesky factor (its inverted diagonal blocks are in cholw)
    // second stream (the Gram of a sample tile runs on it while the next tile's feature rows are
    // formed on the caller's stream; the Cholesky's panel and trailing update run on it beside the
    // diagonal blocks) and its events, created on first use
    hipStream_t s2 = nullptr;
    hipEvent_t ev[7] = {};
    // near-pair slots per wavefront of the mixed-precision sweeps (a multiple of 256, raised by
    // lm_step when a wavefront's near pairs overflow it), and the device word in which the last
    // mixed forward sweep left its largest overflowing count (0: none overflowed)
    int near_slots = 1024;
    int* sweep_need = nullptr;
    double bbox[4] = {0.0, 0.0, 1.0, 1.0};   // outer boundary's bounding box (x0, y0, x1, y1)
    double sigma_n = 0.0, shift = 0.0;
    std::string err;
    bem::ProfState prof;
    // one-time boundary system
    bem::DevBuf A, Apinv, LU, piv, un, vn, flag, scal, egeo;   // egeo: outer elements [M][4] (a, b)
    // per-call workspaces
    bem::DevBuf seg64, seg32, F, U, elem64, elem32, red, tmp0, tmp1, tmp2, tmp3, tmp4, tmp5, lmw, nearw, nearv, nearf, regw, cholw, sortw,
        boxw;
    // Gram work list of the normal equations on the device, uploaded once per (W, H, handle
    // model, Gram arithmetic) and kept, so that later calls enqueue without a host synchronisation
    bem::DevBuf tilew;
    int64_t tiles_key[4] = {-1, -1, -1, -1};
};

namespace bem {

int set_error(bem_ctx* ctx, int code, const char* fmt, ...);
void prof_begin(bem_ctx* ctx, int tag, hipStream_t s, hipEvent_t* start);
void prof_end(bem_ctx* ctx, int tag, hipStream_t s, hipEvent_t start);

// Records HIP events around the launches of its scope when profiling is on.
struct ProfScope {
    bem_ctx* ctx;
    int tag;
    hipStream_t s;
    hipEvent_t start = nullptr;
    ProfScope(bem_ctx* c, int t, hipStream_t st) : ctx(c), tag(t), s(st) { prof_begin(ctx, tag, s, &start); }
    ~ProfScope() { prof_end(ctx, tag, s, start); }
};
int ensure(bem_ctx* ctx, DevBuf& b, size_t bytes, hipStream_t stream);
// argument checks shared by the per-call entry points; makes the context's device current
int check_common(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N);
int aux_stream(bem_ctx* ctx, hipStream_t* out);
int check_launch(bem_ctx* ctx, const char* what);

inline int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

// ---- kernels' host launchers (defined in the .hip files) ----------------------
// factor.hip
int launch_square_elements(bem_ctx* ctx, hipStream_t s);
int launch_assemble(bem_ctx* ctx, hipStream_t s);
int launch_factor(bem_ctx* ctx, hipStream_t s);
// forward.hip
int launch_expand(bem_ctx* ctx, const double* theta, int H, hipStream_t s);
int launch_expand_into(bem_ctx* ctx, const double* theta, int H, double* seg64, float* seg32, hipStream_t s);
int launch_boundary_rhs(bem_ctx* ctx, int K, double* F, bool mixed, hipStream_t s);
int launch_boundary_solve(bem_ctx* ctx, const double* F, double* U, bool transpose, hipStream_t s);
int launch_pack_elements(bem_ctx* ctx, const double* U, hipStream_t s);
int launch_pack_elements_into(bem_ctx* ctx, const double* U, double* el64, float* el32, hipStream_t s);
int launch_sweep_f64(bem_ctx* ctx, const double* x, int64_t N, int K, const double* cbar_host, double* u, hipStream_t s);
// The mixed sweeps share one near-pair list layout (sweep_common.hpp).  The
// forward sweep returns the list it built (valid until the next mixed sweep);
// the adjoint and the normal equations take such a list for the same samples
// and parameters, or classify the samples themselves when given none.
struct NearList;
int launch_sweep_mixed(bem_ctx* ctx, const double* x, int64_t N, int K, const double* cbar_host, float* u, hipStream_t s,
                       NearList* out = nullptr);
int near_classify(bem_ctx* ctx, DevBuf& buf, const double* x, int64_t N, int K, int M, NearList* out, hipStream_t s);
// culling boxes of the current segment table (groups of kBoxGroup segments, then of M outer
// elements) into the context's box buffer
int near_boxes(bem_ctx* ctx, int K, int M, const float4** box, hipStream_t s);
// partition.hip (off_host may be null: no readback and no host synchronisation)
int run_partition(bem_ctx* ctx, const int32_t* labels, int64_t N, int D, const double* x, const double* T, double* xo,
                  double* To, int64_t* off_host, hipStream_t s);
// lm.hip: samples and float32 cotangents reordered cell by cell into the sort workspace
int cell_order_f32(bem_ctx* ctx, const double* x, const float* g, int64_t N, const double** xo, const float** go,
                   hipStream_t s);
// reg.hip
bool reg_active(const bem_ctx* ctx);
int check_reg(const bem_reg& r, char* why, size_t n);
int reg_terms(bem_ctx* ctx, const double* theta, int H, bool choose, double* g, double* Hm, double* value, int* pairs,
              hipStream_t s);
int run_prune(bem_ctx* ctx, double* theta, int H, double thr, int* H_out, hipStream_t s);
// vjp.hip
// Device memory the float64 adjoint may carve every workspace from instead of allocating (the
// allocation-free entry point's static array); null: the context's workspaces.
struct Carve {
    char* base;
    size_t bytes;
};
int run_vjp(bem_ctx* ctx, const double* theta, int H, const double* x, int64_t N, const void* gbar, bool mixed,
            double* grad, hipStream_t s, const NearList* pre = nullptr, const Carve* carve = nullptr);
// api.hip: expand + element tables (no boundary solve); and the whole forward set-up
// (expand, boundary right-hand side (float32 far pairs when mixed), boundary solve, element tables)
int prepare_forward_tables(bem_ctx* ctx, const double* theta, int H, hipStream_t s);
int prepare_forward(bem_ctx* ctx, const double* theta, int H, bool mixed, hipStream_t s);
// gemm.hip
// plain products and the float64 Gram on float64 MFMA; valu selects the VALU kernel (Gram mode FP64_VALU)
int gemm_f64(bem_ctx* ctx, int m, int n, int k, double alpha, const double* A, int64_t lda, bool ta, const double* B,
             int64_t ldb, bool tb, double beta, double* C, int64_t ldc, hipStream_t s, const int* tiles, int ntiles,
             bool valu = false);
// jtj.hip
int fill_f64(bem_ctx* ctx, double* p, int64_t n, double v, hipStream_t s);
int run_jtj(bem_ctx* ctx, const double* theta, int H, const double* x, int64_t N, const void* resid, bool mixed,
            int gram, double* JtJ, double* Jtr, hipStream_t s, const NearList* pre = nullptr, double norm = 0.0);
int run_jacobian(bem_ctx* ctx, const double* theta, int H, const double* x, int64_t N, double* J, hipStream_t s);
// gram_mfma.hip
int launch_gram_mfma(bem_ctx* ctx, int gram, const void* Xhi, const uint16_t* Xlo, int64_t ld, int W, int64_t n,
                     const int* work, int nwork, int64_t kchunk, double* G, int64_t gstride, bool accumulate,
                     hipStream_t s);
int launch_xr(bem_ctx* ctx, int gram, const void* Xhi, const uint16_t* Xlo, int64_t ld, int W, int64_t n,
              const double* r, double* R, double* Rp, hipStream_t s, int f0 = 0);
constexpr int kXrPartials = 32;   // sample-block groups of the split-BF16 X r (workspace kXrPartials * W * 3)
// chol.hip
int chol_factor(bem_ctx* ctx, const double* H, int64_t P, double lam, double* A, int* dflag, double* dscal,
                hipStream_t s);
int chol_solve(bem_ctx* ctx, const double* A, int64_t P, double* B, int nrhs, hipStream_t s);
// lm.hip
int fill_i32(bem_ctx* ctx, int* p, int64_t n, int v, hipStream_t s);
int run_lm_step(bem_ctx* ctx, double* theta, int H, const double* x, int64_t N, const double* T, bem_lm_state* st,
                int gram, bool mixed, hipStream_t s);

}  // namespace bem

namespace bem {
// float32 policy of the mixed sweeps: hardware log2, reciprocal, reciprocal
// square root and square root (about 1 ulp); log1p(z) = log(w) z / (w - 1) with
// w = 1 + z rounded (Goldberg 1991: the rounding error of w cancels between the
// two factors), z itself when w == 1; atan2 by reduction to [0, 1] and a
// degree-7 odd minimax polynomial in z (relative error 1e-7; coefficients from
// csrc/fit_atan.py), reflected about pi/4 and pi/2.
struct DevF32 {
    // v_log_f32 (log2, ~1 ulp) times ln 2; arguments here are normal numbers (>= eps^2 or near 1)
    __device__ static float log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
    __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    __device__ static float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static float log1p(float z)
    {
        const float w = 1.0f + z;
        const float d = w - 1.0f;
        return d == 0.0f ? z : (__builtin_amdgcn_logf(w) * 0.693147180559945309f) * (z * __builtin_amdgcn_rcpf(d));
    }
    __device__ static float atan2(float y, float x)
    {
        const float ax = fabsf(x), ay = fabsf(y);
        const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
        const float z = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
        const float s = z * z;
        float p = -4.693678257e-03f;
        p = p * s + 2.425393176e-02f;
        p = p * s - 5.948871678e-02f;
        p = p * s + 9.914472679e-02f;
        p = p * s - 1.401955544e-01f;
        p = p * s + 1.996973974e-01f;
        p = p * s - 3.333199223e-01f;
        p = p * s + 9.999999014e-01f;
        float r = z * p;
        r = ay > ax ? 1.57079632679489662f - r : r;
        r = x < 0.0f ? 3.14159265358979324f - r : r;
        return __builtin_copysignf(r, y);
    }
};
}  // namespace bem
