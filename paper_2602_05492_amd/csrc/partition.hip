// partition.hip - samples grouped by subdomain (Sec. 4.1: every sample belongs to the one
// subdomain its camera ray hits first; each subdomain's LM problem uses only its samples).
// A stable counting sort by label: per-chunk label histograms (LDS), an exclusive scan in
// label-major order (per label, then over the label totals), and a scatter in which each
// chunk hands out destinations in sample order, so every subdomain's samples keep their
// original order.  The mixed LM step uses the same sort to visit samples cell by cell.
#include "common.hpp"

namespace bem {

namespace {

constexpr int kChunk = 1024;        // samples per block
constexpr int kMaxLabels = 1024;

__global__ void __launch_bounds__(256) k_part_hist(const int32_t* __restrict__ labels, int64_t N, int D, int nb,
                                                   int* __restrict__ cnt)
{
    __shared__ int h[kMaxLabels];
    for (int d = threadIdx.x; d < D; d += 256) h[d] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kChunk, hi = lo + kChunk < N ? lo + kChunk : N;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const int l = labels[i];
        if (l >= 0 && l < D) atomicAdd(&h[l], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < D; d += 256) cnt[(size_t)d * nb + blockIdx.x] = h[d];
}

// Exclusive scan of cnt [D * nb] (label-major) into base, in two steps.  Block d scans its
// label's nb chunk counts into base[d * nb + b] (relative to the label's first row) and writes
// the label's total; then one block scans the D totals into off[d] (first row of label d,
// off[D] = rows kept) and the scatter adds off[d] to base.
__global__ void __launch_bounds__(256) k_part_scan_label(const int* __restrict__ cnt, int nb,
                                                         int64_t* __restrict__ base, int64_t* __restrict__ total)
{
    __shared__ int64_t s[256];
    const int d = blockIdx.x, t = threadIdx.x;
    int64_t run = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + t;
        const int64_t c = b < nb ? cnt[(size_t)d * nb + b] : 0;
        s[t] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {      // inclusive scan of the 256 counts
            const int64_t v = t >= o ? s[t - o] : 0;
            __syncthreads();
            s[t] += v;
            __syncthreads();
        }
        if (b < nb) base[(size_t)d * nb + b] = run + s[t] - c;
        run += s[255];
        __syncthreads();
    }
    if (t == 0) total[d] = run;
}

__global__ void __launch_bounds__(1024) k_part_scan_totals(const int64_t* __restrict__ total, int D,
                                                           int64_t* __restrict__ off)
{
    __shared__ int64_t s[kMaxLabels];
    const int t = threadIdx.x;
    const int64_t c = t < D ? total[t] : 0;
    s[t] = c;
    __syncthreads();
    for (int o = 1; o < kMaxLabels; o <<= 1) {
        const int64_t v = t >= o ? s[t - o] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    if (t < D) off[t] = s[t] - c;
    if (t == kMaxLabels - 1) off[D] = s[t];
}

// Scatter of block b's chunk: 256 samples per round; a sample's destination is its label's
// running position plus the number of earlier samples of the round with the same label.
__global__ void __launch_bounds__(256) k_part_scatter(const int32_t* __restrict__ labels, int64_t N, int D, int nb,
                                                      const int64_t* __restrict__ base, const int64_t* __restrict__ off,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ T, double* __restrict__ xo,
                                                      double* __restrict__ To)
{
    __shared__ int64_t cur[kMaxLabels];
    __shared__ int lab[256];
    const int t = threadIdx.x;
    for (int d = t; d < D; d += 256) cur[d] = off[d] + base[(size_t)d * nb + blockIdx.x];
    const int64_t lo = (int64_t)blockIdx.x * kChunk, hi = lo + kChunk < N ? lo + kChunk : N;
    __syncthreads();
    for (int64_t r0 = lo; r0 < hi; r0 += 256) {
        const int64_t i = r0 + t;
        int l = i < hi ? labels[i] : -1;
        if (l >= D) l = -1;
        lab[t] = l < 0 ? -1 : l;
        __syncthreads();
        int rank = 0;
        bool last = true;
        if (l >= 0) {
            for (int u = 0; u < 256; ++u) {
                if (lab[u] != l) continue;
                if (u < t) ++rank;
                else if (u > t) last = false;
            }
        }
        const int64_t dest = l >= 0 ? cur[l] + rank : -1;
        __syncthreads();
        if (l >= 0 && last) cur[l] += rank + 1;
        if (dest >= 0) {
            xo[2 * dest] = x[2 * i];
            xo[2 * dest + 1] = x[2 * i + 1];
            if (T) {
                To[3 * dest] = T[3 * i];
                To[3 * dest + 1] = T[3 * i + 1];
                To[3 * dest + 2] = T[3 * i + 2];
            }
        }
        __syncthreads();
    }
}

}  // namespace

int run_partition(bem_ctx* ctx, const int32_t* labels, int64_t N, int D, const double* x, const double* T, double* xo,
                  double* To, int64_t* off_host, hipStream_t s)
{
    int rc;
    if (D < 1 || D > kMaxLabels) return set_error(ctx, BEM_EINVAL, "D = %d labels not in [1, %d]", D, kMaxLabels);
    const int nb = N > 0 ? (int)((N + kChunk - 1) / kChunk) : 1;
    const int64_t n = (int64_t)D * nb;
    // tmp5: cnt [D * nb] int | base [D * nb] int64 | off [D + 1] int64 | total [D] int64
    const size_t cnt_bytes = ((size_t)n * sizeof(int) + 255) / 256 * 256;
    if ((rc = ensure(ctx, ctx->tmp5, cnt_bytes + (size_t)(n + 2 * D + 1) * sizeof(int64_t), s))) return rc;
    int* cnt = (int*)ctx->tmp5.ptr;
    int64_t* base = (int64_t*)((char*)ctx->tmp5.ptr + cnt_bytes);
    int64_t* off = base + n;
    int64_t* total = off + D + 1;
    if (N > 0) {
        hipLaunchKernelGGL(k_part_hist, dim3(nb), dim3(256), 0, s, labels, N, D, nb, cnt);
    } else {
        hipLaunchKernelGGL(k_part_hist, dim3(1), dim3(256), 0, s, labels, (int64_t)0, D, nb, cnt);
    }
    hipLaunchKernelGGL(k_part_scan_label, dim3(D), dim3(256), 0, s, (const int*)cnt, nb, base, total);
    hipLaunchKernelGGL(k_part_scan_totals, dim3(1), dim3(kMaxLabels), 0, s, (const int64_t*)total, D, off);
    if (N > 0)
        hipLaunchKernelGGL(k_part_scatter, dim3(nb), dim3(256), 0, s, labels, N, D, nb, (const int64_t*)base,
                           (const int64_t*)off, x, T, xo, To);
    if ((rc = check_launch(ctx, "partition"))) return rc;
    if (!off_host) return BEM_OK;                // no readback (and no host synchronisation)
    if (hipMemcpyAsync(off_host, off, (size_t)(D + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "partition readback");
    return BEM_OK;
}

}  // namespace bem
