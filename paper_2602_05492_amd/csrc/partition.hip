// partition.hip - samples grouped by subdomain (Sec. 4.1: every sample belongs to the one
// subdomain its camera ray hits first; each subdomain's LM problem uses only its samples).
// A stable counting sort by label: per-chunk label histograms (LDS), one exclusive scan in
// label-major order, and a scatter in which each chunk hands out destinations in sample
// order, so every subdomain's samples keep their original order.
#include "common.hpp"

namespace bem {

namespace {

constexpr int kChunk = 4096;        // samples per block
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

// One block: exclusive scan of cnt [D * nb] (label-major) into base; off[d] = first row of
// label d, off[D] = rows kept.  Thread t scans the contiguous chunk [t c, (t + 1) c).
__global__ void __launch_bounds__(1024) k_part_scan(const int* __restrict__ cnt, int64_t n, int D, int nb,
                                                    int64_t* __restrict__ base, int64_t* __restrict__ off)
{
    __shared__ int64_t pre[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = t * chunk < n ? t * chunk : n, hi = lo + chunk < n ? lo + chunk : n;
    int64_t c = 0;
    for (int64_t k = lo; k < hi; ++k) c += cnt[k];
    pre[t] = c;
    __syncthreads();
    for (int s = 1; s < 1024; s <<= 1) {
        const int64_t v = t >= s ? pre[t - s] : 0;
        __syncthreads();
        pre[t] += v;
        __syncthreads();
    }
    int64_t run = pre[t] - c;
    for (int64_t k = lo; k < hi; ++k) {
        base[k] = run;
        run += cnt[k];
    }
    __syncthreads();
    for (int d = t; d < D; d += 1024) off[d] = base[(size_t)d * nb];
    if (t == 1023) off[D] = pre[1023];
}

// Scatter of block b's chunk: 256 samples per round; a sample's destination is its label's
// running position plus the number of earlier samples of the round with the same label.
__global__ void __launch_bounds__(256) k_part_scatter(const int32_t* __restrict__ labels, int64_t N, int D, int nb,
                                                      const int64_t* __restrict__ base, const double* __restrict__ x,
                                                      const double* __restrict__ T, double* __restrict__ xo,
                                                      double* __restrict__ To)
{
    __shared__ int64_t cur[kMaxLabels];
    __shared__ int lab[256];
    const int t = threadIdx.x;
    for (int d = t; d < D; d += 256) cur[d] = base[(size_t)d * nb + blockIdx.x];
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
    // tmp5: cnt [D * nb] int | base [D * nb] int64 | off [D + 1] int64
    const size_t cnt_bytes = ((size_t)n * sizeof(int) + 255) / 256 * 256;
    if ((rc = ensure(ctx, ctx->tmp5, cnt_bytes + (size_t)(n + D + 1) * sizeof(int64_t), s))) return rc;
    int* cnt = (int*)ctx->tmp5.ptr;
    int64_t* base = (int64_t*)((char*)ctx->tmp5.ptr + cnt_bytes);
    int64_t* off = base + n;
    if (N > 0) {
        hipLaunchKernelGGL(k_part_hist, dim3(nb), dim3(256), 0, s, labels, N, D, nb, cnt);
    } else {
        hipLaunchKernelGGL(k_part_hist, dim3(1), dim3(256), 0, s, labels, (int64_t)0, D, nb, cnt);
    }
    hipLaunchKernelGGL(k_part_scan, dim3(1), dim3(1024), 0, s, (const int*)cnt, n, D, nb, base, off);
    if (N > 0)
        hipLaunchKernelGGL(k_part_scatter, dim3(nb), dim3(256), 0, s, labels, N, D, nb, (const int64_t*)base, x, T, xo,
                           To);
    if ((rc = check_launch(ctx, "partition"))) return rc;
    if (hipMemcpyAsync(off_host, off, (size_t)(D + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(ctx, BEM_EHIP, "partition readback");
    return BEM_OK;
}

}  // namespace bem
