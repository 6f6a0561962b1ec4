// Contingency counts of two labelings (the joint histogram behind the
// normalised mutual information used to compare partitions): for labels
// a, b of n nodes, counts[r * kb + c] = #{i : a_i = r, b_i = c}, int64.
// Integer counting is exact and order-free, so the result does not depend on
// how the nodes are split across work-groups.
//
// Small tables (ka * kb <= kConfLdsBins): each work-group histograms its
// share of the nodes into int32 LDS bins (a work-group sees far fewer than
// 2^31 nodes), then adds its non-zero bins to the int64 table with one
// atomic each.  Larger tables take one int64 atomic per node.
#include <algorithm>

#include "kernels.h"

namespace raft {

constexpr int kConfLdsBins = 16384;   // 64 KB of int32 bins

__global__ __launch_bounds__(256) void k_fill_i64(int64_t* __restrict__ p, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_confusion_lds(const int32_t* __restrict__ a,
                                                       const int32_t* __restrict__ b, int64_t n,
                                                       int ka, int kb,
                                                       unsigned long long* __restrict__ counts,
                                                       int32_t* __restrict__ status) {
    extern __shared__ int bins[];
    const int nb = ka * kb;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) bins[t] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int r = a[i], c = b[i];
        if (r < 0 || r >= ka || c < 0 || c >= kb) {
            bad = true;
            continue;
        }
        atomicAdd(&bins[r * kb + c], 1);
    }
    if (bad) atomicOr(status, kStatusLabel);
    __syncthreads();
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
        const int v = bins[t];
        if (v) atomicAdd(&counts[t], (unsigned long long)v);
    }
}

__global__ __launch_bounds__(256) void k_confusion_global(const int32_t* __restrict__ a,
                                                          const int32_t* __restrict__ b,
                                                          int64_t n, int ka, int kb,
                                                          unsigned long long* __restrict__ counts,
                                                          int32_t* __restrict__ status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int r = a[i], c = b[i];
        if (r < 0 || r >= ka || c < 0 || c >= kb) {
            bad = true;
            continue;
        }
        atomicAdd(&counts[(size_t)r * kb + c], 1ull);
    }
    if (bad) atomicOr(status, kStatusLabel);
}

void launch_confusion(const int32_t* a, const int32_t* b, int64_t n, int ka, int kb,
                      int64_t* counts, int32_t* status, int num_cu, hipStream_t st) {
    const int64_t bins = (int64_t)ka * kb;
    {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((bins + 255) / 256, 1024));
        hipLaunchKernelGGL(k_fill_i64, dim3(grid), dim3(256), 0, st, counts, bins);
    }
    if (n == 0) return;
    unsigned long long* c = reinterpret_cast<unsigned long long*>(counts);
    if (bins <= kConfLdsBins) {
        // enough nodes per work-group that the bin flush stays small
        const int64_t per = std::max<int64_t>(4096, 8 * bins);
        const int grid = (int)std::max<int64_t>(
            1, std::min<int64_t>((n + per - 1) / per, (int64_t)num_cu * 4));
        hipLaunchKernelGGL(k_confusion_lds, dim3(grid), dim3(256), (size_t)bins * sizeof(int), st,
                           a, b, n, ka, kb, c, status);
    } else {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256,
                                                                      (int64_t)num_cu * 8));
        hipLaunchKernelGGL(k_confusion_global, dim3(grid), dim3(256), 0, st, a, b, n, ka, kb, c,
                           status);
    }
}

}  // namespace raft
