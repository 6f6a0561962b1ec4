// Seeded Gaussian matrices: the projection matrix Theta (Sec. III-A, Eq. 5,
// entries with spread L^-1/2) and the random GCN weights (Sec. III-B).
// Philox4x64-10 with key (seed, stream), counter (row, col_block, 0, 0); the
// four words give two Box-Muller pairs for columns 4*col_block .. +3; the
// value is FP32(sigma * z), round to nearest even.
#include "kernels.h"

namespace raft {

__device__ __forceinline__ void gaussian_body(uint64_t seed, uint64_t stream, int64_t rows,
                                              int64_t cols, int64_t cblocks, double sigma,
                                              float* __restrict__ out, int64_t idx) {
    if (idx >= rows * cblocks) return;
    const int64_t row = idx / cblocks;
    const int64_t cb = idx - row * cblocks;
    const U64x4 b = philox4x64_10((uint64_t)row, (uint64_t)cb, 0, 0, seed, stream);
    double z[4];
    box_muller(uniform52(b.v[0]), uniform52(b.v[1]), &z[0], &z[1]);
    box_muller(uniform52(b.v[2]), uniform52(b.v[3]), &z[2], &z[3]);
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        double p;
        {
#pragma clang fp contract(off)
            p = sigma * z[t];
        }
        v[t] = (float)p;
    }
    const int64_t c0 = cb * 4;
    float* o = out + row * cols + c0;
    if (c0 + 4 <= cols && (cols % 4) == 0) {
        *reinterpret_cast<float4*>(o) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        for (int t = 0; t < 4 && c0 + t < cols; ++t) o[t] = v[t];
    }
}

__global__ __launch_bounds__(256) void k_gaussian(uint64_t seed, uint64_t stream, int64_t rows,
                                                  int64_t cols, int64_t cblocks, double sigma,
                                                  float* __restrict__ out) {
    gaussian_body(seed, stream, rows, cols, cblocks, sigma, out,
                  (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_gaussian_b(const GaussItem* __restrict__ items,
                                                    BatchTable t) {
    int g;
    Wg w;
    if (!batch_find(t, g, w)) return;
    const GaussItem it = items[g];
    const int64_t cb = (it.cols + 3) / 4;
    gaussian_body(it.seed, it.stream, it.rows, it.cols, cb, it.sigma, it.out,
                  (int64_t)w.x * blockDim.x + threadIdx.x);
}

int gaussian_blocks(int64_t rows, int64_t cols) {
    return (int)((rows * ((cols + 3) / 4) + 255) / 256);
}

void launch_gaussian_batched(const GaussItem* items, const BatchTable& t, int grid,
                             hipStream_t st) {
    if (grid == 0) return;
    hipLaunchKernelGGL(k_gaussian_b, dim3(grid), dim3(256), 0, st, items, t);
}

void launch_gaussian(uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols, double sigma,
                     float* out, hipStream_t st) {
    const int64_t cb = (cols + 3) / 4;
    const int64_t total = rows * cb;
    if (total == 0) return;
    hipLaunchKernelGGL(k_gaussian, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, seed,
                       stream_id, rows, cols, cb, sigma, out);
}

}  // namespace raft
