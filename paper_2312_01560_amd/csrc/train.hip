// Training kernels: relaxed modularity loss on softmax assignments and the
// adjoint of the GCN layer (Eq. 6 with trainable W^(k); the paper keeps W
// random, Sec. III-B).
//   loss = -tr(S^T B S) / 2e,  S = softmax_rows(U),  B = A - d d^T / 2e
//   dloss/dS = -(B S)/e;  softmax: G_U = S o (G_S - rowsum(G_S o S))
//   hidden layer (Zh = tanh(U)/||tanh(U)||): G_Z = (G_Zh - Zh (Zh.G_Zh))/||Z||,
//                 G_U = G_Z o (1 - Z^2)
//   G_W = P^T G_U (MFMA, split over rows, partials combined in fixed order)
#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace raft {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// S = softmax_rows(U), one wave per row.
__global__ __launch_bounds__(256) void k_softmax_rows(const float* __restrict__ U, float* __restrict__ S,
                                                      int n, int K) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (row >= n) return;
    const float* u = U + (size_t)row * K;
    float m = -INFINITY;
    for (int c = lane; c < K; c += kWave) m = fmaxf(m, u[c]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    float s = 0.f;
    for (int c = lane; c < K; c += kWave) s += expf(u[c] - m);
    s = wave_sum(s);
    const float inv = 1.0f / s;
    for (int c = lane; c < K; c += kWave) S[(size_t)row * K + c] = expf(u[c] - m) * inv;
}

// FP64 partials of sum_i S_i . BS_i per work-group (fixed row blocks).
__global__ __launch_bounds__(256) void k_rowdot_part(const float* __restrict__ S,
                                                     const float* __restrict__ BS, int64_t total,
                                                     double* __restrict__ part) {
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = std::min<int64_t>(total, i0 + per);
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
        acc += (double)S[i] * (double)BS[i];
    acc = wave_sum(acc);
    __shared__ double w[4];
    if ((threadIdx.x & (kWave - 1)) == 0) w[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((w[0] + w[1]) + w[2]) + w[3];
}

__global__ void k_loss_finish(const double* __restrict__ part, int parts, double m2,
                              double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < parts; ++b) t += part[b];
    *loss = -t / m2;
}

// G_U = scale * S o (G_S - rowsum(G_S o S)),  G_S = -BS / e.  One wave per row.
__global__ __launch_bounds__(256) void k_modloss_grad(const float* __restrict__ S,
                                                      const float* __restrict__ BS, int n, int K,
                                                      double inv_e, const float* __restrict__ scale,
                                                      float* __restrict__ GU) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (row >= n) return;
    const float sc = scale ? *scale : 1.0f;
    const float ie = (float)inv_e;
    const float* s = S + (size_t)row * K;
    const float* b = BS + (size_t)row * K;
    float dot = 0.f;
    for (int c = lane; c < K; c += kWave) dot += (-b[c] * ie) * s[c];
    dot = wave_sum(dot);
    for (int c = lane; c < K; c += kWave)
        GU[(size_t)row * K + c] = sc * s[c] * ((-b[c] * ie) - dot);
}

// Hidden layer backward through the row normalisation and tanh:
// U (pre-activation, recomputed) and G (gradient w.r.t. the normalised
// output) -> G_U, written over G.  One wave per row.
__global__ __launch_bounds__(256) void k_tanh_norm_backward(const float* __restrict__ U,
                                                            float* __restrict__ G, int n, int L) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (row >= n) return;
    const float* u = U + (size_t)row * L;
    float* gr = G + (size_t)row * L;
    float ss = 0.f;
    for (int c = lane; c < L; c += kWave) {
        const float z = tanhf(u[c]);
        ss += z * z;
    }
    ss = wave_sum(ss);
    const float nrm = fmaxf(sqrtf(ss), 1e-12f);
    const float inv = 1.0f / nrm;
    float dot = 0.f;
    for (int c = lane; c < L; c += kWave) dot += tanhf(u[c]) * inv * gr[c];
    dot = wave_sum(dot);
    for (int c = lane; c < L; c += kWave) {
        const float z = tanhf(u[c]);
        const float gz = (gr[c] - z * inv * dot) * inv;
        gr[c] = gz * (1.0f - z * z);
    }
}

// W^T (rows x cols -> cols x rows).
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ W, int rows, int cols,
                                                   float* __restrict__ WT) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int r = idx / cols, c = idx - (idx / cols) * cols;
    WT[(size_t)c * rows + r] = W[idx];
}

// G_W partial = P^T G_U over one block of rows (MFMA 16x16x4: M = input
// feature, N = output feature, K = rows).  Each wave sums its share of the
// block's rows; the 4 waves are combined in LDS in order.  part: [grid x LI x LO].
template <int LI, int LO>
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ P,
                                               const float* __restrict__ GU, int n,
                                               int rows_per_block, float* __restrict__ part) {
    constexpr int MB = LI / 16, NB = LO / 16;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int g = lane >> 4, li = lane & 15;
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    floatx4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int rb = r0 + wid * 4; rb < r1; rb += 16) {
        const int row = rb + g;
        const bool ok = row < r1;
        float a[MB], b[NB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a[mb] = ok ? P[(size_t)row * LI + mb * 16 + li] : 0.f;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[nb] = ok ? GU[(size_t)row * LO + nb * 16 + li] : 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
    extern __shared__ float red[];   // [4][LI*LO]
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = mb * 16 + 4 * g + v, c = nb * 16 + li;
                red[(size_t)wid * LI * LO + m * LO + c] = acc[mb][nb][v];
            }
    __syncthreads();
    for (int idx = threadIdx.x; idx < LI * LO; idx += blockDim.x) {
        const float s = ((red[idx] + red[LI * LO + idx]) + red[2 * LI * LO + idx]) + red[3 * LI * LO + idx];
        part[(size_t)blockIdx.x * LI * LO + idx] = s;
    }
}

__global__ __launch_bounds__(256) void k_wgrad_finish(const float* __restrict__ part, int parts,
                                                      int total, float* __restrict__ GW) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    double s = 0.0;
    for (int b = 0; b < parts; ++b) s += (double)part[(size_t)b * total + idx];
    GW[idx] = (float)s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
void launch_softmax_rows(const float* U, float* S, int n, int K, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_softmax_rows, dim3((unsigned)(((int64_t)n * kWave + 255) / 256)), dim3(256),
                       0, st, U, S, n, K);
}

int rowdot_parts(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (total + 4095) / 4096));
}

void launch_modloss_value(const float* S, const float* BS, int64_t total, double m2, double* part,
                          double* loss, hipStream_t st) {
    const int parts = rowdot_parts(total);
    hipLaunchKernelGGL(k_rowdot_part, dim3(parts), dim3(256), 0, st, S, BS, total, part);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(64), 0, st, part, parts, m2, loss);
}

void launch_modloss_grad(const float* S, const float* BS, int n, int K, double inv_e,
                         const float* scale, float* GU, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_modloss_grad, dim3((unsigned)(((int64_t)n * kWave + 255) / 256)), dim3(256),
                       0, st, S, BS, n, K, inv_e, scale, GU);
}

void launch_tanh_norm_backward(const float* U, float* G, int n, int L, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_tanh_norm_backward, dim3((unsigned)(((int64_t)n * kWave + 255) / 256)),
                       dim3(256), 0, st, U, G, n, L);
}

void launch_transpose(const float* W, int rows, int cols, float* WT, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose, dim3((rows * cols + 255) / 256), dim3(256), 0, st, W, rows, cols, WT);
}

int wgrad_parts(int n) { return std::max(1, std::min(1024, (n + 1023) / 1024)); }

bool wgrad_supported(int li, int lo) {
    return (li == 16 || li == 32 || li == 64 || li == 128) && (lo == 16 || lo == 32 || lo == 64 || lo == 128) &&
           li * lo <= 64 * 128;
}

template <int LI, int LO>
static void wgrad2(const float* P, const float* GU, int n, float* part, float* GW, hipStream_t st) {
    const int parts = wgrad_parts(n);
    const int rpb = (n + parts - 1) / parts;
    const size_t lds = (size_t)4 * LI * LO * sizeof(float);
    static std::once_flag attr_once;   // contexts may launch from several host threads
    std::call_once(attr_once, [&] {
        (void)hipFuncSetAttribute((const void*)k_wgrad<LI, LO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    });
    hipLaunchKernelGGL((k_wgrad<LI, LO>), dim3(parts), dim3(256), lds, st, P, GU, n, rpb, part);
    hipLaunchKernelGGL(k_wgrad_finish, dim3((LI * LO + 255) / 256), dim3(256), 0, st, part, parts,
                       LI * LO, GW);
}

template <int LI>
static void wgrad1(const float* P, const float* GU, int n, int lo, float* part, float* GW,
                   hipStream_t st) {
    switch (lo) {
        case 16: wgrad2<LI, 16>(P, GU, n, part, GW, st); break;
        case 32: wgrad2<LI, 32>(P, GU, n, part, GW, st); break;
        case 64: wgrad2<LI, 64>(P, GU, n, part, GW, st); break;
        case 128: if constexpr (LI <= 64) wgrad2<LI, 128>(P, GU, n, part, GW, st); break;
        default: break;
    }
}

void launch_wgrad(const float* P, const float* GU, int n, int li, int lo, float* part, float* GW,
                  hipStream_t st) {
    if (!n) return;
    switch (li) {
        case 16: wgrad1<16>(P, GU, n, lo, part, GW, st); break;
        case 32: wgrad1<32>(P, GU, n, lo, part, GW, st); break;
        case 64: wgrad1<64>(P, GU, n, lo, part, GW, st); break;
        case 128: wgrad1<128>(P, GU, n, lo, part, GW, st); break;
        default: break;
    }
}

void launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                 float b2, float eps, int step, hipStream_t st) {
    if (!n) return;
    const float c1 = 1.0f - powf(b1, (float)step);
    const float c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, m, v, g, n, lr,
                       b1, b2, eps, c1, c2);
}

}  // namespace raft
