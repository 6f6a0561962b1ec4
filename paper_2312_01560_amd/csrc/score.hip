// Per-edge segmented scores of every candidate partition and the model
// selection.  For candidate k with labels a:
//   l_r   = 1/2 #{(i,j) stored in the CSR : a_i = a_j = r}   (intra edges)
//   vol_r = sum_{a_i = r} d_i
//   Mod   = sum_r ( l_r / e - (vol_r / 2e)^2 )                 (Eq. 3)
//   NCut  = 1/2 sum_{r: vol_r > 0} (vol_r - 2 l_r) / vol_r      (Eq. 1)
// Counts are integers (exact, order-free); the FP64 finish runs over r in
// ascending order without contraction.  K* is the first maximum of Mod over
// the grid; its labels are renumbered by first occurrence in node order.
//
// Edge kernel: labels are point-major bytes, row stride S (multiple of 4), so
// one uint32 load gives four candidates' labels of a node; LPR lanes cover a
// node's label row and 64/LPR edges are compared per wave step with a
// per-byte equality mask.  Counts are reduced over the edge slots by xor
// shuffles and accumulated per work-group in LDS, then written as partials.
#include <limits.h>

#include <algorithm>

#include "kernels.h"

namespace raft {

__global__ __launch_bounds__(256) void k_transpose_labels(const uint8_t* __restrict__ cm, int n,
                                                          int Kc, uint8_t* __restrict__ pm,
                                                          int S) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * S) return;
    const int i = (int)(idx / S);
    const int k = (int)(idx - (int64_t)i * S);
    pm[idx] = k < Kc ? cm[(size_t)k * n + i] : (uint8_t)0;
}

__global__ __launch_bounds__(256) void k_copy_labels(const uint8_t* __restrict__ pm, int n, int Kc,
                                                     int S, uint8_t* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * Kc) return;
    const int i = (int)(idx / Kc);
    const int k = (int)(idx - (int64_t)i * Kc);
    out[idx] = pm[(size_t)i * S + k];
}

__device__ __forceinline__ uint32_t zero_bytes_mask(uint32_t x) {
    // 0x80 in every byte of x that is zero, exact per byte
    uint32_t y = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    return ~(y | x | 0x7F7F7F7Fu);
}

template <int LPR>
__global__ __launch_bounds__(256) void k_edge_score(GraphView g, ScorePlan p,
                                                    const uint8_t* __restrict__ lab) {
    constexpr int SLOTS = kWave / LPR;
    extern __shared__ int sm[];
    int* sl = sm;
    int* sv = sm + p.SK;
    for (int idx = threadIdx.x; idx < 2 * p.SK; idx += blockDim.x) sm[idx] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int slot = lane / LPR;
    const int m = lane % LPR;
    const bool on = 4 * m < p.S;
    const int waves = gridDim.x * (blockDim.x / kWave);
    const int wave = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    for (int i = wave; i < g.n; i += waves) {
        const uint32_t li = on ? *reinterpret_cast<const uint32_t*>(lab + (size_t)i * p.S + 4 * m) : 0u;
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        const int beg = g.rp[i], end = g.rp[i + 1];
        int e = beg + slot;
        for (; e + 3 * SLOTS < end; e += 4 * SLOTS) {
            int j[4];
            uint32_t lj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) j[u] = g.ci[e + u * SLOTS];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                lj[u] = on ? *reinterpret_cast<const uint32_t*>(lab + (size_t)j[u] * p.S + 4 * m) : 1u;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t z = zero_bytes_mask(li ^ lj[u]);
                c0 += (z >> 7) & 1u;
                c1 += (z >> 15) & 1u;
                c2 += (z >> 23) & 1u;
                c3 += (z >> 31) & 1u;
            }
        }
        for (; e < end; e += SLOTS) {
            const int j = g.ci[e];
            const uint32_t lj = on ? *reinterpret_cast<const uint32_t*>(lab + (size_t)j * p.S + 4 * m) : 1u;
            const uint32_t z = zero_bytes_mask(li ^ lj);
            c0 += (z >> 7) & 1u;
            c1 += (z >> 15) & 1u;
            c2 += (z >> 23) & 1u;
            c3 += (z >> 31) & 1u;
        }
#pragma unroll
        for (int off = LPR; off < kWave; off <<= 1) {
            c0 += __shfl_xor(c0, off, kWave);
            c1 += __shfl_xor(c1, off, kWave);
            c2 += __shfl_xor(c2, off, kWave);
            c3 += __shfl_xor(c3, off, kWave);
        }
        if (slot == 0 && on) {
            const int d = end - beg;
            const int cc[4] = {c0, c1, c2, c3};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int k = 4 * m + b;
                if (k < p.Kc) {
                    const int r = (li >> (8 * b)) & 0xFF;
                    if (r >= p.ks[k]) {
                        atomicOr(p.status, kStatusLabel);
                        continue;
                    }
                    const int slotk = p.koff[k] + r;
                    if (cc[b]) atomicAdd(&sl[slotk], cc[b]);
                    if (d) atomicAdd(&sv[slotk], d);
                }
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < p.SK; idx += blockDim.x) {
        p.lpart[(size_t)blockIdx.x * p.SK + idx] = sl[idx];
        p.vpart[(size_t)blockIdx.x * p.SK + idx] = sv[idx];
    }
}

__global__ __launch_bounds__(256) void k_reduce_counts(ScorePlan p) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= p.SK) return;
    int64_t l = 0, v = 0;
    for (int b = 0; b < p.grid; ++b) {
        l += p.lpart[(size_t)b * p.SK + idx];
        v += p.vpart[(size_t)b * p.SK + idx];
    }
    p.l64[idx] = l / 2;
    p.v64[idx] = v;
}

__global__ __launch_bounds__(256) void k_score_finalize(ScorePlan p) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.Kc) return;
    const int K = p.ks[k];
    const int64_t* l = p.l64 + p.koff[k];
    const int64_t* v = p.v64 + p.koff[k];
    const double e = (double)(p.nnz / 2);
    const double m2 = (double)p.nnz;
    double mod = 0.0;
    for (int r = 0; r < K; ++r) {
        const double t = (double)v[r] / m2;
        const double term = (double)l[r] / e - t * t;
        mod = mod + term;
    }
    double nc = 0.0;
    for (int r = 0; r < K; ++r) {
        if (v[r] > 0) nc = nc + (double)(v[r] - 2 * l[r]) / (double)v[r];
    }
    p.mod[k] = mod;
    p.ncut[k] = 0.5 * nc;
}

// K* = first maximum of Mod; init first-occurrence table.
__global__ void k_select_best(ScorePlan p, int32_t* k_selected) {
    if (threadIdx.x == 0) {
        int best = 0;
        for (int j = 1; j < p.Kc; ++j)
            if (p.mod[j] > p.mod[best]) best = j;
        *p.best = best;
        k_selected[0] = p.ks[best];
        k_selected[2] = best;
    }
    for (int r = threadIdx.x; r <= RAFT_MAX_K_DEV; r += blockDim.x) p.first[r] = INT_MAX;
}

__global__ __launch_bounds__(256) void k_first_occ(ScorePlan p, const uint8_t* __restrict__ lab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const int r = lab[(size_t)i * p.S + *p.best];
    atomicMin(&p.first[r], i);
}

__global__ void k_rank(ScorePlan p, int32_t* k_selected) {
    __shared__ int keff;
    if (threadIdx.x == 0) keff = 0;
    __syncthreads();
    const int K = p.ks[*p.best];
    for (int r = threadIdx.x; r < K; r += blockDim.x) {
        const int f = p.first[r];
        if (f == INT_MAX) {
            p.remap[r] = -1;
            continue;
        }
        int rank = 0;
        for (int q = 0; q < K; ++q) rank += (p.first[q] < f);
        p.remap[r] = rank;
        atomicAdd(&keff, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) k_selected[1] = keff;
}

__global__ __launch_bounds__(256) void k_apply(ScorePlan p, const uint8_t* __restrict__ lab,
                                               int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    out[i] = p.remap[lab[(size_t)i * p.S + *p.best]];
}

int score_grid(int32_t n, int num_cu) {
    const int64_t want = ((int64_t)n + 63) / 64;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * 2));
}

bool score_supported(int SK) { return SK >= 1 && SK <= 16384; }

void launch_transpose_labels(const uint8_t* cm, int32_t n, int Kc, uint8_t* pm, int S,
                             hipStream_t st) {
    const int64_t total = (int64_t)n * S;
    if (!total) return;
    hipLaunchKernelGGL(k_transpose_labels, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       cm, n, Kc, pm, S);
}

void launch_copy_labels(const uint8_t* pm, int32_t n, int Kc, int S, uint8_t* out,
                        hipStream_t st) {
    const int64_t total = (int64_t)n * Kc;
    if (!total) return;
    hipLaunchKernelGGL(k_copy_labels, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, pm,
                       n, Kc, S, out);
}

void launch_edge_score(const GraphView& g, const ScorePlan& p, const uint8_t* lab,
                       hipStream_t st) {
    const size_t lds = (size_t)2 * p.SK * sizeof(int);
    const int words = p.S / 4;
    int lpr = 1;
    while (lpr < words) lpr <<= 1;
#define EDGE(LV)                                                                              \
    {                                                                                         \
        static bool attr = false;                                                             \
        if (!attr) {                                                                          \
            (void)hipFuncSetAttribute((const void*)k_edge_score<LV>,                          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
            attr = true;                                                                      \
        }                                                                                     \
        hipLaunchKernelGGL(k_edge_score<LV>, dim3(p.grid), dim3(256), lds, st, g, p, lab);    \
    }
    switch (lpr) {
        case 1: EDGE(1) break;
        case 2: EDGE(2) break;
        case 4: EDGE(4) break;
        case 8: EDGE(8) break;
        case 16: EDGE(16) break;
        case 32: EDGE(32) break;
        default: EDGE(64) break;
    }
#undef EDGE
}

void launch_score_finish(const ScorePlan& p, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_counts, dim3((p.SK + 255) / 256), dim3(256), 0, st, p);
    hipLaunchKernelGGL(k_score_finalize, dim3((p.Kc + 255) / 256), dim3(256), 0, st, p);
}

void launch_select(const ScorePlan& p, const uint8_t* lab, int32_t* labels_out,
                   int32_t* k_selected, hipStream_t st) {
    hipLaunchKernelGGL(k_select_best, dim3(1), dim3(256), 0, st, p, k_selected);
    if (p.n == 0) return;
    const int grid = (p.n + 255) / 256;
    hipLaunchKernelGGL(k_first_occ, dim3(grid), dim3(256), 0, st, p, lab);
    hipLaunchKernelGGL(k_rank, dim3(1), dim3(256), 0, st, p, k_selected);
    if (labels_out)
        hipLaunchKernelGGL(k_apply, dim3(grid), dim3(256), 0, st, p, lab, labels_out);
}

}  // namespace raft
