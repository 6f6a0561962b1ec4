// Dense part of a GCN layer (Sec. III-B, Eq. 6): U = P W with P = A_hat_n H,
// Z = tanh(U), rows L2-normalised (the normalisation the paper applies before
// the next layer and to the final embedding).
//
// MFMA FP32 (v_mfma_f32_16x16x4f32): a wave computes a 16-row tile against
// all output columns.  The contraction index is permuted so that each lane's
// A operand is a contiguous run of its P row (lane group g = lane/16 owns
// k = g*LIN/4 .. g*LIN/4 + LIN/4 - 1), loaded with float4; B is read from W
// with the same permutation.  The 16x16 result block of a wave keeps rows
// 4g..4g+3 in lane group g, columns in lane%16, so a row norm is an in-lane
// sum over column blocks plus a 16-lane xor reduction.
#include "kernels.h"

namespace raft {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// One wave's 16-row tile from row0 (row0 < n): U = P W on the matrix
// cores, then tanh and the row norm unless LINEAR.  getb(nb, s) returns the
// B operand of this lane for column block nb and contraction step s, i.e.
// W[g*KS + s][nb*16 + li]; where it comes from does not change the result.
template <int LIN, int LOUT, bool LINEAR, class GetB>
__device__ __forceinline__ void dense_tile(const float* __restrict__ P, float* __restrict__ H,
                                           int n, int32_t* __restrict__ status, int row0,
                                           GetB getb) {
    constexpr int KS = LIN / 4;
    constexpr int NB = LOUT / 16;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4;
    const int li = lane & 15;
    const int ra = min(row0 + li, n - 1);
    float a[KS];
    const float* prow = P + (size_t)ra * LIN + g * KS;
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
        const float4 v = *reinterpret_cast<const float4*>(prow + s);
        a[s] = v.x;
        a[s + 1] = v.y;
        a[s + 2] = v.z;
        a[s + 3] = v.w;
    }
    floatx4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], getb(nb, s), acc[nb], 0, 0, 0);
    }
    float inv[4] = {1.f, 1.f, 1.f, 1.f};
    if (!LINEAR) {
        float ss[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float z = tanhf(acc[nb][v]);
                acc[nb][v] = z;
                ss[v] += z * z;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) ss[v] += __shfl_xor(ss[v], off, kWave);
            const float nrm = sqrtf(ss[v]);
            if (!(nrm <= 3.0e38f)) atomicOr(status, kStatusNumeric);
            inv[v] = 1.0f / fmaxf(nrm, 1e-12f);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = row0 + 4 * g + v;
        if (row < n) {
            float* hrow = H + (size_t)row * LOUT + li;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) hrow[nb * 16] = acc[nb][v] * inv[v];
        }
    }
}

template <int LIN, int LOUT, bool LINEAR>
__device__ __forceinline__ void dense_body(const float* __restrict__ P,
                                           const float* __restrict__ W, float* __restrict__ H,
                                           int n, int32_t* __restrict__ status, int bx) {
    constexpr int KS = LIN / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4;
    const int li = lane & 15;
    const int row0 = (bx * 4 + (int)threadIdx.x / kWave) * 16;
    if (row0 >= n) return;
    const float* wcol = W + (size_t)(g * KS) * LOUT + li;
    dense_tile<LIN, LOUT, LINEAR>(P, H, n, status, row0, [&](int nb, int s) {
        return wcol[(size_t)s * LOUT + nb * 16];
    });
}

template <int LIN, int LOUT, bool LINEAR>
__global__ __launch_bounds__(256) void k_dense(const float* __restrict__ P,
                                               const float* __restrict__ W,
                                               float* __restrict__ H, int n,
                                               int32_t* __restrict__ status) {
    dense_body<LIN, LOUT, LINEAR>(P, W, H, n, status, (int)blockIdx.x);
}

// W staged in LDS once per work-group of kDenseLdsWaves waves, which then
// walk 16-row tiles (one per wave at a time, grid-stride).  Layout: for
// column block nb and contraction steps s..s+3 (s a multiple of 4) the 64
// lanes' operands are 64 consecutive float4s, lane-major, so a wave reads
// them with one conflict-free 16-byte load per lane; the staging writes are
// scattered once per work-group.  Used while W fits 64 KB, so that two
// work-groups (four waves per SIMD) share a CU.
constexpr int kDenseLdsWaves = 8;

template <int LIN, int LOUT>
struct DenseLds {
    static constexpr int kFloats = LIN * LOUT;
    static constexpr bool kFits = kFloats * 4 <= 64 * 1024;
};

template <int LIN, int LOUT, bool LINEAR>
__global__ __launch_bounds__(kDenseLdsWaves * kWave, 2) void k_dense_lds(
    const float* __restrict__ P, const float* __restrict__ W, float* __restrict__ H, int n,
    int32_t* __restrict__ status) {
    constexpr int KS = LIN / 4;
    __shared__ float4 wl4[DenseLds<LIN, LOUT>::kFloats / 4];
    float* wl = reinterpret_cast<float*>(wl4);
    for (int e = threadIdx.x; e < LIN * LOUT; e += blockDim.x) {
        const int k = e / LOUT, col = e % LOUT;
        const int g = k / KS, s = k - g * KS;
        const int ln = g * 16 + (col & 15);
        wl[((((col >> 4) * (KS / 4) + (s >> 2)) * kWave + ln) << 2) + (s & 3)] = W[e];
    }
    __syncthreads();
    const int tiles = (n + 15) / 16;
    for (int t = (int)blockIdx.x * kDenseLdsWaves + (int)threadIdx.x / kWave; t < tiles;
         t += (int)gridDim.x * kDenseLdsWaves) {
        // the lane's offset made opaque per tile: W's operands are the same
        // for every tile, and held in registers across tiles they would take
        // 256 of them (one wave per SIMD); read per tile they take four
        int lane = (int)(threadIdx.x & (kWave - 1));
        asm volatile("" : "+v"(lane));
        const float4* wp = wl4 + lane;
        dense_tile<LIN, LOUT, LINEAR>(P, H, n, status, t * 16, [&](int nb, int s) {
            const float4 v = wp[(nb * (KS / 4) + (s >> 2)) * kWave];
            return (s & 3) == 0 ? v.x : (s & 3) == 1 ? v.y : (s & 3) == 2 ? v.z : v.w;
        });
    }
}

// Batched: each graph's rows with its own W (one 64-row block never holds
// two graphs' rows).
template <int LIN, int LOUT, bool LINEAR>
__global__ __launch_bounds__(256) void k_dense_b(const DenseItem* __restrict__ items,
                                                 int32_t* __restrict__ status, BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const DenseItem& it = items[gi];
    dense_body<LIN, LOUT, LINEAR>(it.P, it.W, it.H, it.n, status, (int)w.x);
}

// Row L2 normalisation, one wave per row, lanes over columns.
__device__ __forceinline__ void rownorm_body(float* __restrict__ x, int n, int L, int bx) {
    const int wave = (bx * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (wave >= n) return;
    float* row = x + (size_t)wave * L;
    float ss = 0.f;
    for (int c = lane; c < L; c += kWave) ss += row[c] * row[c];
    ss = wave_sum(ss);
    const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
    for (int c = lane; c < L; c += kWave) row[c] *= inv;
}

__global__ __launch_bounds__(256) void k_rownorm(float* __restrict__ x, int n, int L) {
    rownorm_body(x, n, L, (int)blockIdx.x);
}

// Batched row normalisation: item.H (rows n of width L) of each graph.
__global__ __launch_bounds__(256) void k_rownorm_b(const DenseItem* __restrict__ items, int L,
                                                   BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    rownorm_body(items[gi].H, items[gi].n, L, (int)w.x);
}

// Wide layers (the paper's widths up to 4096, Table I): U = P W as a tiled
// FP32 MFMA GEMM.  A work-group computes a 64 x 128 tile of U; per 16-deep
// slab of the contraction the 256 threads stage the P tile (64 x 16) and the
// W tile (16 x 128) in LDS (double-buffered, the next slab's loads issued
// before this slab's MFMAs), and wave w computes the 64 x 32 columns
// [32 w, 32 w + 32) of the tile as 4 x 2 blocks of v_mfma_f32_16x16x4f32.
// Lane (li, g) supplies A[m + li][k0 + g] and B[k0 + g][n + li] per 4-deep
// step.  Then tanh and the row normalisation run over whole rows in a
// second kernel (a row spans several tiles).
constexpr int kGemmBM = 64, kGemmBN = 128, kGemmBK = 16;

__global__ __launch_bounds__(256) void k_gemm_wide(const float* __restrict__ P,
                                                   const float* __restrict__ W,
                                                   float* __restrict__ U, int n, int lin,
                                                   int lout) {
    __shared__ float As[2][kGemmBM][kGemmBK + 1];
    __shared__ float Bs[2][kGemmBK][kGemmBN + 4];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int g = lane >> 4, li = lane & 15;
    const int tiles_n = lout / kGemmBN;
    const int m0 = (blockIdx.x / tiles_n) * kGemmBM;
    const int n0 = (blockIdx.x % tiles_n) * kGemmBN;
    // staging: P tile 64 x 16 = one float4 per thread; W tile 16 x 128 = two
    const int ar = tid / 4, ac = (tid % 4) * 4;
    const int arow = min(m0 + ar, n - 1);
    const int br = tid / 32, bc = (tid % 32) * 4;
    float4 pa, pb0, pb1;
    auto issue = [&](int k0) {
        pa = *reinterpret_cast<const float4*>(P + (size_t)arow * lin + k0 + ac);
        pb0 = *reinterpret_cast<const float4*>(W + (size_t)(k0 + br) * lout + n0 + bc);
        pb1 = *reinterpret_cast<const float4*>(W + (size_t)(k0 + br + 8) * lout + n0 + bc);
    };
    auto commit = [&](int buf) {
        As[buf][ar][ac + 0] = pa.x;
        As[buf][ar][ac + 1] = pa.y;
        As[buf][ar][ac + 2] = pa.z;
        As[buf][ar][ac + 3] = pa.w;
        *reinterpret_cast<float4*>(&Bs[buf][br][bc]) = pb0;
        *reinterpret_cast<float4*>(&Bs[buf][br + 8][bc]) = pb1;
    };
    floatx4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    issue(0);
    commit(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < lin; k0 += kGemmBK) {
        const bool more = k0 + kGemmBK < lin;
        if (more) issue(k0 + kGemmBK);
#pragma unroll
        for (int s = 0; s < kGemmBK / 4; ++s) {
            float a[4], b[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[buf][16 * i + li][4 * s + g];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[buf][4 * s + g][32 * wid + 16 * j + li];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            commit(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    // block (i, j): rows m0 + 16 i + 4 g + v, column n0 + 32 wid + 16 j + li
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = m0 + 16 * i + 4 * g + v;
            if (row < n) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    U[(size_t)row * lout + n0 + 32 * wid + 16 * j + li] = acc[i][j][v];
            }
        }
}

// tanh and the row normalisation of a wide layer, in place; one wave per row.
__global__ __launch_bounds__(256) void k_tanh_rownorm(float* __restrict__ H, int n, int L,
                                                      int32_t* __restrict__ status) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (row >= n) return;
    float* h = H + (size_t)row * L;
    float ss = 0.f;
    for (int c = lane * 4; c < L; c += kWave * 4) {
        float4 v = *reinterpret_cast<float4*>(h + c);
        v.x = tanhf(v.x);
        v.y = tanhf(v.y);
        v.z = tanhf(v.z);
        v.w = tanhf(v.w);
        *reinterpret_cast<float4*>(h + c) = v;
        ss += v.x * v.x;
        ss += v.y * v.y;
        ss += v.z * v.z;
        ss += v.w * v.w;
    }
    ss = wave_sum(ss);
    const float nrm = sqrtf(ss);
    if (lane == 0 && !(nrm <= 3.0e38f)) atomicOr(status, kStatusNumeric);
    const float inv = 1.0f / fmaxf(nrm, 1e-12f);
    for (int c = lane * 4; c < L; c += kWave * 4) {
        float4 v = *reinterpret_cast<float4*>(h + c);
        v.x *= inv;
        v.y *= inv;
        v.z *= inv;
        v.w *= inv;
        *reinterpret_cast<float4*>(h + c) = v;
    }
}

static bool pow2_width(int v) { return v == 16 || v == 32 || v == 64 || v == 128 || v == 256; }

static bool wide_width(int v) {
    return v == 16 || v == 32 || v == 64 || v == 128 || v == 256 || v == 512 || v == 1024 ||
           v == 2048 || v == 4096;
}

// The register-tile kernel (k_dense) for lin x lout <= 128 x 256; the tiled
// GEMM otherwise (lout a multiple of 128, lin of 16).
static bool dense_small(int lin, int lout) {
    return pow2_width(lin) && pow2_width(lout) && lin * lout <= 128 * 256;
}

bool dense_supported(int lin, int lout) {
    return dense_small(lin, lout) || (wide_width(lin) && wide_width(lout) && lout >= kGemmBN);
}

template <int LIN, int LOUT>
static void dense_launch2(const float* P, const float* W, float* H, int32_t n, bool linear,
                          int32_t* status, int num_cu, hipStream_t st) {
    const int grid = (n + 63) / 64;
    if constexpr (DenseLds<LIN, LOUT>::kFits) {
        // as many work-groups as fit the CUs' LDS at once (at most 4 per CU)
        constexpr int per_cu = std::min(4, (160 * 1024) / (DenseLds<LIN, LOUT>::kFloats * 4));
        const int tiles = (n + 16 * kDenseLdsWaves - 1) / (16 * kDenseLdsWaves);
        const int g2 = std::min(tiles, std::max(1, num_cu) * per_cu);
        const dim3 blk(kDenseLdsWaves * kWave);
        if (linear)
            hipLaunchKernelGGL((k_dense_lds<LIN, LOUT, true>), dim3(g2), blk, 0, st, P, W, H, n,
                               status);
        else
            hipLaunchKernelGGL((k_dense_lds<LIN, LOUT, false>), dim3(g2), blk, 0, st, P, W, H, n,
                               status);
        return;
    }
    if (linear)
        hipLaunchKernelGGL((k_dense<LIN, LOUT, true>), dim3(grid), dim3(256), 0, st, P, W, H, n,
                           status);
    else
        hipLaunchKernelGGL((k_dense<LIN, LOUT, false>), dim3(grid), dim3(256), 0, st, P, W, H, n,
                           status);
}

template <int LIN, int LOUT>
static void dense_batched2(const DenseItem* items, bool linear, int32_t* status,
                           const BatchTable& t, int grid, hipStream_t st) {
    if (linear)
        hipLaunchKernelGGL((k_dense_b<LIN, LOUT, true>), dim3(grid), dim3(256), 0, st, items,
                           status, t);
    else
        hipLaunchKernelGGL((k_dense_b<LIN, LOUT, false>), dim3(grid), dim3(256), 0, st, items,
                           status, t);
}

template <int LIN>
static void dense_batched1(const DenseItem* items, int lout, bool linear, int32_t* status,
                           const BatchTable& t, int grid, hipStream_t st) {
    switch (lout) {
        case 16: dense_batched2<LIN, 16>(items, linear, status, t, grid, st); break;
        case 32: dense_batched2<LIN, 32>(items, linear, status, t, grid, st); break;
        case 64: dense_batched2<LIN, 64>(items, linear, status, t, grid, st); break;
        case 128: dense_batched2<LIN, 128>(items, linear, status, t, grid, st); break;
        case 256:
            if constexpr (LIN <= 128) dense_batched2<LIN, 256>(items, linear, status, t, grid, st);
            break;
        default: break;
    }
}

int dense_blocks(int32_t n) { return (n + 63) / 64; }

void launch_dense_layer_batched(const DenseItem* items, int lin, int lout, bool linear,
                                int32_t* status, const BatchTable& t, int grid, hipStream_t st) {
    if (grid == 0) return;
    switch (lin) {
        case 16: dense_batched1<16>(items, lout, linear, status, t, grid, st); break;
        case 32: dense_batched1<32>(items, lout, linear, status, t, grid, st); break;
        case 64: dense_batched1<64>(items, lout, linear, status, t, grid, st); break;
        case 128: dense_batched1<128>(items, lout, linear, status, t, grid, st); break;
        case 256: dense_batched1<256>(items, lout, linear, status, t, grid, st); break;
        default: break;
    }
}

int rownorm_blocks(int32_t n) { return (int)(((int64_t)n * kWave + 255) / 256); }

void launch_rownorm_batched(const DenseItem* items, int L, const BatchTable& t, int grid,
                            hipStream_t st) {
    if (grid == 0) return;
    hipLaunchKernelGGL(k_rownorm_b, dim3(grid), dim3(256), 0, st, items, L, t);
}

template <int LIN>
static void dense_launch1(const float* P, const float* W, float* H, int32_t n, int lout,
                          bool linear, int32_t* status, int num_cu, hipStream_t st) {
    switch (lout) {
        case 16: dense_launch2<LIN, 16>(P, W, H, n, linear, status, num_cu, st); break;
        case 32: dense_launch2<LIN, 32>(P, W, H, n, linear, status, num_cu, st); break;
        case 64: dense_launch2<LIN, 64>(P, W, H, n, linear, status, num_cu, st); break;
        case 128: dense_launch2<LIN, 128>(P, W, H, n, linear, status, num_cu, st); break;
        case 256:
            if constexpr (LIN <= 128) dense_launch2<LIN, 256>(P, W, H, n, linear, status, num_cu, st);
            break;
        default: break;
    }
}

void launch_dense_layer(const float* P, const float* W, float* H, int32_t n, int lin, int lout,
                        bool linear, int32_t* status, int num_cu, hipStream_t st) {
    if (n == 0) return;
    if (!dense_small(lin, lout)) {
        const int grid = ((n + kGemmBM - 1) / kGemmBM) * (lout / kGemmBN);
        hipLaunchKernelGGL(k_gemm_wide, dim3(grid), dim3(256), 0, st, P, W, H, n, lin, lout);
        if (!linear) {
            const int64_t threads = (int64_t)n * kWave;
            hipLaunchKernelGGL(k_tanh_rownorm, dim3((unsigned)((threads + 255) / 256)), dim3(256),
                               0, st, H, n, lout, status);
        }
        return;
    }
    switch (lin) {
        case 16: dense_launch1<16>(P, W, H, n, lout, linear, status, num_cu, st); break;
        case 32: dense_launch1<32>(P, W, H, n, lout, linear, status, num_cu, st); break;
        case 64: dense_launch1<64>(P, W, H, n, lout, linear, status, num_cu, st); break;
        case 128: dense_launch1<128>(P, W, H, n, lout, linear, status, num_cu, st); break;
        case 256: dense_launch1<256>(P, W, H, n, lout, linear, status, num_cu, st); break;
        default: break;
    }
}

void launch_rownorm(float* x, int32_t n, int L, hipStream_t st) {
    if (n == 0) return;
    const int64_t threads = (int64_t)n * kWave;
    hipLaunchKernelGGL(k_rownorm, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, x, n,
                       L);
}

}  // namespace raft
