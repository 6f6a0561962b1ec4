// Sparse x tall-skinny products of the projection (Sec. III-A) and of the GCN
// aggregation (Sec. III-B, Eq. 6):
//   NCUT        y_i = s_i  sum_{j in N(i)} s_j x_j                   (M, Eq. 2)
//   MOD_FULL    y_i = sum_{j in N(i)} x_j - (d_i/2e) (d^T x)           (B, Eq. 4)
//   MOD_REDUCED y_i = sum_{j in N(i)} x_j - (d_i/2e) sum_j d_j x_j     (Q~)
//   GCN         y_i = sh_i (sum_{j in N(i)} sh_j x_j + sh_i x_i)       (A_hat_n)
// with s = D^-1/2 and sh = (D+1)^-1/2.
//
// Row-split CSR: one wave per row.  The wave reads up to 64 column indices
// coalesced (one per lane), then gathers feature rows: each lane loads a
// float4, L/4 lanes cover one row of x, so 256/L edges are gathered per wave
// instruction and several such steps are kept in flight.  Partial sums of
// the edge slots are folded with xor shuffles.  Rows are assigned in
// contiguous runs per wave; the optional epilogue accumulates FP64 partials
// of d^T y per work-group (the rank-1 term of the next MOD_FULL step), in a
// fixed order so the column sums are deterministic.
#include "kernels.h"

namespace raft {

constexpr int kSpmmWaves = 4;

template <int L, int OP, bool CS>
__global__ __launch_bounds__(256) void k_spmm(GraphView g, const float* __restrict__ x,
                                              float* __restrict__ y,
                                              const float* __restrict__ cvec,
                                              double* __restrict__ cpart, int rpw) {
    constexpr int LANES = L / 4;
    constexpr int SLOTS = kWave / LANES;
    constexpr int UNR = SLOTS >= 16 ? 1 : 16 / SLOTS;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int slot = lane / LANES;
    const int sub = lane % LANES;
    const int row0 = (blockIdx.x * kSpmmWaves + wid) * rpw;
    double cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;

    for (int r = 0; r < rpw; ++r) {
        const int i = row0 + r;
        if (i >= g.n) break;
        const int beg = g.rp[i], end = g.rp[i + 1];
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 acc2 = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int base = beg; base < end; base += kWave) {
            const int e = base + lane;
            int j = i;
            float w = 0.f;
            if (e < end) {
                j = g.ci[e];
                if (OP == kOpNcut) w = g.s[j];
                else if (OP == kOpGcn) w = g.sh[j];
                else if (OP == kOpModReduced) w = (float)g.deg[j];
                else w = 1.f;
            }
            const int cnt = min(kWave, end - base);
            for (int t = 0; t < cnt; t += SLOTS * UNR) {
                float4 v[UNR];
                float ww[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int src = t + u * SLOTS + slot;
                    const int jj = __shfl(j, src & (kWave - 1), kWave);
                    ww[u] = __shfl(w, src & (kWave - 1), kWave);
                    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (src < cnt)
                        v[u] = *reinterpret_cast<const float4*>(x + (size_t)jj * L + sub * 4);
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    if (OP == kOpModFull) {
                        acc.x += v[u].x;
                        acc.y += v[u].y;
                        acc.z += v[u].z;
                        acc.w += v[u].w;
                    } else if (OP == kOpModReduced) {
                        acc.x += v[u].x;
                        acc.y += v[u].y;
                        acc.z += v[u].z;
                        acc.w += v[u].w;
                        acc2.x += ww[u] * v[u].x;
                        acc2.y += ww[u] * v[u].y;
                        acc2.z += ww[u] * v[u].z;
                        acc2.w += ww[u] * v[u].w;
                    } else {
                        acc.x += ww[u] * v[u].x;
                        acc.y += ww[u] * v[u].y;
                        acc.z += ww[u] * v[u].z;
                        acc.w += ww[u] * v[u].w;
                    }
                }
            }
        }
#pragma unroll
        for (int off = LANES; off < kWave; off <<= 1) {
            acc.x += __shfl_xor(acc.x, off, kWave);
            acc.y += __shfl_xor(acc.y, off, kWave);
            acc.z += __shfl_xor(acc.z, off, kWave);
            acc.w += __shfl_xor(acc.w, off, kWave);
            if (OP == kOpModReduced) {
                acc2.x += __shfl_xor(acc2.x, off, kWave);
                acc2.y += __shfl_xor(acc2.y, off, kWave);
                acc2.z += __shfl_xor(acc2.z, off, kWave);
                acc2.w += __shfl_xor(acc2.w, off, kWave);
            }
        }
        float4 o;
        if (OP == kOpNcut) {
            const float si = g.s[i];
            o = make_float4(si * acc.x, si * acc.y, si * acc.z, si * acc.w);
        } else if (OP == kOpGcn) {
            const float si = g.sh[i];
            const float4 xi = *reinterpret_cast<const float4*>(x + (size_t)i * L + sub * 4);
            o = make_float4(si * (acc.x + si * xi.x), si * (acc.y + si * xi.y),
                            si * (acc.z + si * xi.z), si * (acc.w + si * xi.w));
        } else if (OP == kOpModFull) {
            const float ci = g.dcoef[i];
            const float4 c = *reinterpret_cast<const float4*>(cvec + sub * 4);
            o = make_float4(acc.x - ci * c.x, acc.y - ci * c.y, acc.z - ci * c.z,
                            acc.w - ci * c.w);
        } else {
            const float ci = g.dcoef[i];
            o = make_float4(acc.x - ci * acc2.x, acc.y - ci * acc2.y, acc.z - ci * acc2.z,
                            acc.w - ci * acc2.w);
        }
        if (slot == 0) *reinterpret_cast<float4*>(y + (size_t)i * L + sub * 4) = o;
        if (CS) {
            const double di = (double)g.deg[i];
            cs0 += di * (double)o.x;
            cs1 += di * (double)o.y;
            cs2 += di * (double)o.z;
            cs3 += di * (double)o.w;
        }
    }
    if (CS) {
        __shared__ double red[kSpmmWaves][L];
        if (slot == 0) {
            red[wid][sub * 4 + 0] = cs0;
            red[wid][sub * 4 + 1] = cs1;
            red[wid][sub * 4 + 2] = cs2;
            red[wid][sub * 4 + 3] = cs3;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < L; c += blockDim.x) {
            double s = 0;
            for (int w = 0; w < kSpmmWaves; ++w) s += red[w][c];
            cpart[(size_t)blockIdx.x * L + c] = s;
        }
    }
}

// FP64 partials of d^T x, same row mapping as k_spmm.
template <int L>
__global__ __launch_bounds__(256) void k_colsum_part(GraphView g, const float* __restrict__ x,
                                                     double* __restrict__ cpart, int rpw) {
    constexpr int LANES = L / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int row0 = (blockIdx.x * kSpmmWaves + wid) * rpw;
    double cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;
    if (lane < LANES) {
        for (int r = 0; r < rpw; ++r) {
            const int i = row0 + r;
            if (i >= g.n) break;
            const float4 o = *reinterpret_cast<const float4*>(x + (size_t)i * L + lane * 4);
            const double di = (double)g.deg[i];
            cs0 += di * (double)o.x;
            cs1 += di * (double)o.y;
            cs2 += di * (double)o.z;
            cs3 += di * (double)o.w;
        }
    }
    __shared__ double red[kSpmmWaves][L];
    if (lane < LANES) {
        red[wid][lane * 4 + 0] = cs0;
        red[wid][lane * 4 + 1] = cs1;
        red[wid][lane * 4 + 2] = cs2;
        red[wid][lane * 4 + 3] = cs3;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < L; c += blockDim.x) {
        double s = 0;
        for (int w = 0; w < kSpmmWaves; ++w) s += red[w][c];
        cpart[(size_t)blockIdx.x * L + c] = s;
    }
}

// c = sum over parts (fixed split into `per` contiguous slices per column,
// slices combined in order), cvec = FP32(c).
__global__ __launch_bounds__(1024) void k_colsum_finish(const double* __restrict__ part, int parts,
                                                        int L, double* __restrict__ c64,
                                                        float* __restrict__ cvec) {
    const int per = blockDim.x / L;
    const int col = threadIdx.x % L;
    const int sl = threadIdx.x / L;
    __shared__ double red[1024];
    double s = 0;
    if (sl < per) {
        const int len = (parts + per - 1) / per;
        const int b0 = sl * len, b1 = min(parts, b0 + len);
        for (int b = b0; b < b1; ++b) s += part[(size_t)b * L + col];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (sl == 0) {
        double t = 0;
        for (int k = 0; k < per; ++k) t += red[k * L + col];
        c64[col] = t;
        cvec[col] = (float)t;
    }
}

bool spmm_supported(int L) { return L == 16 || L == 32 || L == 64 || L == 128 || L == 256; }

int spmm_grid(int32_t n, int L, int num_cu, int* rows_per_wave) {
    (void)L;
    const int target_waves = num_cu * 32;
    int rpw = (int)((n + (int64_t)target_waves - 1) / target_waves);
    rpw = rpw < 1 ? 1 : (rpw > 64 ? 64 : rpw);
    if (rows_per_wave) *rows_per_wave = rpw;
    const int64_t rows_per_block = (int64_t)rpw * kSpmmWaves;
    return (int)((n + rows_per_block - 1) / rows_per_block);
}

template <int L>
static void spmm_dispatch_op(const GraphView& g, int op, const float* x, float* y,
                             const float* cvec, double* cpart, int grid, int rpw, hipStream_t st) {
#define RAFT_SPMM_CASE(OPV)                                                                  \
    if (op == OPV) {                                                                         \
        if (cpart)                                                                           \
            hipLaunchKernelGGL((k_spmm<L, OPV, true>), dim3(grid), dim3(256), 0, st, g, x, y, \
                               cvec, cpart, rpw);                                            \
        else                                                                                 \
            hipLaunchKernelGGL((k_spmm<L, OPV, false>), dim3(grid), dim3(256), 0, st, g, x,   \
                               y, cvec, cpart, rpw);                                         \
        return;                                                                              \
    }
    RAFT_SPMM_CASE(kOpNcut)
    RAFT_SPMM_CASE(kOpModFull)
    RAFT_SPMM_CASE(kOpModReduced)
    RAFT_SPMM_CASE(kOpGcn)
#undef RAFT_SPMM_CASE
}

void launch_spmm(const GraphView& g, int op, int L, const float* x, float* y, const float* cvec,
                 double* cpart, int num_cu, hipStream_t st) {
    int rpw;
    const int grid = spmm_grid(g.n, L, num_cu, &rpw);
    if (grid == 0) return;
    switch (L) {
        case 16: spmm_dispatch_op<16>(g, op, x, y, cvec, cpart, grid, rpw, st); break;
        case 32: spmm_dispatch_op<32>(g, op, x, y, cvec, cpart, grid, rpw, st); break;
        case 64: spmm_dispatch_op<64>(g, op, x, y, cvec, cpart, grid, rpw, st); break;
        case 128: spmm_dispatch_op<128>(g, op, x, y, cvec, cpart, grid, rpw, st); break;
        case 256: spmm_dispatch_op<256>(g, op, x, y, cvec, cpart, grid, rpw, st); break;
        default: break;
    }
}

void launch_colsum_partials(const GraphView& g, int L, const float* x, double* part, int num_cu,
                            hipStream_t st) {
    int rpw;
    const int grid = spmm_grid(g.n, L, num_cu, &rpw);
    if (grid == 0) return;
    switch (L) {
        case 16: hipLaunchKernelGGL(k_colsum_part<16>, dim3(grid), dim3(256), 0, st, g, x, part, rpw); break;
        case 32: hipLaunchKernelGGL(k_colsum_part<32>, dim3(grid), dim3(256), 0, st, g, x, part, rpw); break;
        case 64: hipLaunchKernelGGL(k_colsum_part<64>, dim3(grid), dim3(256), 0, st, g, x, part, rpw); break;
        case 128: hipLaunchKernelGGL(k_colsum_part<128>, dim3(grid), dim3(256), 0, st, g, x, part, rpw); break;
        case 256: hipLaunchKernelGGL(k_colsum_part<256>, dim3(grid), dim3(256), 0, st, g, x, part, rpw); break;
        default: break;
    }
}

void launch_colsum_finish(const double* part, int parts, int L, double* c64, float* cvec,
                          hipStream_t st) {
    const int threads = (1024 / L) * L;
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(threads), 0, st, part, parts, L, c64, cvec);
}

}  // namespace raft
