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
// Edge kernel: labels are point-major bytes, row stride S (multiple of 8),
// so one 8-byte load gives eight candidates' labels of a node.  LPR lanes
// cover a node's label row and a wave scores 64/LPR rows side by side: per
// batch of 16 edges the lanes of a row group load the same column indices
// (broadcast loads) and gather the neighbours' label words back to back,
// comparing bytes with an exact per-byte zero mask.  Counts are accumulated per work-group in LDS and
// written as partials; all counts are integers, so their sums are exact.
// The heaviest rows (the first `heavy` rows of the degree order) are taken
// one per pass, their edges split over the wave's row groups, so that a
// long row does not leave one row group walking its edges alone at the end
// of the launch; each group adds its share of the count, and the first adds
// the row's degree.
#include <limits.h>

#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace raft {

__device__ __forceinline__ void transpose_labels_body(const uint8_t* __restrict__ cm, int n, int Kc,
                                                      uint8_t* __restrict__ pm, int S, int bx) {
    const int64_t idx = (int64_t)bx * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * S) return;
    const int i = (int)(idx / S);
    const int k = (int)(idx - (int64_t)i * S);
    pm[idx] = k < Kc ? cm[(size_t)k * n + i] : (uint8_t)0;
}

__global__ __launch_bounds__(256) void k_transpose_labels(const uint8_t* __restrict__ cm, int n,
                                                          int Kc, uint8_t* __restrict__ pm,
                                                          int S) {
    transpose_labels_body(cm, n, Kc, pm, S, (int)blockIdx.x);
}

__device__ __forceinline__ void copy_labels_body(const uint8_t* __restrict__ pm, int n, int Kc, int S,
                                                 uint8_t* __restrict__ out, int bx) {
    const int64_t idx = (int64_t)bx * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * Kc) return;
    const int i = (int)(idx / Kc);
    const int k = (int)(idx - (int64_t)i * Kc);
    out[idx] = pm[(size_t)i * S + k];
}

__global__ __launch_bounds__(256) void k_copy_labels(const uint8_t* __restrict__ pm, int n, int Kc,
                                                     int S, uint8_t* __restrict__ out) {
    copy_labels_body(pm, n, Kc, S, out, (int)blockIdx.x);
}

__device__ __forceinline__ uint32_t zero_bytes_mask(uint32_t x) {
    // 0x80 in every byte of x that is zero, exact per byte
    uint32_t y = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    return ~(y | x | 0x7F7F7F7Fu);
}

// Node ids from the graph view are global (a batch's block-diagonal CSR); the
// labels are the graph's own rows, so they are indexed by id - base.
template <int LPR>
__device__ __forceinline__ void edge_score_body(const GraphView& g, const ScorePlan& p,
                                                const uint8_t* __restrict__ lab, Wg w) {
    constexpr int G = kWave / LPR;                  // rows side by side per wave
    extern __shared__ int sm[];
    int* sl = sm;
    int* sv = sm + p.SK;
    for (int idx = threadIdx.x; idx < 2 * p.SK; idx += blockDim.x) sm[idx] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int slot = lane / LPR;
    const int m = lane % LPR;
    const bool on = 8 * m < p.S;
    // passes of G positions of the graph's degree-class order (rows of
    // similar length side by side, the longest first), dealt to the waves
    // round robin so every wave gets its share of long and short rows
    const int nwaves = (int)w.n * (blockDim.x / kWave);
    const int H = p.heavy;
    const int npass = H + (g.n - H + G - 1) / G;
    lab -= (size_t)g.base * p.S;
    for (int pp = (int)w.x * (blockDim.x / kWave) + wid; pp < npass; pp += nwaves) {
        // pass pp < H: row order[pp], row group `slot` takes the slot-th of
        // G equal runs of its edges; else G rows side by side
        const bool split = pp < H;
        const int pos = split ? pp : H + (pp - H) * G + slot;
        const bool valid = pos < g.n;
        const int i = valid ? g.order[pos] : 0;
        const int rbeg = g.rp[i];
        const int rend = valid ? g.rp[i + 1] : rbeg;
        int beg = rbeg, end = rend;
        if (split) {
            const int run = (rend - rbeg + G - 1) / G;
            beg = min(rend, rbeg + slot * run);
            end = min(rend, beg + run);
        }
        const bool first = !split || slot == 0;   // adds the row's degree
        int maxdeg = end - beg;
#pragma unroll
        for (int off = LPR; off < kWave; off <<= 1)
            maxdeg = max(maxdeg, __shfl_xor(maxdeg, off, kWave));
        uint2 li = make_uint2(0u, 0u);
        if (valid && on) li = *reinterpret_cast<const uint2*>(lab + (size_t)i * p.S + 8 * m);
        int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int base = 0; base < maxdeg; base += 16) {
            int jv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = beg + base + q;
                jv[q] = e < end ? g.ci[e] : -1;
            }
            uint2 lj[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                // a non-edge compares against a word with no byte equal to li
                lj[q] = make_uint2(~li.x, ~li.y);
                if (jv[q] >= 0 && on)
                    lj[q] = *reinterpret_cast<const uint2*>(lab + (size_t)jv[q] * p.S + 8 * m);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t z0 = zero_bytes_mask(li.x ^ lj[q].x);
                const uint32_t z1 = zero_bytes_mask(li.y ^ lj[q].y);
                c[0] += (z0 >> 7) & 1u;
                c[1] += (z0 >> 15) & 1u;
                c[2] += (z0 >> 23) & 1u;
                c[3] += (z0 >> 31) & 1u;
                c[4] += (z1 >> 7) & 1u;
                c[5] += (z1 >> 15) & 1u;
                c[6] += (z1 >> 23) & 1u;
                c[7] += (z1 >> 31) & 1u;
            }
        }
        if (valid && on) {
            const int d = first ? rend - rbeg : 0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int k = 8 * m + b;
                if (k < p.Kc) {
                    const int rr = ((b < 4 ? li.x : li.y) >> (8 * (b & 3))) & 0xFF;
                    if (rr >= p.ks[k]) {
                        atomicOr(p.status, kStatusLabel);
                        continue;
                    }
                    const int slotk = p.koff[k] + rr;
                    if (c[b]) atomicAdd(&sl[slotk], c[b]);
                    if (d) atomicAdd(&sv[slotk], d);
                }
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < p.SK; idx += blockDim.x) {
        p.lpart[(size_t)w.x * p.SK + idx] = sl[idx];
        p.vpart[(size_t)w.x * p.SK + idx] = sv[idx];
    }
}

template <int LPR>
__global__ __launch_bounds__(256) void k_edge_score(GraphView g, ScorePlan p,
                                                    const uint8_t* __restrict__ lab) {
    edge_score_body<LPR>(g, p, lab, wg_self());
}

template <int LPR>
__global__ __launch_bounds__(256) void k_edge_score_b(const GraphView* __restrict__ views,
                                                      const ScorePlan* __restrict__ plans,
                                                      BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    edge_score_body<LPR>(views[gi], plans[gi], plans[gi].lab, w);
}

// Sum of the work-group partials: 16 entries x 16 slices per block, slices
// combined through LDS.  Integer sums, exact.
__device__ __forceinline__ void reduce_counts_body(const ScorePlan& p, int bx) {
    __shared__ long long sl[16][17], sv[16][17];
    const int e = threadIdx.x & 15, sl_id = threadIdx.x >> 4;
    const int idx = bx * 16 + e;
    long long l = 0, v = 0;
    if (idx < p.SK) {
        const int per = (p.grid + 15) / 16;
        const int b0 = sl_id * per, b1 = min(p.grid, b0 + per);
#pragma unroll 8
        for (int b = b0; b < b1; ++b) {
            l += p.lpart[(size_t)b * p.SK + idx];
            v += p.vpart[(size_t)b * p.SK + idx];
        }
    }
    sl[e][sl_id] = l;
    sv[e][sl_id] = v;
    __syncthreads();
    if (sl_id == 0 && idx < p.SK) {
        long long tl = 0, tv = 0;
        for (int q = 0; q < 16; ++q) {
            tl += sl[e][q];
            tv += sv[e][q];
        }
        p.l64[idx] = tl / 2;
        p.v64[idx] = tv;
    }
}

__global__ __launch_bounds__(256) void k_reduce_counts(ScorePlan p) {
    reduce_counts_body(p, (int)blockIdx.x);
}

// One wave per candidate: the lanes compute the per-block terms (each with
// its divisions) into LDS, then one lane sums them over r in ascending order
// (the same terms and the same order as a single lane doing both).
__device__ __forceinline__ void score_finalize_body(const ScorePlan& p, int k) {
    __shared__ double tm[RAFT_MAX_K_DEV + 1], tn[RAFT_MAX_K_DEV + 1];
    if (k >= p.Kc) return;
    const int K = p.ks[k];
    {
#pragma clang fp contract(off)
        const double e = (double)(p.nnz / 2);
        const double m2 = (double)p.nnz;
        for (int r = threadIdx.x; r < K; r += blockDim.x) {
            const long long l = p.l64[p.koff[k] + r];
            const long long v = p.v64[p.koff[k] + r];
            const double t = (double)v / m2;
            tm[r] = (double)l / e - t * t;
            tn[r] = v > 0 ? (double)(v - 2 * l) / (double)v : 0.0;
        }
        __syncthreads();
        if (threadIdx.x != 0) return;
        double mod = 0.0;
        for (int r = 0; r < K; ++r) mod = mod + tm[r];
        double nc = 0.0;   // an empty block adds +0.0, which leaves the sum as it is
        for (int r = 0; r < K; ++r) nc = nc + tn[r];
        p.mod[k] = mod;
        p.ncut[k] = 0.5 * nc;
    }
}

__global__ __launch_bounds__(64) void k_score_finalize(ScorePlan p) {
    score_finalize_body(p, (int)blockIdx.x);
}

// K* = first maximum of Mod; init first-occurrence table.
__device__ __forceinline__ void select_best_body(const ScorePlan& p, int32_t* k_selected) {
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

__global__ void k_select_best(ScorePlan p, int32_t* k_selected) { select_best_body(p, k_selected); }

__device__ __forceinline__ void first_occ_body(const ScorePlan& p, const uint8_t* __restrict__ lab,
                                               Wg w) {
    __shared__ int first[RAFT_MAX_K_DEV + 1];
    for (int r = threadIdx.x; r <= RAFT_MAX_K_DEV; r += blockDim.x) first[r] = INT_MAX;
    __syncthreads();
    const int best = *p.best;
    for (int i = (int)w.x * blockDim.x + threadIdx.x; i < p.n; i += (int)w.n * blockDim.x)
        atomicMin(&first[lab[(size_t)i * p.S + best]], i);
    __syncthreads();
    for (int r = threadIdx.x; r <= RAFT_MAX_K_DEV; r += blockDim.x)
        if (first[r] != INT_MAX) atomicMin(&p.first[r], first[r]);
}

__global__ __launch_bounds__(256) void k_first_occ(ScorePlan p, const uint8_t* __restrict__ lab) {
    first_occ_body(p, lab, wg_self());
}

__device__ __forceinline__ void rank_body(const ScorePlan& p, int32_t* k_selected) {
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

__global__ void k_rank(ScorePlan p, int32_t* k_selected) { rank_body(p, k_selected); }

__device__ __forceinline__ void apply_body(const ScorePlan& p, const uint8_t* __restrict__ lab,
                                           int32_t* __restrict__ out, int bx) {
    const int i = bx * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    out[i] = p.remap[lab[(size_t)i * p.S + *p.best]];
}

__global__ __launch_bounds__(256) void k_apply(ScorePlan p, const uint8_t* __restrict__ lab,
                                               int32_t* __restrict__ out) {
    apply_body(p, lab, out, (int)blockIdx.x);
}

// ---- batched forms: one launch per kernel over the graphs of a batch, each
// graph with its own ScorePlan (labels, outputs) in device memory ----

__global__ __launch_bounds__(256) void k_transpose_labels_b(const ScorePlan* __restrict__ plans,
                                                            BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const ScorePlan& p = plans[gi];
    transpose_labels_body(p.lab_cm, p.n, p.Kc, p.lab, p.S, (int)w.x);
}

__global__ __launch_bounds__(256) void k_reduce_counts_b(const ScorePlan* __restrict__ plans,
                                                         BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    reduce_counts_body(plans[gi], (int)w.x);
}

__global__ __launch_bounds__(64) void k_score_finalize_b(const ScorePlan* __restrict__ plans,
                                                         BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    score_finalize_body(plans[gi], (int)w.x);
}

__global__ __launch_bounds__(256) void k_select_best_b(const ScorePlan* __restrict__ plans,
                                                       BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    select_best_body(plans[gi], plans[gi].ksel_out);
}

__global__ __launch_bounds__(256) void k_first_occ_b(const ScorePlan* __restrict__ plans,
                                                     BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    first_occ_body(plans[gi], plans[gi].lab, w);
}

__global__ __launch_bounds__(256) void k_rank_b(const ScorePlan* __restrict__ plans,
                                                BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    rank_body(plans[gi], plans[gi].ksel_out);
}

__global__ __launch_bounds__(256) void k_apply_b(const ScorePlan* __restrict__ plans,
                                                 BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const ScorePlan& p = plans[gi];
    if (p.labels_out) apply_body(p, p.lab, p.labels_out, (int)w.x);
}

__global__ __launch_bounds__(256) void k_copy_labels_b(const ScorePlan* __restrict__ plans,
                                                       BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const ScorePlan& p = plans[gi];
    if (p.labels_all_out) copy_labels_body(p.lab, p.n, p.Kc, p.S, p.labels_all_out, (int)w.x);
}

static int score_lpr(int S) {
    const int words = S / 8;
    int lpr = 1;
    while (lpr < words) lpr <<= 1;
    return lpr;
}

int score_split_batches(int S) { return std::min(16, kWave / score_lpr(S)); }

int score_grid(int32_t n, int num_cu) {
    const int64_t want = ((int64_t)n + 63) / 64;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * 4));
}

// a label row of Kc bytes is covered by at most 32 lanes of 8 bytes; the
// per-work-group counts (2 x SK ints) live in LDS
bool score_supported(int Kc, int SK) {
    return Kc >= 1 && Kc <= 8 * 32 && SK >= 1 && SK <= 16384;
}

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
    const int lpr = score_lpr(p.S);
#define EDGE(LV)                                                                              \
    {                                                                                         \
        static std::once_flag attr_once;                                                      \
        std::call_once(attr_once, [] {                                                        \
            (void)hipFuncSetAttribute((const void*)k_edge_score<LV>,                          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
        });                                                                                   \
        hipLaunchKernelGGL(k_edge_score<LV>, dim3(p.grid), dim3(256), lds, st, g, p, lab);    \
    }
    switch (lpr) {
        case 1: EDGE(1) break;
        case 2: EDGE(2) break;
        case 4: EDGE(4) break;
        case 8: EDGE(8) break;
        case 16: EDGE(16) break;
        default: EDGE(32) break;
    }
#undef EDGE
}

void launch_score_finish(const ScorePlan& p, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_counts, dim3((p.SK + 15) / 16), dim3(256), 0, st, p);
    hipLaunchKernelGGL(k_score_finalize, dim3(p.Kc), dim3(64), 0, st, p);
}

void launch_select(const ScorePlan& p, const uint8_t* lab, int32_t* labels_out,
                   int32_t* k_selected, hipStream_t st) {
    hipLaunchKernelGGL(k_select_best, dim3(1), dim3(256), 0, st, p, k_selected);
    if (p.n == 0) return;
    const int grid = (p.n + 255) / 256;
    hipLaunchKernelGGL(k_first_occ, dim3(std::min(grid, 256)), dim3(256), 0, st, p, lab);
    hipLaunchKernelGGL(k_rank, dim3(1), dim3(256), 0, st, p, k_selected);
    if (labels_out)
        hipLaunchKernelGGL(k_apply, dim3(grid), dim3(256), 0, st, p, lab, labels_out);
}

int score_blocks(const ScorePlan& p, int kind) {
    const int ng = (p.n + 255) / 256;
    switch (kind) {
        case kScTranspose: return (int)(((int64_t)p.n * p.S + 255) / 256);
        case kScEdge: return p.grid;
        case kScReduce: return (p.SK + 15) / 16;
        case kScFinalize: return p.Kc;
        case kScSelect:
        case kScRank: return 1;
        case kScFirst: return p.n == 0 ? 0 : std::min(ng, 256);
        case kScApply: return ng;
        case kScCopy: return (int)(((int64_t)p.n * p.Kc + 255) / 256);
        default: return 0;
    }
}

void launch_score_batched(int kind, const GraphView* views, const ScorePlan* plans, int S, int SK,
                          const BatchTable& t, int grid, hipStream_t st) {
    if (grid == 0) return;
    const dim3 blk(256);
    switch (kind) {
        case kScTranspose:
            hipLaunchKernelGGL(k_transpose_labels_b, dim3(grid), blk, 0, st, plans, t);
            break;
        case kScEdge: {
            const size_t lds = (size_t)2 * SK * sizeof(int);
#define EDGE(LV)                                                                              \
    {                                                                                         \
        static std::once_flag attr_once;                                                      \
        std::call_once(attr_once, [] {                                                        \
            (void)hipFuncSetAttribute((const void*)k_edge_score_b<LV>,                        \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
        });                                                                                   \
        hipLaunchKernelGGL(k_edge_score_b<LV>, dim3(grid), blk, lds, st, views, plans, t);    \
    }
            switch (score_lpr(S)) {
                case 1: EDGE(1) break;
                case 2: EDGE(2) break;
                case 4: EDGE(4) break;
                case 8: EDGE(8) break;
                case 16: EDGE(16) break;
                default: EDGE(32) break;
            }
#undef EDGE
            break;
        }
        case kScReduce: hipLaunchKernelGGL(k_reduce_counts_b, dim3(grid), blk, 0, st, plans, t); break;
        case kScFinalize:
            hipLaunchKernelGGL(k_score_finalize_b, dim3(grid), dim3(64), 0, st, plans, t);
            break;
        case kScSelect: hipLaunchKernelGGL(k_select_best_b, dim3(grid), blk, 0, st, plans, t); break;
        case kScFirst: hipLaunchKernelGGL(k_first_occ_b, dim3(grid), blk, 0, st, plans, t); break;
        case kScRank: hipLaunchKernelGGL(k_rank_b, dim3(grid), blk, 0, st, plans, t); break;
        case kScApply: hipLaunchKernelGGL(k_apply_b, dim3(grid), blk, 0, st, plans, t); break;
        case kScCopy: hipLaunchKernelGGL(k_copy_labels_b, dim3(grid), blk, 0, st, plans, t); break;
        default: break;
    }
}

}  // namespace raft
