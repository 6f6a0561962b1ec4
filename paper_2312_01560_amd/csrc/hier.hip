// Hierarchical model selection (Sec. III-C, Alg. 1) with local modularity
// (Eq. 7), level-synchronous: every set still to be partitioned at one depth
// of the tree is split at once.  Each set U occupies a contiguous segment of
// a node permutation; a launch table gives each set work-groups in
// proportion to its size (the BatchTable of the batched launches).
//
// Per set and level: KMeans with K = 2 on the embeddings of U (k-means++
// seeding by the exponential race with draws keyed by node id and depth,
// Lloyd to a fixed point or T_max, ties to side 0), then the integer counts of
// Eq. 7: edges with both ends in U, edges with both ends in U_1 or in U_2,
// and the G-degree volumes of U_1 and U_2.  The host finishes LMod in FP64
// and decides.  Every result is independent of the order of the nodes in a
// segment (argmins are lexicographic on (value, node id), sums are integers),
// so the children's segments are filled with atomic cursors.
#include <float.h>
#include <limits.h>

#include <algorithm>

#include "kernels.h"

namespace raft {

constexpr uint64_t kStreamHierRace = 0x21;

__device__ __forceinline__ bool hlex_less(double v, int i, double bv, int bi) {
    return v < bv || (v == bv && i < bi);
}

// Race step t of every set: per work-group, the lexicographic minimum of
// (E_{t,i} / w_i, i) over its part of the segment (w > 0 only), and the
// lowest node id other than pick 0 (the fallback when every w is 0).
template <int D>
__global__ __launch_bounds__(256) void k_hier_race(HierPlan h, int t, BatchTable tb) {
    int s;
    Wg w;
    if (!batch_find(tb, s, w)) return;
    const int beg = h.beg[s], cnt = h.cnt[s];
    const int p0 = t > 0 ? h.pick[2 * s] : -1;
    const float* z0 = p0 >= 0 ? h.Z + (size_t)p0 * D : h.Z;
    double best = INFINITY;
    int bidx = INT_MAX, low = INT_MAX;
    for (int pos = (int)w.x * blockDim.x + threadIdx.x; pos < cnt;
         pos += (int)w.n * blockDim.x) {
        const int i = h.perm[beg + pos];
        if (i != p0) low = min(low, i);
        float wi = 1.0f;
        if (t > 0) {
            const float* zi = h.Z + (size_t)i * D;
            float dist = 0.f;
#pragma unroll 4
            for (int c = 0; c < D; c += 4) {
                const float4 a = *reinterpret_cast<const float4*>(zi + c);
                const float4 b = *reinterpret_cast<const float4*>(z0 + c);
                const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
                dist += dx * dx;
                dist += dy * dy;
                dist += dz * dz;
                dist += dw * dw;
            }
            wi = dist;
        }
        if (wi > 0.f) {
            const U64x4 r = philox4x64_10((uint64_t)i, (uint64_t)t, (uint64_t)h.depth, 0, h.seed,
                                          kStreamHierRace);
            const double ratio = -own_ln(uniform52(r.v[0])) / (double)wi;
            if (hlex_less(ratio, i, best, bidx)) {
                best = ratio;
                bidx = i;
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bidx, off, kWave);
        if (hlex_less(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
        }
        low = min(low, __shfl_xor(low, off, kWave));
    }
    __shared__ double sv[4];
    __shared__ int si[4], sl[4];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        sv[wid] = best;
        si[wid] = bidx;
        sl[wid] = low;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q) {
            if (hlex_less(sv[q], si[q], best, bidx)) {
                best = sv[q];
                bidx = si[q];
            }
            low = min(low, sl[q]);
        }
        const int slot = tb.start[s] + (int)w.x;
        h.rval[slot] = best;
        h.ridx[slot] = bidx;
        h.rlow[slot] = low;
    }
}

// One work-group per set: the pick of step t from its work-groups' minima.
__global__ __launch_bounds__(64) void k_hier_pick(HierPlan h, int t, BatchTable tb) {
    const int s = blockIdx.x;
    if (s >= tb.G) return;
    double best = INFINITY;
    int bidx = INT_MAX, low = INT_MAX;
    for (int q = threadIdx.x; q < tb.count[s]; q += blockDim.x) {
        const int slot = tb.start[s] + q;
        if (hlex_less(h.rval[slot], h.ridx[slot], best, bidx)) {
            best = h.rval[slot];
            bidx = h.ridx[slot];
        }
        low = min(low, h.rlow[slot]);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bidx, off, kWave);
        if (hlex_less(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
        }
        low = min(low, __shfl_xor(low, off, kWave));
    }
    if (threadIdx.x == 0) h.pick[2 * s + t] = bidx != INT_MAX ? bidx : low;
}

// Centres of side 0 and 1 from the two picks; sums cleared.
template <int D>
__global__ __launch_bounds__(64) void k_hier_init(HierPlan h, int nsets) {
    const int s = blockIdx.x;
    if (s >= nsets) return;
    if (!h.need[s]) {                                // small set: a block without KMeans
        if (threadIdx.x == 0) h.active[s] = 0;
        return;
    }
    for (int a = 0; a < 2; ++a) {
        const float* z = h.Z + (size_t)h.pick[2 * s + a] * D;
        float ss = 0.f;
        for (int c = threadIdx.x; c < D; c += blockDim.x) {
            const float v = z[c];
            h.C[((size_t)s * 2 + a) * D + c] = v;
            h.S64[((size_t)s * 2 + a) * D + c] = 0;
            ss += v * v;
        }
        ss = wave_sum(ss);
        if (threadIdx.x == 0) {
            h.cnorm[2 * s + a] = ss;
            h.n32[2 * s + a] = 0;
        }
    }
    if (threadIdx.x == 0) {
        h.active[s] = 1;
        h.changed[s] = 0;
    }
}

// Assignment of every point of an active set to the nearer of its two
// centres (score ||c||^2 - 2 z.c in FP32, ties to side 0), with the fixed-point
// sums of the new sides (exact int64, summed per work-group in LDS).
template <int D>
__global__ __launch_bounds__(256) void k_hier_assign(HierPlan h, int it, BatchTable tb) {
    int s;
    Wg w;
    if (!batch_find(tb, s, w)) return;
    if (!h.active[s]) return;                      // uniform: the set has converged
    __shared__ unsigned long long acc[2][D];
    __shared__ int cnt[2];
    __shared__ int anych;
    for (int q = threadIdx.x; q < 2 * D; q += blockDim.x) acc[q / D][q % D] = 0ull;
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) anych = 0;
    __syncthreads();
    const int beg = h.beg[s], n = h.cnt[s];
    const float* c0 = h.C + (size_t)s * 2 * D;
    const float* c1 = c0 + D;
    const float n0 = h.cnorm[2 * s], n1 = h.cnorm[2 * s + 1];
    const float sc = ldexpf(1.0f, h.fexp);
    bool ch = false;
    for (int pos = (int)w.x * blockDim.x + threadIdx.x; pos < n; pos += (int)w.n * blockDim.x) {
        const int i = h.perm[beg + pos];
        const float* zi = h.Z + (size_t)i * D;
        float d0 = 0.f, d1 = 0.f;
#pragma unroll 4
        for (int c = 0; c < D; c += 4) {
            const float4 z = *reinterpret_cast<const float4*>(zi + c);
            const float4 a = *reinterpret_cast<const float4*>(c0 + c);
            const float4 b = *reinterpret_cast<const float4*>(c1 + c);
            d0 += z.x * a.x + z.y * a.y + z.z * a.z + z.w * a.w;
            d1 += z.x * b.x + z.y * b.y + z.z * b.z + z.w * b.w;
        }
        const float s0 = n0 - 2.0f * d0, s1 = n1 - 2.0f * d1;
        const int side = s1 < s0 ? 1 : 0;
        if (it > 1 && h.side[i] != side) ch = true;
        h.side[i] = (int8_t)side;
        atomicAdd(&cnt[side], 1);
        for (int c = 0; c < D; ++c)
            atomicAdd(&acc[side][c], (unsigned long long)(long long)__float2int_rn(zi[c] * sc));
    }
    if (ch) anych = 1;
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * D; q += blockDim.x) {
        const unsigned long long v = acc[q / D][q % D];
        if (v) atomicAdd(reinterpret_cast<unsigned long long*>(&h.S64[(size_t)s * 2 * D + q]), v);
    }
    if (threadIdx.x < 2 && cnt[threadIdx.x]) atomicAdd(&h.n32[2 * s + threadIdx.x], cnt[threadIdx.x]);
    if (threadIdx.x == 0 && anych) h.changed[s] = 1;
}

// One work-group per set: a set whose sides did not change (from the second
// assignment on) or that reached T_max stops; otherwise its centres become
// the means of its sides (an empty side keeps its centre).  Sums cleared.
template <int D>
__global__ __launch_bounds__(64) void k_hier_update(HierPlan h, int it, int t_max, int nsets) {
    const int s = blockIdx.x;
    if (s >= nsets || !h.active[s]) return;
    const bool stop = (it > 1 && h.changed[s] == 0) || it >= t_max;
    const double inv = ldexp(1.0, -h.fexp);
    for (int a = 0; a < 2; ++a) {
        const int cnt = h.n32[2 * s + a];
        float ss = 0.f;
        for (int c = threadIdx.x; c < D; c += blockDim.x) {
            const size_t o = ((size_t)s * 2 + a) * D + c;
            if (!stop && cnt > 0) {
                const float v = (float)((double)h.S64[o] * inv / (double)cnt);
                h.C[o] = v;
                ss += v * v;
            }
            h.S64[o] = 0;
        }
        ss = wave_sum(ss);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (!stop && cnt > 0) h.cnorm[2 * s + a] = ss;
            h.n32[2 * s + a] = 0;
        }
    }
    if (threadIdx.x == 0) {
        h.changed[s] = 0;
        if (stop) {
            h.active[s] = 0;
            h.iters[s] = it;
        } else {
            atomicAdd(h.live, 1);
        }
    }
}

// Integer counts of Eq. 7 for every set of the level: per node of the set,
// its neighbours in U and, among them, those on its own side; per side the
// node count and the G-degree volume.  counts[s] = {2 m_U, 2 m_1, 2 m_2,
// |U_1|, |U_2|, vol_1, vol_2} (int64).
__global__ __launch_bounds__(256) void k_hier_counts(GraphView g, HierPlan h, BatchTable tb) {
    int s;
    Wg w;
    if (!batch_find(tb, s, w)) return;
    const int beg = h.beg[s], n = h.cnt[s];
    long long mu = 0, ms[2] = {0, 0}, nn[2] = {0, 0}, vol[2] = {0, 0};
    for (int pos = (int)w.x * blockDim.x + threadIdx.x; pos < n; pos += (int)w.n * blockDim.x) {
        const int i = h.perm[beg + pos];
        const int a = h.side[i] & 1;
        const int e0 = g.rp[i], e1 = g.rp[i + 1];
        int in_u = 0, same = 0;
        for (int e = e0; e < e1; ++e) {
            const int j = g.ci[e];
            if (h.setid[j] == s) {
                ++in_u;
                same += h.side[j] == a;
            }
        }
        mu += in_u;
        ms[a] += same;
        nn[a] += 1;
        vol[a] += e1 - e0;
    }
    long long v[7] = {mu, ms[0], ms[1], nn[0], nn[1], vol[0], vol[1]};
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        long long x = wave_sum(v[q]);
        if ((threadIdx.x & (kWave - 1)) == 0 && x)
            atomicAdd(reinterpret_cast<unsigned long long*>(&h.counts[(size_t)s * 7 + q]),
                      (unsigned long long)x);
    }
}

// Children's segments: a node of a set that splits goes to the cursor of its
// side's child (order inside a segment does not matter, see above); a node of
// a set that becomes a block records that tree node as its leaf.
__global__ __launch_bounds__(256) void k_hier_scatter(HierPlan h, BatchTable tb) {
    int s;
    Wg w;
    if (!batch_find(tb, s, w)) return;
    const int beg = h.beg[s], n = h.cnt[s];
    const int child0 = h.child[2 * s];
    for (int pos = (int)w.x * blockDim.x + threadIdx.x; pos < n; pos += (int)w.n * blockDim.x) {
        const int i = h.perm[beg + pos];
        if (child0 < 0) {                            // U is a block
            h.leaf[i] = h.tnode[s];
            h.setid[i] = -1;                         // in both arrays: they alternate
            h.setid_next[i] = -1;
            continue;
        }
        const int a = h.side[i] & 1;
        const int c = h.child[2 * s + a];          // index of the child among next level's sets
        const int at = atomicAdd(&h.cursor[c], 1);
        h.perm_next[at] = i;
        h.setid_next[i] = c;
    }
}

// labels[i] = block number of the node's leaf.
__global__ __launch_bounds__(256) void k_hier_labels(const int32_t* __restrict__ leaf,
                                                     const int32_t* __restrict__ block_of,
                                                     int n, int32_t* __restrict__ labels) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) labels[i] = block_of[leaf[i]];
}

// Trace: 2 t + a for every node, with t the tree node of its set at this
// depth and a its side in that set's KMeans split (0 when none ran).
__global__ __launch_bounds__(256) void k_hier_trace(HierPlan h, int32_t* __restrict__ out,
                                                    BatchTable tb) {
    int s;
    Wg w;
    if (!batch_find(tb, s, w)) return;
    const int beg = h.beg[s], n = h.cnt[s];
    const int need = h.need[s];
    for (int pos = (int)w.x * blockDim.x + threadIdx.x; pos < n; pos += (int)w.n * blockDim.x) {
        const int i = h.perm[beg + pos];
        out[i] = 2 * h.tnode[s] + (need ? (h.side[i] & 1) : 0);
    }
}

__global__ __launch_bounds__(256) void k_hier_setup(const float* __restrict__ Z, int64_t total,
                                                    uint32_t* __restrict__ zmax_bits,
                                                    int32_t* __restrict__ perm,
                                                    int32_t* __restrict__ setid,
                                                    int32_t* __restrict__ setid_next,
                                                    int8_t* __restrict__ side,
                                                    int32_t* __restrict__ leaf, int n) {
    float m = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride)
        m = fmaxf(m, fabsf(Z[q]));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        perm[i] = (int32_t)i;
        setid[i] = 0;
        setid_next[i] = 0;
        side[i] = 0;
        leaf[i] = -1;
    }
    if (!(m <= 3.0e38f)) m = 3.0e38f;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(zmax_bits, __float_as_uint(m));
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_i64(long long* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

void launch_fill_i64(long long* p, int64_t n, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

void launch_hier_setup(const float* Z, int64_t total, uint32_t* zmax_bits, int32_t* perm,
                       int32_t* setid, int32_t* setid_next, int8_t* side, int32_t* leaf, int n,
                       hipStream_t st) {
    launch_fill_i32(reinterpret_cast<int32_t*>(zmax_bits), 1, 0, st);
    const int64_t work = std::max<int64_t>(total, n);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 2048));
    hipLaunchKernelGGL(k_hier_setup, dim3(grid), dim3(256), 0, st, Z, total, zmax_bits, perm,
                       setid, setid_next, side, leaf, n);
}

#define RAFT_HD_SWITCH(D_, CALL) \
    switch (D_) {                \
        case 16: CALL(16); break;  \
        case 32: CALL(32); break;  \
        case 64: CALL(64); break;  \
        case 128: CALL(128); break; \
        case 256: CALL(256); break; \
        default: break;            \
    }

void launch_hier(int kind, const HierPlan& h, const GraphView& g, int d, int t, int t_max,
                 int nsets, const BatchTable& tb, int grid, hipStream_t st) {
    switch (kind) {
        case kHierRace:
            if (grid == 0) return;
#define R(DV) hipLaunchKernelGGL(k_hier_race<DV>, dim3(grid), dim3(256), 0, st, h, t, tb)
            RAFT_HD_SWITCH(d, R)
#undef R
            break;
        case kHierPick:
            if (nsets) hipLaunchKernelGGL(k_hier_pick, dim3(nsets), dim3(64), 0, st, h, t, tb);
            break;
        case kHierInit:
#define I(DV) hipLaunchKernelGGL(k_hier_init<DV>, dim3(nsets), dim3(64), 0, st, h, nsets)
            if (nsets) RAFT_HD_SWITCH(d, I)
#undef I
            break;
        case kHierAssign:
            if (grid == 0) return;
#define A(DV) hipLaunchKernelGGL(k_hier_assign<DV>, dim3(grid), dim3(256), 0, st, h, t, tb)
            RAFT_HD_SWITCH(d, A)
#undef A
            break;
        case kHierUpdate:
#define U(DV) hipLaunchKernelGGL(k_hier_update<DV>, dim3(nsets), dim3(64), 0, st, h, t, t_max, nsets)
            if (nsets) RAFT_HD_SWITCH(d, U)
#undef U
            break;
        case kHierCounts:
            if (grid) hipLaunchKernelGGL(k_hier_counts, dim3(grid), dim3(256), 0, st, g, h, tb);
            break;
        case kHierScatter:
            if (grid) hipLaunchKernelGGL(k_hier_scatter, dim3(grid), dim3(256), 0, st, h, tb);
            break;
        default: break;
    }
}

void launch_hier_trace(const HierPlan& h, int32_t* out, const BatchTable& tb, int grid,
                       hipStream_t st) {
    if (grid) hipLaunchKernelGGL(k_hier_trace, dim3(grid), dim3(256), 0, st, h, out, tb);
}

void launch_hier_labels(const int32_t* leaf, const int32_t* block_of, int n, int32_t* labels,
                        hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_hier_labels, dim3((n + 255) / 256), dim3(256), 0, st, leaf, block_of,
                           n, labels);
}

}  // namespace raft
