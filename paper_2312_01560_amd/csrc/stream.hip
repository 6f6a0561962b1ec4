// Streaming update (Sec. III-D) on the device: new edges merged into the
// CSR, hop balls around their endpoints, and row gathers/scatters so the
// projection and GCN levels can be recomputed on their balls only.
//
// New edges come as a directed list (both directions of every edge) sorted
// by (row, column); add_off is the exclusive scan of the per-row counts, so
// row i's new columns are cols[add_off[i] .. add_off[i + 1]) and its first
// entry in the merged CSR is rp[i] + add_off[i].  Each old entry moves past
// the new columns below it and each new entry past the old columns below it
// (binary searches in the two sorted lists), so the merge is one parallel
// pass with no order dependence; a new column equal to an old one flags the
// edge as already present.
#include "kernels.h"

namespace raft {

__global__ __launch_bounds__(256) void k_stream_count(const int32_t* __restrict__ rows, int64_t m,
                                                      int64_t* __restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[rows[e]]), 1ull);
}

// Entries of the sorted list a[0..len) below v; *hit when v is in it.
__device__ __forceinline__ int count_below(const int32_t* __restrict__ a, int len, int32_t v,
                                           bool* hit) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    *hit = lo < len && a[lo] == v;
    return lo;
}

// One wave per row.
__global__ __launch_bounds__(256) void k_stream_merge(const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci,
                                                      const int64_t* __restrict__ add_off,
                                                      const int32_t* __restrict__ cols, int32_t n,
                                                      int32_t* __restrict__ rp_new,
                                                      int32_t* __restrict__ ci_new,
                                                      int32_t* __restrict__ status) {
    const int i = blockIdx.x * (blockDim.x / kWave) + (int)(threadIdx.x / kWave);
    if (i >= n) return;                              // uniform per wave
    const int lane = threadIdx.x & (kWave - 1);
    const int ob = rp[i], olen = rp[i + 1] - ob;
    const int nb = (int)add_off[i], nlen = (int)(add_off[i + 1] - nb);
    const int base = ob + nb;
    if (lane == 0) {
        rp_new[i] = base;
        if (i == n - 1) rp_new[n] = ob + olen + nb + nlen;
    }
    const int32_t* oc = ci + ob;
    const int32_t* nc = cols + nb;
    bool dup = false;
    for (int k = lane; k < olen; k += kWave) {
        const int32_t c = oc[k];
        bool hit = false;
        const int below = nlen ? count_below(nc, nlen, c, &hit) : 0;
        dup |= hit;
        ci_new[base + k + below] = c;
    }
    for (int k = lane; k < nlen; k += kWave) {
        const int32_t c = nc[k];
        bool hit = false;
        const int below = count_below(oc, olen, c, &hit);
        ci_new[base + k + below] = c;
    }
    if (dup) atomicOr(status, kStatusCsrSym);
}

__global__ __launch_bounds__(256) void k_stream_fill(int32_t* __restrict__ p, int32_t n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_stream_seed(const int32_t* __restrict__ v, int32_t nv,
                                                     int32_t* __restrict__ dist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv) dist[v[i]] = 0;
}

// Level t of the breadth-first search: the neighbours of rows at distance
// t - 1 that are farther than t get t.  Rows written here are at distance t
// and are not read as sources in this pass, and every writer stores the
// same value, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_stream_expand(const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, int32_t n,
                                                       int32_t* __restrict__ dist, int32_t t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || dist[i] != t - 1) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        if (dist[j] > t) dist[j] = t;
    }
}

__global__ __launch_bounds__(256) void k_stream_flag(const int32_t* __restrict__ dist, int32_t n,
                                                     int32_t t, int64_t* __restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = dist[i] <= t ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_stream_compact(const int32_t* __restrict__ dist, int32_t n,
                                                        int32_t t, const int64_t* __restrict__ pos,
                                                        int32_t* __restrict__ list) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && dist[i] <= t) list[pos[i]] = i;
}

// dst[r] = src[list[r]] (GATHER) or dst[list[r]] = src[r], rows of L floats
// (L a multiple of 4), a float4 per thread.
template <bool GATHER>
__global__ __launch_bounds__(256) void k_stream_rows(const int32_t* __restrict__ list, int32_t c,
                                                     int L, const float* __restrict__ src,
                                                     float* __restrict__ dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int L4 = L / 4;
    if (q >= (int64_t)c * L4) return;
    const int r = (int)(q / L4), col = (int)(q % L4) * 4;
    const int64_t g = (int64_t)list[r] * L + col, k = (int64_t)r * L + col;
    if (GATHER)
        *reinterpret_cast<float4*>(dst + k) = *reinterpret_cast<const float4*>(src + g);
    else
        *reinterpret_cast<float4*>(dst + g) = *reinterpret_cast<const float4*>(src + k);
}

static unsigned blocks_for(int64_t threads) { return (unsigned)((threads + 255) / 256); }

void launch_stream_merge(const int32_t* rp, const int32_t* ci, int32_t n, const int32_t* rows,
                         const int32_t* cols, int64_t m, int64_t* add_cnt, int64_t* add_off,
                         int64_t* bsum, int64_t* total, int32_t* rp_new, int32_t* ci_new,
                         int32_t* status, hipStream_t st) {
    launch_fill_i64(reinterpret_cast<long long*>(add_cnt), (int64_t)n + 1, st);
    if (m > 0)
        hipLaunchKernelGGL(k_stream_count, dim3(blocks_for(m)), dim3(256), 0, st, rows, m, add_cnt);
    launch_scan_i64(add_cnt, (int64_t)n + 1, add_off, bsum, total, st);
    hipLaunchKernelGGL(k_stream_merge, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, rp, ci,
                       add_off, cols, n, rp_new, ci_new, status);
}

void launch_stream_balls(const int32_t* rp, const int32_t* ci, int32_t n, const int32_t* vprime,
                         int32_t nv, int radius, int32_t* dist, int64_t* flag, int64_t* pos,
                         int64_t* bsum, int64_t* totals, int32_t* lists, hipStream_t st) {
    hipLaunchKernelGGL(k_stream_fill, dim3(blocks_for(n)), dim3(256), 0, st, dist, n, radius + 1);
    if (nv > 0)
        hipLaunchKernelGGL(k_stream_seed, dim3(blocks_for(nv)), dim3(256), 0, st, vprime, nv, dist);
    for (int t = 1; t <= radius; ++t)
        hipLaunchKernelGGL(k_stream_expand, dim3(blocks_for(n)), dim3(256), 0, st, rp, ci, n, dist,
                           t);
    for (int t = 1; t <= radius; ++t) {
        hipLaunchKernelGGL(k_stream_flag, dim3(blocks_for(n)), dim3(256), 0, st, dist, n, t, flag);
        launch_scan_i64(flag, n, pos, bsum, totals + (t - 1), st);
        hipLaunchKernelGGL(k_stream_compact, dim3(blocks_for(n)), dim3(256), 0, st, dist, n, t,
                           pos, lists + (size_t)(t - 1) * n);
    }
}

void launch_stream_rows(bool gather, const int32_t* list, int32_t c, int L, const float* src,
                        float* dst, hipStream_t st) {
    const int64_t threads = (int64_t)c * (L / 4);
    if (threads == 0) return;
    if (gather)
        hipLaunchKernelGGL(k_stream_rows<true>, dim3(blocks_for(threads)), dim3(256), 0, st, list, c,
                           L, src, dst);
    else
        hipLaunchKernelGGL(k_stream_rows<false>, dim3(blocks_for(threads)), dim3(256), 0, st, list,
                           c, L, src, dst);
}

}  // namespace raft
