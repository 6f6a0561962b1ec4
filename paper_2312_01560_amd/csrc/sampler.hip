// Fast sampling from the degree-corrected SBM (Sec. IV, Alg. 2) on the GPU.
//
// Alg. 2 visits the possible edges between blocks C_r and C_s (r <= s) as a
// virtual |C_r| x |C_s| table and jumps from one positive entry to the next:
// from position m, with E = -ln p (p uniform), the next positive entry is the
// smallest t >= m whose range sum of lambda from m to t exceeds E, found by
// binary search on prefix sums of theta.  Here every ROW of every block
// pair's table (node C_r[x] against C_s) is one independent sequence, run by
// one thread: row x of pair (r, s) draws its jumps from Philox4x64-10 with key
// (seed, 0x30) and counter (r K + s, x, jump, 0), and for r = s starts after
// the diagonal (y > x), so each unordered pair is visited once and no self
// pair is.  A counting pass sizes every row's output, a scan gives the
// offsets, and a writing pass repeats the same draws and stores the edges;
// the CSR is then filled by integer atomics and each row sorted, so the graph
// does not depend on scheduling.  FP64 throughout, without contraction:
// RangeSum(m, t) = (Omega_rs theta_i) (P_s[t + 1] - P_s[m]).
#include "kernels.h"

namespace raft {

constexpr uint64_t kStreamSample = 0x30;

// Row `row` of the row space: pair p with rowoff[p] <= row < rowoff[p + 1].
__device__ __forceinline__ int sbm_pair_of(const int64_t* __restrict__ rowoff, int npairs,
                                           int64_t row) {
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rowoff[mid] <= row)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// WRITE = false: cnt[row] = number of edges of the row.  WRITE = true: the
// row's edges stored from off[row] on, in jump order.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_sbm_rows(SbmPlan p, int64_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ off,
                                                  int32_t* __restrict__ src,
                                                  int32_t* __restrict__ dst) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= p.nrows) return;
    const int pi = sbm_pair_of(p.rowoff, p.npairs, row);
    const int r = p.pair_r[pi], s = p.pair_s[pi];
    const int x = (int)(row - p.rowoff[pi]);
    const int ns = p.bcount[s];
    const int32_t* cs = p.members + p.boff[s];
    const double* ps = p.pref + p.boff[s] + s;          // block s prefix: ns + 1 values
    const int i = p.members[p.boff[r] + x];
    double lam;
    {
#pragma clang fp contract(off)
        lam = p.omega[(size_t)r * p.k + s] * p.theta[i];
    }
    int m = r == s ? x + 1 : 0;
    int64_t out = WRITE ? off[row] : 0;
    int64_t count = 0;
    for (uint64_t jump = 0; m < ns; ++jump) {
        const U64x4 b = philox4x64_10((uint64_t)(r * p.k + s), (uint64_t)x, jump, 0, p.seed,
                                      kStreamSample);
        const double e = -own_ln(uniform52(b.v[0]));
        double total;
        {
#pragma clang fp contract(off)
            total = lam * (ps[ns] - ps[m]);
        }
        if (!(e < total)) break;
        int lo = m, hi = ns - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            double sm;
            {
#pragma clang fp contract(off)
                sm = lam * (ps[mid + 1] - ps[m]);
            }
            if (sm > e)
                hi = mid;
            else
                lo = mid + 1;
        }
        if (WRITE) {
            src[out] = i;
            dst[out] = cs[lo];
            ++out;
        }
        ++count;
        m = lo + 1;
    }
    if (!WRITE) cnt[row] = count;
}

// Exclusive scan of int64 values in three passes: per-block sums, a scan of
// the block sums in one work-group, then each block's own scan plus its
// offset.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(256) void k_scan_sums(const int64_t* __restrict__ v, int64_t n,
                                                   int64_t* __restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    long long s = 0;
    for (int q = threadIdx.x; q < kScanBlock; q += blockDim.x)
        if (base + q < n) s += v[base + q];
    s = wave_sum(s);
    __shared__ long long ws[4];
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(64) void k_scan_bsums(int64_t* __restrict__ bsum, int nb,
                                                   int64_t* __restrict__ total) {
    if (threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t v = bsum[b];
        bsum[b] = acc;
        acc += v;
    }
    *total = acc;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int64_t* __restrict__ v, int64_t n,
                                                    const int64_t* __restrict__ bsum,
                                                    int64_t* __restrict__ out) {
    // 256 threads, 4 consecutive values each: thread-local sums, a
    // work-group scan of them in LDS, then the running values
    __shared__ long long t[256];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
    long long loc[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        loc[q] = base + q < n ? v[base + q] : 0;
        s += loc[q];
    }
    t[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const long long add = threadIdx.x >= d ? t[threadIdx.x - d] : 0;
        __syncthreads();
        t[threadIdx.x] += add;
        __syncthreads();
    }
    long long run = bsum[blockIdx.x] + t[threadIdx.x] - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < n) out[base + q] = run;
        run += loc[q];
    }
}

void launch_scan_i64(const int64_t* v, int64_t n, int64_t* out, int64_t* bsum, int64_t* total,
                     hipStream_t st) {
    const int nb = (int)((n + kScanBlock - 1) / kScanBlock);
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(64), 0, st, bsum, 0, total);
        return;
    }
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, st, v, n, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(64), 0, st, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, st, v, n, bsum, out);
}

// CSR of the sampled graph: degrees (both endpoints of every edge), row
// pointers by the scan, fill by per-row cursors, then every row sorted.
__global__ __launch_bounds__(256) void k_sbm_degrees(const int32_t* __restrict__ src,
                                                     const int32_t* __restrict__ dst, int64_t ne,
                                                     int64_t* __restrict__ deg) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    atomicAdd(reinterpret_cast<unsigned long long*>(&deg[src[e]]), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long*>(&deg[dst[e]]), 1ull);
}

__global__ __launch_bounds__(256) void k_sbm_fill(const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ dst, int64_t ne,
                                                  int64_t* __restrict__ cursor,
                                                  int32_t* __restrict__ col) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int a = src[e], b = dst[e];
    col[atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[a]), 1ull)] = b;
    col[atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[b]), 1ull)] = a;
}

// Shell sort of each row's columns (gaps 701, 301, 132, 57, 23, 10, 4, 1;
// Ciura), one thread per row.
__global__ __launch_bounds__(256) void k_sbm_sort_rows(const int64_t* __restrict__ rp, int n,
                                                       int32_t* __restrict__ col) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t* c = col + rp[i];
    const int len = (int)(rp[i + 1] - rp[i]);
    constexpr int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
#pragma unroll
    for (int gi = 0; gi < 8; ++gi) {
        const int gap = gaps[gi];
        for (int a = gap; a < len; ++a) {
            const int32_t v = c[a];
            int b = a;
            while (b >= gap && c[b - gap] > v) {
                c[b] = c[b - gap];
                b -= gap;
            }
            c[b] = v;
        }
    }
}

void launch_sbm_rows(const SbmPlan& p, bool write, int64_t* cnt, const int64_t* off,
                     int32_t* src, int32_t* dst, hipStream_t st) {
    if (p.nrows == 0) return;
    const dim3 grid((unsigned)((p.nrows + 255) / 256));
    if (write)
        hipLaunchKernelGGL(k_sbm_rows<true>, grid, dim3(256), 0, st, p, cnt, off, src, dst);
    else
        hipLaunchKernelGGL(k_sbm_rows<false>, grid, dim3(256), 0, st, p, cnt, off, src, dst);
}

hipError_t launch_sbm_csr(const int32_t* src, const int32_t* dst, int64_t ne, int n,
                          int64_t* deg, int64_t* rp, int64_t* cursor, int64_t* bsum,
                          int64_t* total, int32_t* col, hipStream_t st) {
    launch_fill_i64(reinterpret_cast<long long*>(deg), (int64_t)n + 1, st);
    if (ne > 0)
        hipLaunchKernelGGL(k_sbm_degrees, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st,
                           src, dst, ne, deg);
    // row_ptr[0..n] = exclusive scan of deg[0..n] (deg[n] = 0 gives nnz last)
    launch_scan_i64(deg, (int64_t)n + 1, rp, bsum, total, st);
    const hipError_t e = hipMemcpyAsync(cursor, rp, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    if (ne > 0)
        hipLaunchKernelGGL(k_sbm_fill, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, src,
                           dst, ne, cursor, col);
    if (n > 0)
        hipLaunchKernelGGL(k_sbm_sort_rows, dim3((n + 255) / 256), dim3(256), 0, st, rp, n, col);
    return hipSuccess;
}

}  // namespace raft
