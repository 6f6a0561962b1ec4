// Sparse x tall-skinny products of the projection (Sec. III-A) and of the GCN
// aggregation (Sec. III-B, Eq. 6):
//   NCUT        y_i = s_i  sum_{j in N(i)} s_j x_j                   (M, Eq. 2)
//   MOD_FULL    y_i = sum_{j in N(i)} x_j - (d_i/2e) (d^T x)           (B, Eq. 4)
//   MOD_REDUCED y_i = sum_{j in N(i)} x_j - (d_i/2e) sum_j d_j x_j     (Q~)
//   GCN         y_i = sh_i (sum_{j in N(i)} sh_j x_j + sh_i x_i)       (A_hat_n)
// with s = D^-1/2 and sh = (D+1)^-1/2.
//
// Row-split CSR with one row per lane group: L/4 lanes hold one feature row
// (a float4 each), so a wave works on 256/L rows side by side, taken in the
// graph's degree-class order (rows of similar length together, the longest
// first); per batch of 16 edges the lanes
// of a row group load the same column indices (broadcast loads), then all 16
// neighbour rows are gathered back to back, the edge weight (a per-node
// scale) loaded next to each feature row.  For L >= 64 work-groups take
// 32-column slices, placed per XCD (see SpmmGeom).  The optional
// epilogue accumulates FP64 partials of d^T y per work-group (the rank-1 term
// of the next MOD_FULL step) in a fixed order, so the column sums are
// deterministic.
#include "kernels.h"

namespace raft {

constexpr int kSpmmWaves = 4;

template <int L, int OP>
__device__ __forceinline__ float edge_weight(const GraphView& g, int j) {
    if (OP == kOpNcut) return g.s[j];
    if (OP == kOpGcn) return g.sh[j];
    if (OP == kOpModReduced) return (float)g.deg[j];
    return 1.f;
}

// Column slices: for L >= 64 a work-group handles one slice of W = 32
// columns (one 128-byte line of a feature row) of a block of rows, and the
// work-groups are dealt to the XCDs (work-group b to XCD b mod 8) so that
// each XCD only ever touches its own slices: its L2 then holds N x 128 bytes
// (or 2 slices' worth at L = 64) of X instead of all of it, and the random
// neighbour gathers hit L2 more often.  For L <= 32 there is one slice.
// Wider rows (L > 256, more than 8 slices) give each XCD NS / 8 slices
// (SPX): block b runs slice (b mod 8) SPX + (b / 8) mod SPX of row block
// (b / 8) / SPX.
template <int L>
struct SpmmGeom {
    static constexpr int W = L >= 64 ? 32 : L;   // columns per slice
    static constexpr int NS = L / W;             // slices
    static constexpr int XS = NS <= 8 ? 8 / NS : 1;   // XCDs per slice
    static constexpr int SPX = NS > 8 ? NS / 8 : 1;   // slices per XCD
    static constexpr int LANES = W / 4;          // lanes per feature row slice
    static constexpr int G = kWave / LANES;      // rows side by side per wave
};

// Sum over the edges beg..end-1 of one row (this lane's 4 columns), in
// batches of 16: the lanes of a row group load the same column indices
// (broadcast loads), then all feature rows are gathered; the next batch's
// indices are requested before this batch's gathers, so each batch waits on
// memory once.  maxdeg: the longest range among the wave's row groups.
template <int L, int OP>
__device__ __forceinline__ void spmm_edges(const GraphView& g, const float* __restrict__ x, int cofs,
                                           int beg, int end, int maxdeg, float4& acc,
                                           float4& acc2) {
    int jv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = beg + q;
        jv[q] = e < end ? g.ci[e] : -1;
    }
    for (int base = 0; base < maxdeg; base += 16) {
        int jn[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = beg + base + 16 + q;
            jn[q] = e < end ? g.ci[e] : -1;
        }
        float4 xv[16];
        float wv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            xv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            wv[q] = 0.f;
            if (jv[q] >= 0) {
                xv[q] = *reinterpret_cast<const float4*>(x + (size_t)jv[q] * L + cofs);
                wv[q] = edge_weight<L, OP>(g, jv[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (OP == kOpModFull) {
                acc.x += xv[q].x;
                acc.y += xv[q].y;
                acc.z += xv[q].z;
                acc.w += xv[q].w;
            } else if (OP == kOpModReduced) {
                acc.x += xv[q].x;
                acc.y += xv[q].y;
                acc.z += xv[q].z;
                acc.w += xv[q].w;
                acc2.x += wv[q] * xv[q].x;
                acc2.y += wv[q] * xv[q].y;
                acc2.z += wv[q] * xv[q].z;
                acc2.w += wv[q] * xv[q].w;
            } else {
                acc.x += wv[q] * xv[q].x;
                acc.y += wv[q] * xv[q].y;
                acc.z += wv[q] * xv[q].z;
                acc.w += wv[q] * xv[q].w;
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) jv[q] = jn[q];
    }
}

// Row i's output from its neighbour sum (this lane's 4 columns), written to
// y, and its term d_i y_i added to the column sums.
template <int L, int OP, bool CS>
__device__ __forceinline__ void spmm_row_out(const GraphView& g, const float* __restrict__ x,
                                             float* __restrict__ y, const float* __restrict__ cvec,
                                             int cofs, int i, float4 acc, float4 acc2, double& cs0,
                                             double& cs1, double& cs2, double& cs3) {
    float4 o;
    if (OP == kOpNcut) {
        const float si = g.s[i];
        o = make_float4(si * acc.x, si * acc.y, si * acc.z, si * acc.w);
    } else if (OP == kOpGcn) {
        const float si = g.sh[i];
        const float4 xi = *reinterpret_cast<const float4*>(x + (size_t)i * L + cofs);
        o = make_float4(si * (acc.x + si * xi.x), si * (acc.y + si * xi.y),
                        si * (acc.z + si * xi.z), si * (acc.w + si * xi.w));
    } else if (OP == kOpModFull) {
        const float ci = g.dcoef[i];
        const float4 c = *reinterpret_cast<const float4*>(cvec + cofs);
        o = make_float4(acc.x - ci * c.x, acc.y - ci * c.y, acc.z - ci * c.z, acc.w - ci * c.w);
    } else {
        const float ci = g.dcoef[i];
        o = make_float4(acc.x - ci * acc2.x, acc.y - ci * acc2.y, acc.z - ci * acc2.z,
                        acc.w - ci * acc2.w);
    }
    *reinterpret_cast<float4*>(y + (size_t)i * L + cofs) = o;
    if (CS) {
        const double di = (double)g.deg[i];
        cs0 += di * (double)o.x;
        cs1 += di * (double)o.y;
        cs2 += di * (double)o.z;
        cs3 += di * (double)o.w;
    }
}

// Rows with more stored entries than this are summed by the whole wave: each
// of its G row groups takes one of G equal runs of the row's edges and the
// runs' sums are combined by a fixed butterfly, so a long row does not keep
// one row group walking alone.  The treatment depends only on the row (its
// length), not on where the row order places it, so a row list (the
// streaming levels) sums every row exactly as the full pass does.
constexpr int kSpmmSplit = 512;

template <int L, int OP, bool CS>
__device__ __forceinline__ void spmm_body(const GraphView& g, const float* __restrict__ x,
                                          float* __restrict__ y, const float* __restrict__ cvec,
                                          double* __restrict__ cpart, int R, int nrb, int b) {
    using GE = SpmmGeom<L>;
    constexpr int W = GE::W, LANES = GE::LANES, G = GE::G, XS = GE::XS, SPX = GE::SPX;
    const int xcd = b % 8;
    const int sl = SPX > 1 ? xcd * SPX + (b / 8) % SPX : xcd / XS;        // column slice
    const int rb = SPX > 1 ? (b / 8) / SPX : (b / 8) * XS + xcd % XS;     // row block
    if (rb >= nrb) return;                          // uniform: padding of the grid
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int slot = lane / LANES;
    const int sub = lane % LANES;
    const int cofs = sl * W + sub * 4;              // this lane's 4 columns
    const int rbeg = rb * R, rend = min(g.n, rbeg + R);
    double cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;
    for (int r0 = rbeg + wid * G; r0 < rend; r0 += kSpmmWaves * G) {
        // position r0 + slot of the degree-class order
        const bool valid = r0 + slot < rend;
        const int i = valid ? g.order[r0 + slot] : 0;
        const int beg = g.rp[i];
        const int end = valid ? g.rp[i + 1] : beg;
        const bool heavy = end - beg > kSpmmSplit;
        int maxdeg = heavy ? 0 : end - beg;
#pragma unroll
        for (int off = LANES; off < kWave; off <<= 1)
            maxdeg = max(maxdeg, __shfl_xor(maxdeg, off, kWave));
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 acc2 = make_float4(0.f, 0.f, 0.f, 0.f);
        spmm_edges<L, OP>(g, x, cofs, beg, heavy ? beg : end, maxdeg, acc, acc2);
        if (valid && !heavy)
            spmm_row_out<L, OP, CS>(g, x, y, cvec, cofs, i, acc, acc2, cs0, cs1, cs2, cs3);
        // the pass's long rows, one after another, over all row groups
        for (uint64_t hm = __ballot(heavy && sub == 0); hm != 0; hm &= hm - 1) {
            const int hl = __builtin_ctzll(hm);
            const int hi = __shfl(i, hl, kWave);
            const int hb = __shfl(beg, hl, kWave), he = __shfl(end, hl, kWave);
            const int run = (he - hb + G - 1) / G;
            const int b0 = min(he, hb + slot * run), b1 = min(he, b0 + run);
            float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
            float4 h2 = make_float4(0.f, 0.f, 0.f, 0.f);
            spmm_edges<L, OP>(g, x, cofs, b0, b1, run, h, h2);
#pragma unroll
            for (int off = LANES; off < kWave; off <<= 1) {
                h.x += __shfl_xor(h.x, off, kWave);
                h.y += __shfl_xor(h.y, off, kWave);
                h.z += __shfl_xor(h.z, off, kWave);
                h.w += __shfl_xor(h.w, off, kWave);
                if (OP == kOpModReduced) {
                    h2.x += __shfl_xor(h2.x, off, kWave);
                    h2.y += __shfl_xor(h2.y, off, kWave);
                    h2.z += __shfl_xor(h2.z, off, kWave);
                    h2.w += __shfl_xor(h2.w, off, kWave);
                }
            }
            if (slot == 0) spmm_row_out<L, OP, CS>(g, x, y, cvec, cofs, hi, h, h2, cs0, cs1, cs2, cs3);
        }
    }
    if (CS) {
        // fold the row slots of the wave (fixed butterfly order), then the
        // waves; the row block's partial row gets this slice's W columns
#pragma unroll
        for (int off = LANES; off < kWave; off <<= 1) {
            cs0 += __shfl_xor(cs0, off, kWave);
            cs1 += __shfl_xor(cs1, off, kWave);
            cs2 += __shfl_xor(cs2, off, kWave);
            cs3 += __shfl_xor(cs3, off, kWave);
        }
        __shared__ double red[kSpmmWaves][W];
        if (slot == 0) {
            red[wid][sub * 4 + 0] = cs0;
            red[wid][sub * 4 + 1] = cs1;
            red[wid][sub * 4 + 2] = cs2;
            red[wid][sub * 4 + 3] = cs3;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < W; c += blockDim.x) {
            double s = 0;
            for (int w = 0; w < kSpmmWaves; ++w) s += red[w][c];
            cpart[(size_t)rb * L + sl * W + c] = s;
        }
    }
}

template <int L, int OP, bool CS>
__global__ __launch_bounds__(256) void k_spmm(GraphView g, const float* __restrict__ x,
                                              float* __restrict__ y,
                                              const float* __restrict__ cvec,
                                              double* __restrict__ cpart, int R, int nrb) {
    spmm_body<L, OP, CS>(g, x, y, cvec, cpart, R, nrb, (int)blockIdx.x);
}

// Batched: one launch over the graphs of a block-diagonal CSR, each graph's
// blocks doing exactly what its own launch would (same row blocks, slices
// and partial order), so every graph's result equals its single-graph run.
template <int L, int OP, bool CS>
__global__ __launch_bounds__(256) void k_spmm_b(const SpmmItem* __restrict__ items,
                                                const float* __restrict__ x,
                                                float* __restrict__ y, BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const SpmmItem& it = items[gi];
    spmm_body<L, OP, CS>(it.g, x, y, it.cvec, it.cpart, it.R, it.nrb, (int)w.x);
}

// FP64 partials of d^T x over the same row blocks as k_spmm<L>.
// Rows are the graph's own (local index i, global row base + i).
template <int L>
__device__ __forceinline__ void colsum_part_body(const GraphView& g, const float* __restrict__ x,
                                                 double* __restrict__ cpart, int rpw, int b) {
    constexpr int LANES = L / 4;
    constexpr int G = kWave / LANES;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int slot = lane / LANES;
    const int sub = lane % LANES;
    const int row0 = (b * kSpmmWaves + wid) * rpw * G;
    double cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;
    for (int r = 0; r < rpw; ++r) {
        const int i = row0 + r * G + slot;
        if (i < g.n) {
            const size_t gi = (size_t)g.base + i;
            const float4 o = *reinterpret_cast<const float4*>(x + gi * L + sub * 4);
            const double di = (double)g.deg[gi];
            cs0 += di * (double)o.x;
            cs1 += di * (double)o.y;
            cs2 += di * (double)o.z;
            cs3 += di * (double)o.w;
        }
    }
#pragma unroll
    for (int off = LANES; off < kWave; off <<= 1) {
        cs0 += __shfl_xor(cs0, off, kWave);
        cs1 += __shfl_xor(cs1, off, kWave);
        cs2 += __shfl_xor(cs2, off, kWave);
        cs3 += __shfl_xor(cs3, off, kWave);
    }
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
        cpart[(size_t)b * L + c] = s;
    }
}

template <int L>
__global__ __launch_bounds__(256) void k_colsum_part(GraphView g, const float* __restrict__ x,
                                                     double* __restrict__ cpart, int rpw) {
    colsum_part_body<L>(g, x, cpart, rpw, (int)blockIdx.x);
}

// L > 256: block (row block rb, 256-column chunk cc); a wave takes one row at
// a time, its 64 lanes 4 columns each.
template <int L>
__global__ __launch_bounds__(256) void k_colsum_part_wide(GraphView g, const float* __restrict__ x,
                                                          double* __restrict__ cpart, int rpw) {
    constexpr int CH = L / 256;
    const int rb = blockIdx.x / CH, cc = blockIdx.x % CH;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int col = cc * 256 + lane * 4;
    const int row0 = (rb * kSpmmWaves + wid) * rpw;
    double cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;
    for (int r = 0; r < rpw; ++r) {
        const int i = row0 + r;
        if (i < g.n) {
            const size_t gi = (size_t)g.base + i;
            const float4 o = *reinterpret_cast<const float4*>(x + gi * L + col);
            const double di = (double)g.deg[gi];
            cs0 += di * (double)o.x;
            cs1 += di * (double)o.y;
            cs2 += di * (double)o.z;
            cs3 += di * (double)o.w;
        }
    }
    __shared__ double red[kSpmmWaves][256];
    red[wid][lane * 4 + 0] = cs0;
    red[wid][lane * 4 + 1] = cs1;
    red[wid][lane * 4 + 2] = cs2;
    red[wid][lane * 4 + 3] = cs3;
    __syncthreads();
    for (int c = threadIdx.x; c < 256; c += blockDim.x) {
        double s2 = 0;
        for (int w = 0; w < kSpmmWaves; ++w) s2 += red[w][c];
        cpart[(size_t)rb * L + cc * 256 + c] = s2;
    }
}

template <int L>
__global__ __launch_bounds__(256) void k_colsum_part_b(const ColsumItem* __restrict__ items,
                                                       const float* __restrict__ x, BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const ColsumItem& it = items[gi];
    colsum_part_body<L>(it.g, x, it.part, it.rpw, (int)w.x);
}

// c = sum over the partial rows in two fixed-order levels: block b sums the
// contiguous slice b of the partials into stage[b]; one block then sums the
// stage rows in order.  cvec = FP32(c).
constexpr int kColsumSlices = 64;
static_assert(kColsumSlices == kColsumSliceBlocks && kColsumSlices <= kColsumStageRows,
              "colsum stage rows");

__device__ __forceinline__ void colsum_slices_body(const double* __restrict__ part, int parts,
                                                   int L, double* __restrict__ stage, int bx) {
    const int per = (parts + kColsumSlices - 1) / kColsumSlices;
    const int b0 = bx * per, b1 = min(parts, b0 + per);
    for (int col = threadIdx.x; col < L; col += blockDim.x) {
        double s = 0;
        int b = b0;
        for (; b + 4 <= b1; b += 4)
            s += part[(size_t)b * L + col] + part[(size_t)(b + 1) * L + col] +
                 part[(size_t)(b + 2) * L + col] + part[(size_t)(b + 3) * L + col];
        for (; b < b1; ++b) s += part[(size_t)b * L + col];
        stage[(size_t)bx * L + col] = s;
    }
}

__global__ __launch_bounds__(256) void k_colsum_slices(const double* __restrict__ part, int parts,
                                                       int L, double* __restrict__ stage) {
    colsum_slices_body(part, parts, L, stage, (int)blockIdx.x);
}

__device__ __forceinline__ void colsum_finish_body(const double* __restrict__ stage, int L,
                                                   double* __restrict__ c64,
                                                   float* __restrict__ cvec) {
    for (int col = threadIdx.x; col < L; col += blockDim.x) {
        double t = 0;
        for (int k = 0; k < kColsumSlices; ++k) t += stage[(size_t)k * L + col];
        c64[col] = t;
        cvec[col] = (float)t;
    }
}

__global__ __launch_bounds__(256) void k_colsum_finish(const double* __restrict__ stage, int L,
                                                       double* __restrict__ c64,
                                                       float* __restrict__ cvec) {
    colsum_finish_body(stage, L, c64, cvec);
}

// Batched forms: kColsumSlices blocks per graph, then one block per graph.
__global__ __launch_bounds__(256) void k_colsum_slices_b(const ColsumItem* __restrict__ items,
                                                         int L, BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const ColsumItem& it = items[gi];
    colsum_slices_body(it.part, it.parts, L, it.part + (size_t)it.parts * L, (int)w.x);
}

__global__ __launch_bounds__(256) void k_colsum_finish_b(const ColsumItem* __restrict__ items,
                                                         int L, BatchTable t) {
    int gi;
    Wg w;
    if (!batch_find(t, gi, w)) return;
    const ColsumItem& it = items[gi];
    colsum_finish_body(it.part + (size_t)it.parts * L, L, it.c64, it.cvec);
}

// ---- merge-path SpMM -------------------------------------------------------
// The same products with the work split evenly along the merge path of the
// CSR (Merrill & Garland, SC'16): the path interleaves the N row ends with the
// nnz stored entries (an entry e of row i comes before the end of row i), and
// each lane group takes kMergeT consecutive path items for one column slice,
// whatever the row lengths.  A group finds its start and end coordinates
// (row, entry) by binary search on the row pointers, gathers the feature rows
// of its entries in batches of 16 (indices first, then the rows back to back)
// and sums them row by row in entry order.  A row that ends in the group's
// range and began there is finished in place (epilogue and store); a row
// still open at the end of the range leaves its partial sum as the range's
// carry, and a row that began in an earlier range and ends in this one leaves
// its last partial as the range's head; a fix-up pass adds, for every head,
// the carries of the earlier ranges of that row in range order and applies
// the epilogue, so the result does not depend on scheduling.
constexpr int kMergeT = 256;

// Merge-path coordinate of diagonal k: (row i, entry e) with i + e = k, i the
// number of row ends before the k-th path item.
__device__ __forceinline__ void merge_search(const int32_t* __restrict__ rp, int n, int64_t nnz,
                                             int64_t k, int& i, int& e) {
    int64_t lo = k - nnz > 0 ? k - nnz : 0;
    int64_t hi = k < n ? k : n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid + 1] <= k - mid - 1)
            lo = mid + 1;
        else
            hi = mid;
    }
    i = (int)lo;
    e = (int)(k - lo);
}

template <int OP>
__device__ __forceinline__ float4 merge_epilogue(const GraphView& g, int i, float4 acc, float4 acc2,
                                                 const float* __restrict__ x, int L, int cofs,
                                                 const float* __restrict__ cvec) {
    if (OP == kOpNcut) {
        const float si = g.s[i];
        return make_float4(si * acc.x, si * acc.y, si * acc.z, si * acc.w);
    }
    if (OP == kOpGcn) {
        const float si = g.sh[i];
        const float4 xi = *reinterpret_cast<const float4*>(x + (size_t)i * L + cofs);
        return make_float4(si * (acc.x + si * xi.x), si * (acc.y + si * xi.y),
                           si * (acc.z + si * xi.z), si * (acc.w + si * xi.w));
    }
    if (OP == kOpModFull) {
        const float ci = g.dcoef[i];
        const float4 c = *reinterpret_cast<const float4*>(cvec + cofs);
        return make_float4(acc.x - ci * c.x, acc.y - ci * c.y, acc.z - ci * c.z, acc.w - ci * c.w);
    }
    const float ci = g.dcoef[i];
    return make_float4(acc.x - ci * acc2.x, acc.y - ci * acc2.y, acc.z - ci * acc2.z,
                       acc.w - ci * acc2.w);
}

// Partial buffers: part[(2 r + q) L + col], r = range, q = 0 carry, 1 head;
// MOD_REDUCED keeps its second sum (sum d_j x_j) at part2 with the same
// layout.  prow[2 r + q] = the row of that partial, -1 for none.
template <int L, int OP>
__global__ __launch_bounds__(256) void k_spmm_merge(GraphView g, const float* __restrict__ x,
                                                    float* __restrict__ y,
                                                    const float* __restrict__ cvec,
                                                    float* __restrict__ part,
                                                    float* __restrict__ part2,
                                                    int32_t* __restrict__ prow, int nranges) {
    using GE = SpmmGeom<L>;
    constexpr int W = GE::W, LANES = GE::LANES, G = GE::G, XS = GE::XS;
    const int b = blockIdx.x;
    const int xcd = b % 8;
    const int sl = xcd / XS;
    const int rbk = (b / 8) * XS + xcd % XS;       // block of ranges
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int slot = lane / LANES;
    const int sub = lane % LANES;
    const int r = (rbk * kSpmmWaves + wid) * G + slot;
    const int cofs = sl * W + sub * 4;
    if (r >= nranges) return;                       // whole lane groups: no wave-wide sync below
    const int64_t total = (int64_t)g.n + g.nnz;
    const int64_t k0 = (int64_t)r * kMergeT;
    const int64_t k1 = k0 + kMergeT < total ? k0 + kMergeT : total;
    int i0, e0, i1, e1;
    merge_search(g.rp, g.n, g.nnz, k0, i0, e0);
    merge_search(g.rp, g.n, g.nnz, k1, i1, e1);
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 acc = zero, acc2 = zero;
    int i = i0;
    int rend = i < g.n ? g.rp[i + 1] : e1;
    const bool began_before = i0 < g.n && e0 > g.rp[i0];
    bool first = true;
    bool any = false;                               // an entry of row i summed in this range
    // closes row i (every row ending before entry e, or before the range end)
#define MERGE_CLOSE_ROW()                                                                      \
    {                                                                                          \
        if (first && began_before) {                                                           \
            *reinterpret_cast<float4*>(part + (size_t)(2 * r + 1) * L + cofs) = acc;          \
            if (OP == kOpModReduced)                                                           \
                *reinterpret_cast<float4*>(part2 + (size_t)(2 * r + 1) * L + cofs) = acc2;    \
            if (sub == 0 && sl == 0) prow[2 * r + 1] = i;                                      \
        } else {                                                                               \
            *reinterpret_cast<float4*>(y + (size_t)i * L + cofs) =                            \
                merge_epilogue<OP>(g, i, acc, acc2, x, L, cofs, cvec);                         \
        }                                                                                      \
        first = false;                                                                         \
        any = false;                                                                           \
        acc = zero;                                                                            \
        acc2 = zero;                                                                           \
        ++i;                                                                                   \
        rend = i < g.n ? g.rp[i + 1] : e1;                                                     \
    }
    for (int base = e0; base < e1; base += 16) {
        // the entries [base, base + 16) of the range, gathered back to back
        int jv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) jv[q] = base + q < e1 ? g.ci[base + q] : -1;
        float4 xv[16];
        float wv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            xv[q] = zero;
            wv[q] = 0.f;
            if (jv[q] >= 0) {
                xv[q] = *reinterpret_cast<const float4*>(x + (size_t)jv[q] * L + cofs);
                wv[q] = edge_weight<L, OP>(g, jv[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = base + q;
            if (e < e1) {
                // a row ending before entry e ends inside this range (i < i1)
                while (rend <= e) MERGE_CLOSE_ROW()
                if (OP == kOpModFull) {
                    acc.x += xv[q].x;
                    acc.y += xv[q].y;
                    acc.z += xv[q].z;
                    acc.w += xv[q].w;
                } else if (OP == kOpModReduced) {
                    acc.x += xv[q].x;
                    acc.y += xv[q].y;
                    acc.z += xv[q].z;
                    acc.w += xv[q].w;
                    acc2.x += wv[q] * xv[q].x;
                    acc2.y += wv[q] * xv[q].y;
                    acc2.z += wv[q] * xv[q].z;
                    acc2.w += wv[q] * xv[q].w;
                } else {
                    acc.x += wv[q] * xv[q].x;
                    acc.y += wv[q] * xv[q].y;
                    acc.z += wv[q] * xv[q].z;
                    acc.w += wv[q] * xv[q].w;
                }
                any = true;
            }
        }
    }
    // the row ends after the last entry of the range
    while (i < i1) MERGE_CLOSE_ROW()
#undef MERGE_CLOSE_ROW
    // row i1 still open at the end of the range
    const bool carry = any && i1 < g.n;
    if (carry) {
        *reinterpret_cast<float4*>(part + (size_t)(2 * r) * L + cofs) = acc;
        if (OP == kOpModReduced)
            *reinterpret_cast<float4*>(part2 + (size_t)(2 * r) * L + cofs) = acc2;
    }
    if (sub == 0 && sl == 0) {
        prow[2 * r] = carry ? i1 : -1;
        if (!(began_before && i1 > i0)) prow[2 * r + 1] = -1;
    }
}

// For every range with a head: the carries of the earlier ranges of that row
// (consecutive ranges ending inside it), in range order, then the head, and
// the epilogue.
template <int L, int OP>
__global__ __launch_bounds__(256) void k_spmm_merge_fix(GraphView g, const float* __restrict__ x,
                                                        float* __restrict__ y,
                                                        const float* __restrict__ cvec,
                                                        const float* __restrict__ part,
                                                        const float* __restrict__ part2,
                                                        const int32_t* __restrict__ prow,
                                                        int nranges) {
    using GE = SpmmGeom<L>;
    constexpr int W = GE::W, LANES = GE::LANES, G = GE::G;
    constexpr int NS = GE::NS;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int slot = lane / LANES;
    const int sub = lane % LANES;
    const int gi = (blockIdx.x * kSpmmWaves + wid) * G + slot;   // (range, slice)
    const int r = gi / NS, sl = gi % NS;
    if (r >= nranges) return;
    const int row = prow[2 * r + 1];
    if (row < 0) return;
    const int cofs = sl * W + sub * 4;
    int r0 = r;
    while (r0 > 0 && prow[2 * (r0 - 1)] == row) --r0;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f), acc2 = acc;
    for (int q = r0; q <= r; ++q) {
        const size_t o = (size_t)(2 * q + (q == r ? 1 : 0)) * L + cofs;
        const float4 v = *reinterpret_cast<const float4*>(part + o);
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
        if (OP == kOpModReduced) {
            const float4 v2 = *reinterpret_cast<const float4*>(part2 + o);
            acc2.x += v2.x;
            acc2.y += v2.y;
            acc2.z += v2.z;
            acc2.w += v2.w;
        }
    }
    *reinterpret_cast<float4*>(y + (size_t)row * L + cofs) =
        merge_epilogue<OP>(g, row, acc, acc2, x, L, cofs, cvec);
}

int spmm_merge_ranges(int32_t n, int64_t nnz) {
    return (int)(((int64_t)n + nnz + kMergeT - 1) / kMergeT);
}

size_t spmm_merge_ws_bytes(int32_t n, int64_t nnz, int L, int op) {
    const size_t nr = (size_t)spmm_merge_ranges(n, nnz);
    const size_t part = ((nr * 2 * L * sizeof(float)) + 255) / 256 * 256;
    const size_t rows = ((nr * 2 * sizeof(int32_t)) + 255) / 256 * 256;
    return part * (op == kOpModReduced ? 2 : 1) + rows;
}

template <int L>
static void spmm_merge_op(const GraphView& g, int op, const float* x, float* y, const float* cvec,
                          char* ws, hipStream_t st) {
    using GE = SpmmGeom<L>;
    const int nr = spmm_merge_ranges(g.n, g.nnz);
    if (nr == 0) return;
    const size_t part_b = (((size_t)nr * 2 * L * sizeof(float)) + 255) / 256 * 256;
    float* part = reinterpret_cast<float*>(ws);
    float* part2 = op == kOpModReduced ? reinterpret_cast<float*>(ws + part_b) : part;
    int32_t* prow = reinterpret_cast<int32_t*>(ws + part_b * (op == kOpModReduced ? 2 : 1));
    const int per_block = kSpmmWaves * GE::G;                    // ranges per work-group
    const int rblocks = (nr + per_block - 1) / per_block;
    const int grid = (rblocks + GE::XS - 1) / GE::XS * 8;
    const int fix_grid = (nr * GE::NS + per_block - 1) / per_block;
#define RAFT_MERGE_CASE(OPV)                                                                   \
    if (op == OPV) {                                                                           \
        hipLaunchKernelGGL((k_spmm_merge<L, OPV>), dim3(grid), dim3(256), 0, st, g, x, y, cvec, \
                           part, part2, prow, nr);                                             \
        hipLaunchKernelGGL((k_spmm_merge_fix<L, OPV>), dim3(fix_grid), dim3(256), 0, st, g, x,  \
                           y, cvec, part, part2, prow, nr);                                    \
        return;                                                                                \
    }
    RAFT_MERGE_CASE(kOpNcut)
    RAFT_MERGE_CASE(kOpModFull)
    RAFT_MERGE_CASE(kOpModReduced)
    RAFT_MERGE_CASE(kOpGcn)
#undef RAFT_MERGE_CASE
}

void launch_spmm_merge(const GraphView& g, int op, int L, const float* x, float* y,
                       const float* cvec, void* ws, hipStream_t st) {
    char* w = reinterpret_cast<char*>(ws);
    switch (L) {
        case 16: spmm_merge_op<16>(g, op, x, y, cvec, w, st); break;
        case 32: spmm_merge_op<32>(g, op, x, y, cvec, w, st); break;
        case 64: spmm_merge_op<64>(g, op, x, y, cvec, w, st); break;
        case 128: spmm_merge_op<128>(g, op, x, y, cvec, w, st); break;
        case 256: spmm_merge_op<256>(g, op, x, y, cvec, w, st); break;
        default: break;
    }
}

bool spmm_supported(int L) {
    return L == 16 || L == 32 || L == 64 || L == 128 || L == 256 || L == 512 || L == 1024 ||
           L == 2048 || L == 4096;
}

// Row blocks of the SpMM and the column-sum partials: G full rows per wave
// (one for L >= 256), rpw passes per wave, four waves.
int spmm_grid(int32_t n, int L, int num_cu, int* rows_per_wave) {
    const int G = L >= 256 ? 1 : kWave / (L / 4);
    const int64_t target_waves = (int64_t)num_cu * 32;
    const int64_t per_wave = ((int64_t)n + target_waves - 1) / target_waves;
    int rpw = (int)((per_wave + G - 1) / G);
    rpw = rpw < 1 ? 1 : (rpw > 64 ? 64 : rpw);
    if (rows_per_wave) *rows_per_wave = rpw;
    const int64_t rows_per_block = (int64_t)rpw * G * kSpmmWaves;
    return (int)((n + rows_per_block - 1) / rows_per_block);
}

static int spmm_xs(int L) {
    const int W = L >= 64 ? 32 : L;
    return L / W <= 8 ? 8 / (L / W) : 1;
}

int spmm_launch_shape(int32_t n, int L, int num_cu, int* R, int* nrb) {
    int rpw;
    const int rb = spmm_grid(n, L, num_cu, &rpw);
    // rows per row block, as in spmm_grid (which k_colsum_part also uses)
    if (R) *R = rpw * (L >= 256 ? 1 : kWave / (L / 4)) * kSpmmWaves;
    if (nrb) *nrb = rb;
    if (L > 256) return rb * (L / 32);   // NS / 8 slices per XCD
    // every group of 8 consecutive work-groups covers XS row blocks x NS slices
    const int xs = spmm_xs(L);
    return rb == 0 ? 0 : (rb + xs - 1) / xs * 8;
}

template <int L>
static void spmm_dispatch_op(const GraphView& g, int op, const float* x, float* y,
                             const float* cvec, double* cpart, int num_cu, hipStream_t st) {
    int R, nrb;
    const int grid = spmm_launch_shape(g.n, L, num_cu, &R, &nrb);
    if (grid == 0) return;
#define RAFT_SPMM_CASE(OPV)                                                                  \
    if (op == OPV) {                                                                         \
        if (cpart)                                                                           \
            hipLaunchKernelGGL((k_spmm<L, OPV, true>), dim3(grid), dim3(256), 0, st, g, x, y, \
                               cvec, cpart, R, nrb);                                         \
        else                                                                                 \
            hipLaunchKernelGGL((k_spmm<L, OPV, false>), dim3(grid), dim3(256), 0, st, g, x,   \
                               y, cvec, cpart, R, nrb);                                      \
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
    switch (L) {
        case 16: spmm_dispatch_op<16>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 32: spmm_dispatch_op<32>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 64: spmm_dispatch_op<64>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 128: spmm_dispatch_op<128>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 256: spmm_dispatch_op<256>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 512: spmm_dispatch_op<512>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 1024: spmm_dispatch_op<1024>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 2048: spmm_dispatch_op<2048>(g, op, x, y, cvec, cpart, num_cu, st); break;
        case 4096: spmm_dispatch_op<4096>(g, op, x, y, cvec, cpart, num_cu, st); break;
        default: break;
    }
}

template <int L>
static void spmm_batched_op(const SpmmItem* items, int op, const float* x, float* y, bool cs,
                            const BatchTable& t, int grid, hipStream_t st) {
#define RAFT_SPMM_CASE(OPV)                                                                    \
    if (op == OPV) {                                                                           \
        if (cs)                                                                                \
            hipLaunchKernelGGL((k_spmm_b<L, OPV, true>), dim3(grid), dim3(256), 0, st, items, x, \
                               y, t);                                                          \
        else                                                                                   \
            hipLaunchKernelGGL((k_spmm_b<L, OPV, false>), dim3(grid), dim3(256), 0, st, items,  \
                               x, y, t);                                                       \
        return;                                                                                \
    }
    RAFT_SPMM_CASE(kOpNcut)
    RAFT_SPMM_CASE(kOpModFull)
    RAFT_SPMM_CASE(kOpModReduced)
    RAFT_SPMM_CASE(kOpGcn)
#undef RAFT_SPMM_CASE
}

void launch_spmm_batched(const SpmmItem* items, int op, int L, const float* x, float* y, bool cs,
                         const BatchTable& t, int grid, hipStream_t st) {
    if (grid == 0) return;
    switch (L) {
        case 16: spmm_batched_op<16>(items, op, x, y, cs, t, grid, st); break;
        case 32: spmm_batched_op<32>(items, op, x, y, cs, t, grid, st); break;
        case 64: spmm_batched_op<64>(items, op, x, y, cs, t, grid, st); break;
        case 128: spmm_batched_op<128>(items, op, x, y, cs, t, grid, st); break;
        case 256: spmm_batched_op<256>(items, op, x, y, cs, t, grid, st); break;
        default: break;
    }
}

void launch_colsum_partials_batched(const ColsumItem* items, int L, const float* x,
                                    const BatchTable& t, int grid, hipStream_t st) {
    if (grid == 0) return;
    switch (L) {
        case 16: hipLaunchKernelGGL(k_colsum_part_b<16>, dim3(grid), dim3(256), 0, st, items, x, t); break;
        case 32: hipLaunchKernelGGL(k_colsum_part_b<32>, dim3(grid), dim3(256), 0, st, items, x, t); break;
        case 64: hipLaunchKernelGGL(k_colsum_part_b<64>, dim3(grid), dim3(256), 0, st, items, x, t); break;
        case 128: hipLaunchKernelGGL(k_colsum_part_b<128>, dim3(grid), dim3(256), 0, st, items, x, t); break;
        case 256: hipLaunchKernelGGL(k_colsum_part_b<256>, dim3(grid), dim3(256), 0, st, items, x, t); break;
        default: break;
    }
}

void launch_colsum_finish_batched(const ColsumItem* items, int L, const BatchTable& t_slices,
                                  int grid_slices, const BatchTable& t_one, int grid_one,
                                  hipStream_t st) {
    if (grid_slices == 0) return;
    hipLaunchKernelGGL(k_colsum_slices_b, dim3(grid_slices), dim3(256), 0, st, items, L, t_slices);
    hipLaunchKernelGGL(k_colsum_finish_b, dim3(grid_one), dim3(256), 0, st, items, L, t_one);
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
        case 512: hipLaunchKernelGGL(k_colsum_part_wide<512>, dim3(grid * 2), dim3(256), 0, st, g, x, part, rpw); break;
        case 1024: hipLaunchKernelGGL(k_colsum_part_wide<1024>, dim3(grid * 4), dim3(256), 0, st, g, x, part, rpw); break;
        case 2048: hipLaunchKernelGGL(k_colsum_part_wide<2048>, dim3(grid * 8), dim3(256), 0, st, g, x, part, rpw); break;
        case 4096: hipLaunchKernelGGL(k_colsum_part_wide<4096>, dim3(grid * 16), dim3(256), 0, st, g, x, part, rpw); break;
        default: break;
    }
}

void launch_colsum_finish(const double* part, int parts, int L, double* c64, float* cvec,
                          hipStream_t st) {
    // the caller reserves kColsumSlices more rows after the partials for the stage
    double* stage = const_cast<double*>(part) + (size_t)parts * L;
    hipLaunchKernelGGL(k_colsum_slices, dim3(kColsumSlices), dim3(256), 0, st, part, parts, L, stage);
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(256), 0, st, stage, L, c64, cvec);
}

}  // namespace raft
