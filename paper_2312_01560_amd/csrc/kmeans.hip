// k-means over every candidate block count of the grid at once (the paper
// clusters the embedding with KMeans, Sec. II and Sec. III-C; the grid of
// candidates is scored afterwards).
//
// Seeding: nested k-means++ picks by an exponential race: pick t is
//   argmin_{i: w_i > 0} E_{t,i} / w_i,  E_{t,i} = -ln u(Philox(i, t | seed, 0x20)),
// w_i = 1 before the first pick, then the squared distance to the nearest
// pick (ties to the lowest index; all-zero weights take the lowest unpicked
// index).  One launch per pick; each launch reduces the previous launch's
// per-group minima (lexicographic on (ratio, index), so the result does not
// depend on scheduling).
//
// Lloyd, all candidates together: the assignment is a dense contraction of
// the points against the table of all centres (rows of each candidate padded
// to a multiple of 16) on MFMA, score ||c||^2 - 2 z.c, argmin per candidate
// with ties to the lowest index: split-fp16 operands (k_assign_h) for d a
// multiple of 32, FP32 (k_assign) otherwise.  The update keeps exact integer
// centre sums across iterations and adds or subtracts only the points whose
// label changed (k_update, k_update_finish).
#include <float.h>
#include <limits.h>

#include <algorithm>
#include <mutex>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace raft {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr uint64_t kStreamRace = 0x20;
constexpr int kRaceThreads = 256;

// Split-fp16 scale exponent s: |z| 2^s < 2^10 for every |z| <= zmax.
__device__ __forceinline__ int split_exp(const KmeansPlan& p) {
    const float zmax = __uint_as_float(*p.zmax_bits);
    if (!(zmax > 0.f)) return 0;
    int ez;
    frexpf(zmax, &ez);
    return 10 - ez;
}

// x 2^s = hi + lo with hi = fp16(x 2^s), lo = fp16(x 2^s - hi); the
// difference is exact in FP32, so hi + lo carries 22 bits of x.
__device__ __forceinline__ void split_half(float x, float sc, uint16_t* hi, uint16_t* lo) {
    const float xs = x * sc;
    const _Float16 h = (_Float16)xs;
    const _Float16 l = (_Float16)(xs - (float)h);
    *hi = __builtin_bit_cast(uint16_t, h);
    *lo = __builtin_bit_cast(uint16_t, l);
}

__device__ __forceinline__ bool lex_less(double v, int i, double bv, int bi) {
    return v < bv || (v == bv && i < bi);
}

// Pick t from the per-group minima that launch t wrote (buffer t mod 2).
// Every work-group of the next launch reduces all of them itself, in the
// same fixed order (the minimum of a total order, so the same pick in every
// work-group): no launch needs a grid-wide "last work-group" step.
// Work-group 0 records the pick.  If every weight was zero, the lowest index
// not picked yet.
__device__ int race_resolve(const KmeansPlan& p, int t, int bx) {
    __shared__ double sv[kRaceThreads / kWave];
    __shared__ int si[kRaceThreads / kWave];
    __shared__ int pick;
    const double* rv = p.race_val + (size_t)(t & 1) * p.race_grid;
    const int* ri = p.race_idx + (size_t)(t & 1) * p.race_grid;
    double best = INFINITY;
    int bidx = INT_MAX;
    for (int b = threadIdx.x; b < p.race_grid; b += blockDim.x) {
        const double v = rv[b];
        const int i = ri[b];
        if (lex_less(v, i, best, bidx)) {
            best = v;
            bidx = i;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bidx, off, kWave);
        if (lex_less(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
        }
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        sv[wid] = best;
        si[wid] = bidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sv[0];
        int bi = si[0];
        for (int w = 1; w < kRaceThreads / kWave; ++w)
            if (lex_less(sv[w], si[w], b, bi)) {
                b = sv[w];
                bi = si[w];
            }
        if (bi == INT_MAX) {
            for (int c = 0; c <= t; ++c) {
                bool taken = false;
                for (int q = 0; q < t; ++q) taken |= (p.picks[q] == c);
                if (!taken) {
                    bi = c;
                    break;
                }
            }
        }
        pick = bi;
        if (bx == 0) p.picks[t] = bi;
    }
    __syncthreads();
    return pick;
}

// Launch t: resolves pick t-1, updates the weights with the distances to it
// and writes this work-group's minimum of E / w for pick t.
template <int D>
__device__ __forceinline__ void race_body(const KmeansPlan& p, const float* __restrict__ Z, int t,
                                          Wg w) {
    const uint64_t seed = p.seed;
    const int tid = (int)w.x * blockDim.x + threadIdx.x;
    const int stride = (int)w.n * blockDim.x;
    // Odd picks sweep from the last point: the end of Z, read last by the
    // previous pick, is still in the memory-side cache (the result does not
    // depend on the order: ties go to the lowest index).
    auto point = [&](int idx) { return (t & 1) ? p.n - 1 - idx : idx; };
    // The draws E = -ln u and the old weights of the first kRacePre points
    // of each thread do not depend on the previous pick: they are computed
    // and loaded before it is resolved, overlapping that reduction.
    constexpr int kRacePre = 8;
    double epre[kRacePre];
    float wpre[kRacePre];
#pragma unroll
    for (int k = 0; k < kRacePre; ++k) {
        const int idx = tid + k * stride;
        epre[k] = 0.0;
        wpre[k] = 1.0f;
        if (idx < p.n) {
            const int i = point(idx);
            const U64x4 b = philox4x64_10((uint64_t)i, (uint64_t)t, 0, 0, seed, kStreamRace);
            epre[k] = -own_ln(uniform52(b.v[0]));
            if (t > 1) wpre[k] = p.w[i];
        }
    }
    const int prev = t > 0 ? race_resolve(p, t - 1, (int)w.x) : -1;
    double best = INFINITY;
    int bidx = INT_MAX;
    const float* zp = prev >= 0 ? Z + (size_t)prev * D : Z;
    // A lane walks its own row: each load instruction of a wave touches 64
    // rows' lines.  Eight float4 loads in flight per lane use a whole
    // 128-byte line of every row before it can leave the L1 (N = 1M, d = 128:
    // 10 % less time per pick than four); at d = 64 the extra registers cost
    // more waves than that saves, so four there.
    constexpr int kRaceUnroll = D >= 128 ? 8 : 4;
    auto visit = [&](int i, double e, float wold) {
        float wi = 1.0f;
        if (t > 0) {
            const float* zi = Z + (size_t)i * D;
            float dist = 0.f;
#pragma unroll kRaceUnroll
            for (int c = 0; c < D; c += 4) {
                const float4 a = *reinterpret_cast<const float4*>(zi + c);
                const float4 b = *reinterpret_cast<const float4*>(zp + c);
                const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
                dist += dx * dx;
                dist += dy * dy;
                dist += dz * dz;
                dist += dw * dw;
            }
            wi = (t == 1) ? dist : fminf(wold, dist);
            p.w[i] = wi;
        }
        if (wi > 0.f) {
            // lexicographic on (ratio, index): odd picks sweep from the end,
            // so an exact tie must still go to the lower index
            const double ratio = e / (double)wi;
            if (lex_less(ratio, i, best, bidx)) {
                best = ratio;
                bidx = i;
            }
        }
    };
#pragma unroll
    for (int k = 0; k < kRacePre; ++k) {
        const int idx = tid + k * stride;
        if (idx < p.n) visit(point(idx), epre[k], wpre[k]);
    }
    for (int idx = tid + kRacePre * stride; idx < p.n; idx += stride) {
        const int i = point(idx);
        const U64x4 b = philox4x64_10((uint64_t)i, (uint64_t)t, 0, 0, seed, kStreamRace);
        visit(i, -own_ln(uniform52(b.v[0])), t > 1 ? p.w[i] : 1.0f);
    }
    // work-group minimum, written for the next launch
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bidx, off, kWave);
        if (lex_less(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
        }
    }
    __shared__ double sv[kRaceThreads / kWave];
    __shared__ int si[kRaceThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        sv[wid] = best;
        si[wid] = bidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sv[0];
        int bi = si[0];
        for (int w = 1; w < kRaceThreads / kWave; ++w)
            if (lex_less(sv[w], si[w], b, bi)) {
                b = sv[w];
                bi = si[w];
            }
        p.race_val[(size_t)(t & 1) * p.race_grid + w.x] = b;
        p.race_idx[(size_t)(t & 1) * p.race_grid + w.x] = bi;
    }
}

template <int D>
__global__ __launch_bounds__(kRaceThreads) void k_race(KmeansPlan p, const float* __restrict__ Z,
                                                       int t) {
    race_body<D>(p, Z, t, wg_self());
}

// Batched: pick t of every graph (its points are rows zoff.. of the packed Z).
template <int D>
__global__ __launch_bounds__(kRaceThreads) void k_race_b(const KmeansPlan* __restrict__ plans,
                                                         const float* __restrict__ Z, int t,
                                                         BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    race_body<D>(p, Z + (size_t)p.zoff * D, t, w);
}

// The last pick (one work-group).
__global__ __launch_bounds__(kRaceThreads) void k_race_final(KmeansPlan p) {
    (void)race_resolve(p, p.k_max - 1, 0);
}

__global__ __launch_bounds__(kRaceThreads) void k_race_final_b(
    const KmeansPlan* __restrict__ plans, BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    (void)race_resolve(plans[gi], plans[gi].k_max - 1, 0);
}

// Copy the first K picks of every candidate into its centre rows; padding
// rows are zero with norm +inf.  One wave per padded centre row.
template <int D>
__device__ __forceinline__ void init_centres_body(const KmeansPlan& p, const float* __restrict__ Z,
                                                  int bx) {
    const int c = (bx * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (c >= p.KP) return;
    const int k = p.cand_of[c];
    const int r = c - p.koff16[k];
    float* crow = p.C + (size_t)c * D;
    if (r >= p.ks[k]) {
        for (int dd = lane; dd < D; dd += kWave) {
            crow[dd] = 0.f;
            if (p.split) {
                p.ch[(size_t)c * D + dd] = 0;
                p.cl[(size_t)c * D + dd] = 0;
            }
        }
        if (lane == 0) p.cnorm[c] = INFINITY;
        return;
    }
    const float* z = Z + (size_t)p.picks[r] * D;
    const float sc = ldexpf(1.0f, split_exp(p));
    float ss = 0.f;
    for (int dd = lane; dd < D; dd += kWave) {
        const float v = z[dd];
        crow[dd] = v;
        if (p.split) split_half(v, sc, p.ch + (size_t)c * D + dd, p.cl + (size_t)c * D + dd);
        ss += v * v;
    }
    ss = wave_sum(ss);
    if (lane == 0) p.cnorm[c] = ss;
}

template <int D>
__global__ __launch_bounds__(256) void k_init_centres(KmeansPlan p, const float* __restrict__ Z) {
    init_centres_body<D>(p, Z, (int)blockIdx.x);
}

template <int D>
__global__ __launch_bounds__(256) void k_init_centres_b(const KmeansPlan* __restrict__ plans,
                                                        const float* __restrict__ Z,
                                                        BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    init_centres_body<D>(p, Z + (size_t)p.zoff * D, (int)w.x);
}

// Assignment for all active candidates of one candidate group.
// Grid: x = point tiles (4 waves x 16*PS points), y = candidate group.
// The group's centre tiles are walked as one flat sequence (candidate by
// candidate, 16 centres per tile); the operands of the next tile are loaded
// while the MFMAs of the current one run.
template <int KS>
__device__ __forceinline__ void load_ctile(const KmeansPlan& p, int cb, int li, int g, float* a,
                                           float4& cn) {
    const float* cr = p.C + (size_t)(cb + li) * (KS * 4) + g * KS;
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
        const float4 v = *reinterpret_cast<const float4*>(cr + s);
        a[s] = v.x;
        a[s + 1] = v.y;
        a[s + 2] = v.z;
        a[s + 3] = v.w;
    }
    cn = *reinterpret_cast<const float4*>(p.cnorm + cb + 4 * g);
}

// Block order of the assignment kernels (one-dimensional grid).  When the
// points are too large for the memory-side cache (group_major, set by the
// host), all candidate groups of one point tile run back to back on one
// XCD, so the tile's points come from memory once and then from that XCD's
// L2: work-groups are dealt to the eight XCDs round robin (block b runs on
// XCD b mod 8), so block b = 8 s + x takes point tile 8 (s / agroups) + x
// and candidate group s mod agroups; the host pads the tile count to a
// multiple of 8 and padding blocks exit.  Otherwise the point tile varies
// fastest, which keeps a group's centre tiles hot (9 % faster at N = 50k,
// where all points stay cached).
__device__ __forceinline__ int assign_group(const KmeansPlan& p, Wg w) {
    if (p.group_major) return (int)((w.x >> 3) % (unsigned)p.agroups);
    const int tiles = (int)(w.n / (unsigned)p.agroups);
    return (int)w.x / tiles;
}
__device__ __forceinline__ int assign_tile(const KmeansPlan& p, Wg w) {
    if (p.group_major) return (int)(((w.x >> 3) / (unsigned)p.agroups) * 8u + (w.x & 7u));
    const int tiles = (int)(w.n / (unsigned)p.agroups);
    return (int)w.x % tiles;
}

// End of a candidate in the assignment kernels.  Lane (li, g) holds, for
// each point 16 ps + li of its wave, the best score and row over the centre
// rows 4g..4g+3 of every tile; the four lane groups are folded through a
// wave-private LDS area (fold: PS x 64 floats then PS x 64 ints): each lane
// writes its PS partials, then lane (li, g) reads the four partials of point
// 16 g + li and keeps the lowest score, the lowest row among equal scores.
// Returns that row (0 for lanes with g >= PS) and resets the partials.
template <int PS>
__device__ __forceinline__ int fold_lane_groups(float (&bv)[PS], int (&bi)[PS], float* fold,
                                                int lane) {
    const int li = lane & 15, g = lane >> 4;
    int* foldi = reinterpret_cast<int*>(fold + PS * kWave);
#pragma unroll
    for (int ps = 0; ps < PS; ++ps) {
        fold[lane * PS + ps] = bv[ps];
        foldi[lane * PS + ps] = bi[ps];
        bv[ps] = INFINITY;
        bi[ps] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    int best = 0;
    if (g < PS) {
        float v = fold[li * PS + g];
        best = foldi[li * PS + g];
#pragma unroll
        for (int h = 1; h < 4; ++h) {
            const float ov = fold[(h * 16 + li) * PS + g];
            const int oi = foldi[(h * 16 + li) * PS + g];
            const bool take = (ov < v) | ((ov == v) & (oi < best));
            v = take ? ov : v;
            best = take ? oi : best;
        }
    }
    __builtin_amdgcn_wave_barrier();
    return best;
}

template <int D, int PS>
__device__ __forceinline__ void assign_body(const KmeansPlan& p, const float* __restrict__ Z, Wg w,
                                            int it) {
    constexpr int KS = D / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int g = lane >> 4;
    const int li = lane & 15;
    __shared__ float fold_all[4][2 * PS * kWave];
    float* fold = fold_all[wid];
    const int pbase = (assign_tile(p, w) * 4 + wid) * 16 * PS;
    if (pbase >= p.n) return;
    float b[PS][KS];
#pragma unroll
    for (int ps = 0; ps < PS; ++ps) {
        const int pt = min(pbase + 16 * ps + li, p.n - 1);
        const float* zr = Z + (size_t)pt * D + g * KS;
#pragma unroll
        for (int s = 0; s < KS; s += 4) {
            const float4 v = *reinterpret_cast<const float4*>(zr + s);
            b[ps][s] = v.x;
            b[ps][s + 1] = v.y;
            b[ps][s + 2] = v.z;
            b[ps][s + 3] = v.w;
        }
    }
    const int grp = assign_group(p, w);
    const int t0 = p.agrp[grp], t1 = p.agrp[grp + 1];
    // The group's candidates (at most kWave), one per lane: id, active flag,
    // tile count and centre offset are loaded once, in parallel; the walk
    // below then reads them with lane reads instead of dependent loads.
    const int nc = min(t1 - t0, kWave);
    int my_k = 0, my_tiles = 0, my_off = 0;
    bool my_act = false;
    if (lane < nc) {
        my_k = p.alist[t0 + lane];
        my_act = p.active[my_k] != 0;
        my_tiles = (p.ks[my_k] + 15) >> 4;
        my_off = p.koff16[my_k];
    }
    const uint64_t amask = __ballot(my_act);
    if (amask == 0) return;
    // first active candidate of the group (position in the group)
    int t = __builtin_ctzll(amask);
    int k = __builtin_amdgcn_readlane(my_k, t);
    int ntiles = __builtin_amdgcn_readlane(my_tiles, t);
    int koff = __builtin_amdgcn_readlane(my_off, t);
    int tile = 0;
    float an[KS];
    float4 cnn;
    load_ctile<KS>(p, koff, li, g, an, cnn);
    float bv[PS];
    int bi[PS];
#pragma unroll
    for (int ps = 0; ps < PS; ++ps) {
        bv[ps] = INFINITY;
        bi[ps] = 0;
    }
    while (true) {
        float a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = an[s];
        const float cnv[4] = {cnn.x, cnn.y, cnn.z, cnn.w};
        // coordinates of the next tile, and its prefetch
        int nk = k, ntile = tile + 1, nt = t, nntiles = ntiles, nkoff = koff;
        if (ntile >= ntiles) {
            ntile = 0;
            const uint64_t rest = amask & ~((2ull << t) - 1ull);   // active positions after t
            nt = rest ? __builtin_ctzll(rest) : nc;
            if (nt < nc) {
                nk = __builtin_amdgcn_readlane(my_k, nt);
                nntiles = __builtin_amdgcn_readlane(my_tiles, nt);
                nkoff = __builtin_amdgcn_readlane(my_off, nt);
            }
        }
        if (nt < nc) load_ctile<KS>(p, nkoff + ntile * 16, li, g, an, cnn);
#pragma unroll
        for (int ps = 0; ps < PS; ++ps) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[ps][s], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float sc = cnv[v] - 2.0f * acc[v];
                if (sc < bv[ps]) {
                    bv[ps] = sc;
                    bi[ps] = tile * 16 + 4 * g + v;
                }
            }
        }
        if (tile == ntiles - 1) {
            // candidate finished: fold the lane groups, write labels, count changes
            const int mine = fold_lane_groups<PS>(bv, bi, fold, lane);
            const int pt = pbase + 16 * g + li;
            bool changed = false;
            if (g < PS && pt < p.n) {
                uint8_t* lp = p.lab_cm + (size_t)k * p.n + pt;
                const uint8_t old = *lp;
                const uint8_t nw = (uint8_t)mine;
                changed = old != nw;
                *lp = nw;
                p.lab_old[(size_t)k * p.n + pt] = old;
                if (changed) p.moved_it[(size_t)(pt >> 6) * p.Kc + k] = it;
            }
            const uint64_t m = __ballot(changed);
            if (lane == 0 && m) p.changes[k] = 1;   // only zero / non-zero is read
        }
        if (nt >= nc) break;
        k = nk;
        tile = ntile;
        t = nt;
        ntiles = nntiles;
        koff = nkoff;
    }
}

template <int D, int PS>
__global__ __launch_bounds__(256) void k_assign(KmeansPlan p, const float* __restrict__ Z) {
    assign_body<D, PS>(p, Z, wg_self(), p.it);
}

template <int D, int PS>
__global__ __launch_bounds__(256) void k_assign_b(const KmeansPlan* __restrict__ plans,
                                                  const float* __restrict__ Z, int it,
                                                  BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    assign_body<D, PS>(p, Z + (size_t)p.zoff * D, w, it);
}

// Split-fp16 assignment (d a multiple of 32): the same walk and argmin as
// k_assign, with each 16 x 16 x d score block from v_mfma_f32_16x16x32_f16
// over the split halves: z.c 2^2s = zh.ch + zl.ch + zh.cl (the lo.lo term is
// below 2^-22 relative); products of fp16 values are exact in FP32, which
// accumulates.  Lane l holds A[l%16][8(l/16)+i] (centres) and
// B[8(l/16)+i][l%16] (points) per 32-wide k chunk; D as in the FP32 MFMA.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// -v for eight fp16 values, by their sign bits (exact for every value)
__device__ __forceinline__ half8 neg_half8(half8 v) {
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(half8, u);
}

// Centre tiles pass through LDS: the four waves of a work-group walk the same
// candidate group, so the 256 threads load each 16-centre tile (hi and lo
// halves, norms) once, one tile ahead of the MFMAs, into a double buffer;
// one barrier per tile.  Rows are padded by 8 halves against bank conflicts.
// The new labels of every candidate wait in LDS and leave after the walk,
// together with the previous labels, the move marks and the change flags, in
// coalesced passes; the walk itself holds no label state in registers, which
// leaves the kernel at d = 64 within 128 registers, four waves per SIMD
// (48.8 us per launch at N = 50k against 53.4 us with three).  A work-group
// has AW waves (AW x 16 PS points); more waves share each staged tile (fewer
// centre loads) but wait at more crowded barriers.
template <int D, int PS, int AW>
__device__ __forceinline__ void assign_h_body(const KmeansPlan& p, Wg w, int it) {
    constexpr int NC = D / 32;
    constexpr int RS = D + 8;                 // LDS row stride (halves)
    constexpr int CPR = D / 8;                // 16-byte chunks per row and half
    constexpr int CHUNKS = 16 * CPR * 2;      // chunks per tile (hi and lo)
    constexpr int NT = AW * kWave;            // threads
    __shared__ _Float16 hs[2][16][RS], ls[2][16][RS];
    __shared__ float cs[2][16];
    __shared__ float fold_all[AW][2 * PS * kWave];
    constexpr int WP = AW * 16 * PS;          // points of the work-group
    __shared__ uint8_t labs[kAssignMaxGroup][WP];   // new labels per group position
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int g = lane >> 4;
    const int li = lane & 15;
    // every wave takes part in the barriers; rows beyond n are clamped, and
    // a work-group wholly past n (tile padding) leaves before any barrier
    if (p.group_major && assign_tile(p, w) * WP >= p.n) return;
    const int pbase = (assign_tile(p, w) * AW + wid) * 16 * PS;
    half8 bh[PS][NC], bl[PS][NC];
#pragma unroll
    for (int ps = 0; ps < PS; ++ps) {
        const int pt = min(pbase + 16 * ps + li, p.n - 1);
        const size_t row = (size_t)pt * D + 8 * g;
        const _Float16* hr = reinterpret_cast<const _Float16*>(p.zh) + row;
        const _Float16* lr = reinterpret_cast<const _Float16*>(p.zl) + row;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            bh[ps][c] = neg_half8(*reinterpret_cast<const half8*>(hr + 32 * c));
            bl[ps][c] = neg_half8(*reinterpret_cast<const half8*>(lr + 32 * c));
        }
    }
    // the group's candidates, one per lane (the same in every wave)
    const int grp = assign_group(p, w);
    const int t0 = p.agrp[grp], t1 = p.agrp[grp + 1];
    const int nc = min(t1 - t0, kAssignMaxGroup);
    int my_k = 0, my_tiles = 0, my_off = 0;
    bool my_act = false;
    if (lane < nc) {
        my_k = p.alist[t0 + lane];
        my_act = p.active[my_k] != 0;
        my_tiles = (p.ks[my_k] + 15) >> 4;
        my_off = p.koff16[my_k];
    }
    const uint64_t amask = __ballot(my_act);
    if (amask == 0) return;                   // uniform across the work-group
    // scores in units of 2^(1-2s): cnorm 2^(2s-1) - z.c 2^2s orders the
    // centres exactly as cnorm - 2 z.c does (scaling by a power of two is
    // exact).  The point halves are held negated (exact: a sign flip), so
    // each tile's MFMA chain starts from the staged norms and ends on the
    // score itself, with no subtraction per element.
    const int nexp = 2 * split_exp(p) - 1;
    const _Float16* chp = reinterpret_cast<const _Float16*>(p.ch);
    const _Float16* clp = reinterpret_cast<const _Float16*>(p.cl);
    // tile loader: global -> registers (issued early), registers -> LDS.
    // Written as macros so the staging registers are only ever indexed by
    // unrolled constants (a lambda capturing them put them on the stack).
    constexpr int SQ = (CHUNKS + NT - 1) / NT;
    uint4 stage[SQ];
    float cstage = 0.f;
#define ASSIGN_ISSUE(KOFF, TILE)                                                            \
    {                                                                                      \
        const int base_ = (KOFF) + (TILE) * 16;                                            \
        _Pragma("unroll") for (int q = 0; q < SQ; ++q) {                                   \
            const int c = tid + NT * q;                                                    \
            if (c < CHUNKS) {                                                              \
                const int which = c / (16 * CPR), rem = c - which * (16 * CPR);            \
                const int r = rem / CPR, c8 = rem - r * CPR;                               \
                const _Float16* src = (which ? clp : chp) + (size_t)(base_ + r) * D + 8 * c8; \
                stage[q] = *reinterpret_cast<const uint4*>(src);                           \
            }                                                                              \
        }                                                                                  \
        if (tid < 16) cstage = p.cnorm[base_ + tid];                                       \
    }
#define ASSIGN_COMMIT(BUF)                                                                 \
    {                                                                                      \
        _Pragma("unroll") for (int q = 0; q < SQ; ++q) {                                   \
            const int c = tid + NT * q;                                                    \
            if (c < CHUNKS) {                                                              \
                const int which = c / (16 * CPR), rem = c - which * (16 * CPR);            \
                const int r = rem / CPR, c8 = rem - r * CPR;                               \
                _Float16* dst = (which ? &ls[(BUF)][r][0] : &hs[(BUF)][r][0]) + 8 * c8;    \
                *reinterpret_cast<uint4*>(dst) = stage[q];                                 \
            }                                                                              \
        }                                                                                  \
        if (tid < 16) cs[(BUF)][tid] = ldexpf(cstage, nexp);                               \
    }
    // the walk: position t in the group, tile within the candidate
    int t = __builtin_ctzll(amask);
    int k = __builtin_amdgcn_readlane(my_k, t);
    int ntiles = __builtin_amdgcn_readlane(my_tiles, t);
    int koff = __builtin_amdgcn_readlane(my_off, t);
    int tile = 0;
    ASSIGN_ISSUE(koff, 0)
    ASSIGN_COMMIT(0)
    __syncthreads();
    const int ptw = wid * 16 * PS + 16 * g + li;   // lane's point within the work-group
    float bv[PS];
    int bi[PS];
#pragma unroll
    for (int ps = 0; ps < PS; ++ps) {
        bv[ps] = INFINITY;
        bi[ps] = 0;
    }
    int buf = 0;
    while (true) {
        // next tile of the walk, and the issue of its loads
        int nk = k, ntile = tile + 1, nt = t, nntiles = ntiles, nkoff = koff;
        if (ntile >= ntiles) {
            ntile = 0;
            const uint64_t rest = amask & ~((2ull << t) - 1ull);
            nt = rest ? __builtin_ctzll(rest) : nc;
            if (nt < nc) {
                nk = __builtin_amdgcn_readlane(my_k, nt);
                nntiles = __builtin_amdgcn_readlane(my_tiles, nt);
                nkoff = __builtin_amdgcn_readlane(my_off, nt);
            }
        }
        const bool more = nt < nc;
        if (more) ASSIGN_ISSUE(nkoff, ntile)
        // this tile's operands from LDS
        const float4 cnn = *reinterpret_cast<const float4*>(&cs[buf][4 * g]);
        // the PS accumulators are independent: interleaving them keeps the
        // matrix unit busy instead of waiting on one dependent chain; each
        // 32-wide chunk's A operands are read from LDS just before its MFMAs
        floatx4 acc[PS];
#pragma unroll
        for (int ps = 0; ps < PS; ++ps) acc[ps] = floatx4{cnn.x, cnn.y, cnn.z, cnn.w};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const half8 ah = *reinterpret_cast<const half8*>(&hs[buf][li][8 * g + 32 * c]);
            const half8 al = *reinterpret_cast<const half8*>(&ls[buf][li][8 * g + 32 * c]);
#pragma unroll
            for (int ps = 0; ps < PS; ++ps)
                acc[ps] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[ps][c], acc[ps], 0, 0, 0);
#pragma unroll
            for (int ps = 0; ps < PS; ++ps)
                acc[ps] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[ps][c], acc[ps], 0, 0, 0);
#pragma unroll
            for (int ps = 0; ps < PS; ++ps)
                acc[ps] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[ps][c], acc[ps], 0, 0, 0);
        }
#pragma unroll
        for (int ps = 0; ps < PS; ++ps) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float sc = acc[ps][v];
                if (sc < bv[ps]) {
                    bv[ps] = sc;
                    bi[ps] = tile * 16 + 4 * g + v;
                }
            }
        }
        if (tile == ntiles - 1) {
            const int mine = fold_lane_groups<PS>(bv, bi, fold_all[wid], lane);
            if (g < PS) labs[t][ptw] = (uint8_t)mine;
        }
        if (!more) break;                     // uniform across the work-group
        ASSIGN_COMMIT(buf ^ 1)
        __syncthreads();
        buf ^= 1;
        k = nk;
        tile = ntile;
        t = nt;
        ntiles = nntiles;
        koff = nkoff;
    }
    // the labels: thread = point (64 consecutive points per wave, one move
    // mark chunk), candidate after candidate
    __syncthreads();
    const int wbase = assign_tile(p, w) * WP;
    for (uint64_t rest = amask; rest != 0; rest &= rest - 1) {
        const int tt = __builtin_ctzll(rest);
        const int kk = __builtin_amdgcn_readlane(my_k, tt);
#pragma unroll
        for (int q = 0; q < (WP + NT - 1) / NT; ++q) {
            const int lp = tid + NT * q;
            const int pt = wbase + lp;
            bool changed = false;
            if (lp < WP && pt < p.n) {
                const uint8_t nw = labs[tt][lp];
                const uint8_t ol = p.lab_cm[(size_t)kk * p.n + pt];
                changed = ol != nw;
                p.lab_cm[(size_t)kk * p.n + pt] = nw;
                p.lab_old[(size_t)kk * p.n + pt] = ol;
            }
            const uint64_t m = __ballot(changed);
            if (lane == 0 && m) {
                p.moved_it[(size_t)(pt >> 6) * p.Kc + kk] = it;
                p.changes[kk] = 1;            // only zero / non-zero is read
            }
        }
    }
}

#undef ASSIGN_ISSUE
#undef ASSIGN_COMMIT

// Waves per SIMD the split-fp16 assignment is compiled for: four at
// d <= 64 (its registers fit 128 per lane), three above.
template <int D>
constexpr int assign_wpe() {
    return D <= 64 ? 4 : 3;
}

template <int D, int PS, int AW>
__global__ __launch_bounds__(AW * 64) __attribute__((amdgpu_waves_per_eu(1, assign_wpe<D>()))) void k_assign_h(KmeansPlan p) {
    assign_h_body<D, PS, AW>(p, wg_self(), p.it);
}

template <int D, int PS, int AW>
__global__ __launch_bounds__(AW * 64) __attribute__((amdgpu_waves_per_eu(1, assign_wpe<D>()))) void k_assign_h_b(
    const KmeansPlan* __restrict__ plans, int it, BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    assign_h_body<D, PS, AW>(plans[gi], w, it);
}

// ---- bound-pruned assignment ------------------------------------------------
// Lloyd's assignment keeps a point's label for a candidate whenever the
// label provably cannot change (Hamerly's bounds): u, an upper bound on the
// distance to its own centre a, and l, a lower bound on the distance to
// every other centre, are taken when the point is scored; each update moves
// centre c by drift_c, which can raise the distance to a by at most drift_a
// and lower the distance to any other centre by at most the candidate's
// largest drift.  With Cum_c the summed drifts of centre c and CumMax the
// summed largest drifts, the stored hu = u - Cum_a and hl = l + CumMax give
// at a later iteration U = hu + Cum_a <= and Lb = hl - CumMax >= the true
// distances.  The point is not re-scored when Lb^2 - U^2 > 2E, E a bound on
// the error of a computed score: then the computed score of a is below every
// other computed score, so scoring the point would return a again, and the
// labels, centres and iteration counts are those of the full assignment.
// Every bound is rounded outward (FP64 with relative slack, FP32 storage
// rounded up or down).
//
// Score error.  A computed score is 2^nexp (|c|^2 - 2 z.c) from split
// halves: each half pair carries z 2^s to 2^-22 relative (plus 2^-25
// absolute below the fp16 normal range), the dropped lo.lo product is below
// 2^-22 |z||c|, the 3d exact products and the norm are accumulated in FP32
// (at most (3d + 1) 2^-24 of their absolute sum), and |c|^2 comes from an
// FP32 sum (d 2^-24 |c|^2).  With cm >= every centre norm (centres are means
// of points, or picked points, so cm = the largest |z| with a margin), all
// of this is below (4d + 64) 2^-23 (cm + |z|)^2, twice the sum of the terms.
__device__ __forceinline__ double prune_up(double x, double rel) {
    return __builtin_isfinite(x) ? x + fabs(x) * rel : x;
}
__device__ __forceinline__ double prune_dn(double x, double rel) {
    return __builtin_isfinite(x) ? x - fabs(x) * rel : x;
}
__device__ __forceinline__ float f32_up(double x) {
    float f = (float)x;
    if ((double)f < x) {
        const uint32_t b = __float_as_uint(f);
        f = f == 0.f ? __uint_as_float(1u) : (f > 0.f ? __uint_as_float(b + 1) : __uint_as_float(b - 1));
    }
    return f;
}
__device__ __forceinline__ float f32_dn(double x) {
    float f = (float)x;
    if ((double)f > x) {
        const uint32_t b = __float_as_uint(f);
        f = f == 0.f ? -__uint_as_float(1u) : (f > 0.f ? __uint_as_float(b - 1) : __uint_as_float(b + 1));
    }
    return f;
}
// slack of the running FP64 sums (at most 65536 terms each)
constexpr double kSumSlack = 0x1p-36;
constexpr double kRootSlack = 0x1p-40;

__device__ __forceinline__ double prune_eps(const KmeansPlan& p, double zn2) {
    const double cm = (double)__uint_as_float(*p.znmax_bits) * (1.0 + 0x1p-16);
    const double s = cm + sqrt(zn2) * (1.0 + 0x1p-30);
    return (double)(4 * p.d + 64) * 0x1p-23 * s * s;
}
// summed largest drift of candidate k before assignment `it` (it >= 2)
__device__ __forceinline__ double prune_cummax(const KmeansPlan& p, int k, int it) {
    return p.cmx[k] + p.dmx[2 * (size_t)k + ((it - 1) & 1)];
}

// |z|^2 per point (FP64 sum, rounded up to FP32) and the largest |z|.
// One wave per row (lanes read consecutive columns), rows strided over the
// grid's waves; each wave's largest norm joins the maximum once.
__global__ __launch_bounds__(256) void k_prune_prep(KmeansPlan p, const float* __restrict__ Z) {
    const int lane = threadIdx.x & (kWave - 1);
    const int waves = (int)gridDim.x * (blockDim.x / kWave);
    float m = 0.f;
    for (int i = (int)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < p.n; i += waves) {
        const float* zr = Z + (size_t)i * p.d;
        double s = 0.0;
        for (int j = lane; j < p.d; j += kWave) s += (double)zr[j] * (double)zr[j];
        s = wave_sum(s);
        s = prune_up(s, kRootSlack);
        if (lane == 0) p.zn2[i] = f32_up(s);
        m = fmaxf(m, f32_up(prune_up(sqrt(s), kRootSlack)));
    }
    if (!(m <= 3.0e38f)) m = 3.0e38f;
    if (lane == 0) atomicMax(p.znmax_bits, __float_as_uint(m));
}

// Score error bound E of every point (needs the largest |z| of all points).
__global__ __launch_bounds__(256) void k_prune_eps(KmeansPlan p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) p.pe[i] = f32_up(prune_eps(p, (double)p.zn2[i]));
}

// Bounds at rest: hu = +inf, hl = -inf (every point is listed until scored);
// running sums and list lengths zero.
__global__ __launch_bounds__(256) void k_prune_fill(KmeansPlan p) {
    const size_t total = (size_t)p.Kc * p.n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        p.hu[i] = INFINITY;
        p.hl[i] = -INFINITY;
    }
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < p.KP) p.cum[tid] = 0.0;
    if (tid < p.Kc) {
        p.cmx[tid] = 0.0;
        p.dmx[2 * tid] = 0.0;
        p.dmx[2 * tid + 1] = 0.0;
    }
    if (tid == 0) *p.znmax_bits = 0u;
}

// Points held per lane group of the pruned assignment's waves, and waves
// per scoring work-group.
template <int D>
constexpr int list_ps() {
    return D <= 64 ? 4 : (D <= 128 ? 2 : 1);
}
template <int D>
constexpr int prune_nw() {
    return D <= 64 ? 4 : 16;
}

// Pruned assignment, two launches per iteration.
//
// k_prune_test (grid: x = ranges of kPruneRange points, y = positions of
// alist) tests the bounds of every point of its range for its candidate and
// writes the points they do not hold, in point order, to the range's own
// slots of the candidate's list (plist[k][range start ...]) and their count
// to scnt[k][range]; the previous labels of the others are brought level
// with the current ones (the update reads a difference of the two as a
// move).  Every load of a wave's points is issued before its first test.
//
// k_prune_score (a persistent grid) scores the listed points.  Work items
// are 256 listed points of one (candidate, range) list, numbered candidate
// after candidate; each work-group takes a contiguous range of items, so it
// changes candidate rarely: on a change it stages the candidate's whole
// centre table in LDS (hi and lo halves, scaled norms, running drifts), and
// its waves then walk the table with no barrier per tile.  The scores are
// those of k_assign_h bit for bit (the same split operands, MFMA chain and
// argmin with ties to the lowest row); each scored point also keeps its
// second-lowest score for its new bounds.
__global__ __launch_bounds__(256) void k_prune_test(KmeansPlan p) {
    constexpr int QR = kPruneRange / 4;     // points per wave
    constexpr int QI = QR / kWave;
    __shared__ int lst[4][QR];
    __shared__ int wcnt[4];
    __shared__ double ccum[RAFT_MAX_K_DEV + 17];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int t = blockIdx.y;
    if (t >= p.agrp[p.agroups]) return;     // uniform across the work-group
    const int k = p.alist[t];
    if (!p.active[k]) return;
    const int koff = p.koff16[k];
    const int K = p.ks[k];
    const int r0 = (int)blockIdx.x * kPruneRange + wid * QR;
    const size_t kb = (size_t)k * p.n;
    uint32_t la[QI], lo[QI];
    float fu[QI], fl[QI], fe[QI];
#pragma unroll
    for (int q = 0; q < QI; ++q) {
        const int i = min(r0 + q * kWave + lane, p.n - 1);
        la[q] = p.lab_cm[kb + i];
        lo[q] = p.lab_old[kb + i];
        fu[q] = p.hu[kb + i];
        fl[q] = p.hl[kb + i];
        fe[q] = p.pe[i];
    }
    for (int r = tid; r < K; r += blockDim.x) ccum[r] = p.cum[koff + r];
    const double cx = prune_up(prune_cummax(p, k, p.it), kSumSlack);
    __syncthreads();
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < QI; ++q) {
        const int i = r0 + q * kWave + lane;
        bool need = false;
        if (i < p.n) {
            if (lo[q] != la[q]) p.lab_old[kb + i] = (uint8_t)la[q];
            const double cu = prune_up(ccum[min((int)la[q], K - 1)], kSumSlack);
            const double U = prune_up((double)fu[q] + cu, kRootSlack);
            const double Lb = prune_dn((double)fl[q] - cx, kRootSlack);
            need = !(Lb > U && prune_dn((Lb - U) * (Lb + U), kRootSlack) > 2.0 * (double)fe[q]);
        }
        const uint64_t m = __ballot(need);
        if (need) lst[wid][cnt + __popcll(m & ((1ull << lane) - 1ull))] = i;
        cnt += __popcll(m);
    }
    if (lane == 0) wcnt[wid] = cnt;
    __syncthreads();
    int off = 0;
    for (int q = 0; q < wid; ++q) off += wcnt[q];
    int* dst = p.plist + kb + (size_t)blockIdx.x * kPruneRange + off;
    for (int e = lane; e < cnt; e += kWave) dst[e] = lst[wid][e];
    if (tid == 0)
        p.scnt[(size_t)k * p.nranges + blockIdx.x] = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
}

template <int D, int PS, int NW>
__global__ __launch_bounds__(NW * 64) void k_prune_score(KmeansPlan p) {
    constexpr int NC = D / 32;
    constexpr int RS = D + 8;               // LDS row stride (halves)
    constexpr int CPR = D / 8;              // 16-byte chunks per row and half
    constexpr int WI = 16 * PS;             // points per wave and pass
    constexpr int IP = NW * WI > 256 ? NW * WI : 256;   // points per work item
    extern __shared__ __align__(16) unsigned char list_lds[];
    __shared__ double ccum[RAFT_MAX_K_DEV + 17];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int g = lane >> 4;
    const int li = lane & 15;
    // (alist position, range) lists; at most as many as the LDS was sized for
    const int nact = min(p.agrp[p.agroups], p.lists_nact);
    const int nr = p.nranges;
    const int E = nact * nr;
    const int ctiles = p.list_tiles;
    _Float16* hs = reinterpret_cast<_Float16*>(list_lds);
    _Float16* ls = hs + (size_t)ctiles * 16 * RS;
    float* cs = reinterpret_cast<float*>(ls + (size_t)ctiles * 16 * RS);
    int* pref = reinterpret_cast<int*>(cs + (size_t)ctiles * 16);   // [E + 1] items before list e
    // items (256 listed points) of every list, prefix over the lists in order
    {
        constexpr int NT = NW * 64;
        const int per = (E + NT - 1) / NT;
        const int e0 = tid * per, e1 = min(E, e0 + per);
        int sum = 0;
        for (int e = e0; e < e1; ++e) {
            const int t = e / nr, r = e - t * nr;
            const int k = p.alist[t];
            const int c = p.active[k] ? p.scnt[(size_t)k * nr + r] : 0;
            const int items = (c + IP - 1) / IP;
            pref[e + 1] = items;
            sum += items;
        }
        __shared__ int part[NT];
        part[tid] = sum;
        __syncthreads();
        if (tid == 0) {
            int run = 0;
            for (int q = 0; q < NT; ++q) {
                const int v = part[q];
                part[q] = run;
                run += v;
            }
            pref[0] = 0;
        }
        __syncthreads();
        int run = part[tid];
        for (int e = e0; e < e1; ++e) {
            run += pref[e + 1];
            pref[e + 1] = run;
        }
        __syncthreads();
    }
    const int total = pref[E];
    const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
    const int w0 = (int)blockIdx.x * per, w1 = min(total, w0 + per);
    if (w0 >= w1) return;                    // uniform across the work-group
    const int nexp = 2 * split_exp(p) - 1;
    const _Float16* chp = reinterpret_cast<const _Float16*>(p.ch);
    const _Float16* clp = reinterpret_cast<const _Float16*>(p.cl);
    int e = 0;
    {
        int lo = 0, hi = E;                  // pref[lo] <= w0 < pref[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pref[mid] <= w0) lo = mid;
            else hi = mid;
        }
        e = lo;
    }
    int staged = -1;                         // alist position of the staged table
    for (int w = w0; w < w1; ++w) {
        while (pref[e + 1] <= w) ++e;
        const int t = e / nr, r = e - t * nr;
        const int k = p.alist[t];
        const int len = p.scnt[(size_t)k * nr + r];
        const int koff = p.koff16[k];
        const int ntiles = (p.ks[k] + 15) >> 4;
        const int* lst = p.plist + (size_t)k * p.n + (size_t)r * kPruneRange;
        const int ibase = (w - pref[e]) * IP;
        if (t != staged) {
            __syncthreads();                 // every wave is past the previous table
            const int chunks = ntiles * 16 * CPR * 2;
            for (int c = tid; c < chunks; c += blockDim.x) {
                const int which = c / (ntiles * 16 * CPR);
                const int rem = c - which * (ntiles * 16 * CPR);
                const int rr = rem / CPR, c8 = rem - rr * CPR;
                const uint4 v = *reinterpret_cast<const uint4*>((which ? clp : chp) +
                                                                (size_t)(koff + rr) * D + 8 * c8);
                *reinterpret_cast<uint4*>((which ? ls : hs) + (size_t)rr * RS + 8 * c8) = v;
            }
            for (int rr = tid; rr < ntiles * 16; rr += blockDim.x) {
                cs[rr] = ldexpf(p.cnorm[koff + rr], nexp);
                ccum[rr] = p.cum[koff + rr];
            }
            __syncthreads();
            staged = t;
        }
        // the wave's passes over its quarter of the item's 256 points
        for (int base = ibase + wid * WI; base < min(len, ibase + IP); base += NW * WI) {
            int idx[PS];
#pragma unroll
            for (int ps = 0; ps < PS; ++ps) idx[ps] = lst[min(base + 16 * ps + li, len - 1)];
            half8 bh[PS][NC], bl[PS][NC];
#pragma unroll
            for (int ps = 0; ps < PS; ++ps) {
                const size_t row = (size_t)idx[ps] * D + 8 * g;
                const _Float16* hr = reinterpret_cast<const _Float16*>(p.zh) + row;
                const _Float16* lr = reinterpret_cast<const _Float16*>(p.zl) + row;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    bh[ps][c] = neg_half8(*reinterpret_cast<const half8*>(hr + 32 * c));
                    bl[ps][c] = neg_half8(*reinterpret_cast<const half8*>(lr + 32 * c));
                }
            }
            // the writing lane's point: previous label and norms, loaded ahead
            int mi = 0;
#pragma unroll
            for (int ps = 0; ps < PS; ++ps)
                if (g == ps) mi = idx[ps];
            const bool wr = g < PS && base + 16 * g + li < len;
            uint32_t old = 0;
            float zq = 0.f, eq = 0.f;
            if (wr) {
                old = p.lab_cm[(size_t)k * p.n + mi];
                zq = p.zn2[mi];
                eq = p.pe[mi];
            }
            float bv[PS], b2[PS];
            int bi[PS];
#pragma unroll
            for (int ps = 0; ps < PS; ++ps) {
                bv[ps] = INFINITY;
                b2[ps] = INFINITY;
                bi[ps] = 0;
            }
            for (int tile = 0; tile < ntiles; ++tile) {
                const float4 cnn = *reinterpret_cast<const float4*>(&cs[tile * 16 + 4 * g]);
                floatx4 acc[PS];
#pragma unroll
                for (int ps = 0; ps < PS; ++ps) acc[ps] = floatx4{cnn.x, cnn.y, cnn.z, cnn.w};
                const _Float16* hrow = hs + (size_t)(tile * 16 + li) * RS + 8 * g;
                const _Float16* lrow = ls + (size_t)(tile * 16 + li) * RS + 8 * g;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const half8 ah = *reinterpret_cast<const half8*>(hrow + 32 * c);
                    const half8 al = *reinterpret_cast<const half8*>(lrow + 32 * c);
#pragma unroll
                    for (int ps = 0; ps < PS; ++ps)
                        acc[ps] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[ps][c], acc[ps], 0, 0, 0);
#pragma unroll
                    for (int ps = 0; ps < PS; ++ps)
                        acc[ps] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[ps][c], acc[ps], 0, 0, 0);
#pragma unroll
                    for (int ps = 0; ps < PS; ++ps)
                        acc[ps] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[ps][c], acc[ps], 0, 0, 0);
                }
#pragma unroll
                for (int ps = 0; ps < PS; ++ps) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float sc = acc[ps][v];
                        const bool lt = sc < bv[ps];
                        b2[ps] = lt ? bv[ps] : fminf(b2[ps], sc);
                        bi[ps] = lt ? tile * 16 + 4 * g + v : bi[ps];
                        bv[ps] = lt ? sc : bv[ps];
                    }
                }
            }
            // the four lane groups of each point: lowest score, lowest row
            // among equal ones; the second-lowest over both sides and the
            // other's best
#pragma unroll
            for (int ps = 0; ps < PS; ++ps) {
#pragma unroll
                for (int off = 16; off < kWave; off <<= 1) {
                    const float ov = __shfl_xor(bv[ps], off, kWave);
                    const int oi = __shfl_xor(bi[ps], off, kWave);
                    const float o2 = __shfl_xor(b2[ps], off, kWave);
                    const bool take = (ov < bv[ps]) | ((ov == bv[ps]) & (oi < bi[ps]));
                    b2[ps] = fminf(fminf(b2[ps], o2), take ? bv[ps] : ov);
                    bv[ps] = take ? ov : bv[ps];
                    bi[ps] = take ? oi : bi[ps];
                }
            }
            float mv = 0.f, m2 = 0.f;
            int mb = 0;
#pragma unroll
            for (int ps = 0; ps < PS; ++ps)
                if (g == ps) {
                    mv = bv[ps];
                    m2 = b2[ps];
                    mb = bi[ps];
                }
            bool changed = false;
            if (wr) {
                const size_t o = (size_t)k * p.n + mi;
                const uint8_t nw = (uint8_t)mb;
                changed = old != nw;
                p.lab_cm[o] = nw;
                p.lab_old[o] = (uint8_t)old;
                if (changed) p.moved_it[(size_t)(mi >> 6) * p.Kc + k] = p.it;
                const double zn2 = (double)zq;
                const double Eq = (double)eq;
                const double sa = ldexp((double)mv, -nexp);
                const double s2 = ldexp((double)m2, -nexp);
                const double u =
                    prune_up(sqrt(fmax(0.0, prune_up(zn2 + sa + Eq, kRootSlack))), kRootSlack);
                const double l = prune_dn(
                    sqrt(fmax(0.0, prune_dn(zn2 * (1.0 - 0x1p-20) + s2 - Eq, kRootSlack))), kRootSlack);
                const double cd = prune_dn(ccum[nw], kSumSlack);
                const double cxd = prune_dn(prune_cummax(p, k, p.it), kSumSlack);
                p.hu[o] = f32_up(prune_up(u - cd, kRootSlack));
                p.hl[o] = f32_dn(prune_dn(l + cxd, kRootSlack));
            }
            const uint64_t cm = __ballot(changed);
            if (lane == 0 && cm) p.changes[k] = 1;
        }
    }
}

// Dynamic LDS bytes of k_prune_score: centre tables of up to `tiles` tiles
// and the item prefix over `lists` (candidate, range) lists.
size_t list_lds_bytes(int d, int tiles, int lists) {
    return (size_t)tiles * 16 * ((size_t)2 * (d + 8) * 2 + 4) + (size_t)(lists + 1) * 4;
}

// After an assignment: a candidate whose labels did not change (from the
// second assignment on) has converged; count the remaining active ones.
// changes[k] is a flag (plain stores of 1): a counter updated by every wave
// serialises tens of thousands of atomics on a few cache lines.
// One work-group: the whole candidate table.
__device__ __forceinline__ void finalize_candidates(const KmeansPlan& p, int it, int t_max) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int k = threadIdx.x; k < p.Kc; k += blockDim.x) {
        if (p.prune) {
            // pruned assignment: the previous update's largest drift
            // (complete since that launch ended) joins the running sum and
            // its slot is cleared for the update after the next assignment
            if (it >= 2) {
                double* slot = p.dmx + 2 * (size_t)k + ((it - 1) & 1);
                p.cmx[k] += *slot;
                *slot = 0.0;
            }
        }
        if (!p.active[k]) continue;
        const int ch = p.changes[k];
        p.changes[k] = 0;
        if (it >= 2 && ch == 0) {
            p.active[k] = 0;
            p.iters[k] = it;
        } else if (it >= t_max) {
            p.active[k] = 0;
            p.iters[k] = it;
        } else {
            ++mine;
        }
    }
    atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) *p.active_count = cnt;
}

__global__ __launch_bounds__(256) void k_iter_finalize(KmeansPlan p, int it, int t_max) {
    finalize_candidates(p, it, t_max);
}

__global__ __launch_bounds__(256) void k_iter_finalize_b(const KmeansPlan* __restrict__ plans,
                                                         int it, int t_max, BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    finalize_candidates(plans[gi], it, t_max);
}

// Largest |z| (bit pattern of a non-negative float orders as an integer):
// block maximum, then one atomic per block.
__device__ __forceinline__ void zmax_body(const KmeansPlan& p, const float* __restrict__ Z, Wg w) {
    const int64_t total = (int64_t)p.n * p.d;
    float m = 0.f;
    for (int64_t i = (int64_t)w.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)w.n * blockDim.x)
        m = fmaxf(m, fabsf(Z[i]));
    if (!(m <= 3.0e38f)) m = 3.0e38f;   // non-finite input: keep the exponent sane
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    __shared__ float wm[4];
    if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
        atomicMax(p.zmax_bits, __float_as_uint(b));
    }
}

__global__ __launch_bounds__(256) void k_zmax(KmeansPlan p, const float* __restrict__ Z) {
    zmax_body(p, Z, wg_self());
}

__global__ __launch_bounds__(256) void k_zmax_b(const KmeansPlan* __restrict__ plans,
                                                const float* __restrict__ Z, BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    zmax_body(p, Z + (size_t)p.zoff * p.d, w);
}

// Fixed-point exponent e: |z| * 2^e < 2^30 for every |z| <= zmax.
__device__ __forceinline__ int fixed_exp(const KmeansPlan& p) {
    const float zmax = __uint_as_float(*p.zmax_bits);
    if (!(zmax > 0.f)) return 0;
    int ez;
    frexpf(zmax, &ez);
    return 30 - ez;
}

__device__ __forceinline__ void split_points_body(const KmeansPlan& p, const float* __restrict__ Z,
                                                  Wg w) {
    const int64_t total = (int64_t)p.n * p.d;
    const float sc = ldexpf(1.0f, split_exp(p));
    for (int64_t i = (int64_t)w.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)w.n * blockDim.x)
        split_half(Z[i], sc, p.zh + i, p.zl + i);
}

__global__ __launch_bounds__(256) void k_split_points(KmeansPlan p, const float* __restrict__ Z) {
    split_points_body(p, Z, wg_self());
}

__global__ __launch_bounds__(256) void k_split_points_b(const KmeansPlan* __restrict__ plans,
                                                        const float* __restrict__ Z,
                                                        BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    split_points_body(p, Z + (size_t)p.zoff * p.d, w);
}

// Centre update, incremental and exact.  The sums of every centre are kept
// between iterations as integers: each point is quantised to int32
// (z * 2^e, e fixed for the whole partition) and a centre's sum is an int64
// total of such values.  An assignment records each point's previous label
// next to the new one; the update then adds the points whose label changed
// to their new cluster and subtracts them from their old one (the first
// assignment has no old cluster).  Integer addition is associative, so the
// totals equal those of summing every cluster from scratch, in any order,
// while the work shrinks with the number of moved points.
//
// One work item = (update group, point range) and one slice of up to 64
// columns.  The assignment marks, per candidate and 64-point chunk, the
// iteration in which a label of the chunk last changed; a wave reads those
// marks for four of its chunks at once and passes over every (chunk,
// candidate) without a move, and over chunks without any (most of them once
// the candidates settle).  Per remaining chunk a wave first reads both label
// columns of every marked candidate (lane = point) into LDS and counts the moves,
// then loads z of the points that moved for any candidate (lane = column,
// one register per point), and walks the candidates again applying the +/-
// into int64 LDS accumulators shared by the work-group, one contiguous
// accumulator row per instruction.  A candidate where most points moved and
// none had a cluster before (the first assignment) takes a branch-free sweep
// over the chunk (unmoved points go to a dummy row); otherwise each point is
// a uniform bit test, skipped when it did not move, with the add and the
// subtraction under one test when every moved point had a cluster.  At the end the
// work-group writes, per accumulator row, a flag saying whether any point
// moved in or out and, if so, the row's partial sums and count change;
// k_update_finish folds the flagged partials of each row into the totals.
constexpr int kUpdWaves = 4;
constexpr int kUpdMaxCand = 16;
constexpr int kUpdSlice = 64;
// label staging: [wave][candidate][point] bytes, new and previous labels
constexpr size_t kUpdStageBytes = (size_t)2 * kUpdWaves * kUpdMaxCand * kWave;
constexpr int kUpdSparse = 16;   // moved points per chunk below which the set bits are walked
typedef int i32x32 __attribute__((ext_vector_type(32)));

// Bit q of a uniform 64-bit mask (q a compile-time constant after
// unrolling), tested on its 32-bit half so the AND alone sets the branch
// condition.
__device__ __forceinline__ bool bit_set(uint64_t m, int q) {
    const uint32_t w = q < 32 ? (uint32_t)m : (uint32_t)(m >> 32);
    return (w & (1u << (q & 31))) != 0u;
}

// int32 -> int64 at the point of use: the empty asm keeps the compiler from
// hoisting 64 widened copies out of the candidate loop (128 more registers).
__device__ __forceinline__ unsigned long long widen_at_use(int x) {
    asm volatile("" : "+v"(x));
    return (unsigned long long)(long long)x;
}

__device__ __forceinline__ void update_body(const KmeansPlan& p, const float* __restrict__ Z, int wi,
                                            int it) {
    extern __shared__ unsigned long long acc64[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // work item wi -> (group, range slot): g = the number of groups after the
    // first whose first item is at most wi (the first items increase), read
    // 64 at a time rather than walked one dependent load after another
    int g = 0;
    for (int b0 = 1; b0 < p.ugroups; b0 += kWave) {
        const int q = b0 + lane;
        g += __popcll(__ballot(q < p.ugroups && p.uwi0[q] <= wi));
    }
    const int slot = wi - p.uwi0[g];
    const int sl = blockIdx.y;
    const int t0 = p.ugrp[g], t1 = p.ugrp[g + 1];
    const int nc = t1 - t0;
    // the group's candidates: lane l holds candidate l % 16 (read back with
    // readlane from lanes 0..15, and by lane in the moved-flag loads), its
    // centre count, padded centre offset and first accumulator row
    const int mc = lane & (kUpdMaxCand - 1);
    int my_k = 0, my_K = 0, my_act = 0, my_off = 0;
    if (mc < nc) {
        my_k = p.alist[t0 + mc];
        my_K = p.ks[my_k];
        my_act = p.active[my_k] != 0;
        my_off = p.koff16[my_k];
    }
    int my_base = 0, rows = 0;
    for (int m = 0; m < nc; ++m) {
        if (mc == m) my_base = rows;
        rows += __builtin_amdgcn_readlane(my_K, m);
    }
    if (__ballot(my_act != 0) == 0) return;   // uniform across the work-group
    const int total_rows = rows + 1;                          // + one dummy row
    int* cnt = reinterpret_cast<int*>(acc64 + (size_t)total_rows * kUpdSlice);
    int* touch = cnt + total_rows;
    uint8_t* stage_n = reinterpret_cast<uint8_t*>(touch + total_rows) +
                       (size_t)wid * 2 * kUpdMaxCand * kWave;
    uint8_t* stage_o = stage_n + kUpdMaxCand * kWave;
    for (int idx = threadIdx.x; idx < total_rows * kUpdSlice; idx += blockDim.x) acc64[idx] = 0ull;
    for (int idx = threadIdx.x; idx < total_rows; idx += blockDim.x) {
        cnt[idx] = 0;
        touch[idx] = 0;
    }
    __syncthreads();
    const int fe = fixed_exp(p);
    const int dummy = rows;
    const int col = sl * kUpdSlice + lane;
    const int colc = min(col, p.d - 1);
    const int len = p.ulen[g];
    const int r0 = slot * len;
    const int r1 = min(p.n, r0 + len);
    unsigned long long* acol = acc64 + lane;
    // Chunks of this wave in batches of four: lane (j, m) reads whether
    // candidate m moved a point of chunk j in this iteration; the update skips
    // every (chunk, candidate) without a move, and whole chunks without one.
    constexpr int kStride = kUpdWaves * kWave;
    for (int cb = r0 + wid * kWave; cb < r1; cb += 4 * kStride) {
        uint64_t F;
        {
            const int csj = cb + (lane >> 4) * kStride;
            bool f = false;
            if (mc < nc && my_act != 0 && csj < r1)
                f = p.moved_it[(size_t)(csj >> 6) * p.Kc + my_k] == it;
            F = __ballot(f);
        }
        for (int j = 0; j < 4; ++j) {
            const uint32_t cm = (uint32_t)(F >> (16 * j)) & 0xFFFFu;
            if (cm == 0) continue;                // also every chunk past r1
            const int cs = cb + j * kStride;
            const int np = min(kWave, r1 - cs);
            const bool lv = lane < np;
            // pass 1: labels to LDS, counts, and the points moved for any candidate;
            // every label load of the chunk is issued before the first is used
            uint64_t U = 0;
            {
                int nlv[kUpdMaxCand], olv[kUpdMaxCand];
#pragma unroll
                for (int m = 0; m < kUpdMaxCand; ++m) {
                    nlv[m] = 0;
                    olv[m] = 0;
                    const int k = __builtin_amdgcn_readlane(my_k, m);
                    if (((cm >> m) & 1u) != 0u && lv) {
                        nlv[m] = p.lab_cm[(size_t)k * p.n + cs + lane];
                        olv[m] = p.lab_old[(size_t)k * p.n + cs + lane];
                    }
                }
                for (int m = 0; m < nc; ++m) {
                    if (((cm >> m) & 1u) == 0u) continue;
                    const int base = __builtin_amdgcn_readlane(my_base, m);
                    const int nl = nlv[m], ol = olv[m];
                    stage_n[m * kWave + lane] = (uint8_t)nl;
                    stage_o[m * kWave + lane] = (uint8_t)ol;
                    const bool moved = nl != ol;
                    U |= __ballot(moved);
                    if (moved) {
                        atomicAdd(&touch[base + nl], 1);
                        if (sl == 0) atomicAdd(&cnt[base + nl], 1);
                        if (ol != 0xFF) {
                            atomicAdd(&touch[base + ol], 1);
                            if (sl == 0) atomicSub(&cnt[base + ol], 1);
                        }
                    }
                }
            }
            if (U == 0) continue;
            // z of the moved points (lane = column): every load is issued before
            // the first conversion, so the loads overlap.  Lanes past d read
            // column d-1; they only feed accumulator columns never written out.
            // Only moved points are loaded; the empty asm after the loads keeps
            // the compiler from pulling each conversion into its load's branch
            // (which would wait on every load in turn).
            float zr[kWave];
#pragma unroll
            for (int q = 0; q < kWave; ++q) {
                zr[q] = 0.f;
                if (bit_set(U, q)) zr[q] = Z[(size_t)(cs + q) * p.d + colc];
            }
#pragma unroll
            for (int q = 0; q < kWave; ++q) asm volatile("" : "+v"(zr[q]));
            // quantised z in two 32-wide vectors: constant indices in the unrolled
            // sweeps, a relative register move in the sparse walk
            i32x32 zf0, zf1;
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                zf0[q] = __float2int_rn(ldexpf(zr[q], fe));
                zf1[q] = __float2int_rn(ldexpf(zr[q + 32], fe));
            }
#define ZF(q) ((q) < 32 ? zf0[(q)] : zf1[(q) - 32])
            // pass 2: the adds and subtractions, candidate by candidate
            for (uint32_t rc = cm; rc != 0u; rc &= rc - 1u) {
                const int m = __builtin_ctz(rc);
                const int base = __builtin_amdgcn_readlane(my_base, m);
                const int nl = stage_n[m * kWave + lane];
                const int ol = stage_o[m * kWave + lane];
                const bool moved = nl != ol;
                const bool had = moved && ol != 0xFF;
                const uint64_t mv = __ballot(moved);
                const uint64_t mo = __ballot(had);
                const int nrow = moved ? base + nl : dummy;
                const int orow = had ? base + ol : dummy;
                if (mv == 0) continue;
                if (mo == 0 && __popcll(mv) >= kWave / 2) {
#pragma unroll
                    for (int q = 0; q < kWave; ++q) {
                        const int a = __builtin_amdgcn_readlane(nrow, q);
                        atomicAdd(acol + (size_t)a * kUpdSlice, widen_at_use(ZF(q)));
                    }
                    continue;
                }
                if (mo == mv && __popcll(mv) <= kUpdSparse) {
                    // few moved points, each with a cluster: walk the set bits
                    for (uint64_t r = mv; r != 0; r &= r - 1) {
                        const int q = __builtin_ctzll(r);
                        const int a = __builtin_amdgcn_readlane(nrow, q);
                        const int o = __builtin_amdgcn_readlane(orow, q);
                        const int z = q < 32 ? zf0[q] : zf1[q - 32];
                        atomicAdd(acol + (size_t)a * kUpdSlice, widen_at_use(z));
                        atomicAdd(acol + (size_t)o * kUpdSlice, widen_at_use(-z));
                    }
                    continue;
                }
                if (mo == mv) {
                    // every moved point had a cluster (all iterations after the
                    // first): one bit test per point for both the add and the
                    // subtraction
#pragma unroll
                    for (int q = 0; q < kWave; ++q) {
                        if (bit_set(mv, q)) {
                            const int a = __builtin_amdgcn_readlane(nrow, q);
                            const int o = __builtin_amdgcn_readlane(orow, q);
                            atomicAdd(acol + (size_t)a * kUpdSlice, widen_at_use(ZF(q)));
                            atomicAdd(acol + (size_t)o * kUpdSlice, widen_at_use(-ZF(q)));
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int q = 0; q < kWave; ++q) {
                    if (bit_set(mv, q)) {
                        const int a = __builtin_amdgcn_readlane(nrow, q);
                        atomicAdd(acol + (size_t)a * kUpdSlice, widen_at_use(ZF(q)));
                    }
                }
                if (mo == 0) continue;
#pragma unroll
                for (int q = 0; q < kWave; ++q) {
                    if (bit_set(mo, q)) {
                        const int o = __builtin_amdgcn_readlane(orow, q);
                        atomicAdd(acol + (size_t)o * kUpdSlice, widen_at_use(-ZF(q)));
                    }
                }
            }
        }
    }
#undef ZF
    __syncthreads();
    const int sw = min(kUpdSlice, p.d - sl * kUpdSlice);
    int base = 0;
    for (int m = 0; m < nc; ++m) {
        const int K = __builtin_amdgcn_readlane(my_K, m);
        if (__builtin_amdgcn_readlane(my_act, m)) {
            const size_t row0 = (size_t)slot * p.KP + __builtin_amdgcn_readlane(my_off, m);
            long long* dst = p.pdelta + row0 * p.d + sl * kUpdSlice;
            for (int r = wid; r < K; r += kUpdWaves) {
                if (touch[base + r] == 0) continue;          // uniform per wave
                if (lane < sw)
                    dst[(size_t)r * p.d + lane] =
                        (long long)acc64[(size_t)(base + r) * kUpdSlice + lane];
            }
            if (sl == 0)
                for (int idx = threadIdx.x; idx < K; idx += blockDim.x) {
                    p.pdirty[row0 + idx] = touch[base + idx] != 0 ? 1 : 0;
                    p.pcnt[row0 + idx] = cnt[base + idx];
                }
        }
        base += K;
    }
}

__global__ __launch_bounds__(256) void k_update(KmeansPlan p, const float* __restrict__ Z) {
    update_body(p, Z, (int)blockIdx.x, p.it);
}

__global__ __launch_bounds__(256) void k_update_b(const KmeansPlan* __restrict__ plans,
                                                  const float* __restrict__ Z, int it,
                                                  BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    update_body(p, Z + (size_t)p.zoff * p.d, (int)w.x, it);
}

// Folds the flagged partials of one centre row into its integer totals and
// recomputes the centre as total * 2^-e / count (FP64, then FP32); a row no
// point moved into or out of keeps its centre, and so does an empty cluster.
// One work-group per padded centre row: 4 slices of the ranges x 64 columns;
// the integer sums do not depend on the order.
//
// The extra work-group KP runs the end-of-iteration bookkeeping
// (finalize_candidates) in the same launch: a candidate it retires has no
// moved point, so no other work-group of this launch or of the update
// depends on its flags.
__device__ __forceinline__ void update_finish_body(const KmeansPlan& p, int it, int t_max, int c) {
    if (c == p.KP) {
        finalize_candidates(p, it, t_max);
        return;
    }
    const int k = p.cand_of[c];
    if (!p.active[k]) return;
    if (c - p.koff16[k] >= p.ks[k]) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int q = threadIdx.x / kWave;
    const int nr = p.cranges[k];
    const int per = (nr + 3) / 4;
    const int ch0 = q * per, ch1 = min(nr, ch0 + per);
    __shared__ long long part[4][kWave];
    __shared__ int pc[4], pd[4];
    // a wave's ranges (at most 64, one per lane): which of them saw a move
    const int chl = ch0 + lane;
    const bool dl = chl < ch1 && p.pdirty[(size_t)chl * p.KP + c] != 0;
    const uint64_t dmask = __ballot(dl);
    int count = dl ? p.pcnt[(size_t)chl * p.KP + c] : 0;
    count = wave_sum(count);
    if (lane == 0) {
        pc[q] = count;
        pd[q] = dmask != 0;
    }
    __syncthreads();
    if (pd[0] + pd[1] + pd[2] + pd[3] == 0) return;   // uniform: nothing moved
    const int total = p.N32[c] + ((pc[0] + pc[1]) + pc[2]) + pc[3];
    const double inv = ldexp(1.0, -fixed_exp(p));
    const size_t stride = (size_t)p.KP * p.d;
    float* crow = p.C + (size_t)c * p.d;
    float ss = 0.f;
    double drift2 = 0.0;   // squared move of the centre (exact differences of FP32 values)
    for (int d0 = 0; d0 < p.d; d0 += kWave) {
        const int dd = d0 + lane;
        long long s = 0;
        if (dd < p.d) {
            const long long* src = p.pdelta + (size_t)c * p.d + dd;
            // the flagged ranges, four independent loads at a time
            uint64_t rem = dmask;
            while (rem) {
                long long v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[j] = 0;
                    if (rem) {
                        v[j] = src[(size_t)(ch0 + __builtin_ctzll(rem)) * stride];
                        rem &= rem - 1;
                    }
                }
                s += (v[0] + v[1]) + (v[2] + v[3]);
            }
        }
        __syncthreads();
        part[q][lane] = s;
        __syncthreads();
        if (q == 0 && dd < p.d) {
            const long long t =
                p.S64[(size_t)c * p.d + dd] + part[0][lane] + part[1][lane] + part[2][lane] +
                part[3][lane];
            p.S64[(size_t)c * p.d + dd] = t;
            if (total > 0) {
                const float v = (float)((double)t * inv / (double)total);
                const double mv = (double)v - (double)crow[dd];
                drift2 += mv * mv;
                crow[dd] = v;
                if (p.split)
                    split_half(v, ldexpf(1.0f, split_exp(p)), p.ch + (size_t)c * p.d + dd,
                               p.cl + (size_t)c * p.d + dd);
                ss += v * v;
            }
        }
    }
    if (q == 0) {
        if (lane == 0) p.N32[c] = total;
        ss = wave_sum(ss);
        if (lane == 0 && total > 0) p.cnorm[c] = ss;
        if (p.prune) {
            // drift of the centre, rounded up, into its running sum (one
            // writer per row) and the candidate's largest drift of this update
            drift2 = wave_sum(drift2);
            if (lane == 0 && drift2 > 0.0) {
                const double dl = sqrt(drift2) * (1.0 + 0x1p-40);
                p.cum[c] += dl;
                atomicMax(reinterpret_cast<unsigned long long*>(p.dmx + 2 * (size_t)k + (it & 1)),
                          (unsigned long long)__double_as_longlong(dl));
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_update_finish(KmeansPlan p, int it, int t_max) {
    update_finish_body(p, it, t_max, (int)blockIdx.x);
}

// Batched: a graph's rows (and its bookkeeping, row KP) walked grid-stride by
// its work-groups, so a launch over many graphs does not dispatch one
// work-group per centre row of every graph (most of them exit at once).
__global__ __launch_bounds__(256) void k_update_finish_b(const KmeansPlan* __restrict__ plans,
                                                         int it, int t_max, BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    const KmeansPlan& p = plans[gi];
    for (int c = (int)w.x; c <= p.KP; c += (int)w.n) {
        update_finish_body(p, it, t_max, c);
        __syncthreads();   // the row's LDS staging is reused by the next row
    }
}

__device__ __forceinline__ void kmeans_reset_body(const KmeansPlan& p, Wg w) {
    const int64_t tid = (int64_t)w.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)w.n * blockDim.x;
    for (int64_t i = tid; i < (int64_t)p.Kc * p.n; i += stride) p.lab_cm[i] = 0xFF;
    for (int64_t i = tid; i < (int64_t)p.KP * p.d; i += stride) p.S64[i] = 0;
    for (int64_t i = tid; i < p.KP; i += stride) p.N32[i] = 0;
    for (int64_t i = tid; i < (int64_t)p.nchunks * p.Kc; i += stride) p.moved_it[i] = 0;
    for (int64_t k = tid; k < p.Kc; k += stride) {
        p.active[k] = 1;
        p.changes[k] = 0;
        p.iters[k] = 0;
    }
    if (tid == 0) {
        *p.active_count = p.Kc;
        *p.zmax_bits = 0u;
    }
}

__global__ void k_kmeans_reset(KmeansPlan p) { kmeans_reset_body(p, wg_self()); }

__global__ __launch_bounds__(256) void k_kmeans_reset_b(const KmeansPlan* __restrict__ plans,
                                                        BatchTable tb) {
    int gi;
    Wg w;
    if (!batch_find(tb, gi, w)) return;
    kmeans_reset_body(plans[gi], w);
}

bool kmeans_supported(int d) { return d == 16 || d == 32 || d == 64 || d == 128 || d == 256; }

// Every work-group of the next launch reads all per-group minima, so the
// grid stays at two work-groups per CU or fewer.
int kmeans_race_grid(int32_t n, int num_cu) {
    const int64_t want = ((int64_t)n + kRaceThreads - 1) / kRaceThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * 2));
}

size_t kmeans_update_lds(int sum_rows, int d) {
    (void)d;
    return (size_t)(sum_rows + 1) * (kUpdSlice * sizeof(unsigned long long) + 2 * sizeof(int)) +
           kUpdStageBytes;
}

int kmeans_update_rows(int K) { return K; }

int kmeans_update_max_candidates() { return kUpdMaxCand; }

// Waves per work-group of the assignment: the split-fp16 kernel at d <= 64
// runs kAssignWavesSmallD, every other form four.
static int assign_waves(const KmeansPlan& p) {
    return (p.split && p.d % 32 == 0 && p.d <= 64) ? kAssignWavesSmallD : 4;
}

int kmeans_blocks(const KmeansPlan& p, int kind, int num_cu) {
    const int64_t nd = (int64_t)p.n * p.d;
    switch (kind) {
        case kKmZmax:
            return (int)std::max<int64_t>(1, std::min<int64_t>((nd + 255) / 256, num_cu * 2));
        case kKmReset: {
            const int64_t total = std::max<int64_t>((int64_t)p.Kc * p.n, p.Kc);
            return (int)std::min<int64_t>((total + 255) / 256, 4096);
        }
        case kKmSplit: return nd == 0 ? 0 : (int)std::min<int64_t>((nd + 255) / 256, 8192);
        case kKmRace: return p.race_grid;
        case kKmRaceFinal:
        case kKmFinalize: return 1;
        case kKmInit: return (p.KP * kWave + 255) / 256;
        case kKmAssign: {
            const int ps = p.d <= 64 ? 4 : (p.d == 128 ? 3 : 1);
            const int pts_per_block = assign_waves(p) * 16 * ps;
            int tiles = (p.n + pts_per_block - 1) / pts_per_block;
            if (p.group_major) tiles = (tiles + 7) / 8 * 8;
            return tiles * p.agroups;
        }
        case kKmUpdate: return p.uwork;
        case kKmUpdateFinish: return p.KP + 1;
        default: return 0;
    }
}

void launch_zmax(const KmeansPlan& p, const float* Z, int num_cu, hipStream_t st) {
    const int grid = kmeans_blocks(p, kKmZmax, num_cu);
    hipLaunchKernelGGL(k_zmax, dim3(grid), dim3(256), 0, st, p, Z);
}

void launch_kmeans_reset(const KmeansPlan& p, hipStream_t st) {
    const int grid = kmeans_blocks(p, kKmReset, 0);
    hipLaunchKernelGGL(k_kmeans_reset, dim3(grid), dim3(256), 0, st, p);
}

#define RAFT_D_SWITCH(D_, CALL) \
    switch (D_) {                \
        case 16: CALL(16); break;  \
        case 32: CALL(32); break;  \
        case 64: CALL(64); break;  \
        case 128: CALL(128); break; \
        case 256: CALL(256); break; \
        default: break;            \
    }

void launch_race_pick(const KmeansPlan& p, const float* Z, int t, hipStream_t st) {
#define RACE(DV) \
    hipLaunchKernelGGL(k_race<DV>, dim3(p.race_grid), dim3(kRaceThreads), 0, st, p, Z, t)
    RAFT_D_SWITCH(p.d, RACE)
#undef RACE
    if (t == p.k_max - 1) hipLaunchKernelGGL(k_race_final, dim3(1), dim3(kRaceThreads), 0, st, p);
}

void launch_init_centres(const KmeansPlan& p, const float* Z, hipStream_t st) {
    const int grid = (p.KP * kWave + 255) / 256;
#define INIT(DV) hipLaunchKernelGGL(k_init_centres<DV>, dim3(grid), dim3(256), 0, st, p, Z)
    RAFT_D_SWITCH(p.d, INIT)
#undef INIT
}

template <int D>
static constexpr int assign_ps() {
    return D <= 64 ? 4 : (D == 128 ? 3 : 1);
}

template <int D>
static constexpr int assign_aw() {
    return D <= 64 ? kAssignWavesSmallD : 4;
}

// The point tile of a work-group is 64 PS points (256 at d <= 64, 192 at
// d = 128).  Smaller tiles split a launch into more work-groups but re-read
// the centre tiles more often; measured on gfx950 at N = 50k, 64-point tiles
// ran the assignment 1.7x slower than 256-point tiles, and at N = 1M
// (d = 128) 48 points per wave ran 12 % faster than 32.
void launch_assign(const KmeansPlan& p, const float* Z, int num_cu, hipStream_t st, hipEvent_t e0,
                   hipEvent_t e1) {
    (void)num_cu;
#define ASSIGN(DV)                                                                        \
    {                                                                                     \
        constexpr int PS = assign_ps<DV>();                                               \
        constexpr int AW = assign_aw<DV>();                                               \
        if constexpr (DV % 32 == 0) {                                                     \
            if (p.split) {                                                                \
                const dim3 grid((unsigned)kmeans_blocks(p, kKmAssign, num_cu));           \
                if (e0)                                                                   \
                    hipExtLaunchKernelGGL((k_assign_h<DV, PS, AW>), grid, dim3(AW * 64), 0, st, \
                                          e0, e1, 0, p);                                  \
                else                                                                      \
                    hipLaunchKernelGGL((k_assign_h<DV, PS, AW>), grid, dim3(AW * 64), 0, st, p); \
                break;                                                                    \
            }                                                                             \
        }                                                                                 \
        const int pts_per_block = 4 * 16 * PS;                                            \
        int tiles_ = (p.n + pts_per_block - 1) / pts_per_block;                           \
        if (p.group_major) tiles_ = (tiles_ + 7) / 8 * 8;                                 \
        dim3 grid((unsigned)(tiles_ * p.agroups));                                        \
        if (e0)                                                                           \
            hipExtLaunchKernelGGL((k_assign<DV, PS>), grid, dim3(256), 0, st, e0, e1, 0, p, Z); \
        else                                                                              \
            hipLaunchKernelGGL((k_assign<DV, PS>), grid, dim3(256), 0, st, p, Z);         \
    }
    RAFT_D_SWITCH(p.d, ASSIGN)
#undef ASSIGN
}

// ---- batched launches: the per-graph plans live in device memory, the
// graphs' points are consecutive row ranges of one packed Z (plan.zoff) ----

void launch_kmeans_batched(int kind, const KmeansPlan* plans, int d, bool split, const float* Z,
                           int it, int t_max, size_t lds_max, size_t update_lds,
                           const BatchTable& t, int grid, hipStream_t st) {
    if (grid == 0) return;
    const dim3 blk(256);
    switch (kind) {
        case kKmReset: hipLaunchKernelGGL(k_kmeans_reset_b, dim3(grid), blk, 0, st, plans, t); break;
        case kKmZmax: hipLaunchKernelGGL(k_zmax_b, dim3(grid), blk, 0, st, plans, Z, t); break;
        case kKmSplit: hipLaunchKernelGGL(k_split_points_b, dim3(grid), blk, 0, st, plans, Z, t); break;
        case kKmRace: {
#define RACE(DV) hipLaunchKernelGGL(k_race_b<DV>, dim3(grid), dim3(kRaceThreads), 0, st, plans, Z, it, t)
            RAFT_D_SWITCH(d, RACE)
#undef RACE
            break;
        }
        case kKmRaceFinal:
            hipLaunchKernelGGL(k_race_final_b, dim3(grid), dim3(kRaceThreads), 0, st, plans, t);
            break;
        case kKmInit: {
#define INIT(DV) hipLaunchKernelGGL(k_init_centres_b<DV>, dim3(grid), blk, 0, st, plans, Z, t)
            RAFT_D_SWITCH(d, INIT)
#undef INIT
            break;
        }
        case kKmAssign: {
#define ASSIGN(DV)                                                                         \
    {                                                                                      \
        constexpr int PS = assign_ps<DV>();                                                \
        constexpr int AW = assign_aw<DV>();                                                \
        if constexpr (DV % 32 == 0) {                                                      \
            if (split) {                                                                   \
                hipLaunchKernelGGL((k_assign_h_b<DV, PS, AW>), dim3(grid), dim3(AW * 64), 0, st, \
                                   plans, it, t);                                          \
                break;                                                                     \
            }                                                                              \
        }                                                                                  \
        hipLaunchKernelGGL((k_assign_b<DV, PS>), dim3(grid), blk, 0, st, plans, Z, it, t); \
    }
            RAFT_D_SWITCH(d, ASSIGN)
#undef ASSIGN
            break;
        }
        case kKmFinalize:
            hipLaunchKernelGGL(k_iter_finalize_b, dim3(grid), blk, 0, st, plans, it, t_max, t);
            break;
        case kKmUpdate: {
            static std::once_flag attr_once;
            std::call_once(attr_once, [&] {
                (void)hipFuncSetAttribute((const void*)k_update_b,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds_max);
            });
            const int nsl = (d + kUpdSlice - 1) / kUpdSlice;
            hipLaunchKernelGGL(k_update_b, dim3(grid, nsl), dim3(kUpdWaves * kWave), update_lds, st,
                               plans, Z, it, t);
            break;
        }
        case kKmUpdateFinish:
            hipLaunchKernelGGL(k_update_finish_b, dim3(grid), blk, 0, st, plans, it, t_max, t);
            break;
        default: break;
    }
}

bool kmeans_split_supported(int d) { return d % 32 == 0 && d >= 32 && d <= 256; }

void launch_split_points(const KmeansPlan& p, const float* Z, hipStream_t st) {
    const int64_t total = (int64_t)p.n * p.d;
    if (total == 0) return;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_split_points, dim3(grid), dim3(256), 0, st, p, Z);
}

__global__ __launch_bounds__(256) void k_copy_centres(KmeansPlan p, float* __restrict__ out) {
    const int64_t total = (int64_t)p.KP * p.d;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / p.d), col = (int)(i - (int64_t)c * p.d);
        const int k = p.cand_of[c];
        const int r = c - p.koff16[k];
        if (r < p.ks[k]) out[(size_t)(p.koff[k] + r) * p.d + col] = p.C[i];
    }
}

void launch_copy_centres(const KmeansPlan& p, float* out, hipStream_t st) {
    const int64_t total = (int64_t)p.KP * p.d;
    if (total == 0) return;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_copy_centres, dim3(grid), dim3(256), 0, st, p, out);
}

void launch_prune_init(const KmeansPlan& p, const float* Z, hipStream_t st) {
    const size_t total = (size_t)p.Kc * p.n;
    const int fill = (int)std::max<size_t>(
        (size_t)(std::max(p.KP, p.Kc) + 255) / 256, std::min<size_t>((total + 255) / 256, 4096));
    hipLaunchKernelGGL(k_prune_fill, dim3(fill), dim3(256), 0, st, p);
    if (p.n > 0) {
        hipLaunchKernelGGL(k_prune_prep, dim3((unsigned)std::min((p.n + 3) / 4, 4096)), dim3(256), 0,
                           st, p, Z);
        hipLaunchKernelGGL(k_prune_eps, dim3((p.n + 255) / 256), dim3(256), 0, st, p);
    }
}

void launch_assign_pruned(const KmeansPlan& p, int nact, int num_cu, hipStream_t st, hipEvent_t e0,
                          hipEvent_t e1) {
    if (p.n == 0 || nact <= 0) return;
    hipExtLaunchKernelGGL(k_prune_test, dim3((unsigned)p.nranges, (unsigned)nact), dim3(256), 0, st,
                          e0, nullptr, 0, p);
    // d <= 64: 256-thread work-groups, three per CU; wider: one 1024-thread
    // work-group per CU, its sixteen waves sharing one staged table
    const dim3 grid((unsigned)(num_cu * (p.d <= 64 ? 3 : 1)));
    KmeansPlan q = p;
    q.lists_nact = nact;
    const size_t lds = list_lds_bytes(p.d, p.list_tiles, nact * p.nranges);
#define PRUNED(DV)                                                                                 \
    {                                                                                              \
        static std::once_flag attr_once;                                                           \
        std::call_once(attr_once, [] {                                                             \
            (void)hipFuncSetAttribute((const void*)k_prune_score<DV, list_ps<DV>(), prune_nw<DV>()>, \
                                      hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                      kPruneDynLdsMax);                                            \
        });                                                                                        \
        hipExtLaunchKernelGGL((k_prune_score<DV, list_ps<DV>(), prune_nw<DV>()>), grid,            \
                              dim3(prune_nw<DV>() * 64), lds, st, nullptr, e1, 0, q);              \
    }
    switch (p.d) {
        case 32: PRUNED(32); break;
        case 64: PRUNED(64); break;
        case 128: PRUNED(128); break;
        case 256: PRUNED(256); break;
        default: break;
    }
#undef PRUNED
}

void launch_iter_finalize(const KmeansPlan& p, int it, int t_max, hipStream_t st) {
    hipLaunchKernelGGL(k_iter_finalize, dim3(1), dim3(256), 0, st, p, it, t_max);
}

void launch_update(const KmeansPlan& p, const float* Z, size_t lds_max, int it, int t_max,
                   hipStream_t st) {
    const size_t lds = kmeans_update_lds(p.usk_max, p.d);
    const int nsl = (p.d + kUpdSlice - 1) / kUpdSlice;
    dim3 grid(p.uwork, nsl);
    static std::once_flag attr_once;   // contexts may launch from several host threads
    std::call_once(attr_once, [&] {
        (void)hipFuncSetAttribute((const void*)k_update, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_max);
    });
    hipLaunchKernelGGL(k_update, grid, dim3(kUpdWaves * kWave), lds, st, p, Z);
    hipLaunchKernelGGL(k_update_finish, dim3(p.KP + 1), dim3(256), 0, st, p, it, t_max);
}

}  // namespace raft
