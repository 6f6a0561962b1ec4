// Shared device helpers of the HIP path (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace raft {

constexpr int kWave = 64;
constexpr int RAFT_MAX_K_DEV = 255;   // labels are bytes

// Status bits latched on the device (one int in the context's status word).
constexpr int kStatusCsrRange = 1 << 0;
constexpr int kStatusCsrOrder = 1 << 1;
constexpr int kStatusCsrLoop = 1 << 2;
constexpr int kStatusCsrSym = 1 << 3;
constexpr int kStatusCsrRowPtr = 1 << 4;
constexpr int kStatusNumeric = 1 << 8;
constexpr int kStatusLabel = 1 << 9;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Position of a work-group within the share of a launch that one partition
// owns: index x of n.  A single-graph launch passes (blockIdx.x, gridDim.x);
// a batched launch over several graphs maps each block to its graph first.
struct Wg {
    uint32_t x, n;
};

__device__ __forceinline__ Wg wg_self() { return Wg{blockIdx.x, gridDim.x}; }

// Table of a batched launch: graph g owns blocks [start[g], start[g] +
// count[g]) of the grid; start[g] is a multiple of 8, so a block's XCD
// (blockIdx.x mod 8) is that of its local index, and the padding blocks
// between count[g] and start[g + 1] exit at once.  start holds G + 1 entries
// (the last is the grid size).
struct BatchTable {
    const int32_t* start;
    const int32_t* count;
    int32_t G;
};

// Graph g of this block (the last g with start[g] <= blockIdx.x) and its
// local position; false for a padding block.
__device__ __forceinline__ bool batch_find(const BatchTable& t, int& g, Wg& w) {
    const int b = (int)blockIdx.x;
    int lo = 0, hi = t.G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.start[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    g = lo;
    const int x = b - t.start[lo];
    w.x = (uint32_t)x;
    w.n = (uint32_t)t.count[lo];
    return x >= 0 && x < t.count[lo];
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 10 rounds of two 64x64->128-bit
// multiplies with the published multipliers, Weyl key schedule.
// ---------------------------------------------------------------------------
struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    U64x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// uint64 -> double in (0,1): ((x >> 12) + 0.5) * 2^-52, exact.
__device__ __forceinline__ double uniform52(uint64_t x) {
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// Own FP64 ln and sincos(2*pi*u) from IEEE basic operations only, evaluated
// in a fixed order without contraction, so that every conforming IEEE-754
// implementation of the same sequence returns the same bits.
//   ln x  = e*ln2 + 2*atanh(f), f = (m-1)/(m+1), m in [sqrt(1/2), sqrt(2)),
//           atanh series through f^23;
//   sin/cos(2 pi u): quadrant k = rint(4u), t = (4u-k)*pi/2, |t| <= pi/4,
//           Taylor series through t^19 (sin) and t^20 (cos).
// ---------------------------------------------------------------------------
__device__ __noinline__ double own_ln(double x) {
#pragma clang fp contract(off)
    const double LN2 = 0x1.62e42fefa39efp-1;
    const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;
    int e;
    double m = frexp(x, &e);
    if (m < SQRT_HALF) {
        m = m * 2.0;
        e -= 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double f2 = f * f;
    double s = 1.0 / 23.0;
    s = 1.0 / 21.0 + f2 * s;
    s = 1.0 / 19.0 + f2 * s;
    s = 1.0 / 17.0 + f2 * s;
    s = 1.0 / 15.0 + f2 * s;
    s = 1.0 / 13.0 + f2 * s;
    s = 1.0 / 11.0 + f2 * s;
    s = 1.0 / 9.0 + f2 * s;
    s = 1.0 / 7.0 + f2 * s;
    s = 1.0 / 5.0 + f2 * s;
    s = 1.0 / 3.0 + f2 * s;
    s = f2 * s;
    const double tf = 2.0 * f;
    const double lnm = tf + tf * s;
    return (double)e * LN2 + lnm;
}

__device__ __noinline__ void own_sincos_2pi(double u, double* sn, double* cs) {
#pragma clang fp contract(off)
    const double HALF_PI = 0x1.921fb54442d18p+0;
    const double u4 = u * 4.0;
    const double k = rint(u4);
    const double r = u4 - k;
    const double t = r * HALF_PI;
    const double t2 = t * t;
    // 1/n! with n! exact in binary64
    double ps = -(1.0 / 121645100408832000.0);          // -1/19!
    ps = (1.0 / 355687428096000.0) + t2 * ps;           // +1/17!
    ps = -(1.0 / 1307674368000.0) + t2 * ps;            // -1/15!
    ps = (1.0 / 6227020800.0) + t2 * ps;                // +1/13!
    ps = -(1.0 / 39916800.0) + t2 * ps;                 // -1/11!
    ps = (1.0 / 362880.0) + t2 * ps;                    // +1/9!
    ps = -(1.0 / 5040.0) + t2 * ps;                     // -1/7!
    ps = (1.0 / 120.0) + t2 * ps;                       // +1/5!
    ps = -(1.0 / 6.0) + t2 * ps;                        // -1/3!
    const double s = t + (t * t2) * ps;
    double pc = 1.0 / 2432902008176640000.0;            // +1/20!
    pc = -(1.0 / 6402373705728000.0) + t2 * pc;         // -1/18!
    pc = (1.0 / 20922789888000.0) + t2 * pc;            // +1/16!
    pc = -(1.0 / 87178291200.0) + t2 * pc;              // -1/14!
    pc = (1.0 / 479001600.0) + t2 * pc;                 // +1/12!
    pc = -(1.0 / 3628800.0) + t2 * pc;                  // -1/10!
    pc = (1.0 / 40320.0) + t2 * pc;                     // +1/8!
    pc = -(1.0 / 720.0) + t2 * pc;                      // -1/6!
    pc = (1.0 / 24.0) + t2 * pc;                        // +1/4!
    pc = -(1.0 / 2.0) + t2 * pc;                        // -1/2!
    const double c = 1.0 + t2 * pc;
    const int q = ((int)k) & 3;
    double so, co;
    if (q == 0) {
        so = s;
        co = c;
    } else if (q == 1) {
        so = c;
        co = -s;
    } else if (q == 2) {
        so = -s;
        co = -c;
    } else {
        so = -c;
        co = s;
    }
    *sn = so;
    *cs = co;
}

// Box-Muller on (u0, u1): z0 = rho cos(2 pi u1), z1 = rho sin(2 pi u1).
__device__ __forceinline__ void box_muller(double u0, double u1, double* z0, double* z1) {
#pragma clang fp contract(off)
    const double rho = sqrt(-2.0 * own_ln(u0));
    double s, c;
    own_sincos_2pi(u1, &s, &c);
    *z0 = rho * c;
    *z1 = rho * s;
}

}  // namespace raft
