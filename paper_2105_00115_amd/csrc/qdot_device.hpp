// Device-side building blocks shared by the qdot kernels (gfx950 only).
//
// Everything here is integer or exactly-rounded IEEE arithmetic; the whole
// library is compiled with -ffp-contract=off so that no product is fused
// with the sum that consumes it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qdot.h"

namespace qd {

// Product exponents (keys) span [KMIN, KMAX]: operand exponents are in
// [-1074, 1023] once subnormals are normalised, and the product-mode carry
// adds at most one.
constexpr int KMIN = -2148;
constexpr int KMAX = 2047;
constexpr int W = KMAX - KMIN + 1;          // 4196 histogram slots
constexpr int ZERO_SLOT = W;                // class-table slot of zero products
constexpr int W_LUT = (W + 1 + 15) / 16 * 16;
constexpr int HIST_COPIES = 8;              // one global histogram per XCD

constexpr int BLOCK = 256;                  // threads per block (4 waves)
constexpr int EPT = 4;                      // consecutive elements per lane
constexpr int CHUNK = BLOCK * EPT;          // 1024 elements per block group
constexpr int TILE = 64;                    // FP32 accumulation tile
constexpr int CUT_THREADS = 1024;
constexpr int MAX_GRID = 16 * 256;          // persistent grid cap (16 per CU)

// Class-table code of a single-precision input bin that eq. (precision-def)
// cannot lower (score at or above m_single): the product is formed in FP32,
// the input precision, and added in FP64 with the double leaves relative to
// 2^e_max, since such bins may lie anywhere below e_max.  Counted and
// reported as QDOT_SINGLE; never present for double inputs.
constexpr int SINGLE_IN = 4;

constexpr uint64_t FRAC_MASK = 0x000fffffffffffffull;
constexpr uint64_t ONE_BITS = 0x3ff0000000000000ull;

// Control block in device memory, one per handle.
struct Ws {
    unsigned long long hist[HIST_COPIES][W]; // pass-1 exponent histograms
    unsigned long long n_zero;   // zero products seen by pass 1
    unsigned int nonfinite;      // any Inf/NaN seen by pass 1
    unsigned int pad0;
    int2 block_range[MAX_GRID];  // per scan block: [lo, hi] of its live slots
    // produced by the cutoff kernel for pass 2
    int e_max;
    int t;
    int c32;                     // exponent offset of FP32 leaves
    int skip;                    // nothing to accumulate (result final)
    int flags;                   // result flags known after selection
    int s1_lo, s1_hi;            // live slot range of the last scan
    int mu_single;               // the last selection was for single-precision inputs
    int keep_lo;                 // tile_skip: lowest slot of a kept class (W: none)
    // per scan block: bit 0 = a negative, bit 1 = a positive non-zero product
    unsigned int block_signs[MAX_GRID];
    // guaranteed mode (guard_mode 1)
    long long hsave[W];          // the histogram, kept for the reselection
    double s_last;               // S of the last two-pass combine (units of 2^e_max)
    double g_low;                // lower bound of |x.y| after the first sweep (same units)
    unsigned int signs;          // OR of block_signs over the last scan
    int g_redo;                  // the reselection ran
    unsigned char lut[W_LUT];    // class of every key slot (+ zero slot)
};

// One-pass (exact per-bin) accumulation: a block keeps candidate sums for
// the S1_WIN bins below its running maximum key; S1_PIECES exact FP64 sums
// per bin (half leaf; single leaf in two pieces; double leaf in three).
constexpr int S1_WIN = 256;
constexpr int S1_PIECES = 6;
constexpr int64_t S1_MAX_N = (int64_t)1 << 30;  // bound of the exact-sum argument

// One operand split into unbiased exponent and 52-bit fraction of its
// normalised significand m = 1.frac in [1, 2).  General path (subnormals
// included); the kernels call it only for operands whose biased exponent
// field is zero.
struct Split {
    int e;
    uint64_t frac;
};

__device__ __forceinline__ Split split_bits(uint64_t b)
{
    Split s;
    const uint32_t code = (uint32_t)(b >> 52) & 0x7ffu;
    const uint64_t f = b & FRAC_MASK;
    if (code != 0) {
        s.e = (int)code - 1023;
        s.frac = f;
    } else {
        // subnormal: leading one at bit p (0..51); value 2^(p-1074) * 1.xxx
        const int p = 63 - __clzll(f | 1ull);
        s.e = p - 1074;
        s.frac = (f << (52 - p)) & FRAC_MASK;
    }
    return s;
}

__device__ __forceinline__ double mant(uint64_t frac)
{
    return __longlong_as_double((long long)(frac | ONE_BITS));
}

// One component x_i, y_i reduced to what both passes need:
//   es   = E(x) + E(y)
//   mx, my the significands in [1, 2), mp = fl64(mx * my) in [1, 4)
//   slot = key - KMIN (ZERO_SLOT for a zero product)
//   sgn  = sign bit of x*y in bit 31
// Fast path: both biased exponent fields in 1..2046, all 32-bit integer
// work on the high words.  Zero and subnormal operands (field 0) take a
// rare divergent branch.  Non-finite operands (field 2047) are reported by
// `bad`; their slot is ZERO_SLOT.
struct Comp {
    int es;
    int slot;
    uint32_t sgn;
    bool zero;
    bool bad;
    double mx, my, mp;
};

__device__ __forceinline__ Comp component(double x, double y, int key_mode)
{
    Comp c;
    const uint64_t bx = (uint64_t)__double_as_longlong(x);
    const uint64_t by = (uint64_t)__double_as_longlong(y);
    const uint32_t hx = (uint32_t)(bx >> 32), hy = (uint32_t)(by >> 32);
    const uint32_t cx = (hx >> 20) & 0x7ffu, cy = (hy >> 20) & 0x7ffu;
    c.sgn = (hx ^ hy) & 0x80000000u;
    c.mx = __longlong_as_double((long long)((bx & FRAC_MASK) | ONE_BITS));
    c.my = __longlong_as_double((long long)((by & FRAC_MASK) | ONE_BITS));
    c.es = (int)(cx + cy) - 2046;
    c.zero = false;
    c.bad = max(cx, cy) == 0x7ffu;
    if (__builtin_expect(min(cx, cy) == 0, 0)) {
        c.zero = ((bx << 1) == 0) | ((by << 1) == 0);
        const Split sx = split_bits(bx), sy = split_bits(by);
        c.mx = mant(sx.frac);
        c.my = mant(sy.frac);
        c.es = sx.e + sy.e;
    }
    c.mp = c.mx * c.my;
    const int carry = (key_mode == 0 && c.mp >= 2.0) ? 1 : 0;
    c.slot = (c.zero | c.bad) ? ZERO_SLOT : (c.es + carry - KMIN);
    return c;
}

// Single-precision operands: the same decomposition on 32-bit words.  The
// significands are floats in [1, 2) (exact), and the product key's carry is
// decided exactly from the FP32 product p and its FMA residual r (the exact
// product is p + r; it reaches 2 iff p > 2, or p == 2 and r >= 0).  Zero and
// subnormal operands take the double path: a float widens exactly.
struct CompF {
    int es;
    int slot;
    uint32_t sgn;
    bool zero;
    bool bad;
    float mx, my;
};

__device__ __forceinline__ CompF component_f(float x, float y, int key_mode)
{
    CompF c;
    const uint32_t bx = __float_as_uint(x), by = __float_as_uint(y);
    const uint32_t cx = (bx >> 23) & 0xffu, cy = (by >> 23) & 0xffu;
    c.sgn = (bx ^ by) & 0x80000000u;
    if (__builtin_expect(min(cx, cy) == 0, 0)) {
        const Comp d = component((double)x, (double)y, key_mode);
        c.es = d.es;
        c.slot = d.slot;
        c.zero = d.zero;
        c.bad = d.bad;
        c.mx = (float)d.mx;
        c.my = (float)d.my;
        return c;
    }
    c.mx = __uint_as_float((bx & 0x7fffffu) | 0x3f800000u);
    c.my = __uint_as_float((by & 0x7fffffu) | 0x3f800000u);
    c.es = (int)(cx + cy) - 254;
    c.zero = false;
    c.bad = max(cx, cy) == 0xffu;
    const float p = c.mx * c.my;
    const float r = __builtin_fmaf(c.mx, c.my, -p);
    const int carry = (key_mode == 0 && (p > 2.0f || (p == 2.0f && r >= 0.0f))) ? 1 : 0;
    c.slot = c.bad ? ZERO_SLOT : (c.es + carry - KMIN);
    return c;
}

// Binary16 significand of a float m in [1, 2): adding 2^13 leaves an ulp of
// 2^-10, so the sum rounds m to 10 fraction bits (nearest even) exactly once.
__device__ __forceinline__ float half_round_f(float m)
{
    const float big = 0x1p13f;
    return (m + big) - big;
}

// Binary16 significand of m in [1, 2), round to nearest even in one step
// straight from FP64: m + 2^42 has an ulp of 2^-10, so the addition rounds
// m to the nearest multiple of 2^-10 (ties to even) and the subtraction is
// exact.  Result in [1, 2].
__device__ __forceinline__ double half_round(double m)
{
    const double big = 0x1p42;
    return (m + big) - big;
}

// ---- cross-lane moves (DPP, within 16-lane rows) -------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <- 7 - i within 8
constexpr int DPP_MIRROR = 0x140;      // lane i <- 15 - i within 16

// Levels 3..6 of the adjacent-pairwise tree of a 64-element tile held as
// 16 lanes x 4 consecutive leaves, each lane entering with the sum of its
// own 4 leaves (levels 1..2).  After each level every lane of a group holds
// the same group sum (IEEE addition is commutative), so any partner lane in
// the neighbouring group supplies the same operand.
__device__ __forceinline__ float tile_levels_3to6(float s)
{
    s = s + dpp_f<DPP_XOR1>(s);
    s = s + dpp_f<DPP_XOR2>(s);
    s = s + dpp_f<DPP_HALF_MIRROR>(s);
    s = s + dpp_f<DPP_MIRROR>(s);
    return s;
}

// ---- compensated FP64 accumulation ---------------------------------------
struct Acc {
    double s, c;
};

__device__ __forceinline__ void acc_add(Acc &a, double v)
{
    const double t = a.s + v;
    const double bp = t - a.s;
    const double err = (a.s - (t - bp)) + (v - bp);
    a.s = t;
    a.c = a.c + err;
}

__device__ __forceinline__ Acc acc_merge(Acc a, Acc b)
{
    Acc r = a;
    acc_add(r, b.s);
    r.c = r.c + b.c;
    return r;
}

__device__ __forceinline__ Acc acc_shfl_xor(Acc a, int mask)
{
    Acc b;
    b.s = __shfl_xor(a.s, mask, 64);
    b.c = __shfl_xor(a.c, mask, 64);
    return b;
}

__device__ __forceinline__ Acc wave_reduce(Acc a)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) a = acc_merge(a, acc_shfl_xor(a, m));
    return a;
}

// ceil(log2 m), m >= 1
__device__ __forceinline__ int ceil_log2_u64(unsigned long long m)
{
    return m <= 1 ? 0 : 64 - __clzll(m - 1);
}

}  // namespace qd
