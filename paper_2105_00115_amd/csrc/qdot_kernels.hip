// qdot kernels for gfx950: exponent scan, cutoff selection, fused
// quantize-and-accumulate, and the plain FP64 dot used as the baseline.
//
// Data layout: x and y are FP64 vectors read in groups of 4 consecutive
// elements per lane (two 16-byte loads per operand when both are 16-byte
// aligned).  A block of 256 lanes covers 1024 consecutive elements per
// group; a wave covers 256, i.e. four 64-element FP32 accumulation tiles,
// one per 16-lane DPP row.  Both passes use the same block -> chunk
// mapping, so on inputs that fit in L2 / Infinity Cache the second pass
// re-reads what the same XCD fetched in the first.
#include "qdot_kernels.hpp"

#include <climits>

namespace qd {

template <bool VEC>
__device__ __forceinline__ void load4_full(const double *__restrict__ p, double v[4])
{
    if (VEC) {
        const double2 a = *reinterpret_cast<const double2 *>(p);
        const double2 b = *reinterpret_cast<const double2 *>(p + 2);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    } else {
#pragma unroll
        for (int e = 0; e < 4; e++) v[e] = p[e];
    }
}

__device__ __forceinline__ void load4_tail(const double *__restrict__ p, int lim, double v[4])
{
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = e < lim ? p[e] : 0.0;
}

// Grid-stride walk over groups of CHUNK * U consecutive components.  Whole
// groups are loaded without bounds checks; the single partial group (met by
// one block at most) is loaded with per-lane limits.  body(xv, yv, i0, lim)
// sees 4 consecutive components i0..i0+3 of which the first `lim` are real;
// it is called with every lane of the block active.
template <bool VEC, int U, class Body>
__device__ __forceinline__ void stream_groups(const double *__restrict__ x,
                                              const double *__restrict__ y, int64_t n,
                                              Body &&body)
{
    const int64_t group = (int64_t)CHUNK * U;
    const int64_t step = (int64_t)gridDim.x * group;
    int64_t base = (int64_t)blockIdx.x * group;
    for (; base + group <= n; base += step) {
        double xv[U][4], yv[U][4];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * CHUNK + threadIdx.x * EPT;
            load4_full<VEC>(x + i0, xv[u]);
            load4_full<VEC>(y + i0, yv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            body(xv[u], yv[u], base + (int64_t)u * CHUNK + threadIdx.x * EPT, 4);
    }
    if (base < n) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * CHUNK + threadIdx.x * EPT;
            const int64_t left = n - i0;
            const int lim = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
            double xv[4], yv[4];
            load4_tail(x + i0, lim, xv);
            load4_tail(y + i0, lim, yv);
            body(xv, yv, i0, lim);
        }
    }
}

__device__ __forceinline__ unsigned int wave_sum_u32(unsigned int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Pass 1 (Alg. 2, exponent preprocessing + counting): product exponents into
// a block-private LDS histogram, merged into one of HIST_COPIES global
// histograms (blockIdx % HIST_COPIES, i.e. one per XCD under round-robin
// dispatch) so that the merge atomics of concurrent blocks spread out.
// ---------------------------------------------------------------------------
template <bool VEC, int U>
__global__ __launch_bounds__(BLOCK) void k_scan(const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                int64_t n, int key_mode,
                                                Ws *__restrict__ ws)
{
    __shared__ unsigned int h[W + 1];
    for (int i = threadIdx.x; i < W + 1; i += BLOCK) h[i] = 0;
    __syncthreads();

    unsigned int nz = 0, bad = 0;
    stream_groups<VEC, U>(x, y, n, [&](const double *xv, const double *yv, int64_t, int lim) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const Comp c = component(xv[e], yv[e], key_mode);
            const bool valid = e < lim;
            nz += (valid & c.zero) ? 1u : 0u;
            bad |= (valid & c.bad) ? 1u : 0u;
            // zero and non-finite products land in the spare slot W
            if (valid) atomicAdd(&h[c.slot], 1u);
        }
    });
    __syncthreads();
    unsigned long long *gh = ws->hist[blockIdx.x % HIST_COPIES];
    int lo = W, hi = -1;
    for (int i = threadIdx.x; i < W; i += BLOCK) {
        const unsigned int v = h[i];
        if (v) {
            atomicAdd(&gh[i], (unsigned long long)v);
            lo = min(lo, i);
            hi = max(hi, i);
        }
    }
    nz = wave_sum_u32(nz);
    bad = wave_sum_u32(bad);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        lo = min(lo, __shfl_xor(lo, m, 64));
        hi = max(hi, __shfl_xor(hi, m, 64));
    }
    __shared__ int2 wr[BLOCK / 64];
    if ((threadIdx.x & 63) == 0) {
        if (nz) atomicAdd(&ws->n_zero, (unsigned long long)nz);
        if (bad) atomicOr(&ws->nonfinite, 1u);
        wr[threadIdx.x >> 6] = make_int2(lo, hi);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // plain store, no contention: the cutoff kernel reduces the records
        int2 r = wr[0];
        for (int w = 1; w < BLOCK / 64; w++) r = make_int2(min(r.x, wr[w].x), max(r.y, wr[w].y));
        ws->block_range[blockIdx.x] = r;
    }
}

// ---------------------------------------------------------------------------
// Cutoff selection (Alg. 2, bins -> scores -> precisions), one workgroup.
// ---------------------------------------------------------------------------

// t = floor(log2(eps / nb)): the largest integer tau with nb * 2^tau <= eps,
// by integer comparison of 53-bit significands.  With eps = S * 2^(E - 52),
// S in [2^52, 2^53), and nb scaled to N' = nb * 2^(53 - b) in the same
// range (b = bit length of nb): nb * 2^tau = N' * 2^(tau - 53 + b), so
// tau = E + 1 - b when N' <= S, else E - b.
__device__ int floor_log2_ratio(double eps, unsigned long long nb)
{
    const uint64_t bits = (uint64_t)__double_as_longlong(eps);
    const Split s = split_bits(bits);
    const uint64_t S = s.frac | (1ull << 52);
    const int b = 64 - __clzll(nb);
    const uint64_t Np = nb << (53 - b);
    return s.e + 1 - b - (Np > S ? 1 : 0);
}

__device__ __forceinline__ int class_of(int sigma, int nonstrict)
{
    // eq. (precision-def) with m_half = 10, m_single = 23; the non-strict
    // reading moves every boundary up by one (score <= m qualifies).
    const int o = nonstrict ? 1 : 0;
    if (sigma < 0 + o) return QDOT_PERF;
    if (sigma < 10 + o) return QDOT_HALF;
    if (sigma < 23 + o) return QDOT_SINGLE;
    return QDOT_DOUBLE;
}

__device__ __forceinline__ double eps_of_class(int c)
{
    return c == QDOT_DOUBLE ? 0x1p-52 : c == QDOT_SINGLE ? 0x1p-23
         : c == QDOT_HALF ? 0x1p-10 : 1.0;
}

__global__ __launch_bounds__(CUT_THREADS) void k_cut(Ws *__restrict__ ws, double tol,
                                                     int score_mode, int nonstrict,
                                                     int64_t n, int nscan,
                                                     qdot_result *__restrict__ out,
                                                     long long *__restrict__ hist_out)
{
    constexpr int R = (W + CUT_THREADS - 1) / CUT_THREADS;
    constexpr int NW = CUT_THREADS / 64;
    __shared__ int s_max[NW], s_min[NW], s_nb[NW], s_unatt[NW];
    __shared__ unsigned long long s_cnt[NW][4];
    __shared__ double s_bound[NW];
    __shared__ int s_emax, s_t, s_go;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // only the slot window pass 1 touched holds counts; slots outside it are
    // zero in every copy and their class-table entries are never read
    __shared__ int s_lo[NW], s_hi[NW];
    int lo = W, hi = -1;
    {
        int a = W, b = -1;
        for (int i = tid; i < nscan; i += CUT_THREADS) {
            const int2 r = ws->block_range[i];
            a = min(a, r.x);
            b = max(b, r.y);
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            a = min(a, __shfl_xor(a, m, 64));
            b = max(b, __shfl_xor(b, m, 64));
        }
        if (lane == 0) {
            s_lo[wv] = a;
            s_hi[wv] = b;
        }
        __syncthreads();
        for (int w = 0; w < NW; w++) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
    }
    unsigned long long cnt[R];
    int emax = INT_MIN, emin = INT_MAX, nb = 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int j = lo + tid + r * CUT_THREADS;
        unsigned long long v = 0ull;
        if (j <= hi)
#pragma unroll
            for (int c = 0; c < HIST_COPIES; c++) v += ws->hist[c][j];
        cnt[r] = v;
        if (cnt[r]) {
            const int k = j + KMIN;
            emax = max(emax, k);
            emin = min(emin, k);
            nb++;
        }
    }
    if (hist_out) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int j = lo + tid + r * CUT_THREADS;
            if (j <= hi) hist_out[j] = (long long)cnt[r];
        }
        for (int j = tid; j < W; j += CUT_THREADS)
            if (j < lo || j > hi) hist_out[j] = 0ll;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        emax = max(emax, __shfl_xor(emax, m, 64));
        emin = min(emin, __shfl_xor(emin, m, 64));
        nb += __shfl_xor(nb, m, 64);
    }
    if (lane == 0) {
        s_max[wv] = emax;
        s_min[wv] = emin;
        s_nb[wv] = nb;
    }
    __syncthreads();
    if (tid == 0) {
        int a = INT_MIN, b = INT_MAX, c = 0;
        for (int w = 0; w < NW; w++) {
            a = max(a, s_max[w]);
            b = min(b, s_min[w]);
            c += s_nb[w];
        }
        const unsigned long long nzero = ws->n_zero;
        const unsigned int bad = ws->nonfinite;
        out->n_zero = (long long)nzero;
        out->n_bins = c;
        out->e_max = c ? a : 0;
        out->e_min = c ? b : 0;
        for (int q = 0; q < 3; q++) out->part[q] = 0.0;
        int go = 1, t = 0;
        if (bad) {
            go = 0;
            out->value = __longlong_as_double(0x7ff8000000000000ll);
            for (int q = 0; q < 4; q++) out->count[q] = 0;
            out->status = QDOT_E_NONFINITE;
            out->flags = 0;
            out->t = 0;
            out->bound_rel = out->bound_abs = 0.0;
        } else if (c == 0) {
            go = 0;
            out->value = 0.0;
            for (int q = 0; q < 3; q++) out->count[q] = 0;
            out->count[QDOT_PERF] = n;
            out->status = QDOT_OK;
            out->flags = QDOT_F_ALL_PERF;
            out->t = 0;
            out->bound_rel = out->bound_abs = 0.0;
        } else {
            t = floor_log2_ratio(tol, score_mode == 0 ? (unsigned long long)c : 1ull);
            out->t = t;
            out->status = QDOT_OK;
        }
        s_emax = a;
        s_t = t;
        s_go = go;
        ws->n_zero = 0;
        ws->nonfinite = 0;
    }
    __syncthreads();
    const int go = s_go;
    const int e_max = s_emax, t = s_t;

    unsigned long long cc[4] = {0, 0, 0, 0};
    double bound = 0.0;
    int unatt = 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int j = lo + tid + r * CUT_THREADS;
        if (j > hi) break;
        int cls = QDOT_PERF;
        if (go && cnt[r]) {
            const int k = j + KMIN;
            // eq. (bin-score-def) with exact bins (u_k = k)
            const int sigma = ceil_log2_u64(cnt[r]) + k - e_max - t + 1;
            cls = class_of(sigma, nonstrict);
            unatt |= sigma >= 52 + (nonstrict ? 1 : 0);
            cc[cls] += cnt[r];
            // Thm 3.3 term M_k 2^(k - e_max + 1) eps(class)
            bound += ldexp((double)cnt[r] * eps_of_class(cls), k - e_max + 1);
        }
        ws->lut[j] = (unsigned char)cls;
#pragma unroll
        for (int c = 0; c < HIST_COPIES; c++) ws->hist[c][j] = 0ull;
    }
    if (tid < W_LUT - W) ws->lut[W + tid] = (unsigned char)QDOT_PERF;

#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
        for (int q = 0; q < 4; q++) cc[q] += __shfl_xor(cc[q], m, 64);
        bound += __shfl_xor(bound, m, 64);
        unatt |= __shfl_xor(unatt, m, 64);
    }
    if (lane == 0) {
        for (int q = 0; q < 4; q++) s_cnt[wv][q] = cc[q];
        s_bound[wv] = bound;
        s_unatt[wv] = unatt;
    }
    __syncthreads();
    if (tid == 0 && go) {
        unsigned long long tc[4] = {0, 0, 0, 0};
        double bsum = 0.0;
        int ua = 0;
        for (int w = 0; w < NW; w++) {
            for (int q = 0; q < 4; q++) tc[q] += s_cnt[w][q];
            bsum += s_bound[w];
            ua |= s_unatt[w];
        }
        tc[QDOT_PERF] += (unsigned long long)out->n_zero;
        for (int q = 0; q < 4; q++) out->count[q] = (long long)tc[q];
        out->bound_rel = bsum;
        out->bound_abs = ldexp(bsum, e_max);
        int flags = ua ? QDOT_F_UNATTAINABLE : 0;
        // Thm 3.6: e_max - e_min <= -t - m_single
        if ((long long)e_max - out->e_min <= -(long long)t - 23) flags |= QDOT_F_THM_ALL_DOUBLE;
        const bool none_kept = (tc[0] + tc[1] + tc[2]) == 0;
        if (none_kept) {
            flags |= QDOT_F_ALL_PERF;
            out->value = 0.0;
        }
        out->flags = flags;
        ws->flags = flags;
        ws->e_max = e_max;
        ws->t = t;
        ws->c32 = e_max + t + 22;
        ws->skip = none_kept ? 1 : 0;
    } else if (tid == 0) {
        ws->skip = 1;
    }
}

// ---------------------------------------------------------------------------
// Pass 2 (Alg. 1): per component class -> quantised product (leaf) ->
// 64-element FP32 tile trees (single and half separately) and compensated
// FP64 sums -> per-block partials (combined by k_fin).
//
// Leaves (exact powers of two scale them; the FP64 result is multiplied by
// 2^e_max once at the end):
//   double: fl64(m_x m_y) * 2^(E_x + E_y - e_max)
//   single: fl32(fl32(m_x) fl32(m_y)) * 2^(E_x + E_y - c32)
//   half  : h16(m_x) h16(m_y) * 2^(E_x + E_y - c32)  (22-bit product, exact)
// with c32 = e_max + t + 22, which keeps every FP32 leaf normal and < 4.
// All three candidates are formed without branches and the class selects
// one; the only branch is the rare zero/subnormal operand path.
// ---------------------------------------------------------------------------
template <bool VEC, int U, bool CLS>
__global__ __launch_bounds__(BLOCK) void k_acc(const double *__restrict__ x,
                                               const double *__restrict__ y,
                                               int64_t n, int key_mode,
                                               const Ws *__restrict__ ws,
                                               double *__restrict__ partials,
                                               unsigned char *__restrict__ cls_out)
{
    __shared__ unsigned char lut[W_LUT];
    __shared__ Acc red[3][BLOCK / 64];

    const int skip = ws->skip;
    if (skip && !CLS) return;
    {
        const unsigned int *src = reinterpret_cast<const unsigned int *>(ws->lut);
        unsigned int *dst = reinterpret_cast<unsigned int *>(lut);
        for (int i = threadIdx.x; i < W_LUT / 4; i += BLOCK) dst[i] = src[i];
    }
    const int e_max = ws->e_max;
    const int c32 = ws->c32;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    Acc aD = {0.0, 0.0}, aS = {0.0, 0.0}, aH = {0.0, 0.0};
    stream_groups<VEC, U>(x, y, n, [&](const double *xv, const double *yv, int64_t i0, int lim) {
        float ls[4], lh[4];
        double ld[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const Comp c = component(xv[e], yv[e], key_mode);
            const bool valid = e < lim;
            const int cls = valid ? (int)lut[c.slot] : QDOT_PERF;
            if (CLS && valid) cls_out[i0 + e] = (unsigned char)cls;
            // double candidate
            double dl = ldexp(c.mp, c.es - e_max);
            dl = __longlong_as_double(__double_as_longlong(dl) ^ ((long long)c.sgn << 32));
            // single and half candidates share one scaling
            const float ps = (float)c.mx * (float)c.my;
            const float ph = (float)(half_round(c.mx) * half_round(c.my));
            float l32 = ldexpf(cls == QDOT_HALF ? ph : ps, c.es - c32);
            l32 = __int_as_float(__float_as_int(l32) ^ (int)c.sgn);
            ld[e] = cls == QDOT_DOUBLE ? dl : 0.0;
            ls[e] = cls == QDOT_SINGLE ? l32 : 0.0f;
            lh[e] = cls == QDOT_HALF ? l32 : 0.0f;
        }
        if (!skip) {
            // tile tree levels 1-2 in the lane, 3-6 across the row
            const float s4 = (ls[0] + ls[1]) + (ls[2] + ls[3]);
            const float h4 = (lh[0] + lh[1]) + (lh[2] + lh[3]);
            const float ts = tile_levels_3to6(s4);
            const float th = tile_levels_3to6(h4);
            acc_add(aD, (ld[0] + ld[1]) + (ld[2] + ld[3]));
            if ((lane & 15) == 0) {
                acc_add(aS, (double)ts);
                acc_add(aH, (double)th);
            }
        }
    });
    if (skip) return;

    aD = wave_reduce(aD);
    aS = wave_reduce(aS);
    aH = wave_reduce(aH);
    const int wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = aD;
        red[1][wv] = aS;
        red[2][wv] = aH;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *p = partials + (size_t)blockIdx.x * 6;
        for (int q = 0; q < 3; q++) {
            Acc b = red[q][0];
            for (int w = 1; w < BLOCK / 64; w++) b = acc_merge(b, red[q][w]);
            p[2 * q] = b.s;
            p[2 * q + 1] = b.c;
        }
    }
}

// Combine the per-block partials of k_acc in a fixed order (one block).
__global__ __launch_bounds__(BLOCK) void k_fin(const Ws *__restrict__ ws,
                                               const double *__restrict__ partials, int nblk,
                                               qdot_result *__restrict__ out)
{
    __shared__ Acc red[3][BLOCK / 64];
    if (ws->skip) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Acc c[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int b = threadIdx.x; b < nblk; b += BLOCK) {
        const double *p = partials + (size_t)b * 6;
        for (int q = 0; q < 3; q++) c[q] = acc_merge(c[q], Acc{p[2 * q], p[2 * q + 1]});
    }
    for (int q = 0; q < 3; q++) c[q] = wave_reduce(c[q]);
    if (lane == 0)
        for (int q = 0; q < 3; q++) red[q][wv] = c[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc f[3];
        for (int q = 0; q < 3; q++) {
            f[q] = red[q][0];
            for (int w = 1; w < BLOCK / 64; w++) f[q] = acc_merge(f[q], red[q][w]);
        }
        const int t = ws->t, e_max = ws->e_max, c32 = ws->c32;
        // S = D + 2^(c32 - e_max) (S + H), with c32 - e_max = t + 22
        Acc tot = f[0];
        acc_add(tot, ldexp(f[1].s, t + 22));
        acc_add(tot, ldexp(f[2].s, t + 22));
        tot.c = tot.c + ldexp(f[1].c + f[2].c, t + 22);
        const double S = tot.s + tot.c;
        const double value = ldexp(S, e_max);
        out->value = value;
        out->part[QDOT_DOUBLE] = ldexp(f[0].s + f[0].c, e_max);
        out->part[QDOT_SINGLE] = ldexp(f[1].s + f[1].c, c32);
        out->part[QDOT_HALF] = ldexp(f[2].s + f[2].c, c32);
        out->flags = ws->flags | (__builtin_isinf(value) ? QDOT_F_OVERFLOW : 0);
    }
}

// ---------------------------------------------------------------------------
// Plain FP64 dot (baseline): same skeleton, FP64 products and sums.
// ---------------------------------------------------------------------------
template <bool VEC, int U>
__global__ __launch_bounds__(BLOCK) void k_dot64(const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 int64_t n, double *__restrict__ partials)
{
    __shared__ double red[BLOCK / 64];
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    stream_groups<VEC, U>(x, y, n, [&](const double *xv, const double *yv, int64_t, int) {
#pragma unroll
        for (int e = 0; e < 4; e++) acc = fma(xv[e], yv[e], acc);
    });
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    const int wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < BLOCK / 64; w++) b += red[w];
        partials[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(BLOCK) void k_dot_fin(const double *__restrict__ partials,
                                                   int nblk, double *__restrict__ out)
{
    __shared__ double red[BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double c = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BLOCK) c += partials[b];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
    if (lane == 0) red[wv] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        double f = red[0];
        for (int w = 1; w < BLOCK / 64; w++) f += red[w];
        *out = f;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static int grid_for(int64_t n, int unroll, int cap)
{
    const int64_t groups = (n + (int64_t)CHUNK * unroll - 1) / ((int64_t)CHUNK * unroll);
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, groups));
}

template <bool VEC, int U>
static int launch_scan_u(const Launch &L, const double *x, const double *y, int64_t n,
                         int key_mode)
{
    const int grid = grid_for(n, U, L.scan_blocks);
    hipLaunchKernelGGL((k_scan<VEC, U>), dim3(grid), dim3(BLOCK), 0, L.stream, x, y, n,
                       key_mode, L.ws);
    return grid;
}

template <bool VEC>
static int launch_scan(const Launch &L, const double *x, const double *y, int64_t n,
                       int key_mode)
{
    switch (L.scan_unroll) {
    case 1: return launch_scan_u<VEC, 1>(L, x, y, n, key_mode);
    case 4: return launch_scan_u<VEC, 4>(L, x, y, n, key_mode);
    default: return launch_scan_u<VEC, 2>(L, x, y, n, key_mode);
    }
}

template <bool VEC, int U, bool CLS>
static int launch_acc_u(const Launch &L, const double *x, const double *y, int64_t n,
                        int key_mode, unsigned char *cls_out)
{
    const int grid = grid_for(n, U, L.acc_blocks);
    hipLaunchKernelGGL((k_acc<VEC, U, CLS>), dim3(grid), dim3(BLOCK), 0, L.stream, x, y, n,
                       key_mode, L.ws, L.partials, cls_out);
    return grid;
}

template <bool VEC, bool CLS>
static int launch_acc(const Launch &L, const double *x, const double *y, int64_t n,
                      int key_mode, unsigned char *cls_out)
{
    switch (L.acc_unroll) {
    case 1: return launch_acc_u<VEC, 1, CLS>(L, x, y, n, key_mode, cls_out);
    case 4: return launch_acc_u<VEC, 4, CLS>(L, x, y, n, key_mode, cls_out);
    default: return launch_acc_u<VEC, 2, CLS>(L, x, y, n, key_mode, cls_out);
    }
}

hipError_t launch_qdot(const Launch &L, const double *x, const double *y, int64_t n,
                       double tol, const qdot_options &o, qdot_result *out,
                       unsigned char *cls_out, long long *hist_out)
{
    const bool vec = ((((uintptr_t)x) | ((uintptr_t)y)) & 15) == 0;
    hipStream_t s = L.stream;
    if (L.ev) (void)hipEventRecord(L.ev[0], s);
    const int nscan = vec ? launch_scan<true>(L, x, y, n, o.key_mode)
                          : launch_scan<false>(L, x, y, n, o.key_mode);
    if (L.ev) (void)hipEventRecord(L.ev[1], s);
    hipLaunchKernelGGL(k_cut, dim3(1), dim3(CUT_THREADS), 0, s, L.ws, tol, o.score_mode,
                       o.boundary_mode, n, nscan, out, hist_out);
    if (L.ev) (void)hipEventRecord(L.ev[2], s);
    int grid;
    if (cls_out)
        grid = vec ? launch_acc<true, true>(L, x, y, n, o.key_mode, cls_out)
                   : launch_acc<false, true>(L, x, y, n, o.key_mode, cls_out);
    else
        grid = vec ? launch_acc<true, false>(L, x, y, n, o.key_mode, nullptr)
                   : launch_acc<false, false>(L, x, y, n, o.key_mode, nullptr);
    if (L.ev) (void)hipEventRecord(L.ev[3], s);
    hipLaunchKernelGGL(k_fin, dim3(1), dim3(BLOCK), 0, s, L.ws, L.partials, grid, out);
    if (L.ev) (void)hipEventRecord(L.ev[4], s);
    return hipGetLastError();
}

template <bool VEC, int U>
static int launch_dot64_u(const Launch &L, const double *x, const double *y, int64_t n)
{
    const int grid = grid_for(n, U, L.acc_blocks);
    hipLaunchKernelGGL((k_dot64<VEC, U>), dim3(grid), dim3(BLOCK), 0, L.stream, x, y, n,
                       L.partials);
    return grid;
}

template <bool VEC>
static int launch_dot64_v(const Launch &L, const double *x, const double *y, int64_t n)
{
    switch (L.acc_unroll) {
    case 1: return launch_dot64_u<VEC, 1>(L, x, y, n);
    case 4: return launch_dot64_u<VEC, 4>(L, x, y, n);
    default: return launch_dot64_u<VEC, 2>(L, x, y, n);
    }
}

hipError_t launch_dot64(const Launch &L, const double *x, const double *y, int64_t n,
                        double *out)
{
    const bool vec = ((((uintptr_t)x) | ((uintptr_t)y)) & 15) == 0;
    if (L.ev) (void)hipEventRecord(L.ev[0], L.stream);
    const int grid = vec ? launch_dot64_v<true>(L, x, y, n) : launch_dot64_v<false>(L, x, y, n);
    hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(BLOCK), 0, L.stream, L.partials, grid, out);
    if (L.ev) (void)hipEventRecord(L.ev[1], L.stream);
    return hipGetLastError();
}

}  // namespace qd
