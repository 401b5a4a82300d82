// Block-level pieces shared by the single-vector kernels and the persistent
// batched kernel: streaming loops, the cutoff selection of one qdot by one
// workgroup, the per-group leaf computation, and the final combine.
#pragma once

#include <climits>

#include "qdot_device.hpp"

namespace qd {

// ---- loads ---------------------------------------------------------------
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

// single-precision inputs: 4 consecutive floats are one 16-byte load
template <bool VEC>
__device__ __forceinline__ void load4_full(const float *__restrict__ p, float v[4])
{
    if (VEC) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; e++) v[e] = p[e];
    }
}

template <class T>
__device__ __forceinline__ void load4_tail(const T *__restrict__ p, int lim, T v[4])
{
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = e < lim ? p[e] : T(0);
}

// One block of NT threads walks groups of U * NT * EPT components of x, y:
// the groups that start at first, first + stride, first + 2 * stride, ...
// below n (stride a multiple of the group).  Each thread loads EPT
// consecutive components of each NT * EPT chunk, U chunks in flight; the one
// partial group is bounds-checked.
template <bool VEC, int U, int NT = BLOCK, class T, class Body>
__device__ __forceinline__ void stream_strided(const T *__restrict__ x, const T *__restrict__ y,
                                               int64_t first, int64_t stride, int64_t n,
                                               Body &&body)
{
    constexpr int64_t chunk = (int64_t)NT * EPT;
    const int64_t group = chunk * U;
    int64_t base = first;
    for (; base + group <= n; base += stride) {
        T xv[U][4], yv[U][4];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * chunk + threadIdx.x * EPT;
            load4_full<VEC>(x + i0, xv[u]);
            load4_full<VEC>(y + i0, yv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            body(xv[u], yv[u], base + (int64_t)u * chunk + threadIdx.x * EPT, 4);
    }
    if (base < n) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * chunk + threadIdx.x * EPT;
            const int64_t left = n - i0;
            const int lim = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
            T xv[4], yv[4];
            load4_tail(x + i0, lim, xv);
            load4_tail(y + i0, lim, yv);
            body(xv, yv, i0, lim);
        }
    }
}

// stream_strided for tile_skip.  A 64-component tile (the 4 components of
// 16 consecutive lanes) whose largest key slot tk[i / TILE] lies below
// keep_lo holds only perforated components: its lanes load nothing and pass
// zeros, whose products are zero and perforated too, so body() forms the
// same leaves (zero) and classes (perforated).  A wave none of whose tiles
// of a group is live skips the group: it calls dead(i0, lim) for each of its
// chunks instead of body() (the leaves it skips are +0, and adding +0 leaves
// a compensated sum that starts at +0 unchanged, bit for bit).  The keys of
// the block's full groups are staged in LDS a batch at a time, one key per
// thread (KB = 16 / U groups of U chunks of NT / 16 tiles), the next batch
// loaded while the current one is processed; kl holds 2 x NT keys.  The one
// partial group reads its keys directly.  Every thread of the block must
// call it with the same arguments.
template <bool VEC, int U, int NT = BLOCK, class T, class Body, class Dead>
__device__ __forceinline__ void stream_strided_ts(const T *__restrict__ x,
                                                  const T *__restrict__ y, int64_t first,
                                                  int64_t stride, int64_t n,
                                                  const short *__restrict__ tk, int keep_lo,
                                                  short (*kl)[NT], Body &&body, Dead &&dead)
{
    constexpr int64_t chunk = (int64_t)NT * EPT;
    const int64_t group = chunk * U;
    constexpr int TPC = NT * EPT / TILE;  // tiles per chunk
    constexpr int KB = 16 / U;            // groups per batch: KB * U * TPC == NT
    static_assert(KB * U * TPC == NT, "one staged key per thread");
    const int64_t nfull = n >= first + group ? (n - first - group) / stride + 1 : 0;
    auto key_of = [&](int64_t g0) -> short {
        const int t = threadIdx.x;
        const int64_t gi = g0 + t / (U * TPC);
        if (gi >= nfull) return (short)-1;
        const int64_t i = first + gi * stride + (int64_t)((t / TPC) % U) * chunk +
                          (int64_t)(t % TPC) * TILE;
        return tk[i / TILE];
    };
    int buf = 0;
    short next = nfull > 0 ? key_of(0) : (short)-1;
    const int row = threadIdx.x * EPT / TILE;
    for (int64_t g0 = 0; g0 < nfull; g0 += KB) {
        kl[buf][threadIdx.x] = next;
        __syncthreads();
        if (g0 + KB < nfull) next = key_of(g0 + KB);
        const int gend = (int)std::min<int64_t>(KB, nfull - g0);
        for (int gg = 0; gg < gend; gg++) {
            const int64_t base = first + (g0 + gg) * stride;
            bool live[U];
            bool any = false;
#pragma unroll
            for (int u = 0; u < U; u++) {
                live[u] = kl[buf][(gg * U + u) * TPC + row] >= keep_lo;
                any |= live[u];
            }
            if (__ballot(any) == 0ull) {
#pragma unroll
                for (int u = 0; u < U; u++) dead(base + (int64_t)u * chunk + threadIdx.x * EPT, 4);
                continue;
            }
            T xv[U][4], yv[U][4];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int64_t i0 = base + (int64_t)u * chunk + threadIdx.x * EPT;
                if (live[u]) {
                    load4_full<VEC>(x + i0, xv[u]);
                    load4_full<VEC>(y + i0, yv[u]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; e++) xv[u][e] = yv[u][e] = T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                body(xv[u], yv[u], base + (int64_t)u * chunk + threadIdx.x * EPT, 4);
        }
        buf ^= 1;
    }
    const int64_t base = first + nfull * stride;
    if (base < n) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * chunk + threadIdx.x * EPT;
            const int64_t left = n - i0;
            const int lim = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
            T xv[4], yv[4];
            if (lim > 0 && tk[i0 / TILE] >= keep_lo) {
                load4_tail(x + i0, lim, xv);
                load4_tail(y + i0, lim, yv);
            } else {
#pragma unroll
                for (int e = 0; e < 4; e++) xv[e] = yv[e] = T(0);
            }
            body(xv, yv, i0, lim);
        }
    }
}

// Grid-stride walk over groups of CHUNK * U consecutive components: block b
// takes groups b, b + gridDim.x, ...  Whole groups are loaded without bounds
// checks; the single partial group (met by one block at most) is loaded with
// per-lane limits.  body(xv, yv, i0, lim) sees 4 consecutive components
// i0..i0+3 of which the first `lim` are real; it is called with every lane
// of the block active.
template <bool VEC, int U, int NT = BLOCK, class T, class Body>
__device__ __forceinline__ void stream_groups(const T *__restrict__ x, const T *__restrict__ y,
                                              int64_t n, Body &&body)
{
    const int64_t group = (int64_t)NT * EPT * U;
    stream_strided<VEC, U, NT>(x, y, (int64_t)blockIdx.x * group, (int64_t)gridDim.x * group,
                               n, body);
}

__device__ __forceinline__ unsigned int wave_sum_u32(unsigned int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// block-wide reduction of a range and two counters; result in every thread
__device__ __forceinline__ void block_reduce_range(int &lo, int &hi, unsigned int &nz,
                                                   unsigned int &bad, int4 *scratch)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        lo = min(lo, __shfl_xor(lo, m, 64));
        hi = max(hi, __shfl_xor(hi, m, 64));
        nz += __shfl_xor(nz, m, 64);
        bad |= __shfl_xor(bad, m, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wv] = make_int4(lo, hi, (int)nz, (int)bad);
    __syncthreads();
    lo = W;
    hi = -1;
    nz = 0;
    bad = 0;
    for (int w = 0; w < BLOCK / 64; w++) {
        lo = min(lo, scratch[w].x);
        hi = max(hi, scratch[w].y);
        nz += (unsigned int)scratch[w].z;
        bad |= (unsigned int)scratch[w].w;
    }
}

// End of pass 1 in one block: merges the block's LDS histogram h (W + 1
// slots; slot W takes zero and non-finite products, and is not merged) into
// copy blockIdx % copies of ws's global histograms (copies <= HIST_COPIES;
// the cutoff reads all HIST_COPIES), adds the zero count,
// raises the non-finite flag, and stores the block's record at index rec
// (its live slot range and the signs of its nonzero products: bit 0
// negative, bit 1 positive) for the cutoff kernel.  nz, bad and sg are the
// calling thread's own tallies.  Every thread calls it, after a barrier that
// completes h; it ends with one, so it can be called again.
template <int NT = BLOCK>
__device__ __forceinline__ void scan_flush(const unsigned int *h, unsigned int nz,
                                           unsigned int bad, unsigned int sg, Ws *ws, int rec,
                                           int copies = HIST_COPIES)
{
    unsigned long long *gh = ws->hist[blockIdx.x % copies];
    int lo = W, hi = -1;
    for (int i = threadIdx.x; i < W; i += NT) {
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
        sg |= __shfl_xor(sg, m, 64);
    }
    __shared__ int2 wr[NT / 64];
    __shared__ unsigned int wsg[NT / 64];
    if ((threadIdx.x & 63) == 0) {
        if (nz) atomicAdd(&ws->n_zero, (unsigned long long)nz);
        if (bad) atomicOr(&ws->nonfinite, 1u);
        wr[threadIdx.x >> 6] = make_int2(lo, hi);
        wsg[threadIdx.x >> 6] = sg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // plain stores, no contention: the cutoff kernel reduces the records
        int2 r = wr[0];
        unsigned int g = wsg[0];
        for (int w = 1; w < NT / 64; w++) {
            r = make_int2(min(r.x, wr[w].x), max(r.y, wr[w].y));
            g |= wsg[w];
        }
        ws->block_range[rec] = r;
        ws->block_signs[rec] = g;
    }
    __syncthreads();
}

// ---- hand-over between blocks of one launch ------------------------------
// Data that one block hands to another inside a launch travels only through
// device-scope atomics: read-modify-writes, relaxed stores (written through
// to the device's coherence point) and relaxed loads (served from it).  A
// release then needs no writeback of the XCD's L2: it is enough that the
// publishing thread's own memory operations have completed, which the
// vector-memory counter wait in vmem_drain ensures, before the flag or count
// that announces them is written.  An agent-scope release fence would write
// back the whole L2 of the XCD, and an acquire fence would invalidate it;
// with other blocks streaming that costs far more than the counter wait.
__device__ __forceinline__ void vmem_drain()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <class T>
__device__ __forceinline__ T ld_dev(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void st_dev(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pass-1 merge of a block whose LDS histogram is a window of nwin slots
// starting at slot base (keys outside it were added to the global copy
// directly; lo, hi cover those): as scan_flush.
__device__ __forceinline__ void scan_flush_window(const unsigned int *h, int base, int nwin,
                                                  int lo, int hi, unsigned int nz,
                                                  unsigned int bad, unsigned int sg, Ws *ws,
                                                  int rec, int copies)
{
    unsigned long long *gh = ws->hist[blockIdx.x % copies];
    for (int i = threadIdx.x; i < nwin; i += BLOCK) {
        const unsigned int v = h[i];
        if (v) {
            atomicAdd(&gh[base + i], (unsigned long long)v);
            lo = min(lo, base + i);
            hi = max(hi, base + i);
        }
    }
    nz = wave_sum_u32(nz);
    bad = wave_sum_u32(bad);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        lo = min(lo, __shfl_xor(lo, m, 64));
        hi = max(hi, __shfl_xor(hi, m, 64));
        sg |= __shfl_xor(sg, m, 64);
    }
    __shared__ int2 wr[BLOCK / 64];
    __shared__ unsigned int wsg[BLOCK / 64];
    if ((threadIdx.x & 63) == 0) {
        if (nz) atomicAdd(&ws->n_zero, (unsigned long long)nz);
        if (bad) atomicOr(&ws->nonfinite, 1u);
        wr[threadIdx.x >> 6] = make_int2(lo, hi);
        wsg[threadIdx.x >> 6] = sg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int2 r = wr[0];
        unsigned int g = wsg[0];
        for (int w = 1; w < BLOCK / 64; w++) {
            r = make_int2(min(r.x, wr[w].x), max(r.y, wr[w].y));
            g |= wsg[w];
        }
        ws->block_range[rec] = r;
        ws->block_signs[rec] = g;
    }
}

// ---- cutoff selection (Alg. 2: bins -> scores -> precisions) ------------

// t = floor(log2(eps / nb)): the largest integer tau with nb * 2^tau <= eps,
// by integer comparison of 53-bit significands.  With eps = S * 2^(E - 52),
// S in [2^52, 2^53), and nb scaled to N' = nb * 2^(53 - b) in the same
// range (b = bit length of nb): nb * 2^tau = N' * 2^(tau - 53 + b), so
// tau = E + 1 - b when N' <= S, else E - b.
__device__ __forceinline__ int floor_log2_ratio(double eps, unsigned long long nb)
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
    return c == QDOT_DOUBLE ? 0x1p-52 : (c == QDOT_SINGLE || c == SINGLE_IN) ? 0x1p-23
         : c == QDOT_HALF ? 0x1p-10 : 1.0;
}

struct CutParams {
    int e_max, t, c32, skip, flags;
};

// Cutoff selection of one qdot by one workgroup of NT threads (all of them
// must call it).  Only slots lo..hi may hold counts: get(j) returns the count
// of slot j, clear(j) resets it after use, put(j, cls) stores the class of
// slot j.  Writes every field of *out except value and part (which the
// combine writes) unless nothing is to be accumulated, in which case *out is
// final.  Returns the parameters of pass 2 to every thread.  The scores are
// taken against e_ref = e_max - dref (dref > 0 only when the guaranteed mode
// reselects against a lower estimate of flexp(x.y), Thm 3.4); bound_rel
// stays the Thm 3.3 sum relative to e_max.  mu_single: the inputs are
// single precision, so eq. (precision-def) has no double row.
template <int NT, class Get, class Put, class Clear>
__device__ CutParams block_cutoff(int lo, int hi, unsigned long long nzero, unsigned int bad,
                                  int64_t n, double tol, int score_mode, int nonstrict,
                                  Get get, Put put, Clear clear, qdot_result *out,
                                  long long *hist_out, int dref = 0, int mu_single = 0)
{
    constexpr int NW = NT / 64;
    __shared__ int s_max[NW], s_min[NW], s_nb[NW], s_unatt[NW];
    __shared__ unsigned long long s_cnt[NW][4];
    __shared__ double s_bound[NW];
    __shared__ CutParams s_prm;
    __shared__ int s_go;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // the counts of a thread's first RC slots stay in registers for the
    // classification below (a window of up to RC * NT slots is read once);
    // slots further up are read again there
    constexpr int RC = 2;
    unsigned long long vc[RC];
    int emax = INT_MIN, emin = INT_MAX, nb = 0;
    auto survey = [&](int j, unsigned long long v) {
        if (hist_out) hist_out[j] = (long long)v;
        if (v) {
            const int k = j + KMIN;
            emax = max(emax, k);
            emin = min(emin, k);
            nb++;
        }
    };
#pragma unroll
    for (int r = 0; r < RC; r++) {
        const int j = lo + tid + r * NT;
        vc[r] = j <= hi ? (unsigned long long)get(j) : 0ull;
        if (j <= hi) survey(j, vc[r]);
    }
    for (int j = lo + tid + RC * NT; j <= hi; j += NT) survey(j, (unsigned long long)get(j));
    if (hist_out)
        for (int j = tid; j < W; j += NT)
            if (j < lo || j > hi) hist_out[j] = 0ll;
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
        out->n_zero = (long long)nzero;
        out->n_bins = c;
        out->e_max = c ? a : 0;
        out->e_min = c ? b : 0;
        out->e_ref = c ? a - dref : 0;
        out->lower = 0.0;
        out->passes = 0;
        for (int q = 0; q < 3; q++) out->part[q] = 0.0;
        int go = 1, t = 0;
        const bool tol_ok = tol > 0.0 && !__builtin_isinf(tol) && !__builtin_isnan(tol);
        if (bad || !tol_ok) {
            // an error result: status and a NaN value, every other field 0
            go = 0;
            out->value = __longlong_as_double(0x7ff8000000000000ll);
            for (int q = 0; q < 4; q++) out->count[q] = 0;
            out->n_zero = 0;
            out->n_bins = 0;
            out->e_max = out->e_min = out->e_ref = 0;
            out->status = bad ? QDOT_E_NONFINITE : QDOT_E_INVAL;
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
        s_prm.e_max = a;
        s_prm.t = t;
        s_prm.c32 = a - dref + t + 22;
        s_prm.skip = 1;
        s_prm.flags = 0;
        s_go = go;
    }
    __syncthreads();
    const int go = s_go;
    const int e_max = s_prm.e_max, t = s_prm.t, e_ref = e_max - dref;

    unsigned long long cc[4] = {0, 0, 0, 0};
    double bound = 0.0;
    int unatt = 0;
    auto classify = [&](int j, unsigned long long v) {
        int cls = QDOT_PERF;
        if (go && v) {
            const int k = j + KMIN;
            // eq. (bin-score-def) with exact bins (u_k = k)
            const int sigma = ceil_log2_u64(v) + k - e_ref - t + 1;
            cls = class_of(sigma, nonstrict);
            // single inputs (mu = m_single): no double row; such a bin stays
            // at the input precision and is flagged like a double bin >= 52
            if (mu_single && cls == QDOT_DOUBLE) cls = SINGLE_IN;
            unatt |= sigma >= (mu_single ? 23 : 52) + (nonstrict ? 1 : 0);
            cc[cls == SINGLE_IN ? QDOT_SINGLE : cls] += v;
            // Thm 3.3 term M_k 2^(k - e_max + 1) eps(class)
            bound += ldexp((double)v * eps_of_class(cls), k - e_max + 1);
        }
        put(j, cls);
        clear(j);
    };
#pragma unroll
    for (int r = 0; r < RC; r++) {
        const int j = lo + tid + r * NT;
        if (j <= hi) classify(j, vc[r]);
    }
    for (int j = lo + tid + RC * NT; j <= hi; j += NT) classify(j, (unsigned long long)get(j));
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
        tc[QDOT_PERF] += nzero;
        for (int q = 0; q < 4; q++) out->count[q] = (long long)tc[q];
        out->bound_rel = bsum;
        out->bound_abs = ldexp(bsum, e_max);
        int flags = ua ? QDOT_F_UNATTAINABLE : 0;
        // Thm 3.6: e_ref - e_min <= -t - m, m = m_single (double inputs) or
        // m_half (single inputs): every bin at the input precision
        if ((long long)e_ref - out->e_min <= -(long long)t - (mu_single ? 10 : 23))
            flags |= QDOT_F_THM_ALL_DOUBLE;
        const bool none_kept = (tc[0] + tc[1] + tc[2]) == 0;
        out->passes = none_kept ? 0 : 1;
        if (none_kept) {
            flags |= QDOT_F_ALL_PERF;
            out->value = 0.0;
        }
        out->flags = flags;
        s_prm.flags = flags;
        s_prm.skip = none_kept ? 1 : 0;
    }
    __syncthreads();
    return s_prm;
}

// ---- other binning strategies (Sec. 3.2) ------------------------------------
//
// Exact bins hold one exponent each.  The other two partitions of
// [e_min, e_max] that Sec. 3.2 weighs (its draft text defines them):
//   bin_mode 1: ranged bins of width w = bin_param, (u_k - w, u_k] with
//     u_k = e_min + k w - 1, k = 1, 2, ... (the last may reach past e_max);
//   bin_mode 2: variable-width bins from at most bin_param splits: start
//     from the one bin (e_min - 1, e_max]; each split takes the non-empty bin
//     of more than one exponent whose Thm 3.2 term M_k 2^(u_k) is largest
//     (ties to the higher u_k) and halves it at l + ceil((u - l) / 2).
// A bin's score (eq. bin-score-def) uses its upper exponent u_k, its class
// applies to all its keys, N_bins counts the non-empty bins and the Thm 3.3
// term is M_k 2^(u_k - e_max + 1) eps(class).  Bins are kept as slot ranges
// [lo, u] (slot = key - KMIN; u may pass the last slot for ranged bins).
struct BinLds {
    short lo[W + 1], u[W + 1];
    unsigned long long m[W + 1];
    int nb;
    int best;
    unsigned long long part[CUT_THREADS / 64];
    int bestw[CUT_THREADS / 64];
};

// bin a's term M 2^u exceeds bin b's (ties to the higher u); counts below
// 2^53 convert exactly
__device__ __forceinline__ bool bin_heavier(const BinLds &B, int a, int b)
{
    const int d = (int)B.u[a] - (int)B.u[b];
    if (d >= 64) return true;
    if (d <= -64) return false;
    const double va = ldexp((double)B.m[a], d), vb = (double)B.m[b];
    if (va != vb) return va > vb;
    return B.u[a] > B.u[b];
}

// Sum of get(j) over slots [a, b] by the whole block (result in every thread).
template <int NT, class Get>
__device__ __forceinline__ unsigned long long block_range_sum(BinLds &B, int a, int b, Get get)
{
    unsigned long long v = 0ull;
    for (int j = a + (int)threadIdx.x; j <= b; j += NT) v += (unsigned long long)get(j);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) B.part[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0ull;
    for (int w = 0; w < NT / 64; w++) t += B.part[w];
    return t;
}

// As block_cutoff (same outputs, same pass-2 parameters), for bin_mode 1 or
// 2.  Only slots lo..hi may hold counts.
template <int NT, class Get, class Put, class Clear>
__device__ CutParams block_cutoff_bins(BinLds &B, int lo, int hi, unsigned long long nzero,
                                       unsigned int bad, int64_t n, double tol, int score_mode,
                                       int nonstrict, int bin_mode, int bin_param, Get get,
                                       Put put, Clear clear, qdot_result *out,
                                       long long *hist_out, int mu_single = 0)
{
    constexpr int NW = NT / 64;
    __shared__ int s_max[NW], s_min[NW], s_nb[NW], s_unatt[NW];
    __shared__ unsigned long long s_cnt[NW][4];
    __shared__ double s_bound[NW];
    __shared__ CutParams s_prm;
    __shared__ int s_go;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    // e_max, e_min over the live keys
    int smax = -1, smin = W;
    for (int j = lo + tid; j <= hi; j += NT) {
        const unsigned long long v = (unsigned long long)get(j);
        if (hist_out) hist_out[j] = (long long)v;
        if (v) {
            smax = max(smax, j);
            smin = min(smin, j);
        }
    }
    if (hist_out)
        for (int j = tid; j < W; j += NT)
            if (j < lo || j > hi) hist_out[j] = 0ll;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        smax = max(smax, __shfl_xor(smax, m, 64));
        smin = min(smin, __shfl_xor(smin, m, 64));
    }
    if (lane == 0) {
        s_max[wv] = smax;
        s_min[wv] = smin;
    }
    __syncthreads();
    smax = -1;
    smin = W;
    for (int w = 0; w < NW; w++) {
        smax = max(smax, s_max[w]);
        smin = min(smin, s_min[w]);
    }
    const bool any = smax >= 0;

    // the partition
    if (any && bin_mode == 1) {
        const int w = bin_param;
        const int nbr = (smax - smin) / w + 1;
        for (int b = tid; b < nbr; b += NT) {
            const int a = smin + b * w, u = a + w - 1;
            unsigned long long m = 0ull;
            for (int j = a; j <= min(u, smax); j++) m += (unsigned long long)get(j);
            B.lo[b] = (short)a;
            B.u[b] = (short)u;
            B.m[b] = m;
        }
        if (tid == 0) B.nb = nbr;
    } else if (any) {
        const unsigned long long all = block_range_sum<NT>(B, smin, smax, get);
        if (tid == 0) {
            B.lo[0] = (short)smin;
            B.u[0] = (short)smax;
            B.m[0] = all;
            B.nb = 1;
        }
        __syncthreads();
        for (int sp = 0; sp < bin_param; sp++) {
            // the heaviest splittable bin
            const int nb = B.nb;
            int best = -1;
            for (int i = tid; i < nb; i += NT)
                if (B.m[i] > 0 && B.u[i] > B.lo[i] && (best < 0 || bin_heavier(B, i, best)))
                    best = i;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                const int o = __shfl_xor(best, m, 64);
                if (o >= 0 && (best < 0 || bin_heavier(B, o, best))) best = o;
            }
            if (lane == 0) B.bestw[wv] = best;
            __syncthreads();
            if (tid == 0) {
                int b2 = -1;
                for (int w = 0; w < NW; w++) {
                    const int o = B.bestw[w];
                    if (o >= 0 && (b2 < 0 || bin_heavier(B, o, b2))) b2 = o;
                }
                B.best = b2;
            }
            __syncthreads();
            const int bi = B.best;
            if (bi < 0) break;  // every non-empty bin is a single exponent
            const int l = (int)B.lo[bi] - 1, u = B.u[bi];
            const int mid = l + (u - l + 1) / 2;
            const unsigned long long ml = block_range_sum<NT>(B, l + 1, mid, get);
            if (tid == 0) {
                const unsigned long long mb = B.m[bi];
                const int k = B.nb;
                B.lo[k] = (short)(l + 1);
                B.u[k] = (short)mid;
                B.m[k] = ml;
                B.lo[bi] = (short)(mid + 1);
                B.m[bi] = mb - ml;
                B.nb = k + 1;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    const int nbt = any ? B.nb : 0;
    int nbk = 0;
    for (int i = tid; i < nbt; i += NT) nbk += B.m[i] > 0 ? 1 : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) nbk += __shfl_xor(nbk, m, 64);
    if (lane == 0) s_nb[wv] = nbk;
    __syncthreads();
    if (tid == 0) {
        int c = 0;
        for (int w = 0; w < NW; w++) c += s_nb[w];
        const int a = any ? smax + KMIN : 0;
        out->n_zero = (long long)nzero;
        out->n_bins = c;
        out->e_max = c ? a : 0;
        out->e_min = c ? smin + KMIN : 0;
        out->e_ref = c ? a : 0;
        out->lower = 0.0;
        out->passes = 0;
        for (int q = 0; q < 3; q++) out->part[q] = 0.0;
        int go = 1, t = 0;
        const bool tol_ok = tol > 0.0 && !__builtin_isinf(tol) && !__builtin_isnan(tol);
        if (bad || !tol_ok) {
            // an error result: status and a NaN value, every other field 0
            go = 0;
            out->value = __longlong_as_double(0x7ff8000000000000ll);
            for (int q = 0; q < 4; q++) out->count[q] = 0;
            out->n_zero = 0;
            out->n_bins = 0;
            out->e_max = out->e_min = out->e_ref = 0;
            out->status = bad ? QDOT_E_NONFINITE : QDOT_E_INVAL;
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
        s_prm.e_max = a;
        s_prm.t = t;
        s_prm.c32 = a + t + 22;
        s_prm.skip = 1;
        s_prm.flags = 0;
        s_go = go;
    }
    __syncthreads();
    const int go = s_go;
    const int e_max = s_prm.e_max, t = s_prm.t;
    // every live slot's class is set by its bin below; empty slots of the
    // window outside every bin stay perforated
    for (int j = lo + tid; j <= hi; j += NT)
        if (!go || j < smin || j > smax) put(j, QDOT_PERF);
    unsigned long long cc[4] = {0, 0, 0, 0};
    double bound = 0.0;
    int unatt = 0;
    for (int i = tid; i < nbt; i += NT) {
        const unsigned long long v = B.m[i];
        const int ua = B.u[i], la = B.lo[i];
        int cls = QDOT_PERF;
        if (go && v) {
            const int uk = ua + KMIN;
            const int sigma = ceil_log2_u64(v) + uk - e_max - t + 1;
            cls = class_of(sigma, nonstrict);
            if (mu_single && cls == QDOT_DOUBLE) cls = SINGLE_IN;
            unatt |= sigma >= (mu_single ? 23 : 52) + (nonstrict ? 1 : 0);
            cc[cls == SINGLE_IN ? QDOT_SINGLE : cls] += v;
            bound += ldexp((double)v * eps_of_class(cls), uk - e_max + 1);
        }
        if (go)
            for (int j = max(la, lo); j <= min(ua, hi); j++) put(j, cls);
    }
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
    // the counts are no longer read: clear the window
    for (int j = lo + tid; j <= hi; j += NT) clear(j);
    if (tid == 0 && go) {
        unsigned long long tc[4] = {0, 0, 0, 0};
        double bsum = 0.0;
        int ua = 0;
        for (int w = 0; w < NW; w++) {
            for (int q = 0; q < 4; q++) tc[q] += s_cnt[w][q];
            bsum += s_bound[w];
            ua |= s_unatt[w];
        }
        tc[QDOT_PERF] += nzero;
        for (int q = 0; q < 4; q++) out->count[q] = (long long)tc[q];
        out->bound_rel = bsum;
        out->bound_abs = ldexp(bsum, e_max);
        int flags = ua ? QDOT_F_UNATTAINABLE : 0;
        if ((long long)e_max - out->e_min <= -(long long)t - (mu_single ? 10 : 23))
            flags |= QDOT_F_THM_ALL_DOUBLE;
        const bool none_kept = (tc[0] + tc[1] + tc[2]) == 0;
        out->passes = none_kept ? 0 : 1;
        if (none_kept) {
            flags |= QDOT_F_ALL_PERF;
            out->value = 0.0;
        }
        out->flags = flags;
        s_prm.flags = flags;
        s_prm.skip = none_kept ? 1 : 0;
    }
    __syncthreads();
    return s_prm;
}

// ---- guaranteed mode (Thm 3.4) ---------------------------------------------
// After a sweep of pass 2 with sum S (units of 2^e_max), a bound a of every
// error of the call, evaluated from the histogram and the classes alone,
//   a = (Q + T + F)(1 + 2^-40),
//   Q = sum_k M_k 2^(k-e_max+1) rho(class_k)                  quantisation
//   T = g6 (1 + 2^-9) sum_{single, half bins} M_k 2^(k-e_max+1)  FP32 trees
//   F = 2^-52 |S| + 4 gn^2 (1 + 2^-8) sum_{kept bins} M_k 2^(k-e_max+1)
//       + (2n + 4) 2^-1074                  FP64 stage, subnormal scaling
// gives the lower bound L = |S| (1 - 2^-52) - a of |x.y|, raised to 1 when
// every non-zero product has one sign (|x.y| >= max |x_i y_i| >= 2^e_max).
// When L > 0, E_lo = e_max + flexp(L) <= flexp(x.y), and the call is
// certified when bound_rel 2^(e_max - E_lo) <= eps.  guard_sums gives Q, the
// FP32-class weight and the kept weight; guard_lower gives L.
struct GuardSums {
    double q, f32, kept;
};

__device__ __forceinline__ double guard_rho(int c)
{
    // largest relative error of one leaf of each class
    return c == QDOT_DOUBLE ? 0x1p-53
         : (c == QDOT_SINGLE || c == SINGLE_IN) ? 0x1.8p-23 + 0x1.8p-47 + 0x1p-72  // (1+2^-24)^3 - 1
         : c == QDOT_HALF   ? 0x1p-10 + 0x1p-22                // (1+2^-11)^2 - 1
                            : 1.0;
}

// get(j): the count of slot j (any integer type)
template <int NT, class Get>
__device__ GuardSums guard_sums(Get get, const unsigned char *__restrict__ lut, int lo, int hi,
                                int e_max)
{
    constexpr int NW = NT / 64;
    __shared__ double s_v[3][NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double v[3] = {0.0, 0.0, 0.0};
    for (int j = lo + tid; j <= hi; j += NT) {
        const long long m = (long long)get(j);
        if (m == 0) continue;
        const int e = j + KMIN - e_max + 1;
        const int c = lut[j];
        const double w = ldexp((double)m, e);
        v[0] += ldexp((double)m * guard_rho(c), e);
        v[1] += (c == QDOT_SINGLE || c == QDOT_HALF) ? w : 0.0;
        v[2] += c != QDOT_PERF ? w : 0.0;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int q = 0; q < 3; q++) v[q] += __shfl_xor(v[q], m, 64);
    if (lane == 0)
        for (int q = 0; q < 3; q++) s_v[q][wv] = v[q];
    __syncthreads();
    GuardSums g = {0.0, 0.0, 0.0};
    for (int w = 0; w < NW; w++) {
        g.q += s_v[0][w];
        g.f32 += s_v[1][w];
        g.kept += s_v[2][w];
    }
    __syncthreads();
    return g;
}

__device__ __forceinline__ double guard_lower(const GuardSums &g, double S, int64_t n,
                                              unsigned int signs)
{
    const double g6 = 6.0 * 0x1p-24 / (1.0 - 6.0 * 0x1p-24);
    const double nu = (double)n * 0x1p-53;
    const double gn = nu / (1.0 - nu);
    const double F = 0x1p-52 * fabs(S) + 4.0 * gn * gn * (1.0 + 0x1p-8) * g.kept +
                     (2.0 * (double)n + 4.0) * 0x1p-1074;
    const double a = (g.q + g6 * (1.0 + 0x1p-9) * g.f32 + F) * (1.0 + 0x1p-40);
    double low = fabs(S) * (1.0 - 0x1p-52) - a;
    if (signs != 3u && low < 1.0) low = 1.0;  // one sign: |x.y| >= 2^e_max
    return low;
}

__device__ __forceinline__ bool guard_certified(double bound_rel, double low, double tol)
{
    return low > 0.0 && ldexp(bound_rel, -ilogb(low)) <= tol;
}

// ---- pass 2: leaves of 4 consecutive components ---------------------------
//
// Leaves (exact powers of two scale them; the FP64 result is multiplied by
// 2^e_max once at the end):
//   double: fl64(m_x m_y) * 2^(E_x + E_y - e_max)
//   single: fl32(fl32(m_x) fl32(m_y)) * 2^(E_x + E_y - c32)
//   half  : h16(m_x) h16(m_y) * 2^(E_x + E_y - c32)  (22-bit product, exact)
// with c32 = e_max + t + 22, which keeps every FP32 leaf normal and < 4.
// All three candidates are formed without branches and the class selects
// one; the only branch is the rare zero/subnormal operand path.  The FP32
// leaves of the 64-element tile are reduced by the adjacent-pairwise tree
// (levels 1-2 in the lane, 3-6 across the 16-lane row), and one lane per
// row adds the two tile sums to its FP64 accumulators.  Every lane of the
// wave must be active.
// T is the input type.  Single-precision inputs (whose class table never
// holds the double class) take the float decomposition: the same single and
// half leaves bit for bit, formed in FP32 (the float significands are exact),
// and no double leaf.
template <bool CLS, class T>
__device__ __forceinline__ void acc_group(const T *xv, const T *yv, int lim,
                                          const unsigned char *lut, int key_mode, int e_max,
                                          int c32, bool accumulate, Acc &aD, Acc &aS, Acc &aH,
                                          unsigned char *cls_out)
{
    float ls[4], lh[4];
    if constexpr (sizeof(T) == 4) {
        // bins held at the input precision (SINGLE_IN): the FP32 product,
        // summed in FP64 relative to 2^e_max with the double class's sums
        double li[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const CompF c = component_f(xv[e], yv[e], key_mode);
            const bool valid = e < lim;
            const int cls = valid ? (int)lut[c.slot] : QDOT_PERF;
            if (CLS && valid)
                cls_out[e] = (unsigned char)(cls == SINGLE_IN ? QDOT_SINGLE : cls);
            const float ps = c.mx * c.my;
            const float ph = half_round_f(c.mx) * half_round_f(c.my);  // 22 bits: exact
            float l32 = ldexpf(cls == QDOT_HALF ? ph : ps, c.es - c32);
            l32 = __int_as_float(__float_as_int(l32) ^ (int)c.sgn);
            ls[e] = cls == QDOT_SINGLE ? l32 : 0.0f;
            lh[e] = cls == QDOT_HALF ? l32 : 0.0f;
            double l64 = ldexp((double)ps, c.es - e_max);
            l64 = __longlong_as_double(__double_as_longlong(l64) ^ ((long long)c.sgn << 32));
            li[e] = cls == SINGLE_IN ? l64 : 0.0;
        }
        if (accumulate) {
            const float s4 = (ls[0] + ls[1]) + (ls[2] + ls[3]);
            const float h4 = (lh[0] + lh[1]) + (lh[2] + lh[3]);
            const float ts = tile_levels_3to6(s4);
            const float th = tile_levels_3to6(h4);
            acc_add(aD, (li[0] + li[1]) + (li[2] + li[3]));
            if ((threadIdx.x & 15) == 0) {
                acc_add(aS, (double)ts);
                acc_add(aH, (double)th);
            }
        }
        return;
    }
    double ld[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const Comp c = component((double)xv[e], (double)yv[e], key_mode);
        const bool valid = e < lim;
        const int cls = valid ? (int)lut[c.slot] : QDOT_PERF;
        if (CLS && valid) cls_out[e] = (unsigned char)cls;
        double dl = ldexp(c.mp, c.es - e_max);
        dl = __longlong_as_double(__double_as_longlong(dl) ^ ((long long)c.sgn << 32));
        const float ps = (float)c.mx * (float)c.my;
        const float ph = (float)(half_round(c.mx) * half_round(c.my));
        float l32 = ldexpf(cls == QDOT_HALF ? ph : ps, c.es - c32);
        l32 = __int_as_float(__float_as_int(l32) ^ (int)c.sgn);
        ld[e] = cls == QDOT_DOUBLE ? dl : 0.0;
        ls[e] = cls == QDOT_SINGLE ? l32 : 0.0f;
        lh[e] = cls == QDOT_HALF ? l32 : 0.0f;
    }
    if (accumulate) {
        const float s4 = (ls[0] + ls[1]) + (ls[2] + ls[3]);
        const float h4 = (lh[0] + lh[1]) + (lh[2] + lh[3]);
        const float ts = tile_levels_3to6(s4);
        const float th = tile_levels_3to6(h4);
        acc_add(aD, (ld[0] + ld[1]) + (ld[2] + ld[3]));
        if ((threadIdx.x & 15) == 0) {
            acc_add(aS, (double)ts);
            acc_add(aH, (double)th);
        }
    }
}

// ---- pass 2, compacting form ----------------------------------------------
//
// The same leaves, tile trees and FP64 sums as acc_group, with the leaf work
// done only for kept components.  Each lane classifies its 4 components from
// their keys; the kept ones are compacted per wave into an LDS queue
// (operands, position in the wave's 256-component group, class) and taken
// 64 at a time by the whole wave, which forms each queued component's leaf:
// a double leaf goes straight into the lane's compensated FP64 sum, an FP32
// leaf into the group's leaf slot of its class.  The lanes then read their
// 4 slots of each FP32 class back (zero where nothing was kept), reduce the
// 64-element tiles by the same adjacent-pairwise tree, and clear the slots.
// FP32 tile sums are therefore bit for bit those of acc_group; only the
// order of the FP64 additions differs, which the compensated sums absorb.
struct AccWaveLds {
    double2 q[128];  // queued operands
    int qm[128];     // queued position (bits 0..7) and class (bits 8..)
    float ls[256];   // single leaves of the group's components (0: none)
    float lh[256];   // half leaves
};

// Zero the leaf slots (every thread of the block, before the first group).
template <int NT>
__device__ __forceinline__ void acc_q_begin(AccWaveLds *wl)
{
    for (int i = threadIdx.x; i < (NT / 64) * 256; i += NT) {
        wl[i / 256].ls[i % 256] = 0.0f;
        wl[i / 256].lh[i % 256] = 0.0f;
    }
}

template <bool CLS, class T>
__device__ __forceinline__ void acc_group_q(const T *xv, const T *yv, int lim,
                                            const unsigned char *lut, int key_mode, int e_max,
                                            int c32, bool accumulate, Acc &aD, Acc &aS, Acc &aH,
                                            unsigned char *cls_out, AccWaveLds &wl)
{
    const int lane = threadIdx.x & 63;
    int cls[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        int slot;
        if constexpr (sizeof(T) == 4) slot = component_f(xv[e], yv[e], key_mode).slot;
        else slot = component((double)xv[e], (double)yv[e], key_mode).slot;
        cls[e] = e < lim ? (int)lut[slot] : QDOT_PERF;
        if (CLS && e < lim)
            cls_out[e] = (unsigned char)(cls[e] == SINGLE_IN ? QDOT_SINGLE : cls[e]);
    }
    if (!accumulate) return;
    // leaf of one queued component (lanes below cnt)
    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const double2 v = wl.q[lane];
            const int m = wl.qm[lane];
            const int idx = m & 255, c = m >> 8;
            float l32;
            if constexpr (sizeof(T) == 4) {
                const CompF d = component_f((float)v.x, (float)v.y, key_mode);
                const float ps = d.mx * d.my;
                const float ph = half_round_f(d.mx) * half_round_f(d.my);  // exact
                if (c == SINGLE_IN) {
                    double l64 = ldexp((double)ps, d.es - e_max);
                    l64 = __longlong_as_double(__double_as_longlong(l64) ^
                                               ((long long)d.sgn << 32));
                    acc_add(aD, l64);
                }
                l32 = ldexpf(c == QDOT_HALF ? ph : ps, d.es - c32);
                l32 = __int_as_float(__float_as_int(l32) ^ (int)d.sgn);
            } else {
                const Comp d = component(v.x, v.y, key_mode);
                if (c == QDOT_DOUBLE) {
                    double dl = ldexp(d.mp, d.es - e_max);
                    dl = __longlong_as_double(__double_as_longlong(dl) ^ ((long long)d.sgn << 32));
                    acc_add(aD, dl);
                }
                const float ps = (float)d.mx * (float)d.my;
                const float ph = (float)(half_round(d.mx) * half_round(d.my));
                l32 = ldexpf(c == QDOT_HALF ? ph : ps, d.es - c32);
                l32 = __int_as_float(__float_as_int(l32) ^ (int)d.sgn);
            }
            if (c == QDOT_SINGLE) wl.ls[idx] = l32;
            if (c == QDOT_HALF) wl.lh[idx] = l32;
        }
        __builtin_amdgcn_wave_barrier();
    };
    int qn = 0;  // wave-uniform
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const bool kept = cls[e] != QDOT_PERF;
        const unsigned long long m = __ballot(kept);
        if (kept) {
            const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                     (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            wl.q[pos] = make_double2((double)xv[e], (double)yv[e]);
            wl.qm[pos] = (lane * 4 + e) | (cls[e] << 8);
        }
        qn += __popcll(m);
        if (qn >= 64) {
            drain(64);
            if (lane < qn - 64) {
                wl.q[lane] = wl.q[64 + lane];
                wl.qm[lane] = wl.qm[64 + lane];
            }
            __builtin_amdgcn_wave_barrier();
            qn -= 64;
        }
    }
    if (qn > 0) drain(qn);
    // the group's FP32 tiles: 16 lanes x 4 slots each, levels 1-2 in the
    // lane, 3-6 across the row; then the slots back to zero
    const float4 sv = *reinterpret_cast<const float4 *>(&wl.ls[lane * 4]);
    const float4 hv = *reinterpret_cast<const float4 *>(&wl.lh[lane * 4]);
    *reinterpret_cast<float4 *>(&wl.ls[lane * 4]) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    *reinterpret_cast<float4 *>(&wl.lh[lane * 4]) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float ts = tile_levels_3to6((sv.x + sv.y) + (sv.z + sv.w));
    const float th = tile_levels_3to6((hv.x + hv.y) + (hv.z + hv.w));
    if ((threadIdx.x & 15) == 0) {
        acc_add(aS, (double)ts);
        acc_add(aH, (double)th);
    }
}

// ---- one-pass mode: candidate leaves relative to the component's bin -----
// A component with key k (bin 2^k) has, for every precision, the leaf of
// Alg. 1 divided by 2^k: s * L * 2^(E_x + E_y - k) with L = fl64(m_x m_y),
// fl32(fl32(m_x) fl32(m_y)) or r16(m_x) r16(m_y); the factor is 1 or 1/2
// (the product key's carry), so every candidate lies in (-4, 4) on a fixed
// grid: 2^-21 (half), 2^-24 (single), 2^-52 (double).  The single and
// double candidates are split, by rounding to coarser grids with the
// add-and-subtract trick (exact), into pieces whose sums over up to 2^30
// components stay exact in FP64 in any order:
//   half   h                       grid 2^-21, |sum| < 2^32
//   single a (2^-20) + b           |b| <= 2^-21, grid 2^-24
//   double a (2^-20) + b (2^-40) + c   |b| <= 2^-21, |c| <= 2^-41, grid 2^-52
// so the candidate sums of a bin can be formed by atomic adds in any order
// and the class chosen afterwards.
__device__ __forceinline__ void s1_pieces(const Comp &c, int key_mode, double p[S1_PIECES])
{
    const double c20 = 0x1.8p+32;  // ulp 2^-20 over the whole range of use
    const double c40 = 0x1.8p+12;  // ulp 2^-40
    const double sc = (key_mode == 0 && c.mp >= 2.0) ? 0.5 : 1.0;
    const double sg = c.sgn ? -1.0 : 1.0;
    const double vd = sg * (c.mp * sc);
    const double vs = sg * ((double)((float)c.mx * (float)c.my) * sc);
    const double vh = sg * ((half_round(c.mx) * half_round(c.my)) * sc);
    p[0] = vh;
    const double sa = (vs + c20) - c20;
    p[1] = sa;
    p[2] = vs - sa;
    const double da = (vd + c20) - c20;
    const double dr = vd - da;
    const double db = (dr + c40) - c40;
    p[3] = da;
    p[4] = db;
    p[5] = dr - db;
}

// Reduce three compensated accumulators over the block; the result is valid
// in thread 0.  red must hold 3 * (blockDim / 64) entries.
template <int NT>
__device__ __forceinline__ void block_reduce3(Acc a[3], Acc (*red)[NT / 64])
{
    for (int q = 0; q < 3; q++) a[q] = wave_reduce(a[q]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < 3; q++) red[q][wv] = a[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; q++) {
            Acc b = red[q][0];
            for (int w = 1; w < NT / 64; w++) b = acc_merge(b, red[q][w]);
            a[q] = b;
        }
}

// Number of bins below e_max that can hold kept components, for any
// histogram of n components at tolerance tol (tol finite and > 0): a bin k
// is kept only if ceil(log2 M_k) + k - e_max - t + 1 >= 0, and t is at least
// floor(log2 tol) - ceil(log2 min(n, W)) - 1 (adjusted score) or
// floor(log2 tol) (raw score).  The one-pass mode needs it <= S1_WIN.
__device__ __forceinline__ int s1_depth_dev(int64_t n, double tol, int score_mode)
{
    const int fl = ilogb(tol);
    const long long nb = n < 1 ? 1 : (n < W ? n : W);
    const int t_low = score_mode == 0 ? fl - ceil_log2_u64((unsigned long long)nb) - 1 : fl;
    return ceil_log2_u64((unsigned long long)(n < 1 ? 1 : n)) - t_low + 2;
}

// LDS of one block's one-pass window: candidate sums of the bins within
// `depth` of the running maximum key (slot = bin mod S1_WIN), the two
// alternating words on which each group's new maximum is agreed, and one
// queue per wave of in-window components.
struct S1Lds {
    double win[S1_WIN][S1_PIECES];
    int top2[2];
    double2 q[BLOCK / 64][128];
};

// Start a window (every thread; the caller synchronises before use).
__device__ __forceinline__ void s1_begin(S1Lds &S)
{
    for (int i = threadIdx.x; i < S1_WIN * S1_PIECES; i += BLOCK) (&S.win[0][0])[i] = 0.0;
    if (threadIdx.x < 2) S.top2[threadIdx.x] = -1;
}

// Running state of a block's one-pass window between groups.
struct S1Run {
    int top;  // highest live slot seen so far by the block (-1: none)
    int par;  // which of the two LDS words the next group agrees top in
};

__device__ __forceinline__ S1Run s1_run_start() { return S1Run{-1, 0}; }

// One group of K components per thread (component e of this thread is real
// when valid[e]): keys into the LDS histogram h (W + 1 slots), zero /
// non-finite counts, and the candidate sums of every component whose bin
// lies within `depth` of the block's running maximum live slot run.top.
// The new maximum is agreed at a barrier; when it rises the slots of the
// entering bins are cleared first.  The in-window components are compacted
// per wave and processed 64 at a time.  Every thread of the block must call
// it (with the same depth).  T is the input type: floats are widened
// exactly (their single and half candidates are then those of the float
// path; the double candidate is never picked, the class table having no
// double row).
template <int K, class T>
__device__ __forceinline__ void s1_group(const T (&xv)[K], const T (&yv)[K],
                                         const bool (&valid)[K], int key_mode, int depth,
                                         unsigned int *h, S1Lds &S, S1Run &run,
                                         unsigned int &nz, unsigned int &bad)
{
    const int tid = threadIdx.x, lane = tid & 63;
    int live[K];
    int wmax = -1;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const Comp c = component((double)xv[e], (double)yv[e], key_mode);
        nz += (valid[e] & c.zero) ? 1u : 0u;
        bad |= (valid[e] & c.bad) ? 1u : 0u;
        if (valid[e]) atomicAdd(&h[c.slot], 1u);
        live[e] = (valid[e] && c.slot != ZERO_SLOT) ? c.slot : -1;
        wmax = max(wmax, live[e]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) wmax = max(wmax, __shfl_xor(wmax, m, 64));
    if (lane == 0 && wmax > run.top) atomicMax(&S.top2[run.par], wmax);
    __syncthreads();
    const int nt = S.top2[run.par];
    run.par ^= 1;
    if (nt > run.top) {
        // bins top+1 .. nt enter; their slots held bins now below the window
        const int nclr = min(nt - run.top, S1_WIN);
        for (int i = tid; i < nclr * S1_PIECES; i += BLOCK)
            S.win[(nt - i / S1_PIECES) & (S1_WIN - 1)][i % S1_PIECES] = 0.0;
        __syncthreads();
        run.top = nt;
    }
    const int wlo = run.top - depth + 1;
    double2 *qw = S.q[tid >> 6];
    int qn = 0;  // wave-uniform
    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const double2 v = qw[lane];
            const Comp c = component(v.x, v.y, key_mode);
            double pc[S1_PIECES];
            s1_pieces(c, key_mode, pc);
            double *w = S.win[c.slot & (S1_WIN - 1)];
#pragma unroll
            for (int q = 0; q < S1_PIECES; q++)
                if (pc[q] != 0.0) atomicAdd(&w[q], pc[q]);
        }
        __builtin_amdgcn_wave_barrier();
    };
#pragma unroll
    for (int e = 0; e < K; e++) {
        const bool in = live[e] >= wlo && live[e] >= 0;
        const unsigned long long m = __ballot(in);
        if (in) {
            const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                     (unsigned)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            qw[pos] = make_double2((double)xv[e], (double)yv[e]);
        }
        qn += __popcll(m);
        if (qn >= 64) {
            drain(64);
            if (lane < qn - 64) qw[lane] = qw[64 + lane];
            __builtin_amdgcn_wave_barrier();
            qn -= 64;
        }
    }
    if (qn > 0) drain(qn);
}

// One block streams the groups first, first + stride, ... (GROUP = U * CHUNK
// components each) below n through s1_group (4 consecutive components per
// thread and CHUNK, U CHUNKs per group).  Every thread of the block must call
// it with the same arguments.
template <bool VEC, int U, class T>
__device__ __forceinline__ void s1_stream(const T *__restrict__ x, const T *__restrict__ y,
                                          int64_t first, int64_t stride, int64_t n,
                                          int key_mode, int depth, unsigned int *h, S1Lds &S,
                                          S1Run &run, unsigned int &nz, unsigned int &bad)
{
    const int tid = threadIdx.x;
    const int64_t group = (int64_t)CHUNK * U;
    for (int64_t base = first; base < n; base += stride) {
        T xv[U][4], yv[U][4];
        int lim[U];
        const bool full = base + group <= n;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * CHUNK + tid * EPT;
            if (full) {
                lim[u] = 4;
                load4_full<VEC>(x + i0, xv[u]);
                load4_full<VEC>(y + i0, yv[u]);
            } else {
                const int64_t left = n - i0;
                lim[u] = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
                load4_tail(x + i0, lim[u], xv[u]);
                load4_tail(y + i0, lim[u], yv[u]);
            }
        }
        T xf[U * 4], yf[U * 4];
        bool vf[U * 4];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                xf[u * 4 + e] = xv[u][e];
                yf[u * 4 + e] = yv[u][e];
                vf[u * 4 + e] = e < lim[u];
            }
        s1_group<U * 4>(xf, yf, vf, key_mode, depth, h, S, run, nz, bad);
    }
}

// ---- one-pass mode, one window per wave ----------------------------------
// The same candidate sums as s1_group, kept by each wave in a window of its
// own (S1W_WIN bins below the wave's running maximum live slot), so the
// waves of a block never wait for each other while they stream: a wave
// agrees on its new maximum with a shuffle, clears the slots of the bins
// that enter, and drains its in-window components into its window.  The
// mode needs depth <= S1W_WIN.  Used for single-precision inputs, whose
// groups are half the bytes of double groups.  At the end of the block the wave windows
// are added into one block window below the block's maximum (s1w_merge);
// the sums are exact in any order, so the result is that of s1_group.
constexpr int S1W_WIN = 64;

struct S1WLds {
    double win[BLOCK / 64][S1W_WIN][S1_PIECES];
    double blk[S1W_WIN][S1_PIECES];
    double2 q[BLOCK / 64][128];
    int top[BLOCK / 64];
};

__device__ __forceinline__ void s1w_begin(S1WLds &S)
{
    double *w = &S.win[0][0][0];
    for (int i = threadIdx.x; i < (BLOCK / 64) * S1W_WIN * S1_PIECES; i += BLOCK) w[i] = 0.0;
    double *b = &S.blk[0][0];
    for (int i = threadIdx.x; i < S1W_WIN * S1_PIECES; i += BLOCK) b[i] = 0.0;
}

// One group of K components per thread into the block's LDS histogram h and
// the calling wave's window; top is the wave's running maximum live slot
// (wave-uniform, -1: none).  Every lane of the wave must call it.
template <int K, class T>
__device__ __forceinline__ void s1w_group(const T (&xv)[K], const T (&yv)[K],
                                          const bool (&valid)[K], int key_mode, int depth,
                                          unsigned int *h, S1WLds &S, int &top,
                                          unsigned int &nz, unsigned int &bad)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int live[K];
    int wmax = -1;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const Comp c = component((double)xv[e], (double)yv[e], key_mode);
        nz += (valid[e] & c.zero) ? 1u : 0u;
        bad |= (valid[e] & c.bad) ? 1u : 0u;
        if (valid[e]) atomicAdd(&h[c.slot], 1u);
        live[e] = (valid[e] && c.slot != ZERO_SLOT) ? c.slot : -1;
        wmax = max(wmax, live[e]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) wmax = max(wmax, __shfl_xor(wmax, m, 64));
    double(*win)[S1_PIECES] = S.win[wv];
    if (wmax > top) {
        // bins top+1 .. wmax enter; their slots held bins now below the window
        const int nclr = min(wmax - top, S1W_WIN);
        for (int i = lane; i < nclr * S1_PIECES; i += 64)
            win[(wmax - i / S1_PIECES) & (S1W_WIN - 1)][i % S1_PIECES] = 0.0;
        __builtin_amdgcn_wave_barrier();
        top = wmax;
    }
    const int wlo = top - depth + 1;
    double2 *qw = S.q[wv];
    int qn = 0;  // wave-uniform
    auto drain = [&](int cnt) {
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const double2 v = qw[lane];
            const Comp c = component(v.x, v.y, key_mode);
            double pc[S1_PIECES];
            s1_pieces(c, key_mode, pc);
            double *w = win[c.slot & (S1W_WIN - 1)];
#pragma unroll
            for (int q = 0; q < S1_PIECES; q++)
                if (pc[q] != 0.0) atomicAdd(&w[q], pc[q]);
        }
        __builtin_amdgcn_wave_barrier();
    };
#pragma unroll
    for (int e = 0; e < K; e++) {
        const bool in = live[e] >= wlo && live[e] >= 0;
        const unsigned long long m = __ballot(in);
        if (in) {
            const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                     (unsigned)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            qw[pos] = make_double2((double)xv[e], (double)yv[e]);
        }
        qn += __popcll(m);
        if (qn >= 64) {
            drain(64);
            if (lane < qn - 64) qw[lane] = qw[64 + lane];
            __builtin_amdgcn_wave_barrier();
            qn -= 64;
        }
    }
    if (qn > 0) drain(qn);
}

// s1_stream with a window per wave (s1w_group).
template <bool VEC, int U, class T>
__device__ __forceinline__ void s1w_stream(const T *__restrict__ x, const T *__restrict__ y,
                                           int64_t first, int64_t stride, int64_t n,
                                           int key_mode, int depth, unsigned int *h, S1WLds &S,
                                           int &top, unsigned int &nz, unsigned int &bad)
{
    const int tid = threadIdx.x;
    const int64_t group = (int64_t)CHUNK * U;
    for (int64_t base = first; base < n; base += stride) {
        T xv[U][4], yv[U][4];
        int lim[U];
        const bool full = base + group <= n;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i0 = base + (int64_t)u * CHUNK + tid * EPT;
            if (full) {
                lim[u] = 4;
                load4_full<VEC>(x + i0, xv[u]);
                load4_full<VEC>(y + i0, yv[u]);
            } else {
                const int64_t left = n - i0;
                lim[u] = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
                load4_tail(x + i0, lim[u], xv[u]);
                load4_tail(y + i0, lim[u], yv[u]);
            }
        }
        T xf[U * 4], yf[U * 4];
        bool vf[U * 4];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                xf[u * 4 + e] = xv[u][e];
                yf[u * 4 + e] = yv[u][e];
                vf[u * 4 + e] = e < lim[u];
            }
        s1w_group<U * 4>(xf, yf, vf, key_mode, depth, h, S, top, nz, bad);
    }
}

// The wave windows added into the block window S.blk below the block's
// maximum live slot, which it returns (-1: none); bins of a wave below the
// block's window are perforated whatever the rest of the data holds and are
// left out.  Every thread of the block must call it (top: its wave's).
__device__ __forceinline__ int s1w_merge(S1WLds &S, int top, int depth)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) S.top[wv] = top;
    __syncthreads();
    int T = -1;
    for (int w = 0; w < BLOCK / 64; w++) T = max(T, S.top[w]);
    if (top >= 0) {
        const int lo = max(top, T) - depth + 1;
        const int cnt = top >= lo ? (top - lo + 1) * S1_PIECES : 0;
        for (int i = lane; i < cnt; i += 64) {
            const int bin = top - i / S1_PIECES;
            if (bin < 0) continue;
            const double v = S.win[wv][bin & (S1W_WIN - 1)][i % S1_PIECES];
            if (v != 0.0) atomicAdd(&S.blk[bin & (S1W_WIN - 1)][i % S1_PIECES], v);
        }
    }
    __syncthreads();
    return T;
}

// One-pass pick: each kept bin k in [e_max - S1_WIN + 1, e_max] (and >= lo)
// contributes the candidate sum of its class (get(bin, piece), an exact
// FP64 number), scaled by 2^(k - e_max); the block sums them with
// compensation and thread 0 writes value, parts and flags.  lut holds the
// class of every slot.  Every thread must call it.
template <int NT, class Get>
__device__ __forceinline__ void s1_pick_nt(int e_max, int lo, int flags, const unsigned char *lut,
                                        Get get, Acc (*red)[NT / 64], qdot_result *out)
{
    const int top = e_max - KMIN;
    Acc a[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};  // double, single, half
    for (int j = threadIdx.x; j < S1_WIN; j += NT) {
        const int bin = top - j;
        if (bin < lo) continue;
        const int cls = lut[bin];
        if (cls == QDOT_DOUBLE) {
            acc_add(a[0], ldexp(get(bin, 3), -j));
            acc_add(a[0], ldexp(get(bin, 4), -j));
            acc_add(a[0], ldexp(get(bin, 5), -j));
        } else if (cls == QDOT_SINGLE || cls == SINGLE_IN) {
            acc_add(a[1], ldexp(get(bin, 1), -j));
            acc_add(a[1], ldexp(get(bin, 2), -j));
        } else if (cls == QDOT_HALF) {
            acc_add(a[2], ldexp(get(bin, 0), -j));
        }
    }
    block_reduce3<NT>(a, red);
    if (threadIdx.x == 0) {
        Acc tot = a[0];
        acc_add(tot, a[1].s);
        acc_add(tot, a[2].s);
        tot.c = tot.c + (a[1].c + a[2].c);
        const double value = ldexp(tot.s + tot.c, e_max);
        out->value = value;
        out->part[QDOT_DOUBLE] = ldexp(a[0].s + a[0].c, e_max);
        out->part[QDOT_SINGLE] = ldexp(a[1].s + a[1].c, e_max);
        out->part[QDOT_HALF] = ldexp(a[2].s + a[2].c, e_max);
        out->flags = flags | (__builtin_isinf(value) ? QDOT_F_OVERFLOW : 0);
    }
}

template <class Get>
__device__ __forceinline__ void s1_pick(int e_max, int lo, int flags, const unsigned char *lut,
                                        Get get, Acc (*red)[BLOCK / 64], qdot_result *out)
{
    s1_pick_nt<BLOCK>(e_max, lo, flags, lut, get, red, out);
}

// value = 2^e_max (D + 2^(c32 - e_max) (S + H)), parts, overflow flag;
// returns the FP64 sum D + 2^(c32 - e_max) (S + H) before the scaling.
// mu_single: single-precision inputs, whose D holds the bins kept at the
// input precision (SINGLE_IN); they are reported in part[SINGLE].
__device__ __forceinline__ double combine_value(const Acc f[3], int e_max, int c32, int flags,
                                                qdot_result *out, int mu_single = 0)
{
    // FP32-class sums are in units of 2^c32, the total in units of 2^e_max
    const int sh = c32 - e_max;
    Acc tot = f[0];
    acc_add(tot, ldexp(f[1].s, sh));
    acc_add(tot, ldexp(f[2].s, sh));
    tot.c = tot.c + ldexp(f[1].c + f[2].c, sh);
    const double S = tot.s + tot.c;
    const double value = ldexp(S, e_max);
    out->value = value;
    const double pd = ldexp(f[0].s + f[0].c, e_max);
    const double ps = ldexp(f[1].s + f[1].c, c32);
    out->part[QDOT_DOUBLE] = mu_single ? 0.0 : pd;
    out->part[QDOT_SINGLE] = mu_single ? ps + pd : ps;
    out->part[QDOT_HALF] = ldexp(f[2].s + f[2].c, c32);
    out->flags = flags | (__builtin_isinf(value) ? QDOT_F_OVERFLOW : 0);
    return S;
}

}  // namespace qd
