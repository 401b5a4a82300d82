// qdot kernels for gfx950: exponent scan, cutoff selection, fused
// quantize-and-accumulate (two passes over x, y), the one-pass scan with
// per-bin candidate sums and its final pick (accum_mode 1), and the plain
// FP64 dot used as the baseline.
//
// Data layout: x and y are FP64 vectors read in groups of 4 consecutive
// elements per lane (two 16-byte loads per operand when both are 16-byte
// aligned).  A block of 256 lanes covers 1024 consecutive elements per
// group; a wave covers 256, i.e. four 64-element FP32 accumulation tiles,
// one per 16-lane DPP row.  Both passes use the same block -> chunk
// mapping, so on inputs that fit in L2 / Infinity Cache the second pass
// re-reads what the same XCD fetched in the first.
#include "qdot_kernels.hpp"

#include "qdot_blocks.hpp"

namespace qd {

// ---------------------------------------------------------------------------
// Pass 1 (Alg. 2, exponent preprocessing + counting): product exponents into
// a block-private LDS histogram, merged into one of `copies` (<= HIST_COPIES)
// global histograms (blockIdx % copies; 8: one per XCD under round-robin
// dispatch) so that the merge atomics of concurrent blocks spread out.
// TS (tile_skip): also the largest key slot of the non-zero products of
// every 64-component tile (-1: none) into tk[i / TILE]; a tile is the 4
// components of each of 16 consecutive lanes, one DPP row.
// ---------------------------------------------------------------------------
template <class T, bool VEC, int U, int NT = BLOCK, bool TS = false>
__global__ __launch_bounds__(NT) void k_scan(const T *__restrict__ x,
                                             const T *__restrict__ y,
                                             int64_t n, int key_mode,
                                             Ws *__restrict__ ws, int copies,
                                             short *__restrict__ tk)
{
    __shared__ unsigned int h[W + 1];
    for (int i = threadIdx.x; i < W + 1; i += NT) h[i] = 0;
    __syncthreads();

    unsigned int nz = 0, bad = 0, sg = 0;
    // float inputs: the 32-bit decomposition gives the key of the same values
    stream_groups<VEC, U, NT>(x, y, n, [&](const T *xv, const T *yv, int64_t i0, int lim) {
        int top = -1;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const auto c = [&]() {
                if constexpr (sizeof(T) == 4) return component_f(xv[e], yv[e], key_mode);
                else return component(xv[e], yv[e], key_mode);
            }();
            const bool valid = e < lim;
            nz += (valid & c.zero) ? 1u : 0u;
            bad |= (valid & c.bad) ? 1u : 0u;
            sg |= (valid & !c.zero) ? (c.sgn ? 1u : 2u) : 0u;
            // zero and non-finite products land in the spare slot W
            if (valid) atomicAdd(&h[c.slot], 1u);
            if (TS && valid && c.slot != ZERO_SLOT) top = max(top, c.slot);
        }
        if constexpr (TS) {
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) top = max(top, __shfl_xor(top, m, 64));
            if ((threadIdx.x & 15) == 0 && i0 < n) tk[i0 / TILE] = (short)top;
        }
    });
    __syncthreads();
    scan_flush<NT>(h, nz, bad, sg, ws, blockIdx.x, copies);
}

// ---------------------------------------------------------------------------
// Cutoff selection (Alg. 2, bins -> scores -> precisions), one workgroup over
// the live slot window of the 8 histogram copies.
// ---------------------------------------------------------------------------
// BINS: bin_mode / bin_param select the partition (exact bins when 0; the
// other strategies need the block's BinLds, so only kernels that admit them
// instantiate this).  pre(lo, hi) runs in every thread once the live slot
// window is known, before the counts are read (a caller issues loads there
// that the selection does not need, so that both wait together); a non-null
// lut_mirror (LDS) receives the class table as well.
struct NoPre {
    __device__ void operator()(int, int) const {}
};
template <bool BINS = false, int NT = CUT_THREADS, class Pre = NoPre>
__device__ __forceinline__ CutParams cut_body(Ws *__restrict__ ws, double tol, int score_mode,
                                              int nonstrict, int64_t n, int nscan, int guard,
                                              int mu_single, qdot_result *__restrict__ out,
                                              long long *__restrict__ hist_out,
                                              int bin_mode = 0, int bin_param = 0,
                                              int want_keep_lo = 0, Pre &&pre = Pre(),
                                              unsigned char *lut_mirror = nullptr)
{
    constexpr int NW = NT / 64;
    __shared__ int s_lo[NW], s_hi[NW], s_kl[NW];
    __shared__ unsigned int s_sg[NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // only the slot window pass 1 touched holds counts; slots outside it are
    // zero in every copy and their class-table entries are never read
    int lo = W, hi = -1;
    unsigned int sg = 0;
    const unsigned long long nzero = ws->n_zero;
    const unsigned int bad = ws->nonfinite;
    {
        int a = W, b = -1;
        unsigned int g = 0;
        for (int i = tid; i < nscan; i += NT) {
            const int2 r = ws->block_range[i];
            a = min(a, r.x);
            b = max(b, r.y);
            if (guard) g |= ws->block_signs[i];
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            a = min(a, __shfl_xor(a, m, 64));
            b = max(b, __shfl_xor(b, m, 64));
            g |= __shfl_xor(g, m, 64);
        }
        if (lane == 0) {
            s_lo[wv] = a;
            s_hi[wv] = b;
            s_sg[wv] = g;
        }
        __syncthreads();
        for (int w = 0; w < NW; w++) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
            sg |= s_sg[w];
        }
    }
    pre(lo, hi);
    auto get = [&](int j) {
        unsigned long long v = 0ull;
#pragma unroll
        for (int c = 0; c < HIST_COPIES; c++) v += ws->hist[c][j];
        return v;
    };
    // keep_lo: the lowest slot this thread gave a kept class
    int keep_lo = W;
    auto put = [&](int j, int cls) {
        ws->lut[j] = (unsigned char)cls;
        if (lut_mirror) lut_mirror[j] = (unsigned char)cls;
        if (cls != QDOT_PERF) keep_lo = min(keep_lo, j);
    };
    auto clear = [&](int j) {
#pragma unroll
        for (int c = 0; c < HIST_COPIES; c++) ws->hist[c][j] = 0ull;
    };
    CutParams p;
    if constexpr (BINS) {
        __shared__ BinLds B;
        if (bin_mode != 0)
            p = block_cutoff_bins<NT>(B, lo, hi, nzero, bad, n, tol, score_mode,
                                               nonstrict, bin_mode, bin_param, get, put, clear,
                                               out, hist_out, mu_single);
        else
            p = block_cutoff<NT>(lo, hi, nzero, bad, n, tol, score_mode, nonstrict,
                                          get, put, clear, out, hist_out, 0, mu_single);
    } else {
        p = block_cutoff<NT>(lo, hi, nzero, bad, n, tol, score_mode, nonstrict, get,
                                      put, clear, out, hist_out, 0, mu_single);
    }
    if (tid < W_LUT - W) ws->lut[W + tid] = (unsigned char)QDOT_PERF;
    if (want_keep_lo) {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) keep_lo = min(keep_lo, __shfl_xor(keep_lo, m, 64));
        if (lane == 0) s_kl[wv] = keep_lo;
        __syncthreads();
        if (tid == 0) {
            int kl = W;
            for (int w = 0; w < NW; w++) kl = min(kl, s_kl[w]);
            ws->keep_lo = kl;
        }
    }
    if (tid == 0) {
        ws->n_zero = 0;
        ws->nonfinite = 0;
        ws->e_max = p.e_max;
        ws->t = p.t;
        ws->c32 = p.c32;
        ws->flags = p.flags;
        ws->skip = p.skip;
        ws->s1_lo = lo;
        ws->s1_hi = hi;
        ws->signs = sg;
        ws->mu_single = mu_single;
    }
    return p;
}

__global__ __launch_bounds__(CUT_THREADS) void k_cut(Ws *__restrict__ ws, double tol,
                                                     int score_mode, int nonstrict,
                                                     int64_t n, int nscan, int guard,
                                                     int mu_single,
                                                     qdot_result *__restrict__ out,
                                                     long long *__restrict__ hist_out,
                                                     int want_keep_lo)
{
    cut_body(ws, tol, score_mode, nonstrict, n, nscan, guard, mu_single, out, hist_out, 0, 0,
             want_keep_lo);
}

// k_cut with a binning strategy other than exact bins (Sec. 3.2)
__global__ __launch_bounds__(CUT_THREADS) void k_cut_bins(Ws *__restrict__ ws, double tol,
                                                          int score_mode, int nonstrict,
                                                          int64_t n, int nscan, int mu_single,
                                                          qdot_result *__restrict__ out,
                                                          long long *__restrict__ hist_out,
                                                          int bin_mode, int bin_param,
                                                          int want_keep_lo)
{
    cut_body<true, CUT_THREADS>(ws, tol, score_mode, nonstrict, n, nscan, 0, mu_single, out,
                                hist_out, bin_mode, bin_param, want_keep_lo);
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
// Block `blk` of `nblk` (grid-stride over groups) writes its partials at
// partials + 6 * blk.
// Q: the compacting form of the leaf work (acc_group_q), else acc_group.
// TS (tile_skip, dense form): tiles whose key in tk lies below the lowest
// kept slot are not read (stream_strided_ts).
template <class T, bool VEC, int U, bool CLS, bool Q = false, int NT = BLOCK, bool TS = false>
__device__ __forceinline__ void acc_body(const T *__restrict__ x, const T *__restrict__ y,
                                         int64_t n, int key_mode, const Ws *__restrict__ ws,
                                         double *__restrict__ partials,
                                         unsigned char *__restrict__ cls_out, int blk, int nblk,
                                         const short *__restrict__ tk = nullptr)
{
    static_assert(!(TS && Q), "tile skipping uses the dense form");
    __shared__ unsigned char lut[W_LUT];
    __shared__ Acc red[3][NT / 64];
    __shared__ AccWaveLds wl[Q ? NT / 64 : 1];

    const int skip = ws->skip;
    if (skip && !CLS) return;
    {
        const unsigned int *src = reinterpret_cast<const unsigned int *>(ws->lut);
        unsigned int *dst = reinterpret_cast<unsigned int *>(lut);
        for (int i = threadIdx.x; i < W_LUT / 4; i += NT) dst[i] = src[i];
    }
    const int e_max = ws->e_max;
    const int c32 = ws->c32;
    if (Q) acc_q_begin<NT>(wl);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    Acc aD = {0.0, 0.0}, aS = {0.0, 0.0}, aH = {0.0, 0.0};
    const int64_t group = (int64_t)NT * EPT * U;
    auto body = [&](const T *xv, const T *yv, int64_t i0, int lim) {
        if constexpr (Q)
            acc_group_q<CLS>(xv, yv, lim, lut, key_mode, e_max, c32, !skip, aD, aS, aH,
                             CLS ? cls_out + i0 : nullptr, wl[threadIdx.x >> 6]);
        else
            acc_group<CLS>(xv, yv, lim, lut, key_mode, e_max, c32, !skip, aD, aS, aH,
                           CLS ? cls_out + i0 : nullptr);
    };
    if constexpr (TS) {
        __shared__ short kl[2][NT];
        // a skipped group's components are all perforated
        auto dead = [&](int64_t i0, int lim) {
            if constexpr (CLS)
                for (int e = 0; e < lim; e++) cls_out[i0 + e] = (unsigned char)QDOT_PERF;
        };
        stream_strided_ts<VEC, U, NT>(x, y, (int64_t)blk * group, (int64_t)nblk * group, n, tk,
                                      ws->keep_lo, kl, body, dead);
    } else
        stream_strided<VEC, U, NT>(x, y, (int64_t)blk * group, (int64_t)nblk * group, n, body);
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
        double *p = partials + (size_t)blk * 6;
        for (int q = 0; q < 3; q++) {
            Acc b = red[q][0];
            for (int w = 1; w < NT / 64; w++) b = acc_merge(b, red[q][w]);
            p[2 * q] = b.s;
            p[2 * q + 1] = b.c;
        }
    }
}

template <class T, bool VEC, int U, bool CLS, bool Q, int NT = BLOCK, bool TS = false>
__global__ __launch_bounds__(NT) void k_acc(const T *__restrict__ x,
                                            const T *__restrict__ y,
                                            int64_t n, int key_mode,
                                            const Ws *__restrict__ ws,
                                            double *__restrict__ partials,
                                            unsigned char *__restrict__ cls_out,
                                            const short *__restrict__ tk)
{
    acc_body<T, VEC, U, CLS, Q, NT, TS>(x, y, n, key_mode, ws, partials, cls_out, blockIdx.x,
                                        gridDim.x, tk);
}

// Combine the per-block partials of k_acc in a fixed order (one block).
__device__ __forceinline__ void fin_body(Ws *__restrict__ ws,
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
        ws->s_last = combine_value(f, ws->e_max, ws->c32, ws->flags, out, ws->mu_single);
    }
}

__global__ __launch_bounds__(BLOCK) void k_fin(Ws *__restrict__ ws,
                                               const double *__restrict__ partials, int nblk,
                                               qdot_result *__restrict__ out)
{
    fin_body(ws, partials, nblk, out);
}

// ---------------------------------------------------------------------------
// Guaranteed mode (guard_mode 1, Thm 3.4): the lower bound L of |x.y| and
// the certification test are those of guard_sums / guard_lower.
// Stage 0 (after the first sweep): certify, or reselect against E_lo (or
// make every bin double when L <= 0) so that the second sweep of k_acc and
// k_fin runs.  Stage 1 (after the second sweep; returns unless it ran):
// check again with the larger of the two lower bounds.
// One workgroup of CUT_THREADS threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CUT_THREADS) void k_guard(Ws *__restrict__ ws,
                                                       const long long *__restrict__ hs,
                                                       double tol, int score_mode, int nonstrict,
                                                       int64_t n, int stage, int mu_single,
                                                       qdot_result *__restrict__ out)
{
    __shared__ int s_go, s_dref, s_passes;
    __shared__ unsigned long long s_nz;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int go;
        if (stage == 0) {
            ws->g_redo = 0;
            go = out->status == QDOT_OK && out->n_bins > 0;
            // every product zero: +0 is exact
            if (out->status == QDOT_OK && out->n_bins == 0) out->flags |= QDOT_F_GUARANTEED;
        } else {
            go = ws->g_redo;
        }
        s_go = go;
        s_dref = 0;
        s_passes = out->passes;
        s_nz = (unsigned long long)out->n_zero;
    }
    __syncthreads();
    if (!s_go) return;
    const int e_max = out->e_max;
    const int lo = ws->s1_lo, hi = ws->s1_hi;
    const GuardSums g =
        guard_sums<CUT_THREADS>([&](int j) { return hs[j]; }, ws->lut, lo, hi, e_max);
    if (tid == 0) {
        const double S = ws->skip ? 0.0 : ws->s_last;
        double low = guard_lower(g, S, n, ws->signs);
        if (stage == 0) {
            if (guard_certified(out->bound_rel, low, tol)) {
                out->flags |= QDOT_F_GUARANTEED;
                out->lower = ldexp(low, e_max);
                ws->skip = 1;
            } else {
                // L <= 0: every bin at the input precision (scores >= 23 for
                // double inputs, >= 10 for single; one more non-strict)
                const int ref = low > 0.0 ? e_max + ilogb(low)
                                          : out->e_min - out->t - (mu_single ? 9 : 22) - nonstrict;
                if (ref < e_max) {
                    s_dref = e_max - ref;
                    ws->g_low = low;
                    ws->g_redo = 1;
                } else {
                    out->lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
                    ws->skip = 1;
                }
            }
        } else {
            low = fmax(low, ws->g_low);
            out->flags |= QDOT_F_RESELECTED |
                          (guard_certified(out->bound_rel, low, tol) ? QDOT_F_GUARANTEED : 0);
            out->lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
        }
    }
    __syncthreads();
    if (s_dref == 0) return;
    // stage 0 reselection: scores against e_ref = e_max - dref
    auto get = [&](int j) { return (unsigned long long)hs[j]; };
    auto put = [&](int j, int cls) { ws->lut[j] = (unsigned char)cls; };
    auto clear = [](int) {};
    const CutParams p = block_cutoff<CUT_THREADS>(lo, hi, s_nz, 0u, n, tol, score_mode, nonstrict,
                                                  get, put, clear, out, nullptr, s_dref,
                                                  mu_single);
    if (tid == 0) {
        ws->c32 = p.c32;
        ws->flags = p.flags | QDOT_F_RESELECTED;
        ws->skip = p.skip;
        out->flags |= QDOT_F_RESELECTED;
        out->passes = s_passes + (p.skip ? 0 : 1);
    }
}

// ---------------------------------------------------------------------------
// One-pass mode (exact per-bin accumulation): the scan that also forms, per
// bin, the candidate sums of every precision, so the data is read once.
//
// A component of bin k can be kept only if its score is >= 0, i.e. if
// e_max - k <= ceil(log2 M_k) - t + 1; the host passes `depth`, a bound of
// that over every histogram n components can give, and admits the mode only
// when depth <= S1_WIN.  The block's own running maximum key `top` never
// exceeds e_max, so the bins below top - depth + 1 are perforated whatever
// the rest of the data holds, and the `depth` bins under `top` (slot = bin
// mod S1_WIN) are all a block has to keep.  `top` is block-uniform: each group's new maximum is agreed
// at a barrier (two alternating LDS words, so one barrier per group
// suffices), and when it rises the slots of the entering bins are cleared
// before anyone adds to them.  The candidate pieces are exact in any order
// (s1_pieces), so LDS and global atomic adds give the same sums every run.
// At the end each block adds its window into one of `copies` global
// tables; k_s1_cutfin selects the cutoff, picks each kept bin's class and
// clears the tables.
// ---------------------------------------------------------------------------
template <class T, bool VEC, int U>
__global__ __launch_bounds__(BLOCK) void k_s1_scan(const T *__restrict__ x,
                                                   const T *__restrict__ y,
                                                   int64_t n, int key_mode, int depth,
                                                   Ws *__restrict__ ws,
                                                   double *__restrict__ tab, int copies)
{
    __shared__ unsigned int h[W + 1];
    __shared__ S1Lds S;
    __shared__ int2 wr[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < W + 1; i += BLOCK) h[i] = 0;
    s1_begin(S);
    __syncthreads();

    S1Run run = s1_run_start();
    unsigned int nz = 0, bad = 0;
    const int64_t group = (int64_t)CHUNK * U;
    s1_stream<VEC, U>(x, y, (int64_t)blockIdx.x * group, (int64_t)gridDim.x * group, n, key_mode,
                      depth, h, S, run, nz, bad);
    const int top = run.top;  // highest live slot seen by the block (-1: none)
    __syncthreads();

    // histogram merge and live range, as in k_scan
    unsigned long long *gh = ws->hist[blockIdx.x % copies];
    int lo = W, hi = -1;
    for (int i = tid; i < W; i += BLOCK) {
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
    if (lane == 0) {
        if (nz) atomicAdd(&ws->n_zero, (unsigned long long)nz);
        if (bad) atomicOr(&ws->nonfinite, 1u);
        wr[tid >> 6] = make_int2(lo, hi);
    }
    // window -> global table (bins top .. top - depth + 1, non-zero sums)
    if (top >= 0) {
        double *tb = tab + (size_t)(blockIdx.x % copies) * W * S1_PIECES;
        for (int i = tid; i < depth * S1_PIECES; i += BLOCK) {
            const int bin = top - i / S1_PIECES;
            if (bin < 0) continue;
            const double v = S.win[bin & (S1_WIN - 1)][i % S1_PIECES];
            if (v != 0.0) atomicAdd(&tb[(size_t)bin * S1_PIECES + i % S1_PIECES], v);
        }
    }
    __syncthreads();
    if (tid == 0) {
        int2 r = wr[0];
        for (int w = 1; w < BLOCK / 64; w++) r = make_int2(min(r.x, wr[w].x), max(r.y, wr[w].y));
        ws->block_range[blockIdx.x] = r;
    }
}

// k_s1_scan with a window per wave (s1w_stream; depth <= S1W_WIN): the waves
// of a block meet only once, at the end, where their windows are added into
// the block window that goes to the global table.  Same tables, histogram
// and records as k_s1_scan.
template <class T, bool VEC, int U>
__global__ __launch_bounds__(BLOCK) void k_s1_scan_w(const T *__restrict__ x,
                                                     const T *__restrict__ y,
                                                     int64_t n, int key_mode, int depth,
                                                     Ws *__restrict__ ws,
                                                     double *__restrict__ tab, int copies)
{
    __shared__ unsigned int h[W + 1];
    __shared__ S1WLds S;
    __shared__ int2 wr[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < W + 1; i += BLOCK) h[i] = 0;
    s1w_begin(S);
    __syncthreads();

    int wtop = -1;
    unsigned int nz = 0, bad = 0;
    const int64_t group = (int64_t)CHUNK * U;
    s1w_stream<VEC, U>(x, y, (int64_t)blockIdx.x * group, (int64_t)gridDim.x * group, n, key_mode,
                       depth, h, S, wtop, nz, bad);
    __syncthreads();
    const int top = s1w_merge(S, wtop, depth);  // highest live slot of the block (-1: none)

    // histogram merge and live range, as in k_scan
    unsigned long long *gh = ws->hist[blockIdx.x % copies];
    int lo = W, hi = -1;
    for (int i = tid; i < W; i += BLOCK) {
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
    if (lane == 0) {
        if (nz) atomicAdd(&ws->n_zero, (unsigned long long)nz);
        if (bad) atomicOr(&ws->nonfinite, 1u);
        wr[tid >> 6] = make_int2(lo, hi);
    }
    // block window -> global table (bins top .. top - depth + 1, non-zero sums)
    if (top >= 0) {
        double *tb = tab + (size_t)(blockIdx.x % copies) * W * S1_PIECES;
        for (int i = tid; i < depth * S1_PIECES; i += BLOCK) {
            const int bin = top - i / S1_PIECES;
            if (bin < 0) continue;
            const double v = S.blk[bin & (S1W_WIN - 1)][i % S1_PIECES];
            if (v != 0.0) atomicAdd(&tb[(size_t)bin * S1_PIECES + i % S1_PIECES], v);
        }
    }
    __syncthreads();
    if (tid == 0) {
        int2 r = wr[0];
        for (int w = 1; w < BLOCK / 64; w++) r = make_int2(min(r.x, wr[w].x), max(r.y, wr[w].y));
        ws->block_range[blockIdx.x] = r;
    }
}

// One-pass mode, cutoff and pick in one workgroup: the cutoff of k_cut, then
// (after a barrier) every kept bin contributes the candidate sum of its
// class, summed over the table copies (exact), scaled by 2^(k - e_max); the
// scaled total is summed with compensation and rounded once.  The block then
// clears the tables over the live range for the next call.  The candidate
// sums of the only bins that can be kept (the depth bins below the top live
// slot, which is e_max's) are loaded as soon as the live window is known,
// so that their loads and the histogram's wait together; the classes come
// from an LDS copy of the class table.
constexpr int S1FIN_THREADS = 512;  // 256 VGPRs per lane: the early loads stay in registers

__global__ __launch_bounds__(S1FIN_THREADS) void k_s1_cutfin(Ws *__restrict__ ws, double tol,
                                                           int score_mode, int nonstrict,
                                                           int64_t n, int nscan, int mu_single,
                                                           double *__restrict__ tab,
                                                           qdot_result *__restrict__ out)
{
    __shared__ Acc red[3][S1FIN_THREADS / 64];
    __shared__ unsigned char cls_l[W_LUT];
    __shared__ double pv[S1_WIN][S1_PIECES];
    // admitted by the host: 1 <= depth <= S1_WIN for a valid tolerance
    const int depth = max(1, min(S1_WIN, s1_depth_dev(n, tol, score_mode)));
    // one (bin, piece) pair per thread is loaded early (depth <= 85 bins);
    // the pairs past S1FIN_THREADS (deeper windows) after the cutoff
    double raw[HIST_COPIES];
    int cnt = 0, blo = W, top = -1;
    auto pre = [&](int lo, int hi) {
        top = hi;
        blo = hi >= lo ? max(lo, hi - depth + 1) : W;
        cnt = hi >= lo ? (hi - blo + 1) * S1_PIECES : 0;
        const int i = (int)threadIdx.x;
        if (i < cnt) {
            const int bin = hi - i / S1_PIECES, q = i % S1_PIECES;
#pragma unroll
            for (int c = 0; c < HIST_COPIES; c++)
                raw[c] = tab[((size_t)c * W + bin) * S1_PIECES + q];
        }
    };
    const CutParams p = cut_body<false, S1FIN_THREADS>(ws, tol, score_mode, nonstrict, n, nscan,
                                                       0, mu_single, out, nullptr, 0, 0, 0, pre,
                                                       cls_l);
    for (int i = threadIdx.x; i < cnt; i += S1FIN_THREADS) {
        double v = 0.0;
        if (i < S1FIN_THREADS) {
#pragma unroll
            for (int c = 0; c < HIST_COPIES; c++) v += raw[c];
        } else {
            const int bin = top - i / S1_PIECES, q = i % S1_PIECES;
            for (int c = 0; c < HIST_COPIES; c++) v += tab[((size_t)c * W + bin) * S1_PIECES + q];
        }
        pv[i / S1_PIECES][i % S1_PIECES] = v;
    }
    __syncthreads();
    const int lo = ws->s1_lo, hi = ws->s1_hi;
    if (!p.skip) {
        // bins below blo are perforated (the mode's admission), so they are
        // never picked; pv holds bin top - j at row j
        auto get = [&](int bin, int q) { return bin >= blo ? pv[top - bin][q] : 0.0; };
        s1_pick_nt<S1FIN_THREADS>(p.e_max, lo, p.flags, cls_l, get, red, out);
    }
    if (hi >= lo) {
        const int64_t cnt = (int64_t)(hi - lo + 1) * S1_PIECES;
        for (int c = 0; c < HIST_COPIES; c++) {
            double *tb = tab + ((size_t)c * W + lo) * S1_PIECES;
            for (int64_t i = threadIdx.x; i < cnt; i += S1FIN_THREADS) tb[i] = 0.0;
        }
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
static int grid_for(int64_t n, int unroll, int cap, int nt = BLOCK)
{
    const int64_t g = (int64_t)nt * EPT * unroll;
    const int64_t groups = (n + g - 1) / g;
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, groups));
}

// Threads per block of the scan and accumulate kernels: the tuned value for
// aligned double inputs (the hot path), BLOCK otherwise.  The grid caps of
// the tune entry count blocks of BLOCK threads, so a block of nt threads
// stands for nt / BLOCK of them.
template <class T, bool VEC>
static int block_threads(const Launch &L)
{
    return (sizeof(T) == 8 && VEC && (L.block_threads == 128 || L.block_threads == 512))
               ? L.block_threads
               : BLOCK;
}

static int cap_for(int cap_blocks, int nt)
{
    return std::max(1, (int)((int64_t)cap_blocks * BLOCK / nt));
}

// Groups in flight per wave: a group of single-precision inputs is half the
// bytes of a double group, so float launches keep twice as many (at most 4).
template <class T>
static int unroll_for(int u)
{
    return sizeof(T) == 4 ? std::min(4, 2 * u) : u;
}

template <class T, bool VEC, int U, int NT>
static int launch_scan_nt(const Launch &L, const T *x, const T *y, int64_t n, int key_mode)
{
    const int grid = grid_for(n, U, std::min(MAX_GRID, cap_for(L.scan_blocks, NT)), NT);
    if (L.tiles)
        hipLaunchKernelGGL((k_scan<T, VEC, U, NT, true>), dim3(grid), dim3(NT), 0, L.stream, x,
                           y, n, key_mode, L.ws, L.hist_copies, L.tiles);
    else
        hipLaunchKernelGGL((k_scan<T, VEC, U, NT>), dim3(grid), dim3(NT), 0, L.stream, x, y, n,
                           key_mode, L.ws, L.hist_copies, nullptr);
    return grid;
}

template <class T, bool VEC, int U>
static int launch_scan_u(const Launch &L, const T *x, const T *y, int64_t n, int key_mode)
{
    if constexpr (sizeof(T) == 8 && VEC) {
        switch (block_threads<T, VEC>(L)) {
        case 128: return launch_scan_nt<T, VEC, U, 128>(L, x, y, n, key_mode);
        case 512: return launch_scan_nt<T, VEC, U, 512>(L, x, y, n, key_mode);
        default: break;
        }
    }
    return launch_scan_nt<T, VEC, U, BLOCK>(L, x, y, n, key_mode);
}

template <class T, bool VEC>
static int launch_scan(const Launch &L, const T *x, const T *y, int64_t n, int key_mode)
{
    switch (unroll_for<T>(L.scan_unroll)) {
    case 1: return launch_scan_u<T, VEC, 1>(L, x, y, n, key_mode);
    case 4: return launch_scan_u<T, VEC, 4>(L, x, y, n, key_mode);
    default: return launch_scan_u<T, VEC, 2>(L, x, y, n, key_mode);
    }
}

template <class T, bool VEC, int U, bool CLS, int NT>
static int launch_acc_nt(const Launch &L, const T *x, const T *y, int64_t n, int key_mode,
                         unsigned char *cls_out)
{
    // the partials hold L.partial_cap blocks of any size
    const int grid = grid_for(n, U, std::min(L.partial_cap, cap_for(L.acc_blocks, NT)), NT);
    // tile keys: the dense form (the compacting form's queue holds the
    // components it reads)
    if (L.tiles)
        hipLaunchKernelGGL((k_acc<T, VEC, U, CLS, false, NT, true>), dim3(grid), dim3(NT), 0,
                           L.stream, x, y, n, key_mode, L.ws, L.partials, cls_out, L.tiles);
    else if (L.acc_form == 1)
        hipLaunchKernelGGL((k_acc<T, VEC, U, CLS, true, NT>), dim3(grid), dim3(NT), 0, L.stream,
                           x, y, n, key_mode, L.ws, L.partials, cls_out, nullptr);
    else
        hipLaunchKernelGGL((k_acc<T, VEC, U, CLS, false, NT>), dim3(grid), dim3(NT), 0,
                           L.stream, x, y, n, key_mode, L.ws, L.partials, cls_out, nullptr);
    return grid;
}

template <class T, bool VEC, int U, bool CLS>
static int launch_acc_u(const Launch &L, const T *x, const T *y, int64_t n, int key_mode,
                        unsigned char *cls_out)
{
    if constexpr (sizeof(T) == 8 && VEC && !CLS) {
        switch (block_threads<T, VEC>(L)) {
        case 128: return launch_acc_nt<T, VEC, U, CLS, 128>(L, x, y, n, key_mode, cls_out);
        case 512: return launch_acc_nt<T, VEC, U, CLS, 512>(L, x, y, n, key_mode, cls_out);
        default: break;
        }
    }
    return launch_acc_nt<T, VEC, U, CLS, BLOCK>(L, x, y, n, key_mode, cls_out);
}

template <class T, bool VEC, bool CLS>
static int launch_acc(const Launch &L, const T *x, const T *y, int64_t n, int key_mode,
                      unsigned char *cls_out)
{
    switch (unroll_for<T>(L.acc_unroll)) {
    case 1: return launch_acc_u<T, VEC, 1, CLS>(L, x, y, n, key_mode, cls_out);
    case 4: return launch_acc_u<T, VEC, 4, CLS>(L, x, y, n, key_mode, cls_out);
    default: return launch_acc_u<T, VEC, 2, CLS>(L, x, y, n, key_mode, cls_out);
    }
}

template <class T, bool VEC, int U>
static int launch_s1_u(const Launch &L, const T *x, const T *y, int64_t n, int key_mode,
                       int depth)
{
    const int grid = grid_for(n, U, L.s1_blocks);
    // single-precision inputs: a window per wave when every possibly kept
    // bin fits in S1W_WIN (a group of floats is half the bytes of a group of
    // doubles, and the block barrier per group costs them 10 %; double
    // inputs measured the same either way at their best shapes)
    if (sizeof(T) == 4 && depth <= S1W_WIN)
        hipLaunchKernelGGL((k_s1_scan_w<T, VEC, U>), dim3(grid), dim3(BLOCK), 0, L.stream, x, y,
                           n, key_mode, depth, L.ws, L.s1tab, L.hist_copies);
    else
        hipLaunchKernelGGL((k_s1_scan<T, VEC, U>), dim3(grid), dim3(BLOCK), 0, L.stream, x, y, n,
                           key_mode, depth, L.ws, L.s1tab, L.hist_copies);
    return grid;
}

template <class T, bool VEC>
static int launch_s1(const Launch &L, const T *x, const T *y, int64_t n, int key_mode,
                     int depth)
{
    switch (unroll_for<T>(L.s1_unroll)) {
    case 1: return launch_s1_u<T, VEC, 1>(L, x, y, n, key_mode, depth);
    case 4: return launch_s1_u<T, VEC, 4>(L, x, y, n, key_mode, depth);
    default: return launch_s1_u<T, VEC, 2>(L, x, y, n, key_mode, depth);
    }
}

// One-pass mode: scan with per-bin candidate sums, cutoff, pick per bin.
template <class T>
static hipError_t launch_qdot_s1(const Launch &L, const T *x, const T *y, int64_t n,
                                 double tol, const qdot_options &o, qdot_result *out)
{
    const bool vec = ((((uintptr_t)x) | ((uintptr_t)y)) & 15) == 0;
    const int mu_single = sizeof(T) == 4 ? 1 : 0;
    hipStream_t s = L.stream;
    if (L.ev) (void)hipEventRecord(L.ev[0], s);
    const int depth = s1_depth(n, tol, o);
    const int nscan = vec ? launch_s1<T, true>(L, x, y, n, o.key_mode, depth)
                          : launch_s1<T, false>(L, x, y, n, o.key_mode, depth);
    if (L.ev) (void)hipEventRecord(L.ev[1], s);
    hipLaunchKernelGGL(k_s1_cutfin, dim3(1), dim3(S1FIN_THREADS), 0, s, L.ws, tol, o.score_mode,
                       o.boundary_mode, n, nscan, mu_single, L.s1tab, out);
    if (L.ev) {
        (void)hipEventRecord(L.ev[2], s);
        (void)hipEventRecord(L.ev[3], s);
        (void)hipEventRecord(L.ev[4], s);
    }
    return hipGetLastError();
}

// Two-pass qdot of T inputs (double, or float with mu = m_single): scan,
// cutoff, accumulate, finalize, and in the guaranteed mode the guard stages
// around a second sweep.
// nscan_pre >= 0: pass 1 already ran into L.ws, in an earlier kernel on the
// stream that left nscan_pre block records; the scan is not launched.
template <class T>
static hipError_t launch_qdot_t(const Launch &L, const T *x, const T *y, int64_t n, double tol,
                                const qdot_options &o, qdot_result *out,
                                unsigned char *cls_out, long long *hist_out,
                                int nscan_pre = -1)
{
    const bool vec = ((((uintptr_t)x) | ((uintptr_t)y)) & 15) == 0;
    const int guard = o.guard_mode;
    const int mu_single = sizeof(T) == 4 ? 1 : 0;
    // the guaranteed mode keeps the histogram for its reselection
    long long *hs = hist_out;
    if (guard && !hs)
        hs = reinterpret_cast<long long *>(reinterpret_cast<char *>(L.ws) + offsetof(Ws, hsave));
    hipStream_t s = L.stream;
    if (L.ev) (void)hipEventRecord(L.ev[0], s);
    const int nscan = nscan_pre >= 0 ? nscan_pre
                      : vec          ? launch_scan<T, true>(L, x, y, n, o.key_mode)
                                     : launch_scan<T, false>(L, x, y, n, o.key_mode);
    if (L.ev) (void)hipEventRecord(L.ev[1], s);
    if (o.bin_mode != 0)
        hipLaunchKernelGGL(k_cut_bins, dim3(1), dim3(CUT_THREADS), 0, s, L.ws, tol,
                           o.score_mode, o.boundary_mode, n, nscan, mu_single, out, hs,
                           o.bin_mode, o.bin_param, L.tiles ? 1 : 0);
    else
        hipLaunchKernelGGL(k_cut, dim3(1), dim3(CUT_THREADS), 0, s, L.ws, tol, o.score_mode,
                           o.boundary_mode, n, nscan, guard, mu_single, out, hs,
                           L.tiles ? 1 : 0);
    if (L.ev) (void)hipEventRecord(L.ev[2], s);
    auto sweep = [&]() {
        int grid;
        if (cls_out)
            grid = vec ? launch_acc<T, true, true>(L, x, y, n, o.key_mode, cls_out)
                       : launch_acc<T, false, true>(L, x, y, n, o.key_mode, cls_out);
        else
            grid = vec ? launch_acc<T, true, false>(L, x, y, n, o.key_mode, nullptr)
                       : launch_acc<T, false, false>(L, x, y, n, o.key_mode, nullptr);
        return grid;
    };
    int grid = sweep();
    if (L.ev) (void)hipEventRecord(L.ev[3], s);
    hipLaunchKernelGGL(k_fin, dim3(1), dim3(BLOCK), 0, s, L.ws, L.partials, grid, out);
    if (guard) {
        // certify or reselect; the second sweep returns at once unless the
        // classes were selected again
        hipLaunchKernelGGL(k_guard, dim3(1), dim3(CUT_THREADS), 0, s, L.ws, hs, tol,
                           o.score_mode, o.boundary_mode, n, 0, mu_single, out);
        grid = sweep();
        hipLaunchKernelGGL(k_fin, dim3(1), dim3(BLOCK), 0, s, L.ws, L.partials, grid, out);
        hipLaunchKernelGGL(k_guard, dim3(1), dim3(CUT_THREADS), 0, s, L.ws, hs, tol,
                           o.score_mode, o.boundary_mode, n, 1, mu_single, out);
    }
    if (L.ev) (void)hipEventRecord(L.ev[4], s);
    return hipGetLastError();
}

hipError_t launch_qdot(const Launch &L, const double *x, const double *y, int64_t n,
                       double tol, const qdot_options &o, qdot_result *out,
                       unsigned char *cls_out, long long *hist_out)
{
    if (o.accum_mode == 1) return launch_qdot_s1<double>(L, x, y, n, tol, o, out);
    return launch_qdot_t<double>(L, x, y, n, tol, o, out, cls_out, hist_out);
}

hipError_t launch_qdot_f32(const Launch &L, const float *x, const float *y, int64_t n,
                           double tol, const qdot_options &o, qdot_result *out,
                           unsigned char *cls_out, long long *hist_out)
{
    if (o.accum_mode == 1) return launch_qdot_s1<float>(L, x, y, n, tol, o, out);
    return launch_qdot_t<float>(L, x, y, n, tol, o, out, cls_out, hist_out);
}

// ---------------------------------------------------------------------------
// Two inner products over the same n components, lambda = x . w and
// c = w . w (the power method's pair, Alg. 5), one launch per step: pass 1
// reads x and w once for the keys of both, and the cutoffs, pass-2 sweeps
// and combines of the two run side by side (block 0 / the first half of the
// grid on x . w into wa, the rest on w . w into wb).
// ---------------------------------------------------------------------------
template <bool VEC, int U>
__global__ __launch_bounds__(BLOCK) void k_scan_pair(const double *__restrict__ x,
                                                     const double *__restrict__ w, int64_t n,
                                                     int key_mode, Ws *__restrict__ wa,
                                                     Ws *__restrict__ wb, int copies)
{
    __shared__ unsigned int h[2 * (W + 1)];
    for (int i = threadIdx.x; i < 2 * (W + 1); i += BLOCK) h[i] = 0;
    __syncthreads();
    unsigned int *ha = h, *hb = h + (W + 1);
    unsigned int nza = 0, bada = 0, sga = 0, nzb = 0, badb = 0, sgb = 0;
    stream_groups<VEC, U>(x, w, n, [&](const double *xv, const double *wv, int64_t, int lim) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const Comp a = component(xv[e], wv[e], key_mode);
            const Comp b = component(wv[e], wv[e], key_mode);
            const bool valid = e < lim;
            nza += (valid & a.zero) ? 1u : 0u;
            bada |= (valid & a.bad) ? 1u : 0u;
            sga |= (valid & !a.zero) ? (a.sgn ? 1u : 2u) : 0u;
            nzb += (valid & b.zero) ? 1u : 0u;
            badb |= (valid & b.bad) ? 1u : 0u;
            sgb |= (valid & !b.zero) ? (b.sgn ? 1u : 2u) : 0u;
            if (valid) {
                atomicAdd(&ha[a.slot], 1u);
                atomicAdd(&hb[b.slot], 1u);
            }
        }
    });
    __syncthreads();
    scan_flush(ha, nza, bada, sga, wa, blockIdx.x, copies);
    scan_flush(hb, nzb, badb, sgb, wb, blockIdx.x, copies);
}

__global__ __launch_bounds__(CUT_THREADS) void k_cut_pair(Ws *__restrict__ wa,
                                                          Ws *__restrict__ wb, double tol,
                                                          int score_mode, int nonstrict,
                                                          int64_t n, int nscan,
                                                          qdot_result *__restrict__ out_a,
                                                          qdot_result *__restrict__ out_b)
{
    if (blockIdx.x == 0)
        cut_body(wa, tol, score_mode, nonstrict, n, nscan, 0, 0, out_a, nullptr);
    else
        cut_body(wb, tol, score_mode, nonstrict, n, nscan, 0, 0, out_b, nullptr);
}

// grid 2 * g: partials of x . w at [0, g), of w . w at [g, 2 g)
template <bool VEC, int U>
__global__ __launch_bounds__(BLOCK) void k_acc_pair(const double *__restrict__ x,
                                                    const double *__restrict__ w, int64_t n,
                                                    int key_mode, const Ws *__restrict__ wa,
                                                    const Ws *__restrict__ wb,
                                                    double *__restrict__ partials, int g)
{
    const int b = blockIdx.x;
    if (b < g)
        acc_body<double, VEC, U, false>(x, w, n, key_mode, wa, partials, nullptr, b, g);
    else
        acc_body<double, VEC, U, false>(w, w, n, key_mode, wb, partials + (size_t)6 * g,
                                        nullptr, b - g, g);
}

__global__ __launch_bounds__(BLOCK) void k_fin_pair(Ws *__restrict__ wa, Ws *__restrict__ wb,
                                                    const double *__restrict__ partials, int g,
                                                    qdot_result *__restrict__ out_a,
                                                    qdot_result *__restrict__ out_b)
{
    if (blockIdx.x == 0)
        fin_body(wa, partials, g, out_a);
    else
        fin_body(wb, partials + (size_t)6 * g, g, out_b);
}

template <bool VEC, int U>
static hipError_t launch_pair_u(const Launch &La, const Launch &Lb, const double *x,
                                const double *w, int64_t n, double tol, const qdot_options &o,
                                qdot_result *out_a, qdot_result *out_b, int nscan_pre)
{
    hipStream_t s = La.stream;
    int nscan = nscan_pre;
    if (nscan < 0) {
        nscan = grid_for(n, U, La.scan_blocks);
        hipLaunchKernelGGL((k_scan_pair<VEC, U>), dim3(nscan), dim3(BLOCK), 0, s, x, w, n,
                           o.key_mode, La.ws, Lb.ws, La.hist_copies);
    }
    if (o.guard_mode) {
        // the guard stages run per product, after the shared pass 1
        hipError_t e = launch_qdot_t<double>(La, x, w, n, tol, o, out_a, nullptr, nullptr, nscan);
        if (e == hipSuccess)
            e = launch_qdot_t<double>(Lb, w, w, n, tol, o, out_b, nullptr, nullptr, nscan);
        return e;
    }
    hipLaunchKernelGGL(k_cut_pair, dim3(2), dim3(CUT_THREADS), 0, s, La.ws, Lb.ws, tol,
                       o.score_mode, o.boundary_mode, n, nscan, out_a, out_b);
    const int g = std::min(grid_for(n, U, La.acc_blocks), La.partial_cap / 2);
    hipLaunchKernelGGL((k_acc_pair<VEC, U>), dim3(2 * g), dim3(BLOCK), 0, s, x, w, n,
                       o.key_mode, La.ws, Lb.ws, La.partials, g);
    hipLaunchKernelGGL(k_fin_pair, dim3(2), dim3(BLOCK), 0, s, La.ws, Lb.ws, La.partials, g,
                       out_a, out_b);
    return hipGetLastError();
}

template <bool VEC>
static hipError_t launch_pair_v(const Launch &La, const Launch &Lb, const double *x,
                                const double *w, int64_t n, double tol, const qdot_options &o,
                                qdot_result *out_a, qdot_result *out_b, int nscan_pre)
{
    // one unroll for both passes: the pass-1 kernel reads two operands per
    // key pair, like pass 2
    switch (unroll_for<double>(La.acc_unroll)) {
    case 1: return launch_pair_u<VEC, 1>(La, Lb, x, w, n, tol, o, out_a, out_b, nscan_pre);
    case 4: return launch_pair_u<VEC, 4>(La, Lb, x, w, n, tol, o, out_a, out_b, nscan_pre);
    default: return launch_pair_u<VEC, 2>(La, Lb, x, w, n, tol, o, out_a, out_b, nscan_pre);
    }
}

hipError_t launch_qdot_pair(const Launch &La, const Launch &Lb, const double *x,
                            const double *w, int64_t n, double tol, const qdot_options &o,
                            qdot_result *out_a, qdot_result *out_b, int nscan_pre)
{
    const bool vec = ((((uintptr_t)x) | ((uintptr_t)w)) & 15) == 0;
    return vec ? launch_pair_v<true>(La, Lb, x, w, n, tol, o, out_a, out_b, nscan_pre)
               : launch_pair_v<false>(La, Lb, x, w, n, tol, o, out_a, out_b, nscan_pre);
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
