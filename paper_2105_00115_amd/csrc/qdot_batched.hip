// Batched ragged qdot: B independent instances in one persistent launch.
//
// The host plans a work queue once per offsets layout:
//   P1    pass-1 chunks of the large instances: an instance of n components
//         has nc = ceil(n / chunk) chunks, chunk c taking the GROUP-sized
//         component groups c, c + nc, c + 2 nc, ... so that the blocks on
//         one instance read neighbouring addresses at any moment,
//   SMALL runs of whole small instances (n <= chunk each), grouped so
//         that sum(n + SMALL_COST0) stays within SMALL_GROUP per item (the
//         fixed term stands for the latency chain of one instance), each
//         instance done start to finish by one block with a block-local
//         cutoff,
//   P2    pass-2 chunks of the large instances,
// in that order.  Blocks take items from a global ticket.  The block that
// finishes the last P1 chunk of a large instance runs that instance's cutoff
// and publishes its class table with release semantics; P2 chunks acquire
// that flag before they start (a wait past the spin limit gives up and
// marks the instance QDOT_E_DEVICE).  Every P1 item is dequeued before any P2
// item and a P1 item never waits, so a waiting block only ever waits for
// work that a running block holds: the launch cannot deadlock, whatever the
// number of resident blocks.  The block that finishes the last P2 chunk of
// an instance combines its partials in chunk order and resets the
// instance's counters, so the next call needs no clearing pass: the launch
// performs no allocation and no memset and can be captured in a HIP graph.
//
// Each instance's 64-element FP32 tiles start at its own first component;
// groups are multiples of 1024 components, so tiles never straddle chunks.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "qdot_blocks.hpp"
#include "qdot_cg.hpp"
#include "qdot_handle.hpp"

namespace qd {

// Components per P1 / P2 chunk, and the largest instance one block takes
// whole (SMALL), is the handle's batch_chunk (default 131072).
constexpr int64_t SMALL_COST0 = 8192; // fixed cost of one small instance, in components
constexpr int64_t SMALL_GROUP = 65536; // cost budget of one item of small instances
constexpr int SU = 2;                 // CHUNK groups in flight per thread
constexpr int64_t GROUP = (int64_t)SU * CHUNK;
constexpr int MAX_PLANS = 8;
// A CG system of n rows gets a gang of ceil(n / batch_cg_rows) blocks, at
// most batch_cg_gang_max (handle fields; defaults 16384 and 16).

enum : int { IT_P1 = 0, IT_SMALL = 1, IT_P2 = 2, IT_CG = 3 };

struct BItem {
    int type;
    int inst;   // P1 / P2: instance; SMALL: first entry in the small list; CG: system
    int large;  // P1 / P2: compact index of the large instance; SMALL: count; CG: gang size
    int slot;   // P2: partial slot; CG: block's place in the gang
    int64_t first, stride;  // P1 / P2: the chunk's groups (see stream_strided)
};

struct BLarge {
    unsigned int p1_done, p2_done, ready, nchunks;
    int lo, hi;
    unsigned long long n_zero;
    unsigned int bad;
    int first_slot;
    int e_max, c32, skip, flags;
    unsigned int signs;  // guard_mode 1: OR of the chunks' sign bits
};

struct BState {
    unsigned int next;
    unsigned int exited;
};

struct BatchPlan {
    std::vector<int64_t> offsets;
    std::vector<qdot_cg_system> systems;
    int B = 0, S = 0, accum = 0, n_items = 0, n_large = 0, n_p2 = 0, max_gang = 0;
    double *ltab = nullptr;           // one-pass mode: per large instance W x S1_PIECES sums
    CgSys *sys = nullptr;             // S device descriptors
    Gang *gangs = nullptr;            // S gang states
    double *cgvec = nullptr;          // r, p, q of every system
    qdot_cg_result *cgres = nullptr;  // S results (synchronous CG entry)
    BItem *items = nullptr;
    BLarge *large = nullptr;
    unsigned int *hist = nullptr;
    unsigned char *lut = nullptr;
    double *partials = nullptr;
    BState *state = nullptr;
    int *small_list = nullptr;
    uint64_t last_use = 0;
};

void free_plan(BatchPlan *p)
{
    if (!p) return;
    (void)hipFree(p->items);
    (void)hipFree(p->large);
    (void)hipFree(p->hist);
    (void)hipFree(p->lut);
    (void)hipFree(p->partials);
    (void)hipFree(p->state);
    (void)hipFree(p->small_list);
    (void)hipFree(p->sys);
    (void)hipFree(p->gangs);
    (void)hipFree(p->cgvec);
    (void)hipFree(p->cgres);
    (void)hipFree(p->ltab);
    delete p;
}

// Pass 1 over the groups first, first + stride, ... (below n) of one
// instance into the LDS histogram h; sg collects bit 0 for a negative and
// bit 1 for a positive non-zero product (the guaranteed mode's sign test).
__device__ __forceinline__ void scan_into(const double *xi, const double *yi, int64_t first,
                                          int64_t stride, int64_t n, bool vec, int key_mode, unsigned int *h,
                                          unsigned int &nz, unsigned int &bad, unsigned int &sg)
{
    auto body = [&](const double *xv, const double *yv, int64_t, int lim) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const Comp c = component(xv[k], yv[k], key_mode);
            const bool valid = k < lim;
            nz += (valid & c.zero) ? 1u : 0u;
            bad |= (valid & c.bad) ? 1u : 0u;
            sg |= (valid & !c.zero) ? (c.sgn ? 1u : 2u) : 0u;
            if (valid) atomicAdd(&h[c.slot], 1u);
        }
    };
    if (vec)
        stream_strided<true, SU>(xi, yi, first, stride, n, body);
    else
        stream_strided<false, SU>(xi, yi, first, stride, n, body);
}

__device__ __forceinline__ void accumulate_range(const double *xi, const double *yi,
                                                 int64_t first, int64_t stride, int64_t n,
                                                 bool vec, int key_mode,
                                                 const unsigned char *lut, int e_max, int c32,
                                                 Acc a[3])
{
    auto body = [&](const double *xv, const double *yv, int64_t, int lim) {
        acc_group<false>(xv, yv, lim, lut, key_mode, e_max, c32, true, a[0], a[1], a[2], nullptr);
    };
    if (vec)
        stream_strided<true, SU>(xi, yi, first, stride, n, body);
    else
        stream_strided<false, SU>(xi, yi, first, stride, n, body);
}

// One-pass mode: window depth of an instance, or -1 when its kept bins
// could lie beyond the window (or n is past the exact-sum bound).  An
// invalid tolerance gets depth 1: the cutoff then reports it.
// Window depth of a one-pass instance, or -1 when the mode is refused
// (kept bins could lie beyond the window).  A depth below 1 means that no
// bin can be kept (a tolerance large enough to perforate everything): the
// window then holds the top bin alone, whose class is perforated.
__device__ __forceinline__ int s1_window_depth(int64_t n, double tol, int score_mode)
{
    if (!(tol > 0.0) || __builtin_isinf(tol)) return 1;
    const int d = s1_depth_dev(n, tol, score_mode);
    return (n > S1_MAX_N || d > S1_WIN) ? -1 : max(d, 1);
}

// guard_mode 1 (Thm 3.4) for one instance that one block finishes: the
// steps and flags of the single-vector guard stages.  R holds the result of
// the selection and of the first sweep, S that sweep's sum (units of
// 2^e_max; 0 when nothing was swept), get(j) the instance's counts over
// [lo, hi], nz its zero count and sg its sign bits.  Certify, or select the
// classes again against the certified exponent (put() writes them into the
// block's class table lut) and let resweep(p, flags) sum the instance again
// with them, returning (in thread 0) the new sum while it writes value,
// parts and flags into R; then check again with the larger lower bound.
// Every thread of the block must call it.
template <class Get, class Put, class Sweep>
__device__ void batch_guard(int lo, int hi, unsigned long long nz, unsigned int sg, int64_t n,
                            double tol, int score_mode, int nonstrict, Get get, Put put,
                            const unsigned char *lut, double S, qdot_result &R, Sweep &&resweep)
{
    __shared__ int s_go, s_dref, s_passes;
    __shared__ double s_low, s_sum;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_go = R.status == QDOT_OK && R.n_bins > 0;
        // every product zero: +0 is exact
        if (R.status == QDOT_OK && R.n_bins == 0) R.flags |= QDOT_F_GUARANTEED;
        s_dref = 0;
        s_passes = R.passes;
    }
    __syncthreads();
    if (!s_go) return;
    const int e_max = R.e_max;
    const GuardSums g0 = guard_sums<BLOCK>(get, lut, lo, hi, e_max);
    if (tid == 0) {
        const double low = guard_lower(g0, S, n, sg);
        if (guard_certified(R.bound_rel, low, tol)) {
            R.flags |= QDOT_F_GUARANTEED;
            R.lower = ldexp(low, e_max);
        } else {
            // L <= 0: every bin double (scores >= 23, one more non-strict)
            const int ref = low > 0.0 ? e_max + ilogb(low) : R.e_min - R.t - 22 - nonstrict;
            if (ref < e_max) {
                s_dref = e_max - ref;
                s_low = low;
            } else {
                R.lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
            }
        }
    }
    __syncthreads();
    if (!s_dref) return;
    auto noclear = [](int) {};
    const CutParams p2 = block_cutoff<BLOCK>(lo, hi, nz, 0u, n, tol, score_mode, nonstrict, get,
                                             put, noclear, &R, nullptr, s_dref);
    if (tid == 0) {
        R.flags |= QDOT_F_RESELECTED;
        R.passes = s_passes + (p2.skip ? 0 : 1);
        s_sum = 0.0;
    }
    __syncthreads();
    if (!p2.skip) {
        const double s2 = resweep(p2, p2.flags | QDOT_F_RESELECTED);
        if (tid == 0) s_sum = s2;
    }
    __syncthreads();
    const GuardSums g1 = guard_sums<BLOCK>(get, lut, lo, hi, e_max);
    if (tid == 0) {
        const double low = fmax(guard_lower(g1, s_sum, n, sg), s_low);
        R.flags |= QDOT_F_RESELECTED |
                   (guard_certified(R.bound_rel, low, tol) ? QDOT_F_GUARANTEED : 0);
        R.lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
    }
    __syncthreads();
}

// Copies a block's result (LDS) to its slot in device memory (every thread
// calls it).
__device__ __forceinline__ void put_result(qdot_result *o, const qdot_result &R)
{
    constexpr int NWORD = (int)(sizeof(qdot_result) / sizeof(unsigned long long));
    static_assert(NWORD * sizeof(unsigned long long) == sizeof(qdot_result), "whole words");
    if (threadIdx.x < NWORD)
        reinterpret_cast<unsigned long long *>(o)[threadIdx.x] =
            reinterpret_cast<const unsigned long long *>(&R)[threadIdx.x];
}

__device__ __forceinline__ void write_invalid(qdot_result *o)
{
    o->value = __longlong_as_double(0x7ff8000000000000ll);
    for (int q = 0; q < 4; q++) o->count[q] = 0;
    o->n_zero = 0;
    o->e_min = o->e_max = o->n_bins = o->t = 0;
    for (int q = 0; q < 3; q++) o->part[q] = 0.0;
    o->bound_rel = o->bound_abs = 0.0;
    o->flags = 0;
    o->status = QDOT_E_INVAL;
    o->lower = 0.0;
    o->e_ref = 0;
    o->passes = 0;
}

// One-pass chunk of a large instance: scan with the block's candidate-sum
// window, merge the histogram and add the window into the instance's bin
// table (device-scope atomics; the sums are exact in any order), then count
// the chunk.  The last chunk selects the cutoff, picks each kept bin's class
// sum from the table, writes the whole result, and clears the table and the
// instance's counters for the next launch.
template <class Red>
__device__ __forceinline__ void p1_onepass(const double *xi, const double *yi, int64_t n,
                                           double tol, bool vec, const BItem &I, BLarge *L,
                                           unsigned int *gh, double *tb, qdot_result *o,
                                           unsigned int *h, unsigned char *lut, Red &red,
                                           int4 *scratch, qdot_result &s_res, S1Lds &S1,
                                           int &s_flag, int key_mode, int score_mode,
                                           int nonstrict)
{
    const int tid = threadIdx.x;
    const int depth = s1_window_depth(n, tol, score_mode);
    const int dw = depth < 0 ? 0 : depth;  // no window when the mode is refused
    unsigned int nz = 0, bad = 0;
    S1Run run = s1_run_start();
    s1_begin(S1);
    __syncthreads();
    if (vec)
        s1_stream<true, SU>(xi, yi, I.first, I.stride, n, key_mode, dw, h, S1, run, nz, bad);
    else
        s1_stream<false, SU>(xi, yi, I.first, I.stride, n, key_mode, dw, h, S1, run, nz, bad);
    const int top = run.top;
    __syncthreads();
    int lo = W, hi = -1;
    for (int j = tid; j < W; j += BLOCK) {
        const unsigned int v = h[j];
        if (v) {
            __hip_atomic_fetch_add(&gh[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            h[j] = 0u;
            lo = min(lo, j);
            hi = max(hi, j);
        }
    }
    if (tid == 0) h[W] = 0u;
    if (top >= 0)
        for (int i = tid; i < dw * S1_PIECES; i += BLOCK) {
            const int bin = top - i / S1_PIECES;
            if (bin < 0) continue;
            const double v = S1.win[bin & (S1_WIN - 1)][i % S1_PIECES];
            if (v != 0.0)
                __hip_atomic_fetch_add(&tb[(size_t)bin * S1_PIECES + i % S1_PIECES], v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    block_reduce_range(lo, hi, nz, bad, scratch);
    if (tid == 0) {
        if (hi >= 0) {
            __hip_atomic_fetch_min(&L->lo, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(&L->hi, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (nz)
            __hip_atomic_fetch_add(&L->n_zero, (unsigned long long)nz, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (bad) __hip_atomic_fetch_or(&L->bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the chunk's merges and table adds complete before it counts itself
    vmem_drain();
    __syncthreads();
    if (tid == 0) {
        const unsigned int prev =
            __hip_atomic_fetch_add(&L->p1_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_flag = (prev + 1 == L->nchunks);
    }
    __syncthreads();
    if (!s_flag) return;
    const int glo = ld_dev(&L->lo);
    const int ghi = ld_dev(&L->hi);
    const unsigned long long gnz = ld_dev(&L->n_zero);
    const unsigned int gbad = ld_dev(&L->bad);
    auto get = [&](int j) { return (unsigned long long)ld_dev(&gh[j]); };
    auto put = [&](int j, int c) { lut[j] = (unsigned char)c; };
    auto clear = [&](int j) { st_dev(&gh[j], 0u); };
    const CutParams p = block_cutoff<BLOCK>(glo, ghi, gnz, gbad, n, tol, score_mode, nonstrict,
                                            get, put, clear, &s_res, nullptr);
    if (depth >= 0 && !p.skip)
        s1_pick(p.e_max, max(glo, p.e_max - KMIN - depth + 1), p.flags, lut,
                [&](int bin, int q) { return ld_dev(&tb[(size_t)bin * S1_PIECES + q]); }, red,
                &s_res);
    __syncthreads();
    if (tid == 0) {
        if (depth < 0) write_invalid(o);
        else *o = s_res;
        st_dev(&L->lo, (int)W);
        st_dev(&L->hi, -1);
        st_dev(&L->n_zero, 0ull);
        st_dev(&L->bad, 0u);
        st_dev(&L->p1_done, 0u);
    }
    if (ghi >= glo) {
        const int64_t cnt = (int64_t)(ghi - glo + 1) * S1_PIECES;
        for (int64_t i = tid; i < cnt; i += BLOCK) st_dev(&tb[(size_t)glo * S1_PIECES + i], 0.0);
    }
}

__global__ __launch_bounds__(BLOCK) void k_batch_init(BLarge *large, int n_large,
                                                      unsigned char *lut)
{
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n_large) return;
    large[i].lo = W;
    large[i].hi = -1;
    for (int s = W; s < W_LUT; s++) lut[(size_t)i * W_LUT + s] = (unsigned char)QDOT_PERF;
}

__global__ __launch_bounds__(BLOCK) void k_batch_gangs_init(Gang *gangs, int S)
{
    if (blockIdx.x >= (unsigned)S) return;
    gang_reset(gangs + blockIdx.x);
    if (threadIdx.x == 0) gangs[blockIdx.x].bar_gen = 0;
}

// Re-arms the gangs of a plan whose previous launch aborted (a bounded wait
// ran out); a clean gang leaves its state ready for the next launch.
__global__ __launch_bounds__(BLOCK) void k_gang_rearm(Gang *gangs, int S)
{
    if (blockIdx.x < (unsigned)S && gangs[blockIdx.x].abort) gang_reset(gangs + blockIdx.x);
}

// GUARD: guard_mode 1 for the qdot instances (two-pass) and the CG systems.
// CG: the work list may hold CG items.  AM: the qdot instances' accum_mode.
// Each combination is its own kernel, so a launch of qdot instances alone
// carries neither the CG solver's registers nor (two-pass) the one-pass
// window's LDS: 128 VGPRs and 22 KB (four blocks per CU) for the two-pass
// kernel, 168 VGPRs (three per CU) for the one-pass one, against two per CU
// for the kernel that holds every path.
template <bool GUARD, bool CG, int AM>
__global__ __launch_bounds__(BLOCK, (CG || GUARD) ? 1 : (AM ? 3 : 4)) void k_batch(const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const int64_t *__restrict__ offsets,
                                                 const double *__restrict__ tols,
                                                 const BItem *__restrict__ items, int n_items,
                                                 BLarge *__restrict__ large,
                                                 unsigned int *__restrict__ ghist,
                                                 unsigned char *__restrict__ glut,
                                                 double *__restrict__ partials,
                                                 BState *__restrict__ st,
                                                 const int *__restrict__ small_list,
                                                 qdot_result *__restrict__ out,
                                                 const CgSys *__restrict__ sys,
                                                 Gang *__restrict__ gangs,
                                                 qdot_cg_result *__restrict__ cg_out,
                                                 double *__restrict__ ltab, int key_mode,
                                                 int score_mode, int nonstrict)
{
    constexpr int accum_mode = AM;
    __shared__ CgLds LD;
    __shared__ S1Lds S1;
    unsigned int *h = LD.h;
    unsigned char *lut = LD.lut;
    auto &red = LD.red;
    int4 *scratch = LD.scratch;
    qdot_result &s_res = LD.res;
    __shared__ int s_item, s_flag;
    __shared__ int4 s_prm2;
    const int tid = threadIdx.x;

    for (int i = tid; i < W + 1; i += BLOCK) h[i] = 0;
    for (int i = W + tid; i < W_LUT; i += BLOCK) lut[i] = (unsigned char)QDOT_PERF;
    __syncthreads();

    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(&st->next, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const BItem I = items[it];
        if (CG && I.type == IT_CG) {
            // one block of a CG gang: its other blocks hold the neighbouring
            // tickets, so they are taken by blocks that are running
            cg_solve<GUARD>(sys[I.inst], gangs + I.inst, I.large, I.slot, key_mode, score_mode,
                            nonstrict, LD, cg_out + I.inst);
            __syncthreads();
            continue;
        }
        if (I.type == IT_SMALL) {
          for (int sj = 0; sj < I.large; sj++) {
            const int inst = small_list[I.inst + sj];
            const int64_t off = offsets[inst];
            const int64_t n = offsets[inst + 1] - off;
            const double *xi = x + off;
            const double *yi = y + off;
            const bool vec = ((((uintptr_t)xi) | ((uintptr_t)yi)) & 15) == 0;
            const double tol = tols[inst];
            unsigned int nz = 0, bad = 0, sg = 0;
            int top = -1, depth = 0;
            if (accum_mode == 1) {
                depth = s1_window_depth(n, tol, score_mode);
                if (depth < 0) {  // kept bins could lie beyond the window
                    if (tid == 0) write_invalid(out + inst);
                    __syncthreads();
                    continue;
                }
                s1_begin(S1);
                __syncthreads();
                S1Run run = s1_run_start();
                if (vec)
                    s1_stream<true, SU>(xi, yi, 0, GROUP, n, key_mode, depth, h, S1, run, nz, bad);
                else
                    s1_stream<false, SU>(xi, yi, 0, GROUP, n, key_mode, depth, h, S1, run, nz, bad);
                top = run.top;
            } else {
                scan_into(xi, yi, 0, GROUP, n, vec, key_mode, h, nz, bad, sg);
            }
            __syncthreads();
            int lo = W, hi = -1;
            for (int j = tid; j < W; j += BLOCK)
                if (h[j]) {
                    lo = min(lo, j);
                    hi = max(hi, j);
                }
            unsigned int bs = (bad ? 1u : 0u) | (sg << 1);
            block_reduce_range(lo, hi, nz, bs, scratch);
            bad = bs & 1u;
            sg = bs >> 1;
            auto get = [&](int j) { return (unsigned long long)h[j]; };
            auto put = [&](int j, int c) { lut[j] = (unsigned char)c; };
            // the guaranteed mode reads the counts again after the sweep
            auto clear = [&](int j) {
                if (!GUARD) h[j] = 0u;
            };
            const CutParams p = block_cutoff<BLOCK>(lo, hi, nz, bad, n, tol, score_mode,
                                                    nonstrict, get, put, clear,
                                                    GUARD ? &s_res : out + inst, nullptr);
            if (tid == 0) h[W] = 0u;
            __syncthreads();
            if (accum_mode == 1) {
                // one pass: each kept bin's class sum straight from the window
                if (!p.skip)
                    s1_pick(p.e_max, max(lo, top - depth + 1), p.flags, lut,
                            [&](int bin, int q) { return S1.win[bin & (S1_WIN - 1)][q]; }, red,
                            out + inst);
            } else if constexpr (GUARD) {
                // the whole instance is swept by this block: first sweep,
                // certification, and a second sweep after a reselection
                auto sweep = [&](const CutParams &cp, int flags) {
                    Acc a[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                    accumulate_range(xi, yi, 0, GROUP, n, vec, key_mode, lut, cp.e_max, cp.c32, a);
                    block_reduce3<BLOCK>(a, red);
                    return tid == 0 ? combine_value(a, cp.e_max, cp.c32, flags, &s_res) : 0.0;
                };
                __shared__ double s_first;
                if (tid == 0) s_first = 0.0;
                __syncthreads();
                if (!p.skip) {
                    const double s0 = sweep(p, p.flags);
                    if (tid == 0) s_first = s0;
                }
                __syncthreads();
                batch_guard(lo, hi, nz, sg, n, tol, score_mode, nonstrict, get, put, lut, s_first,
                            s_res, sweep);
                put_result(out + inst, s_res);
                for (int j = lo + tid; j <= hi; j += BLOCK) h[j] = 0u;
            } else if (!p.skip) {
                Acc a[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                accumulate_range(xi, yi, 0, GROUP, n, vec, key_mode, lut, p.e_max, p.c32, a);
                block_reduce3<BLOCK>(a, red);
                if (tid == 0) combine_value(a, p.e_max, p.c32, p.flags, out + inst);
            }
            __syncthreads();
          }
          continue;
        }
        const int64_t off = offsets[I.inst];
        const int64_t n = offsets[I.inst + 1] - off;
        const double *xi = x + off;
        const double *yi = y + off;
        const bool vec = ((((uintptr_t)xi) | ((uintptr_t)yi)) & 15) == 0;
        const double tol = tols[I.inst];
        if (I.type == IT_P1 && accum_mode == 1) {
            p1_onepass(xi, yi, n, tol, vec, I, large + I.large, ghist + (size_t)I.large * W,
                       ltab + (size_t)I.large * W * S1_PIECES, out + I.inst, h, lut, red,
                       scratch, s_res, S1, s_flag, key_mode, score_mode, nonstrict);
        } else if (I.type == IT_P1) {
            BLarge *L = large + I.large;
            unsigned int *gh = ghist + (size_t)I.large * W;
            unsigned int nz = 0, bad = 0, sg = 0;
            scan_into(xi, yi, I.first, I.stride, n, vec, key_mode, h, nz, bad, sg);
            __syncthreads();
            int lo = W, hi = -1;
            for (int j = tid; j < W; j += BLOCK) {
                const unsigned int v = h[j];
                if (v) {
                    __hip_atomic_fetch_add(&gh[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    h[j] = 0u;
                    lo = min(lo, j);
                    hi = max(hi, j);
                }
            }
            if (tid == 0) h[W] = 0u;
            unsigned int bs = (bad ? 1u : 0u) | (sg << 1);
            block_reduce_range(lo, hi, nz, bs, scratch);
            bad = bs & 1u;
            sg = bs >> 1;
            if (tid == 0) {
                if (GUARD && sg)
                    __hip_atomic_fetch_or(&L->signs, sg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (hi >= 0) {
                    __hip_atomic_fetch_min(&L->lo, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_max(&L->hi, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (nz)
                    __hip_atomic_fetch_add(&L->n_zero, (unsigned long long)nz, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                if (bad) __hip_atomic_fetch_or(&L->bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // every thread's merge has completed before the chunk counts itself
            vmem_drain();
            __syncthreads();
            if (tid == 0) {
                const unsigned int prev = __hip_atomic_fetch_add(&L->p1_done, 1u, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                s_flag = (prev + 1 == L->nchunks);
            }
            __syncthreads();
            if (s_flag) {
                // last P1 chunk of this instance: its cutoff selection, on
                // the merged histogram that every other chunk completed
                // before counting itself
                const int glo = ld_dev(&L->lo);
                const int ghi = ld_dev(&L->hi);
                const unsigned long long gnz = ld_dev(&L->n_zero);
                const unsigned int gbad = ld_dev(&L->bad);
                unsigned char *gl = glut + (size_t)I.large * W_LUT;
                auto get = [&](int j) { return (unsigned long long)ld_dev(&gh[j]); };
                auto put = [&](int j, int c) { st_dev(&gl[j], (unsigned char)c); };
                // the guaranteed mode keeps the counts for the block that
                // finishes the instance
                auto clear = [&](int j) {
                    if (!GUARD) st_dev(&gh[j], 0u);
                };
                const CutParams p = block_cutoff<BLOCK>(glo, ghi, gnz, gbad, n, tol, score_mode,
                                                        nonstrict, get, put, clear, &s_res,
                                                        nullptr);
                if (tid == 0 && !GUARD) {
                    // the combining block writes value, part and flags; this
                    // block writes the rest (all of it when nothing is kept)
                    // (with guard_mode 1 the combining block writes it all:
                    // two blocks never store the same bytes)
                    qdot_result *o = out + I.inst;
                    for (int q = 0; q < 4; q++) o->count[q] = s_res.count[q];
                    o->n_zero = s_res.n_zero;
                    o->e_min = s_res.e_min;
                    o->e_max = s_res.e_max;
                    o->n_bins = s_res.n_bins;
                    o->t = s_res.t;
                    o->bound_rel = s_res.bound_rel;
                    o->bound_abs = s_res.bound_abs;
                    o->status = s_res.status;
                    o->lower = s_res.lower;
                    o->e_ref = s_res.e_ref;
                    o->passes = s_res.passes;
                    if (p.skip) {
                        o->value = s_res.value;
                        for (int q = 0; q < 3; q++) o->part[q] = s_res.part[q];
                        o->flags = s_res.flags;
                    }
                }
                if (tid == 0) {
                    st_dev(&L->e_max, p.e_max);
                    st_dev(&L->c32, p.c32);
                    st_dev(&L->skip, p.skip);
                    st_dev(&L->flags, p.flags);
                    if (!GUARD) {
                        st_dev(&L->lo, (int)W);
                        st_dev(&L->hi, -1);
                        st_dev(&L->n_zero, 0ull);
                        st_dev(&L->bad, 0u);
                    }
                }
                vmem_drain();
                __syncthreads();
                if (tid == 0) st_dev(&L->ready, 1u);
            }
        } else {  // IT_P2
            BLarge *L = large + I.large;
            if (tid == 0) {
                // bounded like the gang barriers: a chunk that waits past the
                // spin limit gives up, marks its instance QDOT_E_DEVICE and
                // only counts itself below
                unsigned int spins = 0;
                bool ready = true;
                while (ld_dev(&L->ready) == 0u) {
                    if (++spins > SPIN_LIMIT) {
                        ready = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (ready) {
                    s_prm2 = make_int4(ld_dev(&L->skip), ld_dev(&L->e_max), ld_dev(&L->c32),
                                       ld_dev(&L->flags));
                } else {
                    st_dev(&out[I.inst].status, (int32_t)QDOT_E_DEVICE);
                    s_prm2 = make_int4(1, 0, 0, 0);
                }
            }
            __syncthreads();
            const int skip = s_prm2.x, e_max = s_prm2.y, c32 = s_prm2.z, flags = s_prm2.w;
            __syncthreads();
            if (!skip) {
                const unsigned int *src =
                    reinterpret_cast<const unsigned int *>(glut + (size_t)I.large * W_LUT);
                unsigned int *dst = reinterpret_cast<unsigned int *>(lut);
                for (int i = tid; i < W_LUT / 4; i += BLOCK) dst[i] = ld_dev(&src[i]);
                __syncthreads();
                Acc a[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                accumulate_range(xi, yi, I.first, I.stride, n, vec, key_mode, lut, e_max, c32, a);
                block_reduce3<BLOCK>(a, red);
                if (tid == 0) {
                    double *p = partials + (size_t)I.slot * 6;
                    for (int q = 0; q < 3; q++) {
                        st_dev(&p[2 * q], a[q].s);
                        st_dev(&p[2 * q + 1], a[q].c);
                    }
                }
            }
            vmem_drain();
            __syncthreads();
            if (tid == 0) {
                const unsigned int prev = __hip_atomic_fetch_add(&L->p2_done, 1u, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                s_flag = (prev + 1 == L->nchunks);
            }
            __syncthreads();
            if (s_flag) {
                // last P2 chunk: combine the instance's partials in chunk order
                Acc a[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                if (!skip) {
                    const int nc = (int)L->nchunks;
                    for (int c = tid; c < nc; c += BLOCK) {
                        const double *p = partials + (size_t)(L->first_slot + c) * 6;
                        for (int q = 0; q < 3; q++)
                            a[q] = acc_merge(a[q], Acc{ld_dev(&p[2 * q]), ld_dev(&p[2 * q + 1])});
                    }
                    block_reduce3<BLOCK>(a, red);
                    if (!GUARD && tid == 0) combine_value(a, e_max, c32, flags, out + I.inst);
                }
                if constexpr (GUARD) {
                    // the selection again, from the kept counts, into this
                    // block's result and class table (the same classes as
                    // the chunks used), the combine, then the certification;
                    // a reselection sweeps the instance with this block alone
                    unsigned int *gh = ghist + (size_t)I.large * W;
                    const int glo = ld_dev(&L->lo), ghi = ld_dev(&L->hi);
                    const unsigned long long gnz = ld_dev(&L->n_zero);
                    const unsigned int gbad = ld_dev(&L->bad), gsg = ld_dev(&L->signs);
                    auto get = [&](int j) { return (unsigned long long)ld_dev(&gh[j]); };
                    auto put = [&](int j, int c) { lut[j] = (unsigned char)c; };
                    auto noclear = [](int) {};
                    const CutParams p = block_cutoff<BLOCK>(glo, ghi, gnz, gbad, n, tol,
                                                            score_mode, nonstrict, get, put,
                                                            noclear, &s_res, nullptr);
                    __shared__ double s_first;
                    if (tid == 0)
                        s_first = p.skip ? 0.0 : combine_value(a, p.e_max, p.c32, p.flags, &s_res);
                    __syncthreads();
                    auto sweep = [&](const CutParams &cp, int fl) {
                        Acc b[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                        accumulate_range(xi, yi, 0, GROUP, n, vec, key_mode, lut, cp.e_max,
                                         cp.c32, b);
                        block_reduce3<BLOCK>(b, red);
                        return tid == 0 ? combine_value(b, cp.e_max, cp.c32, fl, &s_res) : 0.0;
                    };
                    batch_guard(glo, ghi, gnz, gsg, n, tol, score_mode, nonstrict, get, put, lut,
                                s_first, s_res, sweep);
                    // a chunk that gave up waiting has marked the instance
                    if (tid == 0 && ld_dev(&out[I.inst].status) == QDOT_E_DEVICE)
                        s_res.status = QDOT_E_DEVICE;
                    __syncthreads();
                    put_result(out + I.inst, s_res);
                    for (int j = glo + tid; j <= ghi; j += BLOCK) st_dev(&gh[j], 0u);
                    if (tid == 0) {
                        st_dev(&L->lo, (int)W);
                        st_dev(&L->hi, -1);
                        st_dev(&L->n_zero, 0ull);
                        st_dev(&L->bad, 0u);
                        st_dev(&L->signs, 0u);
                    }
                }
                if (tid == 0) {
                    st_dev(&L->p1_done, 0u);
                    st_dev(&L->p2_done, 0u);
                    st_dev(&L->ready, 0u);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const unsigned int e = __hip_atomic_fetch_add(&st->exited, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        if (e == gridDim.x - 1) {
            st_dev(&st->next, 0u);
            st_dev(&st->exited, 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// host planning
// ---------------------------------------------------------------------------
static bool same_system(const qdot_cg_system &a, const qdot_cg_system &b)
{
    return a.A.n == b.A.n && a.A.nnz == b.A.nnz && a.A.rowptr == b.A.rowptr &&
           a.A.col == b.A.col && a.A.val == b.A.val && a.b == b.b && a.x == b.x &&
           a.rtol == b.rtol && a.qtol == b.qtol && a.maxit == b.maxit &&
           a.use_qdot == b.use_qdot;
}

static int gang_size(const qdot_handle *h, int64_t n)
{
    const int64_t rows = h->batch_cg_rows;
    return (int)std::max<int64_t>(1, std::min<int64_t>(h->batch_cg_gang_max, (n + rows - 1) / rows));
}

static int32_t build_plan(qdot_handle *h, const int64_t *host_offsets, int32_t B,
                          const qdot_cg_system *systems, int32_t S, int accum, BatchPlan **out)
{
    BatchPlan *p = new BatchPlan();
    p->B = B;
    p->S = S;
    p->accum = accum;
    if (B > 0) p->offsets.assign(host_offsets, host_offsets + B + 1);
    if (S > 0) p->systems.assign(systems, systems + S);
    std::vector<int> big, small;
    for (int j = 0; j < B; j++) {
        const int64_t n = host_offsets[j + 1] - host_offsets[j];
        (n > h->batch_chunk ? big : small).push_back(j);
    }
    auto len = [&](int j) { return host_offsets[j + 1] - host_offsets[j]; };
    std::stable_sort(big.begin(), big.end(), [&](int a, int b) { return len(a) > len(b); });
    std::stable_sort(small.begin(), small.end(), [&](int a, int b) { return len(a) > len(b); });
    std::vector<BItem> items;
    // CG gangs first, largest system first: their solves are the longest
    // chains of the launch, and the qdot items fill the other blocks
    std::vector<int> cg_order(S);
    std::iota(cg_order.begin(), cg_order.end(), 0);
    std::stable_sort(cg_order.begin(), cg_order.end(),
                     [&](int a, int c) { return systems[a].A.n > systems[c].A.n; });
    for (int s : cg_order) {
        const int G = gang_size(h, systems[s].A.n);
        p->max_gang = std::max(p->max_gang, G);
        for (int gb = 0; gb < G; gb++) items.push_back(BItem{IT_CG, s, G, gb, 0, 0});
    }
    std::vector<BLarge> lg(big.size());
    int slot = 0;
    for (size_t L = 0; L < big.size(); L++) {
        const int j = big[L];
        const int64_t n = len(j);
        const unsigned int nc = (unsigned int)((n + h->batch_chunk - 1) / h->batch_chunk);
        std::memset(&lg[L], 0, sizeof(BLarge));
        lg[L].nchunks = nc;
        lg[L].lo = W;
        lg[L].hi = -1;
        lg[L].first_slot = slot;
        for (unsigned int c = 0; c < nc; c++)
            items.push_back(BItem{IT_P1, j, (int)L, -1, (int64_t)c * GROUP, (int64_t)nc * GROUP});
        slot += (int)nc;
    }
    std::vector<int> small_list(small.begin(), small.end());
    for (size_t s0 = 0; s0 < small_list.size();) {
        size_t s1 = s0;
        int64_t cost = 0;
        while (s1 < small_list.size() &&
               (s1 == s0 || cost + len(small_list[s1]) + SMALL_COST0 <= SMALL_GROUP)) {
            cost += len(small_list[s1]) + SMALL_COST0;
            s1++;
        }
        items.push_back(BItem{IT_SMALL, (int)s0, (int)(s1 - s0), -1, 0, 0});
        s0 = s1;
    }
    // the one-pass mode has no second pass
    for (size_t L = 0; accum == 0 && L < big.size(); L++) {
        const int j = big[L];
        for (unsigned int c = 0; c < lg[L].nchunks; c++)
            items.push_back(BItem{IT_P2, j, (int)L, lg[L].first_slot + (int)c, (int64_t)c * GROUP,
                                  (int64_t)lg[L].nchunks * GROUP});
    }
    p->n_items = (int)items.size();
    p->n_large = (int)big.size();
    p->n_p2 = slot;
    int64_t cg_rows = 0;
    for (int s = 0; s < S; s++) cg_rows += systems[s].A.n;
    const size_t nl = std::max<size_t>(1, big.size());
    const size_t ns = std::max<int32_t>(1, S);
    bool ok = hipMalloc((void **)&p->items, sizeof(BItem) * std::max<size_t>(1, items.size())) == hipSuccess &&
              hipMalloc((void **)&p->large, sizeof(BLarge) * nl) == hipSuccess &&
              hipMalloc((void **)&p->hist, sizeof(unsigned int) * W * nl) == hipSuccess &&
              hipMalloc((void **)&p->lut, (size_t)W_LUT * nl) == hipSuccess &&
              hipMalloc((void **)&p->partials, sizeof(double) * 6 * std::max(1, slot)) == hipSuccess &&
              hipMalloc((void **)&p->state, sizeof(BState)) == hipSuccess &&
              hipMalloc((void **)&p->small_list, sizeof(int) * std::max<size_t>(1, small_list.size())) == hipSuccess &&
              hipMalloc((void **)&p->sys, sizeof(CgSys) * ns) == hipSuccess &&
              hipMalloc((void **)&p->gangs, sizeof(Gang) * ns) == hipSuccess &&
              hipMalloc((void **)&p->cgres, sizeof(qdot_cg_result) * ns) == hipSuccess &&
              hipMalloc((void **)&p->cgvec, sizeof(double) * std::max<int64_t>(1, 3 * cg_rows)) == hipSuccess &&
              (accum == 0 ||
               hipMalloc((void **)&p->ltab, sizeof(double) * W * S1_PIECES * nl) == hipSuccess);
    if (!ok) {
        free_plan(p);
        return fail(h, QDOT_E_NOMEM, "batched plan allocation failed");
    }
    std::vector<CgSys> dsys(S);
    int64_t vo = 0;
    for (int s = 0; s < S; s++) {
        const qdot_cg_system &q = systems[s];
        CgSys &d = dsys[s];
        d.n = q.A.n;
        d.rowptr = q.A.rowptr;
        d.col = q.A.col;
        d.val = q.A.val;
        d.b = q.b;
        d.x = q.x;
        d.r = p->cgvec + vo;
        d.p = p->cgvec + vo + q.A.n;
        d.q = p->cgvec + vo + 2 * q.A.n;
        vo += 3 * q.A.n;
        d.rtol = q.rtol;
        d.qtol = q.qtol;
        d.maxit = q.maxit;
        d.use_qdot = q.use_qdot ? 1 : 0;
        d.trace = nullptr;
    }
    hipError_t e = hipMemcpy(p->items, items.data(), sizeof(BItem) * items.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess && !lg.empty())
        e = hipMemcpy(p->large, lg.data(), sizeof(BLarge) * lg.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->hist, 0, sizeof(unsigned int) * W * nl);
    if (e == hipSuccess) e = hipMemset(p->lut, 0, (size_t)W_LUT * nl);
    if (e == hipSuccess) e = hipMemset(p->state, 0, sizeof(BState));
    if (e == hipSuccess && p->ltab) e = hipMemset(p->ltab, 0, sizeof(double) * W * S1_PIECES * nl);
    if (e == hipSuccess && !small_list.empty())
        e = hipMemcpy(p->small_list, small_list.data(), sizeof(int) * small_list.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && S > 0)
        e = hipMemcpy(p->sys, dsys.data(), sizeof(CgSys) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess && !lg.empty()) {
        hipLaunchKernelGGL(k_batch_init, dim3((unsigned)((lg.size() + BLOCK - 1) / BLOCK)),
                           dim3(BLOCK), 0, 0, p->large, (int)lg.size(), p->lut);
        e = hipGetLastError();
    }
    if (e == hipSuccess && S > 0) {
        hipLaunchKernelGGL(k_batch_gangs_init, dim3((unsigned)S), dim3(BLOCK), 0, 0, p->gangs, S);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(h, e, "batched plan upload");
    }
    *out = p;
    return QDOT_OK;
}

static int32_t find_plan(qdot_handle *h, const int64_t *host_offsets, int32_t B,
                         const qdot_cg_system *systems, int32_t S, int accum, BatchPlan **out)
{
    static uint64_t clock = 0;
    for (void *vp : h->plans) {
        BatchPlan *p = (BatchPlan *)vp;
        if (p->B != B || p->S != S || p->accum != accum) continue;
        if (B > 0 && !std::equal(p->offsets.begin(), p->offsets.end(), host_offsets)) continue;
        bool same = true;
        for (int s = 0; s < S && same; s++) same = same_system(p->systems[s], systems[s]);
        if (!same) continue;
        p->last_use = ++clock;
        *out = p;
        return QDOT_OK;
    }
    BatchPlan *p = nullptr;
    int32_t st = build_plan(h, host_offsets, B, systems, S, accum, &p);
    if (st != QDOT_OK) return st;
    p->last_use = ++clock;
    if ((int)h->plans.size() >= MAX_PLANS) {
        auto oldest = std::min_element(h->plans.begin(), h->plans.end(), [](void *a, void *b) {
            return ((BatchPlan *)a)->last_use < ((BatchPlan *)b)->last_use;
        });
        (void)hipDeviceSynchronize();
        free_plan((BatchPlan *)*oldest);
        h->plans.erase(oldest);
    }
    h->plans.push_back(p);
    *out = p;
    return QDOT_OK;
}

void free_plans(qdot_handle *h)
{
    for (void *p : h->plans) free_plan((BatchPlan *)p);
    h->plans.clear();
}

static int32_t check_batch(qdot_handle *h, const int64_t *host_offsets, int32_t B)
{
    if (B < 0 || (B > 0 && !host_offsets)) return fail(h, QDOT_E_INVAL, "bad batch size or offsets");
    if (B > 0 && host_offsets[0] != 0) return fail(h, QDOT_E_INVAL, "offsets[0] must be 0");
    for (int j = 0; j < B; j++)
        if (host_offsets[j + 1] < host_offsets[j])
            return fail(h, QDOT_E_INVAL, "offsets must be non-decreasing");
    return QDOT_OK;
}

static int32_t check_systems(qdot_handle *h, const qdot_cg_system *systems, int32_t S)
{
    if (S < 0 || (S > 0 && !systems)) return fail(h, QDOT_E_INVAL, "bad system count or array");
    for (int s = 0; s < S; s++) {
        const qdot_cg_system &q = systems[s];
        if (q.A.n <= 0 || q.A.nnz < 0 || !q.A.rowptr || !q.A.col || !q.A.val || !q.b || !q.x ||
            q.A.n >= ((int64_t)1 << 31) || q.A.nnz >= ((int64_t)1 << 31))
            return fail(h, QDOT_E_INVAL, "bad CSR or vector in a CG system");
        if (!(q.rtol >= 0.0) || q.maxit < 0) return fail(h, QDOT_E_INVAL, "bad rtol or maxit");
        if (q.use_qdot && (!(q.qtol > 0.0) || !std::isfinite(q.qtol)))
            return fail(h, QDOT_E_INVAL, "qtol must be finite and > 0");
    }
    return QDOT_OK;
}

// Arguments of one k_batch launch.
struct BatchArgs {
    const double *x, *y;
    const int64_t *offsets;
    const double *tols;
    const BatchPlan *p;
    qdot_result *out;
    qdot_cg_result *cg_out;
    int key_mode, score_mode, nonstrict;
};

template <bool GUARD, bool CG, int AM>
static hipError_t batch_kernel_t(const BatchArgs &a, int grid, hipStream_t s, int *per_cu)
{
    if (per_cu)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<GUARD, CG, AM>,
                                                            BLOCK, 0);
    const BatchPlan *p = a.p;
    hipLaunchKernelGGL((k_batch<GUARD, CG, AM>), dim3(grid), dim3(BLOCK), 0, s, a.x, a.y,
                       a.offsets, a.tols, p->items, p->n_items, p->large, p->hist, p->lut,
                       p->partials, p->state, p->small_list, a.out, p->sys, p->gangs, a.cg_out,
                       p->ltab, a.key_mode, a.score_mode, a.nonstrict);
    return hipGetLastError();
}

// per_cu != nullptr: the occupancy query of the kernel the launch would use
// (resident blocks per CU), no launch.
static hipError_t batch_kernel(bool guard, bool cg, int accum, const BatchArgs &a, int grid,
                               hipStream_t s, int *per_cu)
{
    if (guard)
        return cg ? batch_kernel_t<true, true, 0>(a, grid, s, per_cu)
                  : batch_kernel_t<true, false, 0>(a, grid, s, per_cu);
    if (cg)
        return accum ? batch_kernel_t<false, true, 1>(a, grid, s, per_cu)
                     : batch_kernel_t<false, true, 0>(a, grid, s, per_cu);
    return accum ? batch_kernel_t<false, false, 1>(a, grid, s, per_cu)
                 : batch_kernel_t<false, false, 0>(a, grid, s, per_cu);
}

// Plans (when needed) and launches the work of one batch: B qdot instances
// and S CG systems in one persistent launch.
static int32_t batch_launch(qdot_handle *h, const double *x_cat, const double *y_cat,
                            const int64_t *offsets, const int64_t *host_offsets,
                            const double *tols, int32_t B, const qdot_cg_system *systems,
                            int32_t S, const qdot_options *opt, void *stream,
                            qdot_result *dev_out, qdot_cg_result *dev_cg_out, BatchPlan **used)
{
    int32_t st = check_batch(h, host_offsets, B);
    if (st != QDOT_OK) return st;
    if ((st = check_systems(h, systems, S)) != QDOT_OK) return st;
    if (B == 0 && S == 0) return QDOT_OK;
    if (B > 0) {
        const int64_t total = host_offsets[B];
        if ((total > 0 && (!x_cat || !y_cat)) || !offsets || !tols || !dev_out)
            return fail(h, QDOT_E_INVAL, "NULL pointer");
        if (((uintptr_t)x_cat | (uintptr_t)y_cat) & 7)
            return fail(h, QDOT_E_INVAL, "vectors not 8-byte aligned");
    }
    if (S > 0 && !dev_cg_out) return fail(h, QDOT_E_INVAL, "NULL CG result array");
    qdot_options o;
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return fail(h, QDOT_E_INVAL, "unknown option value");
    if (o.bin_mode != 0)
        return fail(h, QDOT_E_INVAL, "bin_mode 1 and 2 are for the single-vector qdot entry points");
    if (o.tile_skip != 0)
        return fail(h, QDOT_E_INVAL, "tile_skip is for the single-vector qdot entry points");
    DeviceGuard g(h->device);
    BatchPlan *p = nullptr;
    const int accum = B > 0 ? o.accum_mode : 0;  // CG systems always use the default reading
    if ((st = find_plan(h, host_offsets, B, systems, S, accum, &p)) != QDOT_OK) return st;
    const int bpc = h->batch_blocks_per_cu;
    const int grid = std::max(1, std::min(p->n_items, bpc * h->num_cus));
    // guard_mode 1 implies accum_mode 0 (options_ok)
    const BatchArgs a = {x_cat, y_cat, offsets, tols, p, dev_out, dev_cg_out,
                         o.key_mode, o.score_mode, o.boundary_mode};
    const bool cg = S > 0;
    if (p->max_gang > 0) {
        // a gang waits for its own blocks only, so it needs that many
        // blocks resident at once
        int per_cu = 0;
        hipError_t e = batch_kernel(o.guard_mode != 0, cg, accum, a, 0, nullptr, &per_cu);
        if (e != hipSuccess) return hip_fail(h, e, "occupancy query");
        if ((int64_t)per_cu * h->num_cus < p->max_gang)
            return fail(h, QDOT_E_DEVICE, "CG gang larger than the resident blocks");
    }
    hipStream_t s = (hipStream_t)stream;
    if (S > 0) hipLaunchKernelGGL(k_gang_rearm, dim3((unsigned)S), dim3(BLOCK), 0, s, p->gangs, S);
    (void)batch_kernel(o.guard_mode != 0, cg, accum, a, grid, s, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "batched launch");
    if (used) *used = p;
    return QDOT_OK;
}

}  // namespace qd

using namespace qd;

extern "C" {

int32_t qdot_set_solver_tune(qdot_handle *h, const qdot_solver_tune *cfg)
{
    if (!h) return QDOT_E_INVAL;
    qdot_solver_tune t = cfg ? *cfg : qdot_solver_tune{4, 131072, 16384, 16, 8, 2, 0};
    if (t.batch_blocks_per_cu < 1 || t.batch_blocks_per_cu > 16 || t.batch_chunk < (1 << 13) ||
        t.batch_chunk > (1 << 22) || t.batch_chunk % GROUP != 0 ||
        t.cg_rows_per_block < CHUNK || t.cg_gang_max < 1 || t.cg_gang_max > MAX_GANG ||
        t.spmv_blocks_per_cu < 1 || t.spmv_blocks_per_cu > 16 || t.cg_blocks_per_cu < 1 ||
        t.cg_blocks_per_cu > 2 || (t.power_scan_in_spmv != 0 && t.power_scan_in_spmv != 1))
        return fail(h, QDOT_E_INVAL, "solver tune out of range (batch blocks per CU 1..16, chunk "
                                     "2^13..2^22 in multiples of 2048, CG rows per block >= "
                                     "1024, gang 1..512, SpMV blocks per CU 1..16, CG blocks "
                                     "per CU 1..2, power scan in SpMV 0/1)");
    DeviceGuard g(h->device);
    // the cached plans were cut with the old shape
    if (!h->plans.empty()) {
        (void)hipDeviceSynchronize();
        free_plans(h);
    }
    h->batch_blocks_per_cu = t.batch_blocks_per_cu;
    h->batch_chunk = t.batch_chunk;
    h->batch_cg_rows = t.cg_rows_per_block;
    h->batch_cg_gang_max = t.cg_gang_max;
    h->spmv_blocks_per_cu = t.spmv_blocks_per_cu;
    h->cg_blocks_per_cu = t.cg_blocks_per_cu;
    h->power_scan_in_spmv = t.power_scan_in_spmv;
    return QDOT_OK;
}

int32_t qdot_get_solver_tune(const qdot_handle *h, qdot_solver_tune *cfg)
{
    if (!h || !cfg) return QDOT_E_INVAL;
    cfg->batch_blocks_per_cu = h->batch_blocks_per_cu;
    cfg->batch_chunk = (int32_t)h->batch_chunk;
    cfg->cg_rows_per_block = (int32_t)h->batch_cg_rows;
    cfg->cg_gang_max = h->batch_cg_gang_max;
    cfg->spmv_blocks_per_cu = h->spmv_blocks_per_cu;
    cfg->cg_blocks_per_cu = h->cg_blocks_per_cu;
    cfg->power_scan_in_spmv = h->power_scan_in_spmv;
    return QDOT_OK;
}

int32_t qdot_batched_plan(qdot_handle *h, const int64_t *host_offsets, int32_t B)
{
    return qdot_batch_plan(h, host_offsets, B, nullptr, 0, nullptr);
}

int32_t qdot_batch_plan(qdot_handle *h, const int64_t *host_offsets, int32_t B,
                        const qdot_cg_system *systems, int32_t S, const qdot_options *opt)
{
    if (!h) return QDOT_E_INVAL;
    int32_t st = check_batch(h, host_offsets, B);
    if (st != QDOT_OK) return st;
    if ((st = check_systems(h, systems, S)) != QDOT_OK) return st;
    qdot_options o;
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return fail(h, QDOT_E_INVAL, "unknown option value");
    if (o.bin_mode != 0)
        return fail(h, QDOT_E_INVAL, "bin_mode 1 and 2 are for the single-vector qdot entry points");
    if (o.tile_skip != 0)
        return fail(h, QDOT_E_INVAL, "tile_skip is for the single-vector qdot entry points");
    if (B == 0 && S == 0) return QDOT_OK;
    DeviceGuard g(h->device);
    BatchPlan *p = nullptr;
    return find_plan(h, host_offsets, B, systems, S, B > 0 ? o.accum_mode : 0, &p);
}

int32_t qdot_batched_async(qdot_handle *h, const double *x_cat, const double *y_cat,
                           const int64_t *offsets, const int64_t *host_offsets,
                           const double *tols, int32_t B, const qdot_options *opt,
                           void *stream, qdot_result *dev_out)
{
    if (!h) return QDOT_E_INVAL;
    return batch_launch(h, x_cat, y_cat, offsets, host_offsets, tols, B, nullptr, 0, opt, stream,
                        dev_out, nullptr, nullptr);
}

int32_t qdot_batch_run_async(qdot_handle *h, const double *x_cat, const double *y_cat,
                             const int64_t *offsets, const int64_t *host_offsets,
                             const double *tols, int32_t B, const qdot_cg_system *systems,
                             int32_t S, const qdot_options *opt, void *stream,
                             qdot_result *dev_out, qdot_cg_result *dev_cg_out)
{
    if (!h) return QDOT_E_INVAL;
    return batch_launch(h, x_cat, y_cat, offsets, host_offsets, tols, B, systems, S, opt, stream,
                        dev_out, dev_cg_out, nullptr);
}

int32_t qdot_cg_batched(qdot_handle *h, const qdot_cg_system *systems, int32_t S,
                        const qdot_options *opt, void *stream, qdot_cg_result *host_out)
{
    if (!h) return QDOT_E_INVAL;
    if (S > 0 && !host_out) return fail(h, QDOT_E_INVAL, "out is NULL");
    if (S <= 0) return S == 0 ? QDOT_OK : fail(h, QDOT_E_INVAL, "bad system count");
    int32_t st = qdot_batch_plan(h, nullptr, 0, systems, S, opt);
    if (st != QDOT_OK) return st;
    DeviceGuard g(h->device);
    BatchPlan *p = nullptr;
    if ((st = find_plan(h, nullptr, 0, systems, S, 0, &p)) != QDOT_OK) return st;
    if ((st = batch_launch(h, nullptr, nullptr, nullptr, nullptr, nullptr, 0, systems, S, opt,
                           stream, nullptr, p->cgres, nullptr)) != QDOT_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(host_out, p->cgres, sizeof(qdot_cg_result) * S,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "batched CG");
    for (int i = 0; i < S; i++)
        if (host_out[i].status == QDOT_E_DEVICE)
            return fail(h, QDOT_E_DEVICE, "CG gang barrier timed out");
    return QDOT_OK;
}

}  // extern "C"
