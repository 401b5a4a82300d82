// Device side of conjugate gradient (Alg. 4) run by a gang of blocks inside
// one launch; used by the single-system CG launch and by the batched launch.
//
// A gang of G blocks solves one system; block b of the gang owns a
// contiguous slice of rows and every vector update, SpMV row and qdot pass
// on that slice.  Gang barriers (an arrival counter and a generation word)
// separate the steps that need data from other slices:
//   before the SpMV (p complete), after a qdot's pass 1 (histogram merged),
//   after its pass 2 (partials written),
// five per iteration (one more for an inner product that the guaranteed
// mode sums again; one fewer per inner product in the one-pass mode).  The
// whole-gang reductions (the blocks' pass-1 records and histogram copies at
// the first barrier of a qdot, its partials at the second) are done once,
// by the last block to arrive, before it releases the others; that block
// also clears the histogram copies.  Every block then computes the cutoff
// itself from the same merged histogram and finishes the combine from the
// same published words, so every block holds bit-identical scalars (alpha,
// beta, c) and takes the same branches: no decision is broadcast.  Two
// buffers alternate between consecutive qdots.
//
// Every wait is bounded: a barrier that does not complete within the spin
// limit raises the gang's abort flag, every block leaves, and the call
// reports QDOT_E_DEVICE.  The launches size their grids so that all blocks
// of a gang are resident together (the single-system launch: up to two
// blocks per CU when the kernel's occupancy allows it).
#pragma once
#include <cmath>

#include "qdot_blocks.hpp"

namespace qd {

constexpr unsigned SPIN_LIMIT = 1u << 26;

struct CgSys {
    int64_t n;
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x;
    double *r, *p, *q;  // scratch, n each
    double rtol, qtol;
    int maxit, use_qdot;
    qdot_result *trace;  // nullable: 2 * maxit + 1 results
};

constexpr int MAX_GANG = 512;
// block gb of a gang merges its histogram into copy gb % GANG_HIST_COPIES:
// the merge atomics of one slot then queue 8 ways instead of G deep, and
// every block waits for its own atomics before it arrives at the barrier
constexpr int GANG_HIST_COPIES = 8;

struct GangQ {  // per gang and qdot buffer
    unsigned int hist[GANG_HIST_COPIES][W];
    // per block: live slot range, zero count, and non-finite flag (bit 0)
    // with the signs of the nonzero products (bit 1 negative, bit 2
    // positive); written by every block for every inner product, so never
    // cleared
    int4 rec[MAX_GANG];
    // published by the last block to arrive at the merge barrier: the
    // reduced records (lo, hi, zeros, flags) and the summed copies over
    // [lo, hi] (the copies are cleared by the same block)
    int4 sum;
    unsigned int hm[W];
};

constexpr int BAR_GROUPS = 8;    // first level of the barrier of a large gang
constexpr int BAR_TWO_LEVEL = 64; // gangs larger than this use two levels

struct Gang {
    unsigned int bar_count;
    unsigned int bar_gen;
    unsigned int abort;
    unsigned int pad;
    GangQ qb[2];
    double partials[2][MAX_GANG * 6];
    // partials[k] combined in block order by the last block to arrive
    double pfin[2][6];
    // one-pass mode: the result of buffer k's qdot, published by the last
    // block to arrive
    qdot_result res[2];
    unsigned int bar_sub[BAR_GROUPS][32];  // group counters, one 128-byte line each
};


// ---------------------------------------------------------------------------
// Gang barrier.  Everything a block hands to the others (vector entries,
// histogram merges, partials, clears) is written with device-scope atomics
// or write-through stores and read with device-scope loads, so arriving
// needs only the block's own memory operations to have completed
// (vmem_drain) and leaving needs no cache invalidation.  A gang of more than
// BAR_TWO_LEVEL blocks arrives in two levels: each block on the counter of
// its group (gb mod BAR_GROUPS), the last of a group on the gang counter, so
// no counter takes more than G / BAR_GROUPS serialised atomics.
//
// gang_barrier_then: the last block to arrive runs work() with all its
// threads before it releases the others.  Reductions over the whole gang
// (the blocks' records, histogram copies, partials) are done there once,
// and every other block reads only the result: when every block reads all
// G contributions the same words are fetched G times at once.
template <class Work>
__device__ bool gang_barrier_then(Gang *gg, int G, int gb, Work &&work)
{
    __shared__ int s_ok, s_last;
    __shared__ unsigned int s_gen;
    vmem_drain();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int gen = ld_dev(&gg->bar_gen);
        bool last;
        if (G > BAR_TWO_LEVEL) {
            const int grp = gb % BAR_GROUPS;
            const unsigned int members = (unsigned)((G - grp + BAR_GROUPS - 1) / BAR_GROUPS);
            unsigned int *sc = &gg->bar_sub[grp][0];
            last = false;
            if (__hip_atomic_fetch_add(sc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 ==
                members) {
                // re-arm the group counter before the gang can be released
                // (its members wait for the generation below)
                st_dev(sc, 0u);
                vmem_drain();
                last = __hip_atomic_fetch_add(&gg->bar_count, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) + 1 ==
                       (unsigned)BAR_GROUPS;
            }
        } else {
            last = __hip_atomic_fetch_add(&gg->bar_count, 1u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) + 1 == (unsigned)G;
        }
        s_ok = 1;
        s_last = last ? 1 : 0;
        s_gen = gen;
    }
    __syncthreads();
    if (s_last) {
        work();
        vmem_drain();
        __syncthreads();
        if (threadIdx.x == 0) {
            st_dev(&gg->bar_count, 0u);
            vmem_drain();
            st_dev(&gg->bar_gen, s_gen + 1);
        }
    } else if (threadIdx.x == 0) {
        unsigned int spins = 0;
        while (ld_dev(&gg->bar_gen) == s_gen) {
            if (ld_dev(&gg->abort) || ++spins > SPIN_LIMIT) {
                __hip_atomic_fetch_or(&gg->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    return s_ok != 0;
}

__device__ __forceinline__ bool gang_barrier(Gang *gg, int G, int gb)
{
    return gang_barrier_then(gg, G, gb, [] {});
}

struct DotOut {
    double value;
    bool all_perf;  // qdot perforated every component of a nonzero vector
    bool ok;        // gang still healthy
};

// Shared-memory workspace of one block (CG and batched kernels).
struct CgLds {
    unsigned int h[W + 1];
    unsigned char lut[W_LUT];
    Acc red[3][BLOCK / 64];
    int4 scratch[BLOCK / 64];
    qdot_result res;
    double dval;
    double sval;  // S of the last qdot combine (units of 2^e_max)
};

// Pass 1 of qdot for one component pair, into the block's LDS histogram.
__device__ __forceinline__ void scan_pair(double a, double b, int key_mode, CgLds &L,
                                          unsigned int &nz, unsigned int &bad, unsigned int &sg)
{
    const Comp c = component(a, b, key_mode);
    nz += c.zero ? 1u : 0u;
    bad |= c.bad ? 1u : 0u;
    sg |= c.zero ? 0u : (c.sgn ? 1u : 2u);
    atomicAdd(&L.h[c.slot], 1u);
}

// a.b over the gang's rows by qdot (buffer k), value identical in every block.
// With `scanned` the caller has already put its rows' keys into L.h (while
// it produced a or b) and passes its zero count, non-finite flag and sign
// bits.  After the histogram merge each block copies the merged window into
// its LDS histogram (counts of one system fit 32 bits) and selects from
// there; the copy is cleared before returning.
//
// GUARD (guard_mode 1): after the combine every block evaluates the lower
// bound of Thm 3.4 from its copy of the histogram and its class table, and
// certifies the result or reselects against E_lo (or makes every bin
// double) and sums its rows again, into the other partials buffer (free:
// every block has read it in the previous inner product), then checks again
// with the larger lower bound: the steps and flags of the single-vector
// guaranteed mode, one more gang barrier when it reselects.
template <bool GUARD>
__device__ __forceinline__ DotOut gang_qdot(const double *a, const double *bv, int64_t n,
                                            int64_t r0, int64_t r1, double tol, int key_mode,
                                            int score_mode, int nonstrict, Gang *gg,
                                            int G, int gb, int k, CgLds &L,
                                            qdot_result *trace_slot, bool scanned = false,
                                            unsigned int nz = 0, unsigned int bad = 0,
                                            unsigned int sg = 0)
{
    DotOut o = {0.0, false, true};
    GangQ &Q = gg->qb[k];
    const bool vec = ((((uintptr_t)a) | ((uintptr_t)bv)) & 15) == 0;
    if (!scanned) {
        // pass 1 over own rows
        auto scan = [&](const double *xv, const double *yv, int64_t, int lim) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const Comp c = component(xv[e], yv[e], key_mode);
                const bool valid = e < lim;
                nz += (valid & c.zero) ? 1u : 0u;
                bad |= (valid & c.bad) ? 1u : 0u;
                sg |= (valid & !c.zero) ? (c.sgn ? 1u : 2u) : 0u;
                if (valid) atomicAdd(&L.h[c.slot], 1u);
            }
        };
        if (vec)
            stream_strided<true, 2>(a, bv, r0, 2 * CHUNK, r1, scan);
        else
            stream_strided<false, 2>(a, bv, r0, 2 * CHUNK, r1, scan);
    }
    __syncthreads();
    int lo = W, hi = -1;
    for (int j = threadIdx.x; j < W; j += BLOCK) {
        const unsigned int v = L.h[j];
        if (v) {
            __hip_atomic_fetch_add(&Q.hist[gb % GANG_HIST_COPIES][j], v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            L.h[j] = 0u;
            lo = min(lo, j);
            hi = max(hi, j);
        }
    }
    if (threadIdx.x == 0) L.h[W] = 0u;
    // the block's record, a plain write-through store: same-word atomics of
    // every block would queue at one address, and the wait for them before
    // the barrier would put that whole queue on every block's path
    unsigned int bs = (bad ? 1u : 0u) | (sg << 1);
    block_reduce_range(lo, hi, nz, bs, L.scratch);
    if (threadIdx.x == 0) {
        int *rec = &Q.rec[gb].x;
        st_dev(rec, lo);
        st_dev(rec + 1, hi);
        st_dev(rec + 2, (int)nz);
        st_dev(rec + 3, (int)bs);
    }
    // the last block to arrive reduces the gang's records (counts of one
    // system fit 32 bits), sums the histogram copies over the live window
    // into hm and clears the copies for the qdot after next
    auto merge = [&]() {
        int lo2 = W, hi2 = -1;
        unsigned int z2 = 0, bs2 = 0;
        for (int c = threadIdx.x; c < G; c += BLOCK) {
            const int *rec = &Q.rec[c].x;
            lo2 = min(lo2, ld_dev(rec));
            hi2 = max(hi2, ld_dev(rec + 1));
            z2 += (unsigned int)ld_dev(rec + 2);
            bs2 |= (unsigned int)ld_dev(rec + 3);
        }
        block_reduce_range(lo2, hi2, z2, bs2, L.scratch);
        const int ncopy = min(G, GANG_HIST_COPIES);
        for (int j = lo2 + (int)threadIdx.x; j <= hi2; j += BLOCK) {
            unsigned int v = 0u;
            for (int c = 0; c < ncopy; c++) {
                v += ld_dev(&Q.hist[c][j]);
                st_dev(&Q.hist[c][j], 0u);
            }
            st_dev(&Q.hm[j], v);
        }
        if (threadIdx.x == 0) {
            int *sm = &Q.sum.x;
            st_dev(sm, lo2);
            st_dev(sm + 1, hi2);
            st_dev(sm + 2, (int)z2);
            st_dev(sm + 3, (int)bs2);
        }
    };
    if (!gang_barrier_then(gg, G, gb, merge)) {
        o.ok = false;
        return o;
    }
    // the merged window into this block's LDS copy
    const int glo = ld_dev(&Q.sum.x);
    const int ghi = ld_dev(&Q.sum.y);
    const unsigned long long gnz = (unsigned int)ld_dev(&Q.sum.z);
    const unsigned int gbs = (unsigned int)ld_dev(&Q.sum.w);
    const unsigned int gbad = gbs & 1u;
    const unsigned int gsg = gbs >> 1;
    for (int j = glo + (int)threadIdx.x; j <= ghi; j += BLOCK) L.h[j] = ld_dev(&Q.hm[j]);
    __syncthreads();
    // cutoff, redundantly in every block, into the block's own class table
    auto get = [&](int j) { return (unsigned long long)L.h[j]; };
    auto put = [&](int j, int c) { L.lut[j] = (unsigned char)c; };
    auto noclear = [&](int) {};
    const CutParams p = block_cutoff<BLOCK>(glo, ghi, gnz, gbad, n, tol, score_mode, nonstrict,
                                            get, put, noclear, &L.res, nullptr);
    // pass 2 over own rows into partials buffer kp, combine in every block
    auto sweep = [&](const CutParams &cp, int kp, int flags) -> bool {
        Acc acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        auto body = [&](const double *xv, const double *yv, int64_t, int lim) {
            acc_group<false>(xv, yv, lim, L.lut, key_mode, cp.e_max, cp.c32, true, acc[0],
                             acc[1], acc[2], nullptr);
        };
        if (vec)
            stream_strided<true, 2>(a, bv, r0, 2 * CHUNK, r1, body);
        else
            stream_strided<false, 2>(a, bv, r0, 2 * CHUNK, r1, body);
        block_reduce3<BLOCK>(acc, L.red);
        if (threadIdx.x == 0) {
            double *pp = gg->partials[kp] + gb * 6;
            for (int q = 0; q < 3; q++) {
                st_dev(&pp[2 * q], acc[q].s);
                st_dev(&pp[2 * q + 1], acc[q].c);
            }
        }
        // the last block to arrive combines the gang's partials in block
        // order; every block then finishes from the same six words
        auto combine = [&]() {
            Acc f[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
            for (int c = threadIdx.x; c < G; c += BLOCK) {
                const double *pp = gg->partials[kp] + c * 6;
                for (int q = 0; q < 3; q++)
                    f[q] = acc_merge(f[q], Acc{ld_dev(&pp[2 * q]), ld_dev(&pp[2 * q + 1])});
            }
            block_reduce3<BLOCK>(f, L.red);
            if (threadIdx.x == 0)
                for (int q = 0; q < 3; q++) {
                    st_dev(&gg->pfin[kp][2 * q], f[q].s);
                    st_dev(&gg->pfin[kp][2 * q + 1], f[q].c);
                }
        };
        if (!gang_barrier_then(gg, G, gb, combine)) return false;
        if (threadIdx.x == 0) {
            Acc f[3];
            for (int q = 0; q < 3; q++)
                f[q] = Acc{ld_dev(&gg->pfin[kp][2 * q]), ld_dev(&gg->pfin[kp][2 * q + 1])};
            L.sval = combine_value(f, cp.e_max, cp.c32, flags, &L.res);
        }
        return true;
    };
    if (threadIdx.x == 0) L.sval = 0.0;
    if (!p.skip) {
        if (!sweep(p, k, p.flags)) {
            o.ok = false;
            return o;
        }
    } else if (!gang_barrier(gg, G, gb)) {
        o.ok = false;
        return o;
    }
    __syncthreads();
    if constexpr (GUARD) {
        __shared__ int s_go, s_dref, s_passes;
        __shared__ double s_low;
        if (threadIdx.x == 0) {
            s_go = L.res.status == QDOT_OK && L.res.n_bins > 0;
            // every product zero: +0 is exact
            if (L.res.status == QDOT_OK && L.res.n_bins == 0) L.res.flags |= QDOT_F_GUARANTEED;
            s_dref = 0;
            s_passes = L.res.passes;
        }
        __syncthreads();
        if (s_go) {
            const int e_max = L.res.e_max;
            const GuardSums g0 = guard_sums<BLOCK>(get, L.lut, glo, ghi, e_max);
            if (threadIdx.x == 0) {
                const double low = guard_lower(g0, L.sval, n, gsg);
                if (guard_certified(L.res.bound_rel, low, tol)) {
                    L.res.flags |= QDOT_F_GUARANTEED;
                    L.res.lower = ldexp(low, e_max);
                } else {
                    // L <= 0: every bin double (scores >= 23, one more
                    // non-strict)
                    const int ref = low > 0.0 ? e_max + ilogb(low)
                                              : L.res.e_min - L.res.t - 22 - nonstrict;
                    if (ref < e_max) {
                        s_dref = e_max - ref;
                        s_low = low;
                    } else {
                        L.res.lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
                    }
                }
            }
            __syncthreads();
            if (s_dref) {
                // reselection against e_ref = e_max - dref, second sweep
                const CutParams p2 = block_cutoff<BLOCK>(glo, ghi, gnz, 0u, n, tol, score_mode,
                                                         nonstrict, get, put, noclear, &L.res,
                                                         nullptr, s_dref);
                if (threadIdx.x == 0) {
                    L.res.flags |= QDOT_F_RESELECTED;
                    L.res.passes = s_passes + (p2.skip ? 0 : 1);
                    L.sval = 0.0;
                }
                if (!p2.skip && !sweep(p2, k ^ 1, p2.flags | QDOT_F_RESELECTED)) {
                    o.ok = false;
                    return o;
                }
                __syncthreads();
                const GuardSums g1 = guard_sums<BLOCK>(get, L.lut, glo, ghi, e_max);
                if (threadIdx.x == 0) {
                    const double low = fmax(guard_lower(g1, L.sval, n, gsg), s_low);
                    L.res.flags |= QDOT_F_RESELECTED |
                                   (guard_certified(L.res.bound_rel, low, tol) ? QDOT_F_GUARANTEED
                                                                               : 0);
                    L.res.lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
                }
            }
        }
        __syncthreads();
    }
    o.value = L.res.value;
    o.all_perf = (L.res.flags & QDOT_F_ALL_PERF) && L.res.n_bins > 0;
    if (threadIdx.x == 0 && trace_slot) *trace_slot = L.res;
    // the LDS copy of the histogram back to zero for the next scan
    for (int j = glo + (int)threadIdx.x; j <= ghi; j += BLOCK) L.h[j] = 0u;
    __syncthreads();
    return o;
}

// a.b over the gang's rows by the one-pass qdot (accum_mode 1, value as the
// exact sum of the kept leaves), buffer k, value identical in every block.
// Each block reads its rows once: keys into its LDS histogram and, for the
// bins within `depth` of its running maximum, the candidate sums of every
// precision into its LDS window (s1_stream), which it adds into the gang's
// table `tab` (W x S1_PIECES sums, exact in any order, zero between calls).
// The last block to arrive at the one barrier merges the records and the
// histogram copies, selects, picks each kept bin's sum from the table,
// clears the copies and the table over the live window and publishes the
// result; the others read it.  No class table or second sweep is needed
// outside that block, so an inner product costs one gang barrier.
__device__ __forceinline__ DotOut gang_qdot_s1(const double *a, const double *bv, int64_t n,
                                               int64_t r0, int64_t r1, double tol, int key_mode,
                                               int score_mode, int nonstrict, Gang *gg, int G,
                                               int gb, int k, CgLds &L, S1Lds &S1, double *tab,
                                               qdot_result *trace_slot)
{
    DotOut o = {0.0, false, true};
    GangQ &Q = gg->qb[k];
    const bool vec = ((((uintptr_t)a) | ((uintptr_t)bv)) & 15) == 0;
    // admitted by the host: depth <= S1_WIN
    const int depth = s1_depth_dev(n, tol, score_mode);
    unsigned int nz = 0, bad = 0;
    S1Run run = s1_run_start();
    s1_begin(S1);
    __syncthreads();
    if (r1 > r0) {
        if (vec)
            s1_stream<true, 2>(a + r0, bv + r0, 0, 2 * CHUNK, r1 - r0, key_mode, depth, L.h, S1,
                               run, nz, bad);
        else
            s1_stream<false, 2>(a + r0, bv + r0, 0, 2 * CHUNK, r1 - r0, key_mode, depth, L.h,
                                S1, run, nz, bad);
    }
    const int top = run.top;
    __syncthreads();
    int lo = W, hi = -1;
    for (int j = threadIdx.x; j < W; j += BLOCK) {
        const unsigned int v = L.h[j];
        if (v) {
            __hip_atomic_fetch_add(&Q.hist[gb % GANG_HIST_COPIES][j], v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            L.h[j] = 0u;
            lo = min(lo, j);
            hi = max(hi, j);
        }
    }
    if (threadIdx.x == 0) L.h[W] = 0u;
    if (top >= 0)
        for (int i = threadIdx.x; i < depth * S1_PIECES; i += BLOCK) {
            const int bin = top - i / S1_PIECES;
            if (bin < 0) continue;
            const double v = S1.win[bin & (S1_WIN - 1)][i % S1_PIECES];
            if (v != 0.0)
                __hip_atomic_fetch_add(&tab[(size_t)bin * S1_PIECES + i % S1_PIECES], v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    unsigned int bs = bad ? 1u : 0u;
    block_reduce_range(lo, hi, nz, bs, L.scratch);
    if (threadIdx.x == 0) {
        int *rec = &Q.rec[gb].x;
        st_dev(rec, lo);
        st_dev(rec + 1, hi);
        st_dev(rec + 2, (int)nz);
        st_dev(rec + 3, (int)bs);
    }
    auto finish = [&]() {
        int lo2 = W, hi2 = -1;
        unsigned int z2 = 0, bs2 = 0;
        for (int c = threadIdx.x; c < G; c += BLOCK) {
            const int *rec = &Q.rec[c].x;
            lo2 = min(lo2, ld_dev(rec));
            hi2 = max(hi2, ld_dev(rec + 1));
            z2 += (unsigned int)ld_dev(rec + 2);
            bs2 |= (unsigned int)ld_dev(rec + 3);
        }
        block_reduce_range(lo2, hi2, z2, bs2, L.scratch);
        const int ncopy = min(G, GANG_HIST_COPIES);
        for (int j = lo2 + (int)threadIdx.x; j <= hi2; j += BLOCK) {
            unsigned int v = 0u;
            for (int c = 0; c < ncopy; c++) {
                v += ld_dev(&Q.hist[c][j]);
                st_dev(&Q.hist[c][j], 0u);
            }
            L.h[j] = v;
        }
        __syncthreads();
        auto get = [&](int j) { return (unsigned long long)L.h[j]; };
        auto put = [&](int j, int c) { L.lut[j] = (unsigned char)c; };
        auto noclear = [&](int) {};
        const CutParams p = block_cutoff<BLOCK>(lo2, hi2, z2, bs2 & 1u, n, tol, score_mode,
                                                nonstrict, get, put, noclear, &L.res, nullptr);
        if (!p.skip)
            s1_pick(p.e_max, max(lo2, p.e_max - KMIN - depth + 1), p.flags, L.lut,
                    [&](int bin, int q) { return ld_dev(&tab[(size_t)bin * S1_PIECES + q]); },
                    L.red, &L.res);
        __syncthreads();
        // the table and the LDS copy back to zero over the live window
        if (hi2 >= lo2) {
            for (int i = lo2 * S1_PIECES + (int)threadIdx.x; i < (hi2 + 1) * S1_PIECES;
                 i += BLOCK)
                st_dev(&tab[i], 0.0);
            for (int j = lo2 + (int)threadIdx.x; j <= hi2; j += BLOCK) L.h[j] = 0u;
        }
        constexpr int NWORD = (int)(sizeof(qdot_result) / sizeof(unsigned long long));
        if (threadIdx.x < NWORD)
            st_dev(reinterpret_cast<unsigned long long *>(&gg->res[k]) + threadIdx.x,
                   reinterpret_cast<const unsigned long long *>(&L.res)[threadIdx.x]);
    };
    if (!gang_barrier_then(gg, G, gb, finish)) {
        o.ok = false;
        return o;
    }
    constexpr int NWORD = (int)(sizeof(qdot_result) / sizeof(unsigned long long));
    if (threadIdx.x < NWORD)
        reinterpret_cast<unsigned long long *>(&L.res)[threadIdx.x] =
            ld_dev(reinterpret_cast<const unsigned long long *>(&gg->res[k]) + threadIdx.x);
    __syncthreads();
    o.value = L.res.value;
    o.all_perf = (L.res.flags & QDOT_F_ALL_PERF) && L.res.n_bins > 0;
    if (threadIdx.x == 0 && trace_slot) *trace_slot = L.res;
    __syncthreads();
    return o;
}

// a.b over the gang's rows in plain FP64 (partials buffer k).
__device__ __forceinline__ DotOut gang_dot64(const double *a, const double *bv, int64_t r0, int64_t r1, Gang *gg,
                             int G, int gb, int k, CgLds &L)
{
    DotOut o = {0.0, false, true};
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = r0 + threadIdx.x;
    for (; i + 3 * BLOCK < r1; i += 4 * BLOCK) {
#pragma unroll
        for (int u = 0; u < 4; u++) s[u] = fma(a[i + u * BLOCK], bv[i + u * BLOCK], s[u]);
    }
    for (; i < r1; i += BLOCK) s[0] = fma(a[i], bv[i], s[0]);
    Acc acc[3] = {{(s[0] + s[1]) + (s[2] + s[3]), 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    block_reduce3<BLOCK>(acc, L.red);
    if (threadIdx.x == 0) st_dev(&gg->partials[k][gb * 6], acc[0].s + acc[0].c);
    if (!gang_barrier(gg, G, gb)) {
        o.ok = false;
        return o;
    }
    // every block sums the gang's partials in the same fixed order (thread
    // c loads partial c, then a fixed tree), so all hold the same value
    double v = 0.0;
    for (int c = threadIdx.x; c < G; c += BLOCK) v += ld_dev(&gg->partials[k][c * 6]);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) L.red[0][threadIdx.x >> 6].s = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double f = L.red[0][0].s;
        for (int w = 1; w < BLOCK / 64; w++) f += L.red[0][w].s;
        L.dval = f;
    }
    __syncthreads();
    o.value = L.dval;
    __syncthreads();
    return o;
}

// out[i] = sum_j val[j] * v[col[j]] over rows [r0, r1), each row summed in
// column-storage order (plain multiply, then add).  v may hold entries that
// other blocks wrote in this launch, so it is read with device-scope loads.
// A thread takes SR rows at once and issues the column and value loads of
// their first SNZ entries, then every gather, before it adds: two memory
// latencies per SR rows instead of two per entry.  Longer rows finish in a
// plain loop.
constexpr int SR = 2;
constexpr int SNZ = 8;
// With SCAN the row result is also keyed against v's own entry (pass 1 of
// the qdot v . out that follows, fused here so that v and out are not read
// again for it).
template <bool SCAN = false>
__device__ __forceinline__ void spmv_rows(const CgSys &S, const double *v, double *out, int64_t r0,
                                          int64_t r1, int key_mode = 0, CgLds *L = nullptr,
                                          unsigned int *nz = nullptr, unsigned int *bad = nullptr,
                                          unsigned int *sg = nullptr)
{
    for (int64_t base = r0; base < r1; base += (int64_t)SR * BLOCK) {
        int32_t beg[SR], len[SR];
#pragma unroll
        for (int u = 0; u < SR; u++) {
            const int64_t i = base + u * BLOCK + threadIdx.x;
            beg[u] = 0;
            len[u] = 0;
            if (i < r1) {
                beg[u] = S.rowptr[i];
                len[u] = S.rowptr[i + 1] - beg[u];
            }
        }
        int32_t ci[SR][SNZ];
        double pv[SR][SNZ];
#pragma unroll
        for (int u = 0; u < SR; u++)
#pragma unroll
            for (int jj = 0; jj < SNZ; jj++) {
                ci[u][jj] = 0;
                pv[u][jj] = 0.0;
                if (jj < len[u]) {
                    ci[u][jj] = S.col[beg[u] + jj];
                    pv[u][jj] = S.val[beg[u] + jj];
                }
            }
#pragma unroll
        for (int u = 0; u < SR; u++)
#pragma unroll
            for (int jj = 0; jj < SNZ; jj++)
                if (jj < len[u]) pv[u][jj] = pv[u][jj] * ld_dev(&v[ci[u][jj]]);
#pragma unroll
        for (int u = 0; u < SR; u++) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < SNZ; jj++)
                if (jj < len[u]) s = s + pv[u][jj];
            for (int32_t j = beg[u] + SNZ; j < beg[u] + len[u]; j++) {
                const double pr = S.val[j] * ld_dev(&v[S.col[j]]);
                s = s + pr;
            }
            const int64_t i = base + u * BLOCK + threadIdx.x;
            if (i < r1) {
                out[i] = s;
                if (SCAN) scan_pair(v[i], s, key_mode, *L, *nz, *bad, *sg);
            }
        }
    }
}

// One CG solve by one gang.
// ACC1: every inner product by the one-pass qdot (gang_qdot_s1, with the
// caller's LDS window S1 and the gang's table tab, 2 W S1_PIECES doubles);
// otherwise by the two-pass qdot, guaranteed with GUARD.
template <bool GUARD, bool ACC1 = false>
__device__ __forceinline__ void cg_solve(const CgSys &S, Gang *gg, int G, int gb, int key_mode,
                                         int score_mode, int nonstrict, CgLds &L,
                                         qdot_cg_result *res, S1Lds *S1 = nullptr,
                                         double *tab = nullptr)
{
    const int64_t n = S.n;
    // rows of this block: a multiple of CHUNK each, so qdot tiles line up
    const int64_t per = ((n + G - 1) / G + CHUNK - 1) / CHUNK * CHUNK;
    const int64_t r0 = min(n, (int64_t)gb * per), r1 = min(n, r0 + per);
    int k = 0;  // qdot buffer / partials parity
    int ntr = 0;
    auto dot = [&](const double *a, const double *bv, bool scanned = false, unsigned int nz = 0,
                   unsigned int bad = 0, unsigned int sg = 0) {
        DotOut o;
        if (S.use_qdot) {
            qdot_result *ts = (gb == 0 && S.trace) ? S.trace + ntr : nullptr;
            if constexpr (ACC1)
                o = gang_qdot_s1(a, bv, n, r0, r1, S.qtol, key_mode, score_mode, nonstrict, gg,
                                 G, gb, k, L, *S1, tab + (size_t)k * W * S1_PIECES, ts);
            else
                o = gang_qdot<GUARD>(a, bv, n, r0, r1, S.qtol, key_mode, score_mode, nonstrict,
                                     gg, G, gb, k, L, ts, scanned, nz, bad, sg);
            ntr++;
        } else {
            o = gang_dot64(a, bv, r0, r1, gg, G, gb, k, L);
        }
        k ^= 1;
        return o;
    };
    int status = QDOT_OK, iters = 0;
    bool healthy = true;
    // r0 = b - A x0, p0 = r0
    spmv_rows(S, S.x, S.q, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) {
        const double v = S.b[i] - S.q[i];
        S.r[i] = v;
        st_dev(&S.p[i], v);
    }
    __syncthreads();
    DotOut bb = gang_dot64(S.b, S.b, r0, r1, gg, G, gb, k, L);
    k ^= 1;
    const double bnorm = sqrt(bb.value);
    const double thresh = S.rtol * bnorm;
    DotOut c0 = dot(S.r, S.r);
    healthy = bb.ok && c0.ok;
    double c = c0.value;
    bool done = false;
    if (healthy && c0.all_perf) {
        status = QDOT_E_BREAKDOWN;
        done = true;
    } else if (healthy && !(sqrt(c) > thresh)) {
        done = true;
    }
    while (healthy && !done) {
        if (iters >= S.maxit) {
            status = QDOT_E_MAXIT;
            break;
        }
        if (!(healthy = gang_barrier(gg, G, gb))) break;  // p complete
        // pass 1 of the two-pass qdot(p, q) rides in the SpMV; the one-pass
        // qdot reads its rows itself
        const bool scan_q = S.use_qdot != 0 && !ACC1;
        unsigned int nz1 = 0, bad1 = 0, sg1 = 0;
        if (scan_q)
            spmv_rows<true>(S, S.p, S.q, r0, r1, key_mode, &L, &nz1, &bad1, &sg1);
        else
            spmv_rows(S, S.p, S.q, r0, r1);
        __syncthreads();
        const DotOut d = dot(S.p, S.q, scan_q, nz1, bad1, sg1);
        if (!(healthy = d.ok)) break;
        if (!(d.value > 0.0) || !isfinite(d.value) || d.all_perf) {
            status = QDOT_E_BREAKDOWN;
            break;
        }
        const double alpha = c / d.value;
        // x += alpha p, r -= alpha q (four rows' loads in flight per thread),
        // with pass 1 of the qdot r . r that follows fused in
        unsigned int nz2 = 0, bad2 = 0, sg2 = 0;
        const bool scan_r = S.use_qdot != 0 && !ACC1;
        auto xr_row = [&](int64_t i, double pi, double xi, double qi, double ri) {
            const double ap = alpha * pi;
            st_dev(&S.x[i], xi + ap);
            const double aq = alpha * qi;
            const double rn = ri - aq;
            S.r[i] = rn;
            if (scan_r) scan_pair(rn, rn, key_mode, L, nz2, bad2, sg2);
        };
        {
            int64_t i = r0 + threadIdx.x;
            for (; i + 3 * BLOCK < r1; i += 4 * BLOCK) {
                double pi[4], xi[4], qi[4], ri[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    pi[u] = S.p[i + u * BLOCK];
                    xi[u] = S.x[i + u * BLOCK];
                    qi[u] = S.q[i + u * BLOCK];
                    ri[u] = S.r[i + u * BLOCK];
                }
#pragma unroll
                for (int u = 0; u < 4; u++) xr_row(i + u * BLOCK, pi[u], xi[u], qi[u], ri[u]);
            }
            for (; i < r1; i += BLOCK) xr_row(i, S.p[i], S.x[i], S.q[i], S.r[i]);
        }
        __syncthreads();
        const DotOut cn = dot(S.r, S.r, scan_r, nz2, bad2, sg2);
        if (!(healthy = cn.ok)) break;
        if (cn.all_perf) {
            status = QDOT_E_BREAKDOWN;
            break;
        }
        const double beta = cn.value / c;
        // p = r + beta p (four rows' loads in flight per thread)
        {
            int64_t i = r0 + threadIdx.x;
            for (; i + 3 * BLOCK < r1; i += 4 * BLOCK) {
                double pi[4], ri[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    pi[u] = S.p[i + u * BLOCK];
                    ri[u] = S.r[i + u * BLOCK];
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const double bp = beta * pi[u];
                    st_dev(&S.p[i + u * BLOCK], ri[u] + bp);
                }
            }
            for (; i < r1; i += BLOCK) {
                const double bp = beta * S.p[i];
                st_dev(&S.p[i], S.r[i] + bp);
            }
        }
        c = cn.value;
        iters++;
        if (!(sqrt(c) > thresh)) done = true;
    }
    double relres_true = 0.0;
    if (healthy) healthy = gang_barrier(gg, G, gb);  // x complete
    if (healthy) {
        spmv_rows(S, S.x, S.q, r0, r1);
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) S.q[i] = S.b[i] - S.q[i];
        __syncthreads();
        const DotOut rq = gang_dot64(S.q, S.q, r0, r1, gg, G, gb, k, L);
        k ^= 1;
        healthy = rq.ok;
        relres_true = bnorm > 0.0 ? sqrt(rq.value) / bnorm : 0.0;
    }
    if (gb == 0 && threadIdx.x == 0) {
        res->iters = iters;
        res->status = healthy ? status : QDOT_E_DEVICE;
        res->relres_est = bnorm > 0.0 ? sqrt(c) / bnorm : 0.0;
        res->relres_true = relres_true;
    }
    // leave the gang buffers clean and every block past its last use of them
    if (healthy) gang_barrier(gg, G, gb);
}

// Clears a gang's barrier, abort flag and histogram buffers (plain stores;
// used by a kernel of its own, before the launch that uses the gang).
__device__ __forceinline__ void gang_reset(Gang *gg)
{
    for (int i = threadIdx.x; i < W; i += blockDim.x) {
        for (int c = 0; c < GANG_HIST_COPIES; c++) {
            gg->qb[0].hist[c][i] = 0u;
            gg->qb[1].hist[c][i] = 0u;
        }
    }
    if (threadIdx.x < BAR_GROUPS) gg->bar_sub[threadIdx.x][0] = 0u;
    if (threadIdx.x == 0) {
        gg->bar_count = 0;
        gg->abort = 0;
    }
}

}  // namespace qd
