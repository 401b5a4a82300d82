// Conjugate gradient (Alg. 4) on the device in one persistent launch.
//
// A gang of G blocks solves one system; block b of the gang owns a
// contiguous slice of rows and every vector update, SpMV row and qdot pass
// on that slice.  Gang barriers (an arrival counter and a generation word)
// separate the steps that need data from other slices:
//   before the SpMV (p complete), after a qdot's pass 1 (histogram merged),
//   after its pass 2 (partials written),
// five per iteration.  Between those barriers every block computes the
// cutoff and the final combine of each qdot itself, from the same merged
// histogram and the same partials in the same order, so every block holds
// bit-identical scalars (alpha, beta, c) and takes the same branches: the
// gang never needs to broadcast a decision.  Two histogram buffers rotate so
// that block 0 can clear the one just used without an extra barrier.
//
// Every wait is bounded: a barrier that does not complete within the spin
// limit raises the gang's abort flag, every block leaves, and the call
// reports QDOT_E_DEVICE.  The grid never exceeds one block per CU per gang
// slot, so all blocks of a gang are resident together.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "qdot_blocks.hpp"
#include "qdot_handle.hpp"

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
    qdot_cg_result *res; // device result of this system
};

struct GangQ {  // per gang and qdot buffer
    unsigned int hist[W];
    int lo, hi;
    unsigned long long n_zero;
    unsigned int bad;
    unsigned int pad;
};

struct Gang {
    unsigned int bar_count;
    unsigned int bar_gen;
    unsigned int abort;
    unsigned int pad;
    GangQ qb[2];
    double partials[2][256 * 6];  // up to MAX_GANG blocks per gang
};

constexpr int MAX_GANG = 256;

// ---------------------------------------------------------------------------
__device__ bool gang_barrier(Gang *gg, int G)
{
    __shared__ int s_ok;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned int gen =
            __hip_atomic_load(&gg->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int arrived =
            __hip_atomic_fetch_add(&gg->bar_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (arrived == (unsigned)G) {
            __hip_atomic_store(&gg->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&gg->bar_gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // poll with relaxed loads (an acquire load would invalidate the
            // XCD's L2 on every poll); one acquire fence follows the barrier
            unsigned int spins = 0;
            while (__hip_atomic_load(&gg->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&gg->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    ++spins > SPIN_LIMIT) {
                    __hip_atomic_fetch_or(&gg->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return s_ok != 0;
}

struct DotOut {
    double value;
    bool all_perf;  // qdot perforated every component of a nonzero vector
    bool ok;        // gang still healthy
};

// Shared-memory workspace of one block of the CG kernel.
struct CgLds {
    unsigned int h[W + 1];
    unsigned char lut[W_LUT];
    Acc red[3][BLOCK / 64];
    int4 scratch[BLOCK / 64];
    qdot_result res;
    double dval;
};

__device__ __forceinline__ void block_range_reduce(int &lo, int &hi, unsigned int &nz,
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

// a.b over the gang's rows by qdot (buffer k), value identical in every block.
__device__ __noinline__ DotOut gang_qdot(const double *a, const double *bv, int64_t n, int64_t r0, int64_t r1,
                            double tol, int key_mode, int score_mode, int nonstrict, Gang *gg,
                            int G, int gb, int k, CgLds &L, qdot_result *trace_slot)
{
    DotOut o = {0.0, false, true};
    GangQ &Q = gg->qb[k];
    const bool vec = ((((uintptr_t)a) | ((uintptr_t)bv)) & 15) == 0;
    // pass 1 over own rows
    unsigned int nz = 0, bad = 0;
    auto scan = [&](const double *xv, const double *yv, int64_t, int lim) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const Comp c = component(xv[e], yv[e], key_mode);
            const bool valid = e < lim;
            nz += (valid & c.zero) ? 1u : 0u;
            bad |= (valid & c.bad) ? 1u : 0u;
            if (valid) atomicAdd(&L.h[c.slot], 1u);
        }
    };
    if (vec)
        stream_block_range<true>(a, bv, r0, r1, scan);
    else
        stream_block_range<false>(a, bv, r0, r1, scan);
    __syncthreads();
    int lo = W, hi = -1;
    for (int j = threadIdx.x; j < W; j += BLOCK) {
        const unsigned int v = L.h[j];
        if (v) {
            atomicAdd(&Q.hist[j], v);
            L.h[j] = 0u;
            lo = min(lo, j);
            hi = max(hi, j);
        }
    }
    if (threadIdx.x == 0) L.h[W] = 0u;
    block_range_reduce(lo, hi, nz, bad, L.scratch);
    if (threadIdx.x == 0) {
        if (hi >= 0) {
            atomicMin(&Q.lo, lo);
            atomicMax(&Q.hi, hi);
        }
        if (nz) atomicAdd(&Q.n_zero, (unsigned long long)nz);
        if (bad) atomicOr(&Q.bad, 1u);
    }
    if (!gang_barrier(gg, G)) {
        o.ok = false;
        return o;
    }
    // cutoff, redundantly in every block, into the block's own class table
    const int glo = __hip_atomic_load(&Q.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int ghi = __hip_atomic_load(&Q.hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long gnz =
        __hip_atomic_load(&Q.n_zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int gbad = __hip_atomic_load(&Q.bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    auto get = [&](int j) {
        return (unsigned long long)__hip_atomic_load(&Q.hist[j], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    };
    auto put = [&](int j, int c) { L.lut[j] = (unsigned char)c; };
    auto noclear = [&](int) {};
    const CutParams p = block_cutoff<BLOCK>(glo, ghi, gnz, gbad, n, tol, score_mode, nonstrict,
                                            get, put, noclear, &L.res, nullptr);
    // pass 2 over own rows
    if (!p.skip) {
        Acc acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        auto body = [&](const double *xv, const double *yv, int64_t, int lim) {
            acc_group<false>(xv, yv, lim, L.lut, key_mode, p.e_max, p.c32, true, acc[0], acc[1],
                             acc[2], nullptr);
        };
        if (vec)
            stream_block_range<true>(a, bv, r0, r1, body);
        else
            stream_block_range<false>(a, bv, r0, r1, body);
        block_reduce3<BLOCK>(acc, L.red);
        if (threadIdx.x == 0) {
            double *pp = gg->partials[k] + gb * 6;
            for (int q = 0; q < 3; q++) {
                pp[2 * q] = acc[q].s;
                pp[2 * q + 1] = acc[q].c;
            }
        }
    }
    if (!gang_barrier(gg, G)) {
        o.ok = false;
        return o;
    }
    if (!p.skip) {
        // combine the gang's partials in block order, in every block
        Acc acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        for (int c = threadIdx.x; c < G; c += BLOCK) {
            const double *pp = gg->partials[k] + c * 6;
            for (int q = 0; q < 3; q++) acc[q] = acc_merge(acc[q], Acc{pp[2 * q], pp[2 * q + 1]});
        }
        block_reduce3<BLOCK>(acc, L.red);
        if (threadIdx.x == 0) combine_value(acc, p.e_max, p.t, p.c32, p.flags, &L.res);
    }
    __syncthreads();
    o.value = L.res.value;
    o.all_perf = (L.res.flags & QDOT_F_ALL_PERF) && L.res.n_bins > 0;
    if (threadIdx.x == 0 && trace_slot) *trace_slot = L.res;
    // block 0 clears this buffer for the qdot after next; every block has
    // finished reading it (it passed the barrier above after its cutoff)
    if (gb == 0) {
        for (int j = glo + (int)threadIdx.x; j <= ghi; j += BLOCK) Q.hist[j] = 0u;
        if (threadIdx.x == 0) {
            Q.lo = W;
            Q.hi = -1;
            Q.n_zero = 0;
            Q.bad = 0;
        }
    }
    __syncthreads();
    return o;
}

// a.b over the gang's rows in plain FP64 (partials buffer k).
__device__ __noinline__ DotOut gang_dot64(const double *a, const double *bv, int64_t r0, int64_t r1, Gang *gg,
                             int G, int gb, int k, CgLds &L)
{
    DotOut o = {0.0, false, true};
    double s = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) s = fma(a[i], bv[i], s);
    Acc acc[3] = {{s, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    block_reduce3<BLOCK>(acc, L.red);
    if (threadIdx.x == 0) gg->partials[k][gb * 6] = acc[0].s + acc[0].c;
    if (!gang_barrier(gg, G)) {
        o.ok = false;
        return o;
    }
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int c = 0; c < G; c++) v += gg->partials[k][c * 6];
        L.dval = v;
    }
    __syncthreads();
    o.value = L.dval;
    __syncthreads();
    return o;
}

__device__ __forceinline__ void spmv_rows(const CgSys &S, const double *v, double *out, int64_t r0,
                                          int64_t r1)
{
    for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) {
        double s = 0.0;
        for (int32_t j = S.rowptr[i]; j < S.rowptr[i + 1]; j++) {
            const double pr = S.val[j] * v[S.col[j]];
            s = s + pr;
        }
        out[i] = s;
    }
}

// One CG solve by one gang.
__device__ void cg_solve(const CgSys &S, Gang *gg, int G, int gb, int key_mode, int score_mode,
                         int nonstrict, CgLds &L)
{
    const int64_t n = S.n;
    // rows of this block: a multiple of CHUNK each, so qdot tiles line up
    const int64_t per = ((n + G - 1) / G + CHUNK - 1) / CHUNK * CHUNK;
    const int64_t r0 = min(n, (int64_t)gb * per), r1 = min(n, r0 + per);
    int k = 0;  // qdot buffer / partials parity
    int ntr = 0;
    auto dot = [&](const double *a, const double *bv) {
        DotOut o;
        if (S.use_qdot) {
            o = gang_qdot(a, bv, n, r0, r1, S.qtol, key_mode, score_mode, nonstrict, gg, G, gb, k,
                          L, (gb == 0 && S.trace) ? S.trace + ntr : nullptr);
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
        S.p[i] = v;
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
        if (!(healthy = gang_barrier(gg, G))) break;  // p complete
        spmv_rows(S, S.p, S.q, r0, r1);
        __syncthreads();
        const DotOut d = dot(S.p, S.q);
        if (!(healthy = d.ok)) break;
        if (!(d.value > 0.0) || !isfinite(d.value) || d.all_perf) {
            status = QDOT_E_BREAKDOWN;
            break;
        }
        const double alpha = c / d.value;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) {
            const double ap = alpha * S.p[i];
            S.x[i] = S.x[i] + ap;
            const double aq = alpha * S.q[i];
            S.r[i] = S.r[i] - aq;
        }
        __syncthreads();
        const DotOut cn = dot(S.r, S.r);
        if (!(healthy = cn.ok)) break;
        if (cn.all_perf) {
            status = QDOT_E_BREAKDOWN;
            break;
        }
        const double beta = cn.value / c;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) {
            const double bp = beta * S.p[i];
            S.p[i] = S.r[i] + bp;
        }
        c = cn.value;
        iters++;
        if (!(sqrt(c) > thresh)) done = true;
    }
    double relres_true = 0.0;
    if (healthy) healthy = gang_barrier(gg, G);  // x complete
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
        S.res->iters = iters;
        S.res->status = healthy ? status : QDOT_E_DEVICE;
        S.res->relres_est = bnorm > 0.0 ? sqrt(c) / bnorm : 0.0;
        S.res->relres_true = relres_true;
    }
    // leave the gang buffers clean and every block past its last use of them
    if (healthy) gang_barrier(gg, G);
}

__global__ __launch_bounds__(BLOCK) void k_cg_gangs(const CgSys *__restrict__ sys,
                                                    const int *__restrict__ gang_sys,
                                                    const int *__restrict__ gang_sys_off,
                                                    Gang *__restrict__ gangs, int G,
                                                    int key_mode, int score_mode, int nonstrict)
{
    __shared__ CgLds L;
    for (int i = threadIdx.x; i < W + 1; i += BLOCK) L.h[i] = 0u;
    for (int i = W + threadIdx.x; i < W_LUT; i += BLOCK) L.lut[i] = (unsigned char)QDOT_PERF;
    __syncthreads();
    const int g = blockIdx.x / G, gb = blockIdx.x % G;
    Gang *gg = gangs + g;
    for (int s = gang_sys_off[g]; s < gang_sys_off[g + 1]; s++) {
        cg_solve(sys[gang_sys[s]], gg, G, gb, key_mode, score_mode, nonstrict, L);
        if (__hip_atomic_load(&gg->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
}

__global__ void k_gang_init(Gang *gangs, int n)
{
    const int g = blockIdx.x;
    if (g >= n) return;
    Gang *gg = gangs + g;
    for (int i = threadIdx.x; i < W; i += blockDim.x) {
        gg->qb[0].hist[i] = 0u;
        gg->qb[1].hist[i] = 0u;
    }
    if (threadIdx.x == 0) {
        gg->bar_count = 0;
        gg->bar_gen = 0;
        gg->abort = 0;
        for (int k = 0; k < 2; k++) {
            gg->qb[k].lo = W;
            gg->qb[k].hi = -1;
            gg->qb[k].n_zero = 0;
            gg->qb[k].bad = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct CgDev {
    CgSys *sys = nullptr;
    int *gsys = nullptr;
    Gang *gangs = nullptr;
    qdot_cg_result *res = nullptr;
    int n_gangs = 0, n_sys = 0;
};

int32_t ensure_cg_buffers(qdot_handle *h, int n_sys, int n_gangs)
{
    CgDev *d = (CgDev *)h->cg;
    if (!d) {
        d = new CgDev();
        h->cg = d;
    }
    if (d->n_sys < n_sys) {
        (void)hipFree(d->sys);
        (void)hipFree(d->gsys);
        (void)hipFree(d->res);
        d->sys = nullptr;
        d->gsys = nullptr;
        d->res = nullptr;
        d->n_sys = 0;
        if (hipMalloc((void **)&d->sys, sizeof(CgSys) * n_sys) != hipSuccess ||
            hipMalloc((void **)&d->gsys, sizeof(int) * (2 * n_sys + 2 * n_gangs + 2)) != hipSuccess ||
            hipMalloc((void **)&d->res, sizeof(qdot_cg_result) * n_sys) != hipSuccess)
            return fail(h, QDOT_E_NOMEM, "CG buffers");
        d->n_sys = n_sys;
    }
    if (d->n_gangs < n_gangs) {
        (void)hipFree(d->gangs);
        d->gangs = nullptr;
        d->n_gangs = 0;
        if (hipMalloc((void **)&d->gangs, sizeof(Gang) * n_gangs) != hipSuccess)
            return fail(h, QDOT_E_NOMEM, "CG gang state");
        d->n_gangs = n_gangs;
    }
    return QDOT_OK;
}

void free_cg(qdot_handle *h)
{
    CgDev *d = (CgDev *)h->cg;
    if (!d) return;
    (void)hipFree(d->sys);
    (void)hipFree(d->gsys);
    (void)hipFree(d->gangs);
    (void)hipFree(d->res);
    delete d;
    h->cg = nullptr;
}

}  // namespace qd

using namespace qd;

extern "C" {

int32_t qdot_cg(qdot_handle *h, const qdot_csr *A, const double *b, double *x, double rtol,
                double qtol, int32_t maxit, int32_t use_qdot, const qdot_options *opt,
                void *stream, qdot_cg_result *out, qdot_result *trace)
{
    if (!h) return QDOT_E_INVAL;
    if (!out) return fail(h, QDOT_E_INVAL, "out is NULL");
    std::memset(out, 0, sizeof *out);
    if (!A || A->n <= 0 || A->nnz < 0 || !A->rowptr || !A->col || !A->val || !b || !x ||
        A->n >= ((int64_t)1 << 31) || A->nnz >= ((int64_t)1 << 31))
        return fail(h, QDOT_E_INVAL, "bad CSR or vector");
    if (!(rtol >= 0.0) || maxit < 0) return fail(h, QDOT_E_INVAL, "bad rtol or maxit");
    qdot_options o;
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return fail(h, QDOT_E_INVAL, "unknown option value");
    if (use_qdot && (!(qtol > 0.0) || !std::isfinite(qtol)))
        return fail(h, QDOT_E_INVAL, "qtol must be finite and > 0");
    DeviceGuard g(h->device);
    const int64_t n = A->n;
    int32_t st = ensure_solver_vectors(h, n);
    if (st != QDOT_OK) return st;
    if ((st = ensure_cg_buffers(h, 1, 1)) != QDOT_OK) return st;
    CgDev *d = (CgDev *)h->cg;
    hipStream_t s = (hipStream_t)stream;
    // one gang: up to one block per CU, at least CHUNK rows per block
    int cap = std::min(MAX_GANG, h->num_cus);
    if (const char *e = std::getenv("QDOT_CG_BLOCKS")) cap = std::max(1, std::min(cap, std::atoi(e)));
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + CHUNK - 1) / CHUNK));
    CgSys S;
    S.n = n;
    S.rowptr = A->rowptr;
    S.col = A->col;
    S.val = A->val;
    S.b = b;
    S.x = x;
    S.r = h->vec;
    S.p = h->vec + n;
    S.q = h->vec + 2 * n;
    S.rtol = rtol;
    S.qtol = qtol;
    S.maxit = maxit;
    S.use_qdot = use_qdot ? 1 : 0;
    S.trace = trace;
    S.res = d->res;
    const int gl[3] = {0, 0, 1};  // gang_sys = {0}; gang_sys_off = {0, 1}
    hipError_t e = hipMemcpyAsync(d->sys, &S, sizeof S, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->gsys, gl, sizeof gl, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gang_init, dim3(1), dim3(BLOCK), 0, s, d->gangs, 1);
        hipLaunchKernelGGL(k_cg_gangs, dim3(G), dim3(BLOCK), 0, s, d->sys, d->gsys, d->gsys + 1,
                           d->gangs, G, o.key_mode, o.score_mode, o.boundary_mode);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d->res, sizeof(qdot_cg_result), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "cg");
    if (out->status == QDOT_E_DEVICE) return fail(h, QDOT_E_DEVICE, "cg gang barrier timed out");
    return out->status;
}

}  // extern "C"
