// Conjugate gradient (Alg. 4) on the device in one persistent launch: one
// gang of blocks solves the system (device code in qdot_cg.hpp).
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "qdot_cg.hpp"
#include "qdot_handle.hpp"

namespace qd {

// GUARD: guard_mode 1; ACC1: accum_mode 1 (tab: the gang's one-pass
// tables, zero on entry and on exit).
template <bool GUARD, bool ACC1>
__global__ __launch_bounds__(BLOCK) void k_cg_gangs(const CgSys *__restrict__ sys,
                                                    const int *__restrict__ gang_sys,
                                                    const int *__restrict__ gang_sys_off,
                                                    Gang *__restrict__ gangs, int G,
                                                    qdot_cg_result *__restrict__ res,
                                                    int key_mode, int score_mode, int nonstrict,
                                                    double *__restrict__ tab)
{
    __shared__ CgLds L;
    for (int i = threadIdx.x; i < W + 1; i += BLOCK) L.h[i] = 0u;
    for (int i = W + threadIdx.x; i < W_LUT; i += BLOCK) L.lut[i] = (unsigned char)QDOT_PERF;
    __syncthreads();
    const int g = blockIdx.x / G, gb = blockIdx.x % G;
    Gang *gg = gangs + g;
    auto run = [&](S1Lds *S1) {
        for (int s = gang_sys_off[g]; s < gang_sys_off[g + 1]; s++) {
            cg_solve<GUARD, ACC1>(sys[gang_sys[s]], gg, G, gb, key_mode, score_mode, nonstrict,
                                  L, res + gang_sys[s], S1, tab);
            if (__hip_atomic_load(&gg->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        }
    };
    if constexpr (ACC1) {
        __shared__ S1Lds S1;
        run(&S1);
    } else {
        run(nullptr);
    }
}

__global__ void k_gang_init(Gang *gangs, int n)
{
    const int g = blockIdx.x;
    if (g >= n) return;
    gang_reset(gangs + g);
    if (threadIdx.x == 0) gangs[g].bar_gen = 0;
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
    double *s1tab = nullptr;  // one-pass tables of the gang (2 W S1_PIECES), zero between calls
};

constexpr size_t CG_S1TAB = (size_t)2 * W * S1_PIECES;

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
    (void)hipFree(d->s1tab);
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
    if (o.bin_mode != 0)
        return fail(h, QDOT_E_INVAL, "bin_mode 1 and 2 are for the single-vector qdot entry points");
    if (o.tile_skip != 0)
        return fail(h, QDOT_E_INVAL, "tile_skip is for the single-vector qdot entry points");
    if (use_qdot && (!(qtol > 0.0) || !std::isfinite(qtol)))
        return fail(h, QDOT_E_INVAL, "qtol must be finite and > 0");
    const bool acc1 = use_qdot && o.accum_mode == 1;
    if (acc1 && !s1_admissible(A->n, qtol, o))
        return fail(h, QDOT_E_INVAL, "accum_mode 1 not admissible for this n and qtol");
    DeviceGuard g(h->device);
    const int64_t n = A->n;
    int32_t st = ensure_solver_vectors(h, 3 * n);  // r, p, q
    if (st != QDOT_OK) return st;
    if ((st = ensure_cg_buffers(h, 1, 1)) != QDOT_OK) return st;
    CgDev *d = (CgDev *)h->cg;
    hipStream_t s = (hipStream_t)stream;
    // one gang: up to two blocks per CU (as many as are resident together),
    // at least CHUNK rows per block.  Two blocks per CU keep twice the
    // SpMV's gathers in flight; measured on Poisson 1024^2 the iteration
    // took 87 us instead of 92 with qdot and 49 instead of 59 with the FP64
    // dot.
    int per_cu = 0;
    hipError_t oe =
        acc1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg_gangs<false, true>,
                                                           BLOCK, 0)
        : o.guard_mode
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg_gangs<true, false>, BLOCK,
                                                           0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg_gangs<false, false>,
                                                           BLOCK, 0);
    if (oe != hipSuccess) return hip_fail(h, oe, "occupancy query");
    if (per_cu < 1) return fail(h, QDOT_E_DEVICE, "the CG kernel cannot be resident");
    const int cap = std::min(MAX_GANG, std::min(per_cu, h->cg_blocks_per_cu) * h->num_cus);
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
    const int gl[3] = {0, 0, 1};  // gang_sys = {0}; gang_sys_off = {0, 1}
    hipError_t e = hipMemcpyAsync(d->sys, &S, sizeof S, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->gsys, gl, sizeof gl, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && acc1 && !d->s1tab) {
        e = hipMalloc((void **)&d->s1tab, sizeof(double) * CG_S1TAB);
        if (e != hipSuccess) {
            d->s1tab = nullptr;
            return fail(h, QDOT_E_NOMEM, "CG one-pass tables");
        }
        e = hipMemsetAsync(d->s1tab, 0, sizeof(double) * CG_S1TAB, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gang_init, dim3(1), dim3(BLOCK), 0, s, d->gangs, 1);
        if (acc1)
            hipLaunchKernelGGL((k_cg_gangs<false, true>), dim3(G), dim3(BLOCK), 0, s, d->sys,
                               d->gsys, d->gsys + 1, d->gangs, G, d->res, o.key_mode,
                               o.score_mode, o.boundary_mode, d->s1tab);
        else if (o.guard_mode)
            hipLaunchKernelGGL((k_cg_gangs<true, false>), dim3(G), dim3(BLOCK), 0, s, d->sys,
                               d->gsys, d->gsys + 1, d->gangs, G, d->res, o.key_mode,
                               o.score_mode, o.boundary_mode, (double *)nullptr);
        else
            hipLaunchKernelGGL((k_cg_gangs<false, false>), dim3(G), dim3(BLOCK), 0, s, d->sys,
                               d->gsys, d->gsys + 1, d->gangs, G, d->res, o.key_mode,
                               o.score_mode, o.boundary_mode, (double *)nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d->res, sizeof(qdot_cg_result), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "cg");
    if (out->status == QDOT_E_DEVICE) {
        // an abandoned solve may leave one-pass table entries behind
        if (d->s1tab && (hipMemsetAsync(d->s1tab, 0, sizeof(double) * CG_S1TAB, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess)) {
            (void)hipFree(d->s1tab);
            d->s1tab = nullptr;
        }
        return fail(h, QDOT_E_DEVICE, "cg gang barrier timed out");
    }
    return out->status;
}

}  // extern "C"
