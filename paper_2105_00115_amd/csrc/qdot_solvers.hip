// CSR SpMV and the power method (Alg. 5), with both inner products of every
// iteration by qdot or by the plain FP64 dot.  (Conjugate gradient runs as
// a persistent launch: qdot_cg.hip, qdot_cg.hpp.)
//
// All state stays in device memory.  The host enqueues iterations in
// batches and reads a small control block between batches; kernels of
// iterations enqueued after a breakdown see the `done` flag and return, so
// the host syncs only once per batch.  Vector updates are one IEEE operation
// per product and per sum (no fused multiply-add), the same arithmetic as a
// plain sequential loop.
#include <cmath>
#include <cstring>

#include "qdot_handle.hpp"

namespace qd {

struct SolverCtl {
    double c;          // last lambda
    int iters;
    int done;
    int broke;
    int status;
};

constexpr int VB = 256;

static inline int vgrid(int64_t n) { return (int)std::max<int64_t>(1, (n + VB - 1) / VB); }

__global__ __launch_bounds__(VB) void k_spmv(int64_t n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ col,
                                             const double *__restrict__ val,
                                             const double *__restrict__ x, double *__restrict__ y,
                                             const SolverCtl *__restrict__ ctl)
{
    if (ctl && ctl->done) return;
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    // the first SNZ entries' column and value loads, then their gathers, are
    // all in flight before the row is summed in storage order
    constexpr int SNZ = 8;
    const int32_t beg = rowptr[i], len = rowptr[i + 1] - beg;
    int32_t ci[SNZ];
    double pv[SNZ];
#pragma unroll
    for (int jj = 0; jj < SNZ; jj++) {
        ci[jj] = 0;
        pv[jj] = 0.0;
        if (jj < len) {
            ci[jj] = col[beg + jj];
            pv[jj] = val[beg + jj];
        }
    }
#pragma unroll
    for (int jj = 0; jj < SNZ; jj++)
        if (jj < len) pv[jj] = pv[jj] * x[ci[jj]];
    double s = 0.0;
#pragma unroll
    for (int jj = 0; jj < SNZ; jj++)
        if (jj < len) s = s + pv[jj];
    for (int32_t j = beg + SNZ; j < beg + len; j++) {
        const double p = val[j] * x[col[j]];
        s = s + p;
    }
    y[i] = s;
}

// dot-product result flags: a qdot that perforated every component of a
// nonzero vector breaks the solver down
__device__ __forceinline__ bool all_perforated(const qdot_result *r)
{
    return r && (r->flags & QDOT_F_ALL_PERF) && r->n_bins > 0;
}

// power method: x = w / sqrt(c), lambda recorded
__global__ __launch_bounds__(VB) void k_pm_update(int64_t n, SolverCtl *ctl,
                                                  const double *lamval,
                                                  const qdot_result *lamres,
                                                  const double *cval, const qdot_result *cres,
                                                  double *__restrict__ x,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ trace, int k)
{
    if (ctl->done) return;
    const double c = *cval;
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (!(c > 0.0) || !isfinite(c) || all_perforated(cres) || all_perforated(lamres)) {
        if (i == 0) ctl->broke = 1;
        return;
    }
    if (i == 0) {
        if (trace) trace[k] = *lamval;
    }
    if (i >= n) return;
    const double s = sqrt(c);
    x[i] = w[i] / s;
}

__global__ void k_pm_step(SolverCtl *ctl, const double *lamval)
{
    if (ctl->done) return;
    if (ctl->broke) {
        ctl->status = QDOT_E_BREAKDOWN;
        ctl->done = 1;
        return;
    }
    ctl->c = *lamval;
    ctl->iters += 1;
}

__global__ void k_ctl_reset(SolverCtl *ctl)
{
    ctl->c = 0.0;
    ctl->iters = 0;
    ctl->done = 0;
    ctl->broke = 0;
    ctl->status = QDOT_OK;
}

static bool csr_ok(const qdot_csr *A)
{
    return A && A->n >= 0 && A->nnz >= 0 && (A->n == 0 || (A->rowptr && A->col && A->val)) &&
           A->n < (int64_t)1 << 31 && A->nnz < (int64_t)1 << 31;
}

int32_t ensure_solver_vectors(qdot_handle *h, int64_t doubles)
{
    if (!h->ctl) {
        if (hipMalloc(&h->ctl, sizeof(SolverCtl)) != hipSuccess ||
            hipMalloc((void **)&h->res_ring, 4 * sizeof(qdot_result)) != hipSuccess ||
            hipMalloc((void **)&h->dres, 4 * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&h->host_ctl, sizeof(SolverCtl), hipHostMallocDefault) != hipSuccess)
            return fail(h, QDOT_E_NOMEM, "solver control allocation failed");
    }
    if (h->vec_n < doubles) {
        if (h->vec) (void)hipFree(h->vec);
        h->vec = nullptr;
        h->vec_n = 0;
        if (hipMalloc((void **)&h->vec, sizeof(double) * (size_t)std::max<int64_t>(doubles, 1)) !=
            hipSuccess)
            return fail(h, QDOT_E_NOMEM, "solver vector allocation failed");
        h->vec_n = doubles;
    }
    return QDOT_OK;
}

// One inner product into the slot given; returns the device address of its
// value and (for qdot) of its full result.
static hipError_t enqueue_dot(qdot_handle *h, const Launch &L, const double *a, const double *b,
                              int64_t n, int use_qdot, double qtol, const qdot_options &o,
                              qdot_result *qslot, double *dslot, const double **val,
                              const qdot_result **res)
{
    if (use_qdot) {
        *val = &qslot->value;
        *res = qslot;
        return launch_qdot(L, a, b, n, qtol, o, qslot, nullptr, nullptr);
    }
    *val = dslot;
    *res = nullptr;
    return launch_dot64(L, a, b, n, dslot);
}

static int32_t read_ctl(qdot_handle *h, hipStream_t s, SolverCtl &out)
{
    hipError_t e = hipMemcpyAsync(h->host_ctl, h->ctl, sizeof(SolverCtl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "solver control read");
    std::memcpy(&out, h->host_ctl, sizeof(SolverCtl));
    return QDOT_OK;
}

}  // namespace qd

using namespace qd;

extern "C" {

int32_t qdot_spmv_async(qdot_handle *h, const qdot_csr *A, const double *x, double *y,
                        void *stream)
{
    if (!h) return QDOT_E_INVAL;
    if (!csr_ok(A) || (A->n > 0 && (!x || !y))) return fail(h, QDOT_E_INVAL, "bad CSR or vector");
    if (A->n == 0) return QDOT_OK;
    DeviceGuard g(h->device);
    hipLaunchKernelGGL(k_spmv, dim3(vgrid(A->n)), dim3(VB), 0, (hipStream_t)stream, A->n,
                       A->rowptr, A->col, A->val, x, y, (const SolverCtl *)nullptr);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "spmv launch");
}

int32_t qdot_power(qdot_handle *h, const qdot_csr *A, double *x, int32_t iters, double qtol,
                   int32_t use_qdot, const qdot_options *opt, void *stream, double *lambda,
                   double *lambda_trace)
{
    if (!h) return QDOT_E_INVAL;
    if (!csr_ok(A) || A->n == 0 || !x || iters < 0) return fail(h, QDOT_E_INVAL, "bad argument");
    qdot_options o;
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return fail(h, QDOT_E_INVAL, "unknown option value");
    if (use_qdot && (!(qtol > 0.0) || !std::isfinite(qtol)))
        return fail(h, QDOT_E_INVAL, "qtol must be finite and > 0");
    if (use_qdot && o.accum_mode == 1 && !s1_admissible(A->n, qtol, o))
        return fail(h, QDOT_E_INVAL, "accum_mode 1 not admissible for this n and qtol");
    DeviceGuard g(h->device);
    const int64_t n = A->n;
    int32_t st = ensure_solver_vectors(h, n);
    if (st != QDOT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Launch L = make_launch(h, s, n);
    double *w = h->vec;
    SolverCtl *ctl = (SolverCtl *)h->ctl;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x_) {
        if (e == hipSuccess && x_ != hipSuccess) e = x_;
        return e == hipSuccess;
    };
    const int gv = vgrid(n);
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(1), 0, s, ctl);
    ok(hipGetLastError());
    SolverCtl hc;
    std::memset(&hc, 0, sizeof hc);
    for (int32_t k = 0; k < iters && e == hipSuccess; k++) {
        const double *lv, *cv;
        const qdot_result *lr, *cr;
        hipLaunchKernelGGL(k_spmv, dim3(gv), dim3(VB), 0, s, n, A->rowptr, A->col, A->val, x, w,
                           (const SolverCtl *)ctl);
        ok(enqueue_dot(h, L, x, w, n, use_qdot, qtol, o, h->res_ring, h->dres, &lv, &lr));
        ok(enqueue_dot(h, L, w, w, n, use_qdot, qtol, o, h->res_ring + 1, h->dres + 1, &cv, &cr));
        hipLaunchKernelGGL(k_pm_update, dim3(gv), dim3(VB), 0, s, n, ctl, lv, lr, cv, cr, x, w,
                           lambda_trace, k);
        hipLaunchKernelGGL(k_pm_step, dim3(1), dim3(1), 0, s, ctl, lv);
        ok(hipGetLastError());
        if ((k + 1) % 64 == 0) {
            if ((st = read_ctl(h, s, hc)) != QDOT_OK) return st;
            if (hc.done) break;
        }
    }
    if (e != hipSuccess) return hip_fail(h, e, "power launch");
    if ((st = read_ctl(h, s, hc)) != QDOT_OK) return st;
    if (lambda) *lambda = hc.c;
    return hc.status;
}

}  // extern "C"
