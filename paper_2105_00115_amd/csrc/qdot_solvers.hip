// Applications of qdot: CSR SpMV, conjugate gradient (Alg. 4) and the power
// method (Alg. 5), with every inner product by qdot or by the plain FP64 dot.
//
// All state stays in device memory.  The host enqueues iterations in
// batches and reads a small control block between batches; kernels of
// iterations enqueued after convergence see the `done` flag and return, so
// the iteration count is exact while the host syncs only once per batch.
// Vector updates are one IEEE operation per product and per sum (no fused
// multiply-add), the same arithmetic as a plain sequential loop.
#include <cmath>
#include <cstring>

#include "qdot_handle.hpp"

namespace qd {

struct SolverCtl {
    double c;          // CG: current r.r;  power: last lambda
    double thresh;     // CG: rtol * ||b||
    double bnorm;      // CG: ||b||
    int iters;
    int done;
    int broke;
    int status;
};

constexpr int VB = 256;
constexpr int CHECK_EVERY = 16;

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
    double s = 0.0;
    for (int32_t j = rowptr[i]; j < rowptr[i + 1]; j++) {
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

__global__ void k_cg_init(SolverCtl *ctl, const double *c0, const qdot_result *c0res,
                          const double *bb, double rtol)
{
    const double bn = sqrt(*bb);
    ctl->bnorm = bn;
    ctl->thresh = rtol * bn;
    ctl->c = *c0;
    ctl->iters = 0;
    ctl->broke = 0;
    ctl->status = QDOT_OK;
    ctl->done = 0;
    if (all_perforated(c0res)) {
        ctl->status = QDOT_E_BREAKDOWN;
        ctl->done = 1;
    } else if (!(sqrt(ctl->c) > ctl->thresh)) {
        ctl->done = 1;
    }
}

// r0 = b - A x0 (q holds A x0), p0 = r0
__global__ __launch_bounds__(VB) void k_cg_residual(int64_t n, const double *__restrict__ b,
                                                    const double *__restrict__ q,
                                                    double *__restrict__ r,
                                                    double *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    const double v = b[i] - q[i];
    r[i] = v;
    if (p) p[i] = v;
}

// alpha = c / (p.q);  x += alpha p;  r -= alpha q
__global__ __launch_bounds__(VB) void k_cg_update1(int64_t n, SolverCtl *ctl,
                                                   const double *dval, const qdot_result *dres,
                                                   double *__restrict__ x,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ r)
{
    if (ctl->done) return;
    const double d = *dval;
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (!(d > 0.0) || !isfinite(d) || all_perforated(dres)) {
        if (i == 0) ctl->broke = 1;
        return;
    }
    if (i >= n) return;
    const double alpha = ctl->c / d;
    const double ap = alpha * p[i];
    x[i] = x[i] + ap;
    const double aq = alpha * q[i];
    r[i] = r[i] - aq;
}

// beta = c' / c;  p = r + beta p
__global__ __launch_bounds__(VB) void k_cg_update2(int64_t n, const SolverCtl *ctl,
                                                   const double *cnval,
                                                   double *__restrict__ p,
                                                   const double *__restrict__ r)
{
    if (ctl->done || ctl->broke) return;
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    const double beta = *cnval / ctl->c;
    const double bp = beta * p[i];
    p[i] = r[i] + bp;
}

__global__ void k_cg_step(SolverCtl *ctl, const double *cnval, const qdot_result *cnres)
{
    if (ctl->done) return;
    if (ctl->broke || all_perforated(cnres)) {
        ctl->status = QDOT_E_BREAKDOWN;
        ctl->done = 1;
        return;
    }
    ctl->c = *cnval;
    ctl->iters += 1;
    if (!(sqrt(ctl->c) > ctl->thresh)) ctl->done = 1;
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

static int32_t ensure_scratch(qdot_handle *h, int64_t n)
{
    if (!h->ctl) {
        if (hipMalloc(&h->ctl, sizeof(SolverCtl)) != hipSuccess ||
            hipMalloc((void **)&h->res_ring, 4 * sizeof(qdot_result)) != hipSuccess ||
            hipMalloc((void **)&h->dres, 4 * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&h->host_ctl, sizeof(SolverCtl), hipHostMallocDefault) != hipSuccess)
            return fail(h, QDOT_E_NOMEM, "solver control allocation failed");
    }
    if (h->vec_n < n) {
        if (h->vec) (void)hipFree(h->vec);
        h->vec = nullptr;
        h->vec_n = 0;
        if (hipMalloc((void **)&h->vec, sizeof(double) * 4 * (size_t)std::max<int64_t>(n, 1)) !=
            hipSuccess)
            return fail(h, QDOT_E_NOMEM, "solver vector allocation failed");
        h->vec_n = n;
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

int32_t qdot_cg(qdot_handle *h, const qdot_csr *A, const double *b, double *x, double rtol,
                double qtol, int32_t maxit, int32_t use_qdot, const qdot_options *opt,
                void *stream, qdot_cg_result *out, qdot_result *trace)
{
    if (!h) return QDOT_E_INVAL;
    if (!out) return fail(h, QDOT_E_INVAL, "out is NULL");
    std::memset(out, 0, sizeof *out);
    if (!csr_ok(A) || A->n == 0 || !b || !x) return fail(h, QDOT_E_INVAL, "bad CSR or vector");
    if (!(rtol >= 0.0) || maxit < 0) return fail(h, QDOT_E_INVAL, "bad rtol or maxit");
    qdot_options o;
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return fail(h, QDOT_E_INVAL, "unknown option value");
    if (use_qdot && (!(qtol > 0.0) || !std::isfinite(qtol)))
        return fail(h, QDOT_E_INVAL, "qtol must be finite and > 0");
    DeviceGuard g(h->device);
    const int64_t n = A->n;
    int32_t st = ensure_scratch(h, n);
    if (st != QDOT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Launch L = make_launch(h, s, n);
    double *r = h->vec, *p = h->vec + n, *q = h->vec + 2 * n;
    SolverCtl *ctl = (SolverCtl *)h->ctl;
    qdot_result *rr_slot = h->res_ring, *pq_slot = h->res_ring + 1;
    double *d_rr = h->dres, *d_pq = h->dres + 1, *d_bb = h->dres + 2;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x_) {
        if (e == hipSuccess && x_ != hipSuccess) e = x_;
        return e == hipSuccess;
    };
    const int gv = vgrid(n);

    // r0 = b - A x0, p0 = r0, c0 = dot(r0, r0), ||b|| by the FP64 dot
    hipLaunchKernelGGL(k_spmv, dim3(gv), dim3(VB), 0, s, n, A->rowptr, A->col, A->val, x, q,
                       (const SolverCtl *)nullptr);
    hipLaunchKernelGGL(k_cg_residual, dim3(gv), dim3(VB), 0, s, n, b, q, r, p);
    ok(hipGetLastError());
    ok(launch_dot64(L, b, b, n, d_bb));
    const double *cval;
    const qdot_result *cres;
    ok(enqueue_dot(h, L, r, r, n, use_qdot, qtol, o, trace ? &trace[0] : rr_slot, d_rr, &cval,
                   &cres));
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1), 0, s, ctl, cval, cres, d_bb, rtol);
    ok(hipGetLastError());

    SolverCtl hc;
    std::memset(&hc, 0, sizeof hc);
    int32_t enq = 0;
    while (e == hipSuccess) {
        if ((st = read_ctl(h, s, hc)) != QDOT_OK) return st;
        if (hc.done || enq >= maxit) break;
        const int32_t batch = std::min<int32_t>(CHECK_EVERY, maxit - enq);
        for (int32_t it = 0; it < batch && e == hipSuccess; it++, enq++) {
            const double *dval, *cnval;
            const qdot_result *dres, *cnres;
            hipLaunchKernelGGL(k_spmv, dim3(gv), dim3(VB), 0, s, n, A->rowptr, A->col, A->val,
                               p, q, (const SolverCtl *)ctl);
            ok(enqueue_dot(h, L, p, q, n, use_qdot, qtol, o,
                           trace ? &trace[1 + 2 * enq] : pq_slot, d_pq, &dval, &dres));
            hipLaunchKernelGGL(k_cg_update1, dim3(gv), dim3(VB), 0, s, n, ctl, dval, dres, x, p,
                               q, r);
            ok(enqueue_dot(h, L, r, r, n, use_qdot, qtol, o,
                           trace ? &trace[2 + 2 * enq] : rr_slot, d_rr, &cnval, &cnres));
            hipLaunchKernelGGL(k_cg_update2, dim3(gv), dim3(VB), 0, s, n, ctl, cnval, p, r);
            hipLaunchKernelGGL(k_cg_step, dim3(1), dim3(1), 0, s, ctl, cnval, cnres);
            ok(hipGetLastError());
        }
    }
    if (e != hipSuccess) return hip_fail(h, e, "cg launch");
    // true residual ||b - A x|| / ||b||
    hipLaunchKernelGGL(k_spmv, dim3(gv), dim3(VB), 0, s, n, A->rowptr, A->col, A->val, x, q,
                       (const SolverCtl *)nullptr);
    hipLaunchKernelGGL(k_cg_residual, dim3(gv), dim3(VB), 0, s, n, b, q, q, (double *)nullptr);
    ok(hipGetLastError());
    ok(launch_dot64(L, q, q, n, d_pq));
    if (e != hipSuccess) return hip_fail(h, e, "cg residual launch");
    double rq = 0.0;
    e = hipMemcpyAsync(&rq, d_pq, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "cg residual read");
    out->iters = hc.iters;
    out->status = hc.status != QDOT_OK ? hc.status : (hc.done ? QDOT_OK : QDOT_E_MAXIT);
    out->relres_est = hc.bnorm > 0 ? std::sqrt(hc.c) / hc.bnorm : 0.0;
    out->relres_true = hc.bnorm > 0 ? std::sqrt(rq) / hc.bnorm : 0.0;
    return out->status;
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
    DeviceGuard g(h->device);
    const int64_t n = A->n;
    int32_t st = ensure_scratch(h, n);
    if (st != QDOT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Launch L = make_launch(h, s, n);
    double *w = h->vec + 3 * n;
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
