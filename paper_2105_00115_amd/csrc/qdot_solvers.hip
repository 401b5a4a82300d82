// CSR SpMV and the power method (Alg. 5), with both inner products of every
// iteration by qdot or by the plain FP64 dot.  (Conjugate gradient runs as
// a persistent launch: qdot_cg.hip, qdot_cg.hpp.)
//
// All state stays in device memory.  The host enqueues iterations in
// batches of 64 and reads a small control block between batches, so it
// syncs only once per batch.  After a breakdown the SpMV and the update of
// the iterations still enqueued see the `done` flag and return; their inner
// products run on the unchanged vectors and their results are not used.
// Vector updates are one IEEE operation per product and per sum (no fused
// multiply-add), the same arithmetic as a plain sequential loop.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "qdot_blocks.hpp"
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

// ---------------------------------------------------------------------------
// CSR SpMV, y = A v, every row summed in column-storage order (plain
// multiply, then add: the arithmetic of a sequential loop).
//
// A block takes BLOCK consecutive rows at a time (grid-stride over row
// groups).  Their entries are one contiguous range of col/val, read
// coalesced SP_NZ at a time: each thread loads SP_U (col, val) pairs, then
// their gathers v[col], and leaves the products in LDS; after a barrier
// each thread adds its own row's products from LDS in order.  A row that
// runs past the staged range continues with the next one, so rows of any
// length keep their order.
constexpr int SP_U = 8;
constexpr int SP_NZ = SP_U * BLOCK;

// The SpMV loop over a block's row groups.  gather(c) gives the vector entry
// of column c; own(i, yi) is called once per row with its result.
// Row groups go to the XCDs in eight contiguous ranges: the hardware deals
// blocks out to the 8 XCDs in turn (block b to XCD b mod 8), so the blocks
// of one XCD take the groups of one range, and a row's neighbours a few
// groups away (a stencil's next grid line) are gathered from that XCD's own
// L2 instead of being fetched again by another XCD.  Grids that are not a
// multiple of 8 walk the groups in plain grid-stride order.
template <class Gather, class Own>
__device__ __forceinline__ void spmv_lds(int64_t n, const int32_t *__restrict__ rowptr,
                                         const int32_t *__restrict__ col,
                                         const double *__restrict__ val, Gather &&gather,
                                         Own &&own, double *prod)
{
    constexpr int XCDS = 8;
    const int64_t ng = (n + BLOCK - 1) / BLOCK;
    const int grid = (int)gridDim.x;
    int64_t g0 = blockIdx.x, gstep = grid, gend = ng;
    if (grid % XCDS == 0) {
        const int64_t x = blockIdx.x % XCDS;
        g0 = ng * x / XCDS + blockIdx.x / XCDS;
        gstep = grid / XCDS;
        gend = ng * (x + 1) / XCDS;
    }
    for (int64_t g = g0; g < gend; g += gstep) {
        const int64_t r0 = g * BLOCK;
        const int64_t r1 = min(n, r0 + (int64_t)BLOCK);
        const int64_t i = r0 + threadIdx.x;
        const bool row = i < r1;
        int64_t beg = 0, end = 0;
        if (row) {
            beg = rowptr[i];
            end = rowptr[i + 1];
        }
        const int64_t b0 = rowptr[r0], b1 = rowptr[r1];
        double s = 0.0;
        for (int64_t c0 = b0; c0 < b1; c0 += SP_NZ) {
            const int64_t c1 = min(b1, c0 + (int64_t)SP_NZ);
            __syncthreads();  // the previous range's products are consumed
            int32_t ci[SP_U];
            double pv[SP_U];
#pragma unroll
            for (int u = 0; u < SP_U; u++) {
                const int64_t j = c0 + u * BLOCK + threadIdx.x;
                ci[u] = 0;
                pv[u] = 0.0;
                if (j < c1) {
                    ci[u] = col[j];
                    pv[u] = val[j];
                }
            }
#pragma unroll
            for (int u = 0; u < SP_U; u++)
                if (c0 + u * BLOCK + threadIdx.x < c1) pv[u] = pv[u] * gather(ci[u]);
#pragma unroll
            for (int u = 0; u < SP_U; u++) prod[u * BLOCK + threadIdx.x] = pv[u];
            __syncthreads();
            if (row) {
                const int64_t lo = max(beg, c0), hi = min(end, c1);
                for (int64_t j = lo; j < hi; j++) s = s + prod[j - c0];
            }
        }
        if (row) own(i, s);
    }
}

__global__ __launch_bounds__(BLOCK) void k_spmv(int64_t n, const int32_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const double *__restrict__ val,
                                                const double *__restrict__ v,
                                                double *__restrict__ y)
{
    __shared__ double prod[SP_NZ];
    spmv_lds(
        n, rowptr, col, val, [&](int32_t c) { return v[c]; },
        [&](int64_t i, double yi) { y[i] = yi; }, prod);
}

// dot-product result flags: a qdot that perforated every component of a
// nonzero vector breaks the solver down
__device__ __forceinline__ bool all_perforated(const qdot_result *r)
{
    return r && (r->flags & QDOT_F_ALL_PERF) && r->n_bins > 0;
}

// Pass 1 of the iteration's two inner products, lambda = x . w and c = w . w
// (two-pass qdot), can ride in the SpMV, which forms both vectors row by
// row: each row's keys go into a block-private LDS window of PM_HWIN slots
// per product, placed below the previous iteration's e_max of that product
// (PM_HWIN_ABOVE slots above it); a key outside the window, rare for the
// slowly changing vectors of the method, goes straight into the block's
// global histogram copy.  The windows are then merged as k_scan merges its
// histogram, with the same per-block records, so the qdot kernels that
// follow run without their own pass 1.
constexpr int PM_HWIN = 512;
constexpr int PM_HWIN_ABOVE = 64;

struct PmScan {
    Ws *ws[2];             // workspaces of x . w and w . w
    const qdot_result *prev[2];  // previous iteration's results (window placement)
    int key_mode;
    int copies;
};

// Power method, iteration k: it first finishes iteration k - 1 (k > 0),
// whose results lamval / cval are in device memory: breakdown, or lambda
// recorded and x = w_{k-1} / sqrt(c).  It does not wait for that division
// to be stored: the SpMV w_k = A x gathers w_{k-1}[c] / sqrt(c) itself, the
// same rounded quotient, and each row writes its own x entry.  At k = 0 the
// source is x itself, read as it is.  Every block takes the same decision
// from the same results; block 0 alone writes the control block (the others
// read only its `done` word at their start, and a breakdown makes them
// return whichever value they see).
// With SCAN (k > 0) the SpMV also takes pass 1 of both inner products of
// iteration k (PmScan).
template <bool SCAN>
__global__ __launch_bounds__(BLOCK) void k_pm_spmv(
    int64_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ src, double *__restrict__ w,
    double *__restrict__ x, SolverCtl *ctl, const double *lamval, const qdot_result *lamres,
    const double *cval, const qdot_result *cres, double *__restrict__ trace, int k, PmScan ps)
{
    __shared__ double prod[SP_NZ];
    __shared__ unsigned int hw[SCAN ? 2 : 1][SCAN ? PM_HWIN : 1];
    if (ctl->done) return;
    double sc = 1.0;
    if (k > 0) {
        const double c = *cval;
        const bool first_block = blockIdx.x == 0 && threadIdx.x == 0;
        if (!(c > 0.0) || !isfinite(c) || all_perforated(cres) || all_perforated(lamres)) {
            if (first_block) {
                ctl->broke = 1;
                ctl->status = QDOT_E_BREAKDOWN;
                ctl->done = 1;
            }
            return;
        }
        if (first_block) {
            const double lam = *lamval;
            if (trace) trace[k - 1] = lam;
            ctl->c = lam;
            ctl->iters += 1;
        }
        sc = sqrt(c);
    }
    if constexpr (!SCAN) {
        if (k == 0)
            spmv_lds(
                n, rowptr, col, val, [&](int32_t c) { return src[c]; },
                [&](int64_t i, double yi) { w[i] = yi; }, prod);
        else
            spmv_lds(
                n, rowptr, col, val, [&](int32_t c) { return src[c] / sc; },
                [&](int64_t i, double yi) {
                    w[i] = yi;
                    x[i] = src[i] / sc;
                },
                prod);
    } else {
        int base[2];
        unsigned long long *gh[2];
        unsigned int nz[2] = {0u, 0u}, bad[2] = {0u, 0u}, sg[2] = {0u, 0u};
        int lo[2] = {W, W}, hi[2] = {-1, -1};
        for (int p = 0; p < 2; p++) {
            const qdot_result *pr = ps.prev[p];
            const int top = (pr->status == QDOT_OK && pr->n_bins > 0)
                                ? pr->e_max - KMIN + PM_HWIN_ABOVE
                                : W / 2;
            base[p] = max(0, min(W - PM_HWIN, top - PM_HWIN + 1));
            gh[p] = ps.ws[p]->hist[blockIdx.x % ps.copies];
            for (int j = threadIdx.x; j < PM_HWIN; j += BLOCK) hw[p][j] = 0u;
        }
        __syncthreads();
        auto key = [&](int p, double a, double b) {
            const Comp c = component(a, b, ps.key_mode);
            nz[p] += c.zero ? 1u : 0u;
            bad[p] |= c.bad ? 1u : 0u;
            sg[p] |= c.zero ? 0u : (c.sgn ? 1u : 2u);
            if (c.slot == ZERO_SLOT) return;
            const int j = c.slot - base[p];
            if ((unsigned)j < (unsigned)PM_HWIN) {
                atomicAdd(&hw[p][j], 1u);
            } else {
                atomicAdd(&gh[p][c.slot], 1ull);
                lo[p] = min(lo[p], c.slot);
                hi[p] = max(hi[p], c.slot);
            }
        };
        spmv_lds(
            n, rowptr, col, val, [&](int32_t c) { return src[c] / sc; },
            [&](int64_t i, double yi) {
                w[i] = yi;
                const double xi = src[i] / sc;
                x[i] = xi;
                key(0, xi, yi);
                key(1, yi, yi);
            },
            prod);
        __syncthreads();
        for (int p = 0; p < 2; p++) {
            scan_flush_window(hw[p], base[p], PM_HWIN, lo[p], hi[p], nz[p], bad[p], sg[p],
                              ps.ws[p], blockIdx.x, ps.copies);
            __syncthreads();
        }
    }
}

static int spmv_grid(const qdot_handle *h, int64_t n)
{
    const int bpc = h->spmv_blocks_per_cu;
    const int64_t cap = std::min<int64_t>(MAX_GRID, (int64_t)bpc * h->num_cus);
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + BLOCK - 1) / BLOCK));
}

// Power method, end of the last iteration k: x = w / sqrt(c) and lambda
// recorded, or the breakdown recorded (the step k_pm_spmv does for the
// iteration before its own), with the same decision in every block.
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
        if (i == 0) {
            ctl->broke = 1;
            ctl->status = QDOT_E_BREAKDOWN;
            ctl->done = 1;
        }
        return;
    }
    if (i == 0) {
        const double lam = *lamval;
        if (trace) trace[k] = lam;
        ctl->c = lam;
        ctl->iters += 1;
    }
    if (i >= n) return;
    const double s = sqrt(c);
    x[i] = w[i] / s;
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

// A second qdot workspace: the power method's two inner products of an
// iteration are selected and summed side by side.
// It is cleared on the stream of the call that first needs it, ahead of
// that call's kernels.
static int32_t ensure_second_ws(qdot_handle *h, hipStream_t s)
{
    if (h->ws2) return QDOT_OK;
    if (hipMalloc((void **)&h->ws2, sizeof(Ws)) != hipSuccess) {
        h->ws2 = nullptr;
        return fail(h, QDOT_E_NOMEM, "second workspace allocation failed");
    }
    if (hipMemsetAsync(h->ws2, 0, sizeof(Ws), s) != hipSuccess) {
        (void)hipFree(h->ws2);
        h->ws2 = nullptr;
        return fail(h, QDOT_E_DEVICE, "second workspace clear failed");
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
    hipLaunchKernelGGL(k_spmv, dim3(spmv_grid(h, A->n)), dim3(BLOCK), 0, (hipStream_t)stream,
                       A->n, A->rowptr, A->col, A->val, x, y);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "spmv launch");
}

int32_t qdot_power(qdot_handle *h, const qdot_csr *A, double *x, int32_t iters, double qtol,
                   int32_t use_qdot, const qdot_options *opt, void *stream, double *lambda,
                   double *lambda_trace, qdot_result *trace)
{
    if (!h) return QDOT_E_INVAL;
    if (!csr_ok(A) || A->n == 0 || !x || iters < 0) return fail(h, QDOT_E_INVAL, "bad argument");
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
    if (use_qdot && o.accum_mode == 1 && !s1_admissible(A->n, qtol, o))
        return fail(h, QDOT_E_INVAL, "accum_mode 1 not admissible for this n and qtol");
    DeviceGuard g(h->device);
    const int64_t n = A->n;
    int32_t st = ensure_solver_vectors(h, 2 * n);  // w of the iteration and the previous one
    if (st != QDOT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Launch L = make_launch(h, s, n);
    double *wbuf[2] = {h->vec, h->vec + n};
    SolverCtl *ctl = (SolverCtl *)h->ctl;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x_) {
        if (e == hipSuccess && x_ != hipSuccess) e = x_;
        return e == hipSuccess;
    };
    const int gv = vgrid(n);
    // with the two-pass qdot both inner products of an iteration share
    // their launches (launch_qdot_pair); the one-pass mode and the FP64 dot
    // take them one after the other
    const bool paired = use_qdot && o.accum_mode == 0;
    if (paired && (st = ensure_second_ws(h, s)) != QDOT_OK) return st;
    Launch L2 = L;
    L2.ws = h->ws2;
    const int sg = spmv_grid(h, n);
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(1), 0, s, ctl);
    ok(hipGetLastError());
    SolverCtl hc;
    std::memset(&hc, 0, sizeof hc);
    // results of the last enqueued iteration (read by the next one's SpMV)
    const double *lv = nullptr, *cv = nullptr;
    const qdot_result *lr = nullptr, *cr = nullptr;
    int32_t k = 0;
    for (; k < iters && e == hipSuccess; k++) {
        double *w = wbuf[k & 1];
        const double *src = k == 0 ? x : wbuf[(k - 1) & 1];
        // the qdot results of iteration k: straight into the caller's trace
        // when one is given, else the handle's two slots
        qdot_result *ra = trace && use_qdot ? trace + 2 * (int64_t)k : h->res_ring;
        qdot_result *rb = ra + 1;
        // after the first iteration the paired qdot's pass 1 rides in the
        // SpMV (its windows placed by the previous iteration's results)
        const bool fused = paired && k > 0 && h->power_scan_in_spmv;
        const PmScan ps = {{L.ws, L2.ws}, {lr, cr}, o.key_mode, L.hist_copies};
        if (fused)
            hipLaunchKernelGGL(k_pm_spmv<true>, dim3(sg), dim3(BLOCK), 0, s, n, A->rowptr,
                               A->col, A->val, src, w, x, ctl, lv, lr, cv, cr, lambda_trace, k,
                               ps);
        else
            hipLaunchKernelGGL(k_pm_spmv<false>, dim3(sg), dim3(BLOCK), 0, s, n, A->rowptr,
                               A->col, A->val, src, w, x, ctl, lv, lr, cv, cr, lambda_trace, k,
                               ps);
        if (paired) {
            ok(launch_qdot_pair(L, L2, x, w, n, qtol, o, ra, rb, fused ? sg : -1));
            lv = &ra->value;
            lr = ra;
            cv = &rb->value;
            cr = rb;
        } else {
            ok(enqueue_dot(h, L, x, w, n, use_qdot, qtol, o, ra, h->dres, &lv, &lr));
            ok(enqueue_dot(h, L, w, w, n, use_qdot, qtol, o, rb, h->dres + 1, &cv, &cr));
        }
        ok(hipGetLastError());
        if ((k + 1) % 64 == 0) {
            if ((st = read_ctl(h, s, hc)) != QDOT_OK) return st;
            if (hc.done) break;
        }
    }
    // the last enqueued iteration's update (returns at once after a
    // breakdown)
    if (k > 0 && e == hipSuccess) {
        hipLaunchKernelGGL(k_pm_update, dim3(gv), dim3(VB), 0, s, n, ctl, lv, lr, cv, cr, x,
                           wbuf[(k - 1) & 1], lambda_trace, k - 1);
        ok(hipGetLastError());
    }
    if (e != hipSuccess) return hip_fail(h, e, "power launch");
    if ((st = read_ctl(h, s, hc)) != QDOT_OK) return st;
    if (lambda) *lambda = hc.c;
    return hc.status;
}

}  // extern "C"
