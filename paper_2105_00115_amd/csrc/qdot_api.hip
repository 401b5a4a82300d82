// C ABI: handle management and the single-vector qdot entry points.
#include <cmath>
#include <cstring>

#include "qdot_handle.hpp"

namespace qd {

int32_t fail(qdot_handle *h, int32_t code, const std::string &msg)
{
    if (h) h->err = msg;
    return code;
}

int32_t hip_fail(qdot_handle *h, hipError_t e, const char *where)
{
    return fail(h, QDOT_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

Launch make_launch(qdot_handle *h, hipStream_t s)
{
    Launch L;
    L.stream = s;
    L.ws = h->ws;
    L.partials = h->partials;
    L.max_blocks = std::min(h->partial_blocks, std::max(1, h->tune.blocks_per_cu) * h->num_cus);
    L.unroll = h->tune.unroll;
    L.ev = nullptr;
    return L;
}

hipEvent_t *take_events(qdot_handle *h, int kind)
{
    if (!h->timing) return nullptr;
    const size_t k = kind == 0 ? 4 : 2;
    while (h->ev_pool.size() < h->ev_used + k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->ev_pool.push_back(e);
    }
    hipEvent_t *ev = h->ev_pool.data() + h->ev_used;
    h->ev_used += k;
    h->ev_kind.push_back(kind);
    return ev;
}

bool options_ok(const qdot_options &o)
{
    return (o.key_mode == 0 || o.key_mode == 1) && (o.score_mode == 0 || o.score_mode == 1) &&
           (o.boundary_mode == 0 || o.boundary_mode == 1) && o.accum_mode == 0;
}

static int32_t check_qdot_args(qdot_handle *h, const double *x, const double *y, int64_t n,
                               double tol, const qdot_options *opt, qdot_options &o)
{
    if (!h) return QDOT_E_INVAL;
    if (n < 0) return fail(h, QDOT_E_INVAL, "n < 0");
    if (n > 0 && (!x || !y)) return fail(h, QDOT_E_INVAL, "NULL vector with n > 0");
    if (((uintptr_t)x | (uintptr_t)y) & 7) return fail(h, QDOT_E_INVAL, "vectors not 8-byte aligned");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(h, QDOT_E_INVAL, "tol must be finite and > 0");
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return fail(h, QDOT_E_INVAL, "unknown option value");
    return QDOT_OK;
}

}  // namespace qd

using namespace qd;

extern "C" {

int32_t qdot_create(qdot_handle **out, int32_t device)
{
    if (!out) return QDOT_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return QDOT_E_INVAL;
    qdot_handle *h = new qdot_handle();
    h->device = device;
    DeviceGuard g(device);
    hipError_t e;
    if ((e = hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, device)) !=
        hipSuccess) {
        delete h;
        return QDOT_E_DEVICE;
    }
    h->partial_blocks = 16 * h->num_cus;
    bool ok = hipMalloc((void **)&h->ws, sizeof(Ws)) == hipSuccess &&
              hipMalloc((void **)&h->partials, sizeof(double) * 6 * h->partial_blocks) == hipSuccess &&
              hipMalloc((void **)&h->dev_res, sizeof(qdot_result)) == hipSuccess &&
              hipHostMalloc((void **)&h->host_res, sizeof(qdot_result), hipHostMallocDefault) ==
                  hipSuccess;
    if (ok) ok = hipMemset(h->ws, 0, sizeof(Ws)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        qdot_destroy(h);
        return QDOT_E_NOMEM;
    }
    *out = h;
    return QDOT_OK;
}

int32_t qdot_destroy(qdot_handle *h)
{
    if (!h) return QDOT_OK;
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    if (h->ws) (void)hipFree(h->ws);
    if (h->partials) (void)hipFree(h->partials);
    if (h->dev_res) (void)hipFree(h->dev_res);
    if (h->host_res) (void)hipHostFree(h->host_res);
    if (h->vec) (void)hipFree(h->vec);
    if (h->ctl) (void)hipFree(h->ctl);
    if (h->res_ring) (void)hipFree(h->res_ring);
    if (h->dres) (void)hipFree(h->dres);
    if (h->host_ctl) (void)hipHostFree(h->host_ctl);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
    return QDOT_OK;
}

const char *qdot_last_error(const qdot_handle *h) { return h ? h->err.c_str() : "null handle"; }

int32_t qdot_device_info(const qdot_handle *h, int32_t *device, int32_t *num_cus)
{
    if (!h) return QDOT_E_INVAL;
    if (device) *device = h->device;
    if (num_cus) *num_cus = h->num_cus;
    return QDOT_OK;
}

int32_t qdot_set_tune(qdot_handle *h, const qdot_tune *cfg)
{
    if (!h) return QDOT_E_INVAL;
    qdot_tune t = {4, 2};
    if (cfg) t = *cfg;
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 16 ||
        !(t.unroll == 1 || t.unroll == 2 || t.unroll == 4))
        return fail(h, QDOT_E_INVAL, "tune out of range (blocks_per_cu 1..16, unroll 1/2/4)");
    h->tune = t;
    return QDOT_OK;
}

int32_t qdot_get_tune(const qdot_handle *h, qdot_tune *cfg)
{
    if (!h || !cfg) return QDOT_E_INVAL;
    *cfg = h->tune;
    return QDOT_OK;
}

int32_t qdot_async(qdot_handle *h, const double *x, const double *y, int64_t n, double tol,
                   const qdot_options *opt, void *stream, qdot_result *dev_out)
{
    qdot_options o;
    int32_t st = check_qdot_args(h, x, y, n, tol, opt, o);
    if (st != QDOT_OK) return st;
    if (!dev_out) return fail(h, QDOT_E_INVAL, "dev_out is NULL");
    DeviceGuard g(h->device);
    Launch L = make_launch(h, (hipStream_t)stream);
    L.ev = take_events(h, 0);
    hipError_t e = launch_qdot(L, x, y, n, tol, o, dev_out, nullptr, nullptr);
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "qdot launch");
}

int32_t qdot(qdot_handle *h, const double *x, const double *y, int64_t n, double tol,
             const qdot_options *opt, void *stream, qdot_result *host_out)
{
    if (!host_out) return fail(h, QDOT_E_INVAL, "host_out is NULL");
    int32_t st = qdot_async(h, x, y, n, tol, opt, stream, h ? h->dev_res : nullptr);
    if (st != QDOT_OK) return st;
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h->host_res, h->dev_res, sizeof(qdot_result),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "qdot result copy");
    *host_out = *h->host_res;
    return host_out->status;
}

int32_t qdot_classes_async(qdot_handle *h, const double *x, const double *y, int64_t n,
                           double tol, const qdot_options *opt, void *stream,
                           uint8_t *dev_cls, int64_t *dev_hist, qdot_result *dev_out)
{
    qdot_options o;
    int32_t st = check_qdot_args(h, x, y, n, tol, opt, o);
    if (st != QDOT_OK) return st;
    if (!dev_out || (n > 0 && !dev_cls)) return fail(h, QDOT_E_INVAL, "NULL output");
    DeviceGuard g(h->device);
    hipError_t e = launch_qdot(make_launch(h, (hipStream_t)stream), x, y, n, tol, o, dev_out,
                               dev_cls, (long long *)dev_hist);
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "qdot_classes launch");
}

int32_t qdot_fp64_dot_async(qdot_handle *h, const double *x, const double *y, int64_t n,
                            void *stream, double *dev_out)
{
    if (!h) return QDOT_E_INVAL;
    if (n < 0 || (n > 0 && (!x || !y)) || !dev_out) return fail(h, QDOT_E_INVAL, "bad argument");
    if (((uintptr_t)x | (uintptr_t)y) & 7) return fail(h, QDOT_E_INVAL, "vectors not 8-byte aligned");
    DeviceGuard g(h->device);
    Launch L = make_launch(h, (hipStream_t)stream);
    L.ev = take_events(h, 1);
    hipError_t e = launch_dot64(L, x, y, n, dev_out);
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "fp64 dot launch");
}

int32_t qdot_timing_enable(qdot_handle *h, int32_t enable)
{
    if (!h) return QDOT_E_INVAL;
    h->timing = enable != 0;
    return QDOT_OK;
}

int32_t qdot_timing_read(qdot_handle *h, double ms[4], int32_t calls[2])
{
    if (!h || !ms || !calls) return QDOT_E_INVAL;
    DeviceGuard g(h->device);
    for (int i = 0; i < 4; i++) ms[i] = 0.0;
    calls[0] = calls[1] = 0;
    size_t at = 0;
    hipError_t e = hipSuccess;
    for (int kind : h->ev_kind) {
        hipEvent_t *ev = h->ev_pool.data() + at;
        const int k = kind == 0 ? 4 : 2;
        if (e == hipSuccess) e = hipEventSynchronize(ev[k - 1]);
        for (int j = 0; j + 1 < k && e == hipSuccess; j++) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ev[j], ev[j + 1]);
            ms[kind == 0 ? j : 3] += t;
        }
        calls[kind]++;
        at += k;
    }
    h->ev_used = 0;
    h->ev_kind.clear();
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "timing read");
}

}  // extern "C"
