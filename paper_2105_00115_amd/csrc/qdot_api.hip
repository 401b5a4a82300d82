// C ABI: handle management and the single-vector qdot entry points.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

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

int bucket_of(int64_t n)
{
    return n < ((int64_t)1 << 16) ? 0 : n < ((int64_t)1 << 20) ? 1 : n < ((int64_t)1 << 24) ? 2 : 3;
}

qdot_tune default_tune(int bucket)
{
    // measured on MI355X (256 CUs) at n = 2^27; small sizes keep both passes
    // on the same block -> chunk mapping so the second pass finds the data
    // in the same XCD's L2; the one-pass scan wants more resident blocks
    if (bucket < 3) return qdot_tune{2, 1, 2, 1, 4, 1, 0, HIST_COPIES, BLOCK};
    return qdot_tune{2, 1, 2, 2, 4, 1, 0, HIST_COPIES, BLOCK};
}

bool tune_ok(const qdot_tune &t)
{
    auto u_ok = [](int u) { return u == 1 || u == 2 || u == 4; };
    auto b_ok = [](int b) { return b >= 1 && b <= 16; };
    auto c_ok = [](int c) { return c == 1 || c == 2 || c == 4 || c == HIST_COPIES; };
    return b_ok(t.scan_blocks_per_cu) && b_ok(t.acc_blocks_per_cu) &&
           b_ok(t.onepass_blocks_per_cu) && u_ok(t.scan_unroll) && u_ok(t.acc_unroll) &&
           u_ok(t.onepass_unroll) && (t.acc_form == 0 || t.acc_form == 1) &&
           c_ok(t.hist_copies) &&
           (t.block_threads == 128 || t.block_threads == BLOCK || t.block_threads == 512);
}

Launch make_launch_tuned(const qdot_tune &t, int num_cus, Ws *ws, double *partials,
                         int partial_cap, double *s1tab, hipStream_t s, bool single)
{
    // single-precision inputs: a group is half the bytes, so twice the
    // blocks per CU (at most 8; the kernels also double the groups in
    // flight), which measured fastest for both passes on 2^27 floats
    const int f = single ? 2 : 1;
    Launch L;
    L.stream = s;
    L.ws = ws;
    L.partials = partials;
    L.partial_cap = partial_cap;
    L.scan_blocks = std::min(MAX_GRID, std::min(8, f * t.scan_blocks_per_cu) * num_cus);
    L.scan_unroll = t.scan_unroll;
    L.acc_blocks = std::min(partial_cap, std::min(8, f * t.acc_blocks_per_cu) * num_cus);
    L.acc_unroll = t.acc_unroll;
    L.s1_blocks = std::min(MAX_GRID, t.onepass_blocks_per_cu * num_cus);
    L.s1_unroll = t.onepass_unroll;
    L.s1tab = s1tab;
    L.tiles = nullptr;
    // the compacting form is tuned on double inputs; float inputs keep the
    // dense form of their own tuning
    L.acc_form = single ? 0 : t.acc_form;
    // single-precision inputs run twice the scan blocks: they keep every copy
    L.hist_copies = single ? HIST_COPIES : t.hist_copies;
    L.block_threads = t.block_threads;
    L.ev = nullptr;
    return L;
}

Launch make_launch(qdot_handle *h, hipStream_t s, int64_t n, bool single)
{
    return make_launch_tuned(h->tune[bucket_of(n)], h->num_cus, h->ws, h->partials,
                             h->partial_blocks, h->s1tab, s, single);
}

hipEvent_t *take_events(qdot_handle *h, int kind)
{
    if (!h->timing) return nullptr;
    const size_t k = kind == 0 ? 5 : 2;
    while (h->ev_pool.size() < h->ev_used + k) {
        hipEvent_t e;
        // timing only: no system-scope fence (an L2 writeback and
        // invalidation) at each record between two kernels
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        h->ev_pool.push_back(e);
    }
    hipEvent_t *ev = h->ev_pool.data() + h->ev_used;
    h->ev_used += k;
    h->ev_kind.push_back(kind);
    return ev;
}

bool options_ok(const qdot_options &o)
{
    // the guaranteed mode bins on the exponent of the product (the theorems'
    // bins) and repeats pass 2, so it needs key_mode 0 and accum_mode 0
    // the other binning strategies select once, for the two-pass reading
    const bool bins_ok =
        o.bin_mode == 0 ||
        ((o.bin_mode == 1 ? (o.bin_param >= 1 && o.bin_param <= W)
                          : o.bin_mode == 2 && o.bin_param >= 0 && o.bin_param <= W) &&
         o.accum_mode == 0 && o.guard_mode == 0);
    return (o.key_mode == 0 || o.key_mode == 1) && (o.score_mode == 0 || o.score_mode == 1) &&
           (o.boundary_mode == 0 || o.boundary_mode == 1) &&
           (o.accum_mode == 0 || o.accum_mode == 1) &&
           (o.guard_mode == 0 || (o.guard_mode == 1 && o.key_mode == 0 && o.accum_mode == 0)) &&
           bins_ok &&
           // tile keys serve the second pass of one selection
           (o.tile_skip == 0 || (o.tile_skip == 1 && o.accum_mode == 0 && o.guard_mode == 0));
}

static int ceil_log2_host(int64_t v)
{
    int c = 0;
    while (((int64_t)1 << c) < v) c++;
    return c;
}

// A bin k can be kept only if its score ceil(log2 M_k) + k - e_max - t + 1
// reaches the lowest class boundary (0, or 1 in the non-strict reading is
// higher, so 0 bounds both): e_max - k <= ceil(log2 n) - t + 1.  t is
// smallest for the largest possible bin count min(n, W): t >= floor(log2
// tol) - ceil(log2 min(n, W)) - 1 (adjusted score) or floor(log2 tol) (raw).
int s1_depth(int64_t n, double tol, const qdot_options &o)
{
    int e2 = 0;
    (void)std::frexp(tol, &e2);  // tol = f 2^e2, f in [0.5, 1)
    const int fl = e2 - 1;       // floor(log2 tol)
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(n, W));
    const int t_low = o.score_mode == 0 ? fl - ceil_log2_host(nb) - 1 : fl;
    // bins e_max - d for d = 0 .. ceil(log2 n) - t_low + 1
    return ceil_log2_host(std::max<int64_t>(1, n)) - t_low + 2;
}

bool s1_admissible(int64_t n, double tol, const qdot_options &o)
{
    return n <= S1_MAX_N && s1_depth(n, tol, o) <= S1_WIN;
}

template <class T>
int32_t qdot_args(const T *x, const T *y, int64_t n, double tol, const qdot_options *opt,
                  qdot_options &o, const char **msg)
{
    *msg = "";
    if (n < 0) return *msg = "n < 0", QDOT_E_INVAL;
    if (n > 0 && (!x || !y)) return *msg = "NULL vector with n > 0", QDOT_E_INVAL;
    if (((uintptr_t)x | (uintptr_t)y) & (sizeof(T) - 1))
        return *msg = "vectors not aligned to their element size", QDOT_E_INVAL;
    if (!(tol > 0.0) || !std::isfinite(tol))
        return *msg = "tol must be finite and > 0", QDOT_E_INVAL;
    std::memset(&o, 0, sizeof o);
    if (opt) o = *opt;
    if (!options_ok(o)) return *msg = "unknown option value", QDOT_E_INVAL;
    if (o.accum_mode == 1 && !s1_admissible(n, tol, o))
        return *msg = "accum_mode 1 needs n <= 2^30 and a tolerance whose "
                      "kept bins fit the one-pass window",
               QDOT_E_INVAL;
    return QDOT_OK;
}
template int32_t qdot_args<double>(const double *, const double *, int64_t, double,
                                   const qdot_options *, qdot_options &, const char **);
template int32_t qdot_args<float>(const float *, const float *, int64_t, double,
                                  const qdot_options *, qdot_options &, const char **);

// tile_skip: make the handle's tile keys cover n components and point L at
// them.  Growing the buffer allocates (after the device has drained, since
// earlier calls may still read the old one), so it is refused while the
// stream is being captured.
static int32_t attach_tiles(qdot_handle *h, hipStream_t s, int64_t n, const qdot_options &o,
                            Launch &L)
{
    if (!o.tile_skip) return QDOT_OK;
    const int64_t need = std::max<int64_t>(1, (n + TILE - 1) / TILE);
    if (h->tiles_cap < need) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
            return fail(h, QDOT_E_INVAL,
                        "tile_skip: the tile keys must grow (first call with this n) "
                        "outside graph capture");
        if (h->tiles) (void)hipFree(h->tiles);
        h->tiles = nullptr;
        h->tiles_cap = 0;
        if (hipMalloc((void **)&h->tiles, sizeof(short) * (size_t)need) != hipSuccess) {
            h->tiles = nullptr;
            return fail(h, QDOT_E_NOMEM, "tile key allocation failed");
        }
        h->tiles_cap = need;
    }
    L.tiles = h->tiles;
    return QDOT_OK;
}

template <class T>
static int32_t check_qdot_args(qdot_handle *h, const T *x, const T *y, int64_t n, double tol,
                               const qdot_options *opt, qdot_options &o)
{
    if (!h) return QDOT_E_INVAL;
    const char *msg;
    const int32_t st = qdot_args(x, y, n, tol, opt, o, &msg);
    return st == QDOT_OK ? st : fail(h, st, msg);
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
    h->partial_blocks = std::min(MAX_GRID, 16 * h->num_cus);
    for (int b = 0; b < QDOT_TUNE_BUCKETS; b++) h->tune[b] = default_tune(b);
    bool ok = hipMalloc((void **)&h->ws, sizeof(Ws)) == hipSuccess &&
              hipMalloc((void **)&h->partials, sizeof(double) * 6 * h->partial_blocks) == hipSuccess &&
              hipMalloc((void **)&h->dev_res, sizeof(qdot_result)) == hipSuccess &&
              hipMalloc((void **)&h->s1tab, sizeof(double) * HIST_COPIES * W * S1_PIECES) ==
                  hipSuccess &&
              hipHostMalloc((void **)&h->host_res, sizeof(qdot_result), hipHostMallocDefault) ==
                  hipSuccess;
    if (ok) {
        ok = hipMemset(h->ws, 0, sizeof(Ws)) == hipSuccess &&
             hipMemset(h->s1tab, 0, sizeof(double) * HIST_COPIES * W * S1_PIECES) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        qdot_destroy(h);
        return QDOT_E_NOMEM;
    }
    if (const char *p = std::getenv("QDOT_TUNE_FILE")) (void)qdot_load_tune(h, p);
    *out = h;
    return QDOT_OK;
}

int32_t qdot_destroy(qdot_handle *h)
{
    if (!h) return QDOT_OK;
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    if (h->ws) (void)hipFree(h->ws);
    if (h->ws2) (void)hipFree(h->ws2);
    if (h->s1tab) (void)hipFree(h->s1tab);
    if (h->partials) (void)hipFree(h->partials);
    if (h->dev_res) (void)hipFree(h->dev_res);
    if (h->host_res) (void)hipHostFree(h->host_res);
    if (h->vec) (void)hipFree(h->vec);
    if (h->tiles) (void)hipFree(h->tiles);
    if (h->ctl) (void)hipFree(h->ctl);
    if (h->res_ring) (void)hipFree(h->res_ring);
    if (h->dres) (void)hipFree(h->dres);
    if (h->host_ctl) (void)hipHostFree(h->host_ctl);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    free_plans(h);
    free_cg(h);
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

int32_t qdot_set_tune(qdot_handle *h, int32_t bucket, const qdot_tune *cfg)
{
    if (!h) return QDOT_E_INVAL;
    if (bucket < -1 || bucket >= QDOT_TUNE_BUCKETS) return fail(h, QDOT_E_INVAL, "bad bucket");
    for (int b = 0; b < QDOT_TUNE_BUCKETS; b++) {
        if (bucket != -1 && b != bucket) continue;
        const qdot_tune t = cfg ? *cfg : default_tune(b);
        if (!tune_ok(t))
            return fail(h, QDOT_E_INVAL, "tune out of range (blocks per CU 1..16, unroll "
                                         "1/2/4, acc_form 0/1, hist_copies 1/2/4/8, "
                                         "block_threads 128/256/512)");
        h->tune[b] = t;
    }
    return QDOT_OK;
}

int32_t qdot_get_tune(const qdot_handle *h, int32_t bucket, qdot_tune *cfg)
{
    if (!h || !cfg || bucket < 0 || bucket >= QDOT_TUNE_BUCKETS) return QDOT_E_INVAL;
    *cfg = h->tune[bucket];
    return QDOT_OK;
}

int32_t qdot_load_tune(qdot_handle *h, const char *path)
{
    if (!h || !path) return QDOT_E_INVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(h, QDOT_E_INVAL, std::string("cannot open tune file ") + path);
    qdot_tune t[QDOT_TUNE_BUCKETS];
    for (int b = 0; b < QDOT_TUNE_BUCKETS; b++) t[b] = h->tune[b];
    qdot_solver_tune bt;
    (void)qdot_get_solver_tune(h, &bt);
    bool have_solver = false;
    char line[256];
    bool ok = true;
    while (ok && std::fgets(line, sizeof line, f)) {
        char *hash = std::strchr(line, '#');
        if (hash) *hash = 0;
        // "solver batch_bpc batch_chunk cg_rows_per_block cg_gang_max spmv_bpc cg_bpc
        // power_scan_in_spmv"
        int bv[7];
        if (std::sscanf(line, " solver %d %d %d %d %d %d %d", &bv[0], &bv[1], &bv[2], &bv[3],
                        &bv[4], &bv[5], &bv[6]) == 7) {
            bt = qdot_solver_tune{bv[0], bv[1], bv[2], bv[3], bv[4], bv[5], bv[6]};
            have_solver = true;
            continue;
        }
        if (std::strstr(line, "solver")) {
            ok = false;
            continue;
        }
        int b = -1, v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const int got = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d", &b, &v[0], &v[1],
                                    &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8]);
        if (got <= 0) continue;  // blank or comment
        if ((got != 5 && got != 7 && got != 9 && got != 10) || b < 0 ||
            b >= QDOT_TUNE_BUCKETS) {
            ok = false;
            continue;
        }
        qdot_tune c = t[b];
        c.scan_blocks_per_cu = v[0];
        c.scan_unroll = v[1];
        c.acc_blocks_per_cu = v[2];
        c.acc_unroll = v[3];
        if (got >= 7) {
            c.onepass_blocks_per_cu = v[4];
            c.onepass_unroll = v[5];
        }
        if (got >= 9) {
            c.acc_form = v[6];
            c.hist_copies = v[7];
        }
        if (got == 10) c.block_threads = v[8];
        if (!tune_ok(c)) ok = false;
        else t[b] = c;
    }
    std::fclose(f);
    if (!ok) return fail(h, QDOT_E_INVAL, std::string("malformed tune file ") + path);
    qdot_solver_tune cur;
    (void)qdot_get_solver_tune(h, &cur);
    if (have_solver && std::memcmp(&cur, &bt, sizeof bt) != 0) {
        const int32_t st = qdot_set_solver_tune(h, &bt);
        if (st != QDOT_OK) return st;
    }
    for (int b = 0; b < QDOT_TUNE_BUCKETS; b++) h->tune[b] = t[b];
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
    Launch L = make_launch(h, (hipStream_t)stream, n);
    if ((st = attach_tiles(h, (hipStream_t)stream, n, o, L)) != QDOT_OK) return st;
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

int32_t qdot_f32_async(qdot_handle *h, const float *x, const float *y, int64_t n, double tol,
                       const qdot_options *opt, void *stream, qdot_result *dev_out)
{
    qdot_options o;
    int32_t st = check_qdot_args(h, x, y, n, tol, opt, o);
    if (st != QDOT_OK) return st;
    if (!dev_out) return fail(h, QDOT_E_INVAL, "dev_out is NULL");
    DeviceGuard g(h->device);
    Launch L = make_launch(h, (hipStream_t)stream, n, true);
    if ((st = attach_tiles(h, (hipStream_t)stream, n, o, L)) != QDOT_OK) return st;
    L.ev = take_events(h, 0);
    hipError_t e = launch_qdot_f32(L, x, y, n, tol, o, dev_out, nullptr, nullptr);
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "qdot_f32 launch");
}

int32_t qdot_f32(qdot_handle *h, const float *x, const float *y, int64_t n, double tol,
                 const qdot_options *opt, void *stream, qdot_result *host_out)
{
    if (!host_out) return fail(h, QDOT_E_INVAL, "host_out is NULL");
    int32_t st = qdot_f32_async(h, x, y, n, tol, opt, stream, h ? h->dev_res : nullptr);
    if (st != QDOT_OK) return st;
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h->host_res, h->dev_res, sizeof(qdot_result),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "qdot_f32 result copy");
    *host_out = *h->host_res;
    return host_out->status;
}

int32_t qdot_f32_classes_async(qdot_handle *h, const float *x, const float *y, int64_t n,
                               double tol, const qdot_options *opt, void *stream,
                               uint8_t *dev_cls, int64_t *dev_hist, qdot_result *dev_out)
{
    qdot_options o;
    int32_t st = check_qdot_args(h, x, y, n, tol, opt, o);
    if (st != QDOT_OK) return st;
    if (!dev_out || (n > 0 && !dev_cls)) return fail(h, QDOT_E_INVAL, "NULL output");
    if (o.accum_mode != 0)
        return fail(h, QDOT_E_INVAL, "qdot_f32_classes_async needs accum_mode 0");
    DeviceGuard g(h->device);
    Launch L = make_launch(h, (hipStream_t)stream, n, true);
    if ((st = attach_tiles(h, (hipStream_t)stream, n, o, L)) != QDOT_OK) return st;
    hipError_t e = launch_qdot_f32(L, x, y, n, tol, o, dev_out, dev_cls, (long long *)dev_hist);
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "qdot_f32_classes launch");
}

int32_t qdot_simple(const double *x, const double *y, int64_t n, double tol, double *value,
                    int64_t counts[4])
{
    if (!value) return QDOT_E_INVAL;
    static std::mutex mu;
    static std::map<int, qdot_handle *> handles;  // per device, kept for the process
    std::lock_guard<std::mutex> lock(mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return QDOT_E_DEVICE;
    qdot_handle *&h = handles[dev];
    if (!h) {
        const int32_t st = qdot_create(&h, dev);
        if (st != QDOT_OK) {
            h = nullptr;
            return st;
        }
    }
    qdot_result r;
    const int32_t st = qdot(h, x, y, n, tol, nullptr, nullptr, &r);
    if (st != QDOT_OK && st != QDOT_E_NONFINITE) return st;
    *value = r.value;
    if (counts)
        for (int q = 0; q < 4; q++) counts[q] = r.count[q];
    return st;
}

int32_t qdot_classes_async(qdot_handle *h, const double *x, const double *y, int64_t n,
                           double tol, const qdot_options *opt, void *stream,
                           uint8_t *dev_cls, int64_t *dev_hist, qdot_result *dev_out)
{
    qdot_options o;
    int32_t st = check_qdot_args(h, x, y, n, tol, opt, o);
    if (st != QDOT_OK) return st;
    if (!dev_out || (n > 0 && !dev_cls)) return fail(h, QDOT_E_INVAL, "NULL output");
    if (o.accum_mode != 0) return fail(h, QDOT_E_INVAL, "qdot_classes_async needs accum_mode 0");
    DeviceGuard g(h->device);
    Launch L = make_launch(h, (hipStream_t)stream, n);
    if ((st = attach_tiles(h, (hipStream_t)stream, n, o, L)) != QDOT_OK) return st;
    hipError_t e = launch_qdot(L, x, y, n, tol, o, dev_out, dev_cls, (long long *)dev_hist);
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "qdot_classes launch");
}

int32_t qdot_fp64_dot_async(qdot_handle *h, const double *x, const double *y, int64_t n,
                            void *stream, double *dev_out)
{
    if (!h) return QDOT_E_INVAL;
    if (n < 0 || (n > 0 && (!x || !y)) || !dev_out) return fail(h, QDOT_E_INVAL, "bad argument");
    if (((uintptr_t)x | (uintptr_t)y) & 7) return fail(h, QDOT_E_INVAL, "vectors not 8-byte aligned");
    DeviceGuard g(h->device);
    Launch L = make_launch(h, (hipStream_t)stream, n);
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

int32_t qdot_timing_read(qdot_handle *h, double ms[5], int32_t calls[2])
{
    if (!h || !ms || !calls) return QDOT_E_INVAL;
    DeviceGuard g(h->device);
    for (int i = 0; i < 5; i++) ms[i] = 0.0;
    calls[0] = calls[1] = 0;
    size_t at = 0;
    hipError_t e = hipSuccess;
    for (int kind : h->ev_kind) {
        hipEvent_t *ev = h->ev_pool.data() + at;
        const int k = kind == 0 ? 5 : 2;
        if (e == hipSuccess) e = hipEventSynchronize(ev[k - 1]);
        for (int j = 0; j + 1 < k && e == hipSuccess; j++) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ev[j], ev[j + 1]);
            ms[kind == 0 ? j : 4] += t;
        }
        calls[kind]++;
        at += k;
    }
    h->ev_used = 0;
    h->ev_kind.clear();
    return e == hipSuccess ? QDOT_OK : hip_fail(h, e, "timing read");
}

}  // extern "C"
