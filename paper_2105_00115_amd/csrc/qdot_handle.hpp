// Host-side handle shared by the C ABI translation units.
#pragma once

#include <string>
#include <vector>

#include "qdot_kernels.hpp"

struct qdot_handle {
    int device = 0;
    int num_cus = 0;
    qd::Ws *ws = nullptr;            // device control block
    qd::Ws *ws2 = nullptr;           // second one, for the power method's paired products
    double *partials = nullptr;      // per-block partials
    int partial_blocks = 0;          // capacity in blocks
    double *s1tab = nullptr;         // one-pass mode per-bin sums (kept zero between calls)
    qdot_result *dev_res = nullptr;  // device result slot for the sync API
    qdot_result *host_res = nullptr; // pinned host mirror
    qdot_tune tune[QDOT_TUNE_BUCKETS];
    std::string err;

    // solver scratch, grown on demand: the power method keeps w = A x of
    // the current and the previous iteration (2 n doubles), the
    // single-system CG keeps r, p, q (3 n doubles)
    double *vec = nullptr;
    int64_t vec_n = 0;               // doubles held at vec
    void *ctl = nullptr;             // solver control block
    qdot_result *res_ring = nullptr; // solver result slots
    double *dres = nullptr;          // FP64-dot result slots
    void *host_ctl = nullptr;        // pinned mirror of ctl

    // batched qdot: cached work plans (one per offsets layout) and grid size
    std::vector<void *> plans;
    int batch_blocks_per_cu = 4;
    int64_t batch_chunk = 131072;    // components per chunk of a large instance
    int64_t batch_cg_rows = 16384;   // CG rows per gang block
    int batch_cg_gang_max = 16;      // CG gang blocks at most
    int spmv_blocks_per_cu = 8;      // SpMV grid
    int cg_blocks_per_cu = 2;        // single-system CG gang
    int power_scan_in_spmv = 0;      // power method: pass 1 inside the SpMV
    void *cg = nullptr;              // persistent CG buffers

    // tile_skip: largest key slot of every 64-component tile, grown on demand
    short *tiles = nullptr;
    int64_t tiles_cap = 0;           // tiles held at `tiles`

    // kernel timing (diagnostics)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool; // created events, reused after each read
    std::vector<int> ev_kind;        // per timed call: 0 qdot (5 events), 1 dot (2)
    size_t ev_used = 0;
};

namespace qd {

// Make `h->device` current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int32_t fail(qdot_handle *h, int32_t code, const std::string &msg);
int32_t hip_fail(qdot_handle *h, hipError_t e, const char *where);
// Launch shape of a call on n components (the tune bucket of n); single:
// single-precision inputs.
Launch make_launch(qdot_handle *h, hipStream_t s, int64_t n, bool single = false);
// The same from explicit parts: tune entry t, CU count, and the workspace
// (control block, partials for partial_cap blocks, one-pass tables).
Launch make_launch_tuned(const qdot_tune &t, int num_cus, Ws *ws, double *partials,
                         int partial_cap, double *s1tab, hipStream_t s, bool single);
// Tune bucket of a call on n components.
int bucket_of(int64_t n);
// Host-side argument check of a single qdot call (T = double or float):
// QDOT_OK, or QDOT_E_INVAL with a static message in *msg.  o receives the
// options (zero-initialised defaults when opt is NULL).
template <class T>
int32_t qdot_args(const T *x, const T *y, int64_t n, double tol, const qdot_options *opt,
                  qdot_options &o, const char **msg);
qdot_tune default_tune(int bucket);
bool tune_ok(const qdot_tune &t);
// Events for one timed call of `kind` (0: qdot, 5 events; 1: FP64 dot, 2),
// or NULL when timing is off or events cannot be created.
hipEvent_t *take_events(qdot_handle *h, int kind);
bool options_ok(const qdot_options &o);
// One-pass mode (accum_mode 1) preconditions: n within the exact-sum bound
// and a kept-bin depth below the window for any histogram of n components.
bool s1_admissible(int64_t n, double tol, const qdot_options &o);
void free_plans(qdot_handle *h);
void free_cg(qdot_handle *h);
// Grows the solver scratch to at least `doubles` doubles.
int32_t ensure_solver_vectors(qdot_handle *h, int64_t doubles);

}  // namespace qd
