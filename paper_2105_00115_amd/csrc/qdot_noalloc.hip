// C ABI: qdot_noalloc_async, the variant of qdot_async that allocates
// nothing.  Its workspace (the control block with the exponent histograms
// and class table, the per-block partials, and the one-pass per-bin tables)
// lives in `scratch`, a file-scope device array of fixed size that every
// GPU running the library holds until the process ends.  The kernels and
// their launch shapes are qdot_async's (default tune entries); only the
// workspace differs.
//
// The kernels leave the parts of the workspace that must start at zero
// (histogram copies, zero and non-finite counters, one-pass tables) zero
// when a call ends; the first call on a device clears the whole array in
// stream order before its own kernels.  All calls on one GPU share its
// array, so calls that overlap on one GPU race.
#include <mutex>

#include "qdot_handle.hpp"

namespace qd {
namespace {

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// scratch layout: [Ws][partials of NOALLOC_BLOCKS blocks][one-pass tables]
constexpr int NOALLOC_BLOCKS = MAX_GRID;
constexpr size_t OFF_PARTIALS = align256(sizeof(Ws));
constexpr size_t OFF_S1TAB = OFF_PARTIALS + align256(sizeof(double) * 6 * NOALLOC_BLOCKS);
constexpr size_t SCRATCH_BYTES =
    OFF_S1TAB + align256(sizeof(double) * HIST_COPIES * W * S1_PIECES);
static_assert(SCRATCH_BYTES % 8 == 0, "scratch is cleared in 8-byte words");

constexpr int MAX_DEVICES = 64;

struct DevScratch {
    bool ready = false;
    int num_cus = 0;
    unsigned char *ptr = nullptr;  // device address of this GPU's copy
};

std::mutex g_mu;
DevScratch g_dev[MAX_DEVICES];

}  // namespace
}  // namespace qd

static __device__ __align__(256) unsigned char scratch[qd::SCRATCH_BYTES];

namespace qd {

__global__ __launch_bounds__(256) void k_scratch_clear(unsigned long long *p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * 256)
        p[i] = 0ull;
}

// This device's scratch address and CU count; on the first call for the
// device, the address is looked up and the array cleared on `s`.
static int32_t scratch_for(int dev, hipStream_t s, DevScratch &out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return QDOT_E_INVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    DevScratch &d = g_dev[dev];
    if (!d.ready) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return QDOT_E_DEVICE;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            cus <= 0)
            return QDOT_E_DEVICE;
        hipLaunchKernelGGL(k_scratch_clear, dim3(256), dim3(256), 0, s,
                           reinterpret_cast<unsigned long long *>(p),
                           (int64_t)(SCRATCH_BYTES / 8));
        if (hipGetLastError() != hipSuccess) return QDOT_E_DEVICE;
        d.ptr = static_cast<unsigned char *>(p);
        d.num_cus = cus;
        d.ready = true;
    }
    out = d;
    return QDOT_OK;
}

}  // namespace qd

using namespace qd;

extern "C" {

int32_t qdot_noalloc_async(const double *x, const double *y, int64_t n, double tol,
                           const qdot_options *opt, void *stream, qdot_result *dev_out)
{
    qdot_options o;
    const char *msg;
    int32_t st = qdot_args(x, y, n, tol, opt, o, &msg);
    if (st != QDOT_OK) return st;
    // tile keys would need memory of their own
    if (!dev_out || o.tile_skip) return QDOT_E_INVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return QDOT_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    DevScratch d;
    if ((st = scratch_for(dev, s, d)) != QDOT_OK) return st;
    Launch L = make_launch_tuned(default_tune(bucket_of(n)), d.num_cus,
                                 reinterpret_cast<Ws *>(d.ptr),
                                 reinterpret_cast<double *>(d.ptr + OFF_PARTIALS),
                                 NOALLOC_BLOCKS, reinterpret_cast<double *>(d.ptr + OFF_S1TAB),
                                 s, false);
    // every grid of the call fits the partials held in the array
    if (L.acc_blocks > NOALLOC_BLOCKS || L.scan_blocks > MAX_GRID || L.s1_blocks > MAX_GRID)
        return QDOT_E_INVAL;
    const hipError_t e = launch_qdot(L, x, y, n, tol, o, dev_out, nullptr, nullptr);
    return e == hipSuccess ? QDOT_OK : QDOT_E_DEVICE;
}

}  // extern "C"
