// Internal launch interface between the C ABI layer and the kernels.
#pragma once

#include <algorithm>

#include "qdot_device.hpp"

namespace qd {

struct Launch {
    hipStream_t stream;
    Ws *ws;             // device control block of the handle
    double *partials;   // 6 * partial_cap doubles
    int partial_cap;    // blocks whose partials fit
    int scan_blocks;    // persistent grid cap of the exponent scan
    int scan_unroll;    // 1, 2 or 4 groups of 4 elements in flight per lane
    int acc_blocks;     // grid cap of the accumulate pass / FP64 dot
    int acc_unroll;
    int s1_blocks;      // grid cap and unroll of the one-pass scan
    int s1_unroll;
    int acc_form;       // accumulate pass: 0 every leaf formed in place, 1 compacting
    int hist_copies;    // global histogram copies the scan blocks spread over (1..8)
    int block_threads;  // threads per block of the scan and accumulate (128, 256, 512)
    double *s1tab;      // one-pass mode: HIST_COPIES x W x S1_PIECES sums (zero between calls)
    short *tiles;       // tile_skip: ceil(n / TILE) tile keys, else NULL
    hipEvent_t *ev;     // NULL, or events recorded around each kernel
};

// One-pass mode: number of bins below e_max that can hold kept components,
// for any histogram of n components at this tolerance (the mode is admitted
// when it is <= S1_WIN).
int s1_depth(int64_t n, double tol, const qdot_options &o);

// Enqueue one qdot: scan -> cutoff -> accumulate -> combine (accum_mode 0),
// or one-pass scan -> cutoff -> pick (accum_mode 1).  cls_out (n bytes) and
// hist_out (W int64) are optional debug outputs of mode 0.
hipError_t launch_qdot(const Launch &L, const double *x, const double *y, int64_t n,
                       double tol, const qdot_options &o, qdot_result *out,
                       unsigned char *cls_out, long long *hist_out);

// The power method's pair of inner products, lambda = x . w into out_a and
// c = w . w into out_b, two-pass (accum_mode 0), with one shared pass-1
// kernel and the cutoffs, sweeps and combines of both in one launch each
// (guard_mode 1: its stages per product after the shared pass 1).  La and
// Lb differ only in their workspace; the partials of La hold both sweeps.
// nscan_pre >= 0: pass 1 of both products already ran (into La.ws and
// Lb.ws, nscan_pre block records each) in an earlier kernel on the stream.
hipError_t launch_qdot_pair(const Launch &La, const Launch &Lb, const double *x,
                            const double *w, int64_t n, double tol, const qdot_options &o,
                            qdot_result *out_a, qdot_result *out_b, int nscan_pre = -1);

// The two-pass qdot of single-precision inputs (mu = m_single: no double
// class); accum_mode and guard_mode must be 0.
hipError_t launch_qdot_f32(const Launch &L, const float *x, const float *y, int64_t n,
                           double tol, const qdot_options &o, qdot_result *out,
                           unsigned char *cls_out, long long *hist_out);

// Enqueue the plain FP64 dot; *out receives sum x_i y_i.
hipError_t launch_dot64(const Launch &L, const double *x, const double *y, int64_t n,
                        double *out);

}  // namespace qd
