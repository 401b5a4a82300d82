/*
 * qdot oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of qdot (the
 * error-bounded quantized dot product of Diffenderfer, Osei-Kuffuor and
 * Menon, arXiv 2105.00115) plus an exact FP64 dot product.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may call it.
 * It shares no code with the device library: different sources, different
 * headers, different result type.
 */
#ifndef QDOT_ORACLE_H
#define QDOT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Keys (exponents of component products) live in [ORC_KMIN, ORC_KMAX]:
 * each operand exponent is in [-1074, 1023] (subnormals included) and the
 * product-mode carry adds at most one. */
#define ORC_KMIN (-2148)
#define ORC_KMAX 2047
#define ORC_W (ORC_KMAX - ORC_KMIN + 1)

/* precision classes */
#define ORC_DOUBLE 0
#define ORC_SINGLE 1
#define ORC_HALF 2
#define ORC_PERF 3

/* flags */
#define ORC_F_UNATTAINABLE 1 /* a bin scored at or above the double mantissa width */
#define ORC_F_THM_ALL_DOUBLE 2 /* early-termination condition (Thm 3.6) holds */
#define ORC_F_ALL_PERF 4     /* no component kept; value is +0 */
#define ORC_F_OVERFLOW 8     /* final scaling overflowed */
#define ORC_F_GUARANTEED 16  /* guaranteed mode: Thm 3.4 bound with a certified E_lo <= tol */
#define ORC_F_RESELECTED 32  /* guaranteed mode: classes selected again, Alg. 1 repeated */

/* status */
#define ORC_OK 0
#define ORC_E_INVAL 1
#define ORC_E_NONFINITE 2
#define ORC_E_BREAKDOWN 5
#define ORC_E_MAXIT 6

typedef struct {
    double value;
    int64_t count[4]; /* DOUBLE, SINGLE, HALF, PERF (PERF includes zeros) */
    int64_t n_zero;
    int32_t e_min, e_max, n_bins, t;
    double part[3];   /* per-class sums (DOUBLE, SINGLE, HALF), absolute */
    double bound_rel; /* Thm 3.3 sum  sum_k M_k 2^(k-e_max+1) eps(class_k) */
    double bound_abs; /* Thm 3.2 sum  2^e_max * bound_rel */
    double bound_rig; /* rigorous absolute bound on |value - x.y| */
    int32_t flags;
    int32_t status;
    double lower;     /* guaranteed mode: certified lower bound of |x.y| (0: none) */
    int32_t e_ref;    /* exponent the scores were taken against */
    int32_t passes;   /* Alg. 1 sweeps that kept a component (0, 1 or 2) */
} orc_result;

/* opt: NULL or 7 ints {key_mode, score_mode, boundary_mode, accum_mode,
 * guard_mode, bin_mode, bin_param}; guard_mode 1 needs key_mode 0 and
 * accum_mode 0.  bin_mode: 0 exact bins, 1 ranged bins of width bin_param
 * (1..ORC_W), 2 variable-width bins from at most bin_param splits
 * (0..ORC_W); modes 1 and 2 need accum_mode 0 and guard_mode 0.
 * cls (n bytes), keys (n int32; zero products get INT32_MIN) and hist
 * (ORC_W int64) are optional outputs. */
int orc_qdot(const double *x, const double *y, int64_t n, double tol,
             const int32_t *opt, orc_result *out, uint8_t *cls,
             int32_t *keys, int64_t *hist);

/* The same for single-precision inputs (mu = m_single): no double class; a
 * bin scoring at or above m_single stays single and is flagged
 * unattainable. */
int orc_qdot_f32(const float *x, const float *y, int64_t n, double tol,
                 const int32_t *opt, orc_result *out, uint8_t *cls,
                 int32_t *keys, int64_t *hist);

/* correctly rounded sum_i x_i y_i (valid while no product over- or
 * underflows), and correctly rounded sum_i |x_i y_i| */
double orc_dot_exact(const double *x, const double *y, int64_t n);
/* Ogita-Rump-Oishi Dot2: compensated dot product, result as if computed
 * in twice FP64 precision and rounded (error bound u|xy| + gamma_n^2 sum|x_i y_i|). */
double orc_dot_dot2(const double *x, const double *y, int64_t n);
double orc_abs_dot(const double *x, const double *y, int64_t n);
/* correctly rounded sum of n doubles */
double orc_sum_exact(const double *v, int64_t n);

/* building blocks exported for the oracle's own pins */
void orc_split(double v, int32_t *E, double *m);
int32_t orc_key(double x, double y, int32_t key_mode);
double orc_r16(double m);
int32_t orc_t(int64_t n_bins, double eps);
int32_t orc_ceil_log2(int64_t m);
int32_t orc_precision(int32_t sigma, int32_t nonstrict);
float orc_tree64(const float *leaves);

/* CSR y = A x (rows summed in stored order, no fused multiply-add) */
void orc_spmv(int64_t n, const int32_t *rowptr, const int32_t *col,
              const double *val, const double *x, double *y);

/* Conjugate gradient (Alg. 4) from x = x0 (in/out).  use_qdot selects qdot
 * at tolerance qtol for both inner products, else the exact dot.  Stops when
 * sqrt(c_k) <= rtol * ||b|| or after maxit iterations.  trace (nullable,
 * 2*maxit+1 results) receives every qdot result in call order. */
int orc_cg(int64_t n, const int32_t *rowptr, const int32_t *col,
           const double *val, const double *b, double *x, double rtol,
           double qtol, int32_t maxit, int32_t use_qdot, const int32_t *opt,
           int32_t *iters, double *relres_est, double *relres_true,
           orc_result *trace);

/* Power method: per iteration w = A x, lambda = dot(x, w), c = dot(w, w),
 * x = w / sqrt(c).  x is a unit vector on entry and exit. lambda_trace
 * (nullable, iters) receives every lambda; trace (nullable, 2*iters) the
 * results of both inner products of every iteration, lambda's first. */
int orc_power(int64_t n, const int32_t *rowptr, const int32_t *col,
              const double *val, double *x, int32_t iters, double qtol,
              int32_t use_qdot, const int32_t *opt, double *lambda,
              double *lambda_trace, orc_result *trace);

#ifdef __cplusplus
}
#endif
#endif
