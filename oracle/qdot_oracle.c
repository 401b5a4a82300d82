/*
 * qdot oracle -- TEST INFRASTRUCTURE ONLY (see qdot_oracle.h).
 *
 * Plain, single-threaded, unblocked.  Every step follows the paper in its
 * own order and notation:
 *
 *   Alg. 3 (qdot)  = Alg. 2 (parameter selection) then Alg. 1 (computation).
 *   Alg. 2: exponents of the component products, min/max, exact bins
 *           (Sec. 3.2, "exact binning"), bin scores eq. (bin-score-def),
 *           precisions eq. (precision-def).
 *   Alg. 1: per-bin products at the bin's precision after scaling to
 *           exponent 0 (Sec. 3.2 and 3.3), then accumulation at input
 *           precision.
 *
 * Readings of passages the paper leaves open are stated where they are used;
 * the list of them is kept with the design notes.
 *
 * Build with -ffp-contract=off: every product and sum below is one IEEE
 * operation in the type written.
 */
#include "qdot_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Internal class of single-precision inputs for the bins that eq.
 * (precision-def) cannot lower: the product is formed at the input
 * precision (FP32) and added at input precision or better, here exactly,
 * with the double leaves (Alg. 1's accumulation at the precision of x and
 * y; the FP32 tile trees are for the narrower classes).  Counted and
 * reported as single. */
#define ORC_SINGLE_IN 4

/* mantissa widths m_half, m_single, m_double of eq. (precision-def) */
#define M_HALF 10
#define M_SINGLE 23
#define M_DOUBLE 52

/* ------------------------------------------------------------------ */
/* Exact summation: Shewchuk's non-overlapping expansion ("Adaptive    */
/* precision floating-point arithmetic", 1997), with a correctly        */
/* rounded read-out.  Used for the exact dot and for every "sum this     */
/* exactly, round once" step.                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    double *p; /* non-overlapping partials, increasing magnitude */
    int n;
    int cap;
} xsum;

static void xs_init(xsum *s)
{
    s->cap = 64;
    s->n = 0;
    s->p = (double *)malloc(sizeof(double) * (size_t)s->cap);
}

static void xs_free(xsum *s) { free(s->p); }

/* Add one double exactly: run it up the expansion with error-free
 * two-sums, keeping every non-zero error term. */
static void xs_add(xsum *s, double v)
{
    int kept = 0;
    for (int j = 0; j < s->n; j++) {
        double a = v, b = s->p[j];
        if (fabs(a) < fabs(b)) {
            double tmp = a;
            a = b;
            b = tmp;
        }
        double sum = a + b;            /* |a| >= |b|: Fast2Sum is exact */
        double err = b - (sum - a);
        if (err != 0.0) s->p[kept++] = err;
        v = sum;
    }
    if (kept + 1 > s->cap) {
        s->cap *= 2;
        s->p = (double *)realloc(s->p, sizeof(double) * (size_t)s->cap);
    }
    s->p[kept++] = v;
    s->n = kept;
}

/* Nearest double to the exact value of the expansion (ties to even). */
static double xs_round(const xsum *s)
{
    int k = s->n;
    /* drop zero top partials */
    while (k > 0 && s->p[k - 1] == 0.0) k--;
    if (k == 0) return 0.0;
    double hi = s->p[--k];
    double lo = 0.0;
    /* Fold partials in from the top while the fold stays exact. */
    while (k > 0) {
        double b = s->p[--k];
        double sum = hi + b;
        double err = b - (sum - hi);
        hi = sum;
        if (err != 0.0) {
            lo = err;
            break;
        }
    }
    /* hi + lo is exact; lo is at most half an ulp of hi.  If lo is exactly
     * half an ulp the rounding of hi + lo went to even, but smaller partials
     * of lo's sign push the true value past the midpoint: round away. */
    if (lo != 0.0 && k > 0) {
        double below = s->p[k - 1];
        if ((lo > 0.0 && below > 0.0) || (lo < 0.0 && below < 0.0)) {
            double twice = lo * 2.0;
            double cand = hi + twice;
            if (cand - hi == twice) hi = cand;
        }
    }
    return hi;
}

double orc_sum_exact(const double *v, int64_t n)
{
    xsum s;
    xs_init(&s);
    for (int64_t i = 0; i < n; i++) xs_add(&s, v[i]);
    double r = xs_round(&s);
    xs_free(&s);
    return r;
}

/* x.y exactly: each product split into fl(x y) and its rounding error
 * (fma gives the error exactly while it does not underflow), then the 2n
 * terms summed exactly. */
double orc_dot_exact(const double *x, const double *y, int64_t n)
{
    xsum s;
    xs_init(&s);
    for (int64_t i = 0; i < n; i++) {
        double p = x[i] * y[i];
        double e = fma(x[i], y[i], -p);
        xs_add(&s, p);
        xs_add(&s, e);
    }
    double r = xs_round(&s);
    xs_free(&s);
    return r;
}

/* Dot2 (Ogita, Rump and Oishi, "Accurate sum and dot product", SIAM J. Sci.
 * Comput. 2005): the running sum p and a running correction s; every
 * product is split exactly (TwoProduct, here by fma) and every addition to
 * p exactly (Knuth's TwoSum); the errors are added in plain FP64.  Result as
 * if computed in twice the working precision, then rounded. */
double orc_dot_dot2(const double *x, const double *y, int64_t n)
{
    if (n <= 0) return 0.0;
    double p = x[0] * y[0];
    double s = fma(x[0], y[0], -p);
    for (int64_t i = 1; i < n; i++) {
        const double h = x[i] * y[i];
        const double r = fma(x[i], y[i], -h);
        const double q = p + h;            /* TwoSum(p, h) = (q, e) */
        const double z = q - p;
        const double e = (p - (q - z)) + (h - z);
        p = q;
        s = s + (e + r);
    }
    return p + s;
}

double orc_abs_dot(const double *x, const double *y, int64_t n)
{
    xsum s;
    xs_init(&s);
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(x[i]), b = fabs(y[i]);
        double p = a * b;
        double e = fma(a, b, -p);
        xs_add(&s, p);
        xs_add(&s, e);
    }
    double r = xs_round(&s);
    xs_free(&s);
    return r;
}

/* ------------------------------------------------------------------ */
/* Parameter selection (Alg. 2)                                          */
/* ------------------------------------------------------------------ */

/* Unbiased exponent and significand of a nonzero finite double (Sec. 1.1:
 * flexp).  Read as floor(log2|v|) for every |v| (subnormals normalised):
 * the proofs of Thms 3.2-3.4 need |v| >= 2^flexp(v), which the ceiling
 * branch printed for |v| < 1 would break. */
void orc_split(double v, int32_t *E, double *m)
{
    *E = ilogb(v);
    *m = scalbn(fabs(v), -*E); /* exact, in [1, 2) */
}

/* Key of one component product x*y (both nonzero, finite).
 * key_mode 0 (product): the exponent of x*y itself, as Def. 3.1 and the
 *   theorems bin on flexp(x (.) y): E(x) + E(y), plus one when the
 *   significand product m_x m_y reaches 2.
 * key_mode 1 (sum): E(x) + E(y), as the exponent-preprocessing step of
 *   Alg. 2 writes it. */
int32_t orc_key(double x, double y, int32_t key_mode)
{
    int32_t ex, ey;
    double mx, my;
    orc_split(x, &ex, &mx);
    orc_split(y, &ey, &my);
    int32_t k = ex + ey;
    if (key_mode == 0 && mx * my >= 2.0) k += 1;
    return k;
}

/* Binary16 rounding of a significand m in [1, 2): nearest multiple of
 * 2^-10, ties to even, taken directly from the FP64 value (one rounding).
 * Returned as the integer m16 * 2^10 in [1024, 2048]. */
double orc_r16(double m) { return nearbyint(ldexp(m, 10)); }

/* ceil(log2 m) for m >= 1 */
int32_t orc_ceil_log2(int64_t m)
{
    int32_t c = 0;
    while (c < 63 && ((int64_t)1 << c) < m) c++;
    return c;
}

/* t = floor(log2(eps / N_bins)) exactly: the largest integer tau with
 * N_bins * 2^tau <= eps.  (Bin score with eps replaced by eps / N_bins, as
 * the experiments of Sec. 4.1 do so that the bound of Thm 3.5 becomes eps.)
 * Each comparison is exact: eps is first moved into the normal range by an
 * exact power-of-two scaling. */
int32_t orc_t(int64_t n_bins, double eps)
{
    int shift = 0;
    if (eps < 0x1p-900) shift = 600;
    else if (eps > 0x1p900) shift = -600;
    double e2 = ldexp(eps, shift);
    double nb = (double)n_bins;
    int32_t tau = ilogb(e2) - orc_ceil_log2(n_bins);
    while (ldexp(nb, tau + 1) <= e2) tau++;
    while (ldexp(nb, tau) > e2) tau--;
    return tau - shift;
}

/* eq. (precision-def): Double on [m_single, m_double), Single on
 * [m_half, m_single), Half on [0, m_half), Perforate below 0 (strict,
 * half-open as printed).  The non-strict reading takes the proof's wording
 * instead (perforate when the score is <= 0, otherwise the narrowest format
 * whose mantissa width is >= the score).  Scores at or above m_double have
 * no row; they stay double (and are flagged by the caller). */
int32_t orc_precision(int32_t sigma, int32_t nonstrict)
{
    if (!nonstrict) {
        if (sigma < 0) return ORC_PERF;
        if (sigma < M_HALF) return ORC_HALF;
        if (sigma < M_SINGLE) return ORC_SINGLE;
        return ORC_DOUBLE;
    }
    if (sigma <= 0) return ORC_PERF;
    if (sigma <= M_HALF) return ORC_HALF;
    if (sigma <= M_SINGLE) return ORC_SINGLE;
    return ORC_DOUBLE;
}

/* FP32 sum of one 64-leaf tile by the adjacent-pairwise tree: level 1 adds
 * leaves (2m, 2m+1), each later level adds neighbouring results, six levels
 * in all, each addition one FP32 rounding. */
float orc_tree64(const float *leaves)
{
    float v[64];
    memcpy(v, leaves, sizeof v);
    for (int w = 64; w > 1; w >>= 1)
        for (int m = 0; m < w / 2; m++) v[m] = v[2 * m] + v[2 * m + 1];
    return v[0];
}

static double eps_of(int cls)
{
    switch (cls) {
    case ORC_DOUBLE: return 0x1p-52;
    case ORC_SINGLE:
    case ORC_SINGLE_IN: return 0x1p-23;
    case ORC_HALF: return 0x1p-10;
    default: return 1.0; /* perforated: the whole term is the error */
    }
}

/* One (l, u]-exponent bin (Def. 3.1) over the keys: it holds the keys
 * lo = l + 1 .. u, M components in all. */
typedef struct {
    int32_t lo, u;
    int64_t M;
} orc_bin;

/* M_a 2^u_a > M_b 2^u_b (the bins' terms of the Thm 3.2 bound before
 * eps(k)), ties to the higher u.  Counts below 2^53 convert exactly. */
static int orc_bin_heavier(const orc_bin *a, const orc_bin *b)
{
    int32_t d = a->u - b->u;
    if (d >= 64) return 1;
    if (d <= -64) return 0;
    double va = ldexp((double)a->M, d), vb = (double)b->M;
    if (va != vb) return va > vb;
    return a->u > b->u;
}

/* Partition of [e_min, e_max] into exponent bins, by the binning strategies
 * Sec. 3.2 weighs (the passage the typeset paper keeps names exact binning;
 * the authors' draft of it also defines the other two):
 *   bin_mode 0, exact: singletons (u - 1, u], u = e_min .. e_max;
 *   bin_mode 1, ranged of width w = bin_param: (u_k - w, u_k] with
 *     u_k = e_min + k w - 1, k = 1, 2, ... (the last may reach past e_max);
 *   bin_mode 2, variable width (bin splitting) with at most s = bin_param
 *     splits: start from the single bin (e_min - 1, e_max]; each split takes
 *     the non-empty bin of more than one exponent with the largest term
 *     M_k 2^(u_k) of the Thm 3.2 bound (ties to the higher u_k) and halves
 *     it: (l, u] -> (l, m], (m, u] with m = l + ceil((u - l) / 2).  The
 *     draft fixes neither the bin that is split nor where; this reading
 *     splits where the bound is largest, at the middle.  s >= e_max - e_min
 *     splits reach exact binning.
 * Empty bins are kept (they have no score and do not count in N_bins).
 * Returns the number of bins written to `bins` (at most ORC_W + 1). */
static int orc_partition(const int64_t *M, int32_t e_min, int32_t e_max, int32_t bin_mode,
                         int32_t bin_param, orc_bin *bins)
{
    int nb = 0;
    if (bin_mode != 2) {
        int32_t w = bin_mode == 1 ? bin_param : 1;
        for (int32_t lo = e_min; lo <= e_max; lo += w) {
            orc_bin b = {lo, lo + w - 1, 0};
            for (int32_t k = lo; k <= b.u && k <= e_max; k++) b.M += M[k - ORC_KMIN];
            bins[nb++] = b;
        }
        return nb;
    }
    orc_bin all = {e_min, e_max, 0};
    for (int32_t k = e_min; k <= e_max; k++) all.M += M[k - ORC_KMIN];
    bins[nb++] = all;
    for (int32_t s = 0; s < bin_param; s++) {
        int best = -1;
        for (int i = 0; i < nb; i++) {
            if (bins[i].M == 0 || bins[i].u == bins[i].lo) continue;
            if (best < 0 || orc_bin_heavier(&bins[i], &bins[best])) best = i;
        }
        if (best < 0) break; /* every non-empty bin is a single exponent */
        orc_bin b = bins[best];
        int32_t l = b.lo - 1;
        int32_t m = l + (b.u - l + 1) / 2;   /* l + ceil((u - l) / 2) */
        orc_bin lower = {b.lo, m, 0}, upper = {m + 1, b.u, 0};
        for (int32_t k = lower.lo; k <= lower.u; k++) lower.M += M[k - ORC_KMIN];
        upper.M = b.M - lower.M;
        bins[best] = upper;
        bins[nb++] = lower;
    }
    return nb;
}

/* Classes of every bin (eq. (bin-score-def), eq. (precision-def)) with the
 * scores taken against the reference exponent e_ref: e_max as Alg. 2 has
 * it, or a lower estimate of flexp(x.y) when the guaranteed mode reselects
 * (Thm 3.4 puts E in place of e_max).  Fills the class table C (per key:
 * the class of the key's bin), the class counts, the Thm 3.3 sum relative
 * to e_max and the selection flags. */
static void orc_select(const orc_bin *bins, int nbins, int32_t e_max, int32_t e_min,
                       int32_t e_ref, int32_t t, int32_t nonstrict, int mu_single,
                       int64_t n_zero, uint8_t *C, orc_result *r)
{
    /* eq. (precision-def) admits a row only when mu is at least the row's
     * mantissa width: with single inputs (mu = m_single) there is no double
     * row, a bin scoring at or above m_single stays at the input precision
     * (ORC_SINGLE_IN) and is flagged, as a double bin scoring at or above
     * m_double is. */
    const int32_t m_top = mu_single ? M_SINGLE : M_DOUBLE;
    xsum brel;
    xs_init(&brel);
    for (int c = 0; c < 4; c++) r->count[c] = 0;
    r->flags = 0;
    for (int32_t k = ORC_KMIN; k <= ORC_KMAX; k++) C[k - ORC_KMIN] = ORC_PERF;
    for (int i = 0; i < nbins; i++) {
        int64_t Mk = bins[i].M;
        int32_t u = bins[i].u;
        if (Mk == 0) continue; /* empty bin: score -inf */
        int32_t sigma = orc_ceil_log2(Mk) + u - e_ref - t + 1;
        int32_t c = orc_precision(sigma, nonstrict);
        if (mu_single && c == ORC_DOUBLE) c = ORC_SINGLE_IN;
        if (nonstrict ? sigma > m_top : sigma >= m_top)
            r->flags |= ORC_F_UNATTAINABLE;
        for (int32_t k = bins[i].lo; k <= u && k <= ORC_KMAX; k++) C[k - ORC_KMIN] = (uint8_t)c;
        r->count[c == ORC_SINGLE_IN ? ORC_SINGLE : c] += Mk;
        /* Thm 3.3 term M_k 2^(u_k - e_max + 1) eps(k) */
        xs_add(&brel, ldexp((double)Mk * eps_of(c), u - e_max + 1));
    }
    r->count[ORC_PERF] += n_zero;
    r->bound_rel = xs_round(&brel);
    r->bound_abs = ldexp(r->bound_rel, e_max);
    xs_free(&brel);
    /* Thm 3.6 (early termination): all bins at input precision when
     * e_ref - e_min <= -floor(log2 eps) - m, m the mantissa width of the
     * precision just below the input's (m_single for double inputs, m_half
     * for single inputs). */
    if ((int64_t)e_ref - e_min <= -(int64_t)t - (mu_single ? M_HALF : M_SINGLE))
        r->flags |= ORC_F_THM_ALL_DOUBLE;
    if (r->count[ORC_DOUBLE] + r->count[ORC_SINGLE] + r->count[ORC_HALF] == 0)
        r->flags |= ORC_F_ALL_PERF;
}

/* Alg. 1 over the classes C.  Every kept component is scaled to exponent 0
 * (x_i -> m_x, y_i -> m_y), cast to its bin's precision, multiplied there,
 * and scaled back by 2^(E(x)+E(y)).  Scaling back is written relative to
 * 2^e_max (double leaves) or 2^c32 (FP32 leaves); both offsets are exact
 * powers of two and the final result is multiplied by 2^e_max once.
 *   double: fl64(m_x m_y)
 *   single: fl32(fl32(m_x) fl32(m_y))            (FP32 product)
 *   half:   r16(m_x) r16(m_y), exact in FP32     (FP16 operands, FP32
 *                                                 product/accumulation)
 *   single inputs held at their own precision (ORC_SINGLE_IN): the single
 *   product, summed with the double leaves relative to 2^e_max (a range no
 *   FP32 tile could hold: such bins may sit anywhere below e_max).
 * accum_mode 0: FP32 leaves are summed in FP32 only inside 64-element tiles
 * of the original index order (adjacent-pairwise tree); tile sums and
 * double leaves are then summed at input precision: exactly, rounded once.
 * accum_mode 1: every leaf is summed exactly, rounded once.
 * c32 = e_ref + t + 22 keeps every single/half leaf a normal FP32 number
 * below 4 whatever the tolerance.  Returns S, the sum in units of 2^e_max;
 * writes value, part, bound_rig and the overflow flag. */
static double orc_compute(const double *x, const double *y, int64_t n, const int32_t *key,
                          const uint8_t *C, int32_t e_max, int32_t c32, int32_t accum_mode,
                          uint8_t *cls_out, orc_result *r)
{
    xsum all, pd, ps, ph, rig;
    xs_init(&all);
    xs_init(&pd);
    xs_init(&ps);
    xs_init(&ph);
    xs_init(&rig);
    const double dS = 0x1.8p-23 + 0x1.8p-47 + 0x1p-72; /* (1+2^-24)^3 - 1 */
    const double dH = 0x1p-10 + 0x1p-22;              /* (1+2^-11)^2 - 1 */
    const double u32 = 0x1p-24;
    const double g6 = 6.0 * u32 / (1.0 - 6.0 * u32);  /* depth-6 tree */
    const double up = 1.0 + 0x1p-50;                   /* bound slack */
    /* roundings that may land in the subnormal range of the scaled sum:
     * one per component (leaf scaling or a perforated term too small to
     * register), two per tile, the rounding of S and the final scaling */
    int64_t n_round_sub = n + 2 * ((n + 63) / 64) + 2;
    double xy_abs_rel; /* |x_i y_i| / 2^e_max, rounded up */

    for (int64_t base = 0; base < n; base += 64) {
        float lh[64], ls[64];
        double tile_abs = 0.0; /* sum |FP32 leaves| in units 2^c32 */
        for (int j = 0; j < 64; j++) lh[j] = ls[j] = 0.0f;
        for (int j = 0; j < 64 && base + j < n; j++) {
            int64_t i = base + j;
            uint8_t c = ORC_PERF;
            if (key[i] != INT32_MIN) {
                int32_t ex, ey;
                double mx, my;
                orc_split(x[i], &ex, &mx);
                orc_split(y[i], &ey, &my);
                int32_t es = ex + ey;
                int neg = (x[i] < 0.0) != (y[i] < 0.0);
                c = C[key[i] - ORC_KMIN];
                double pm = mx * my; /* exact value lies within 2^-53 rel. */
                xy_abs_rel = ldexp(pm, es - e_max) * (1.0 + 0x1p-52) * up;
                if (c == ORC_DOUBLE) {
                    double leaf = ldexp(neg ? -pm : pm, es - e_max);
                    xs_add(&all, leaf);
                    xs_add(&pd, leaf);
                    xs_add(&rig, xy_abs_rel * 0x1p-53);
                } else if (c == ORC_SINGLE_IN) {
                    float a = (float)mx, b = (float)my;
                    float p = a * b;
                    double leaf = ldexp((double)(neg ? -p : p), es - e_max);
                    xs_add(&all, leaf);
                    xs_add(&ps, leaf);
                    xs_add(&rig, xy_abs_rel * dS);
                } else if (c == ORC_SINGLE) {
                    float a = (float)mx, b = (float)my;
                    float p = a * b;
                    ls[j] = ldexpf(neg ? -p : p, es - c32);
                    xs_add(&rig, xy_abs_rel * dS);
                    /* a leaf below the FP32 normal range (possible only in a
                     * bin wider than exact) is rounded to a multiple of
                     * 2^-149: absolute error <= 2^-150 (units 2^c32) */
                    if (fabsf(ls[j]) <= 0x1p-126f) xs_add(&rig, ldexp(1.0, c32 - e_max - 150));
                    tile_abs += fabs((double)ls[j]);
                } else if (c == ORC_HALF) {
                    double hx = orc_r16(mx), hy = orc_r16(my);
                    float p = (float)(hx * hy); /* < 2^22: exact */
                    lh[j] = ldexpf(neg ? -p : p, es - c32 - 20);
                    xs_add(&rig, xy_abs_rel * dH);
                    if (fabsf(lh[j]) <= 0x1p-126f) xs_add(&rig, ldexp(1.0, c32 - e_max - 150));
                    tile_abs += fabs((double)lh[j]);
                } else {
                    xs_add(&rig, xy_abs_rel); /* perforated: whole term */
                }
            }
            if (cls_out) cls_out[i] = c == ORC_SINGLE_IN ? ORC_SINGLE : c;
        }
        if (accum_mode == 0) {
            double th = ldexp((double)orc_tree64(lh), c32 - e_max);
            double ts = ldexp((double)orc_tree64(ls), c32 - e_max);
            xs_add(&all, th);
            xs_add(&ph, th);
            xs_add(&all, ts);
            xs_add(&ps, ts);
            xs_add(&rig, ldexp(tile_abs * g6 * up, c32 - e_max));
        } else {
            for (int j = 0; j < 64; j++) {
                double vh = ldexp((double)lh[j], c32 - e_max);
                double vs = ldexp((double)ls[j], c32 - e_max);
                xs_add(&all, vh);
                xs_add(&ph, vh);
                xs_add(&all, vs);
                xs_add(&ps, vs);
            }
        }
    }
    double S = xs_round(&all);
    r->value = ldexp(S, e_max);
    if (isinf(r->value)) r->flags |= ORC_F_OVERFLOW;
    r->part[ORC_DOUBLE] = ldexp(xs_round(&pd), e_max);
    r->part[ORC_SINGLE] = ldexp(xs_round(&ps), e_max);
    r->part[ORC_HALF] = ldexp(xs_round(&ph), e_max);
    /* rounding of S to FP64, plus every rounding that can land in the
     * subnormal range of the scaled sum, plus the final scaling */
    xs_add(&rig, fabs(S) * 0x1p-53 * up);
    xs_add(&rig, (double)n_round_sub * 0x1p-1074);
    r->bound_rig = ldexp(xs_round(&rig) * up, e_max) + 0x1p-1074;

    xs_free(&all);
    xs_free(&pd);
    xs_free(&ps);
    xs_free(&ph);
    xs_free(&rig);
    return S;
}

/* Guaranteed mode: a bound, in units of 2^e_max, of every error of one
 * call (quantisation, FP32 tile trees, FP64 stage, subnormal scaling),
 * computed from the histogram, the classes and the computed sum S alone so
 * that the library can evaluate the same formula after pass 2:
 *   a = (Q + T + F)(1 + 2^-40),
 *   Q = sum_k M_k 2^(k-e_max+1) rho(class_k)   (|x_i y_i| < 2^(k+1) in bin
 *       k; rho = the largest relative error of one leaf: 2^-53 double,
 *       (1+2^-24)^3 - 1 single, (1+2^-11)^2 - 1 half, 1 perforated),
 *   T = g6 (1 + 2^-9) sum over single/half bins of M_k 2^(k-e_max+1),
 *   F = 2^-52 |S| + 4 gn^2 (1 + 2^-8) sum over kept bins of
 *       M_k 2^(k-e_max+1) + (2n + 4) 2^-1074. */
static double orc_guard_slack(const int64_t *M, const uint8_t *C, int32_t e_max, double S,
                              int64_t n)
{
    /* indexed by class; ORC_SINGLE_IN (4) takes single's */
    const double rho[5] = {0x1p-53, 0x1.8p-23 + 0x1.8p-47 + 0x1p-72, 0x1p-10 + 0x1p-22, 1.0,
                           0x1.8p-23 + 0x1.8p-47 + 0x1p-72};
    const double u32 = 0x1p-24, u64 = 0x1p-53;
    const double g6 = 6.0 * u32 / (1.0 - 6.0 * u32);
    const double nu = (double)n * u64;
    const double gn = nu / (1.0 - nu);
    xsum q, f32, kept;
    xs_init(&q);
    xs_init(&f32);
    xs_init(&kept);
    for (int32_t k = ORC_KMIN; k <= ORC_KMAX; k++) {
        int64_t Mk = M[k - ORC_KMIN];
        if (Mk == 0) continue;
        int c = C[k - ORC_KMIN];
        double w = ldexp((double)Mk, k - e_max + 1);
        xs_add(&q, ldexp((double)Mk * rho[c], k - e_max + 1));
        if (c == ORC_SINGLE || c == ORC_HALF) xs_add(&f32, w);
        if (c != ORC_PERF) xs_add(&kept, w);
    }
    double Q = xs_round(&q);
    double T = g6 * (1.0 + 0x1p-9) * xs_round(&f32);
    double F = 0x1p-52 * fabs(S) + 4.0 * gn * gn * (1.0 + 0x1p-8) * xs_round(&kept) +
               (2.0 * (double)n + 4.0) * 0x1p-1074;
    xs_free(&q);
    xs_free(&f32);
    xs_free(&kept);
    return (Q + T + F) * (1.0 + 0x1p-40);
}

/* Lower bound of |x.y| in units of 2^e_max from one computed sum: |S|
 * less the slack; raised to 1 when every non-zero product has one sign
 * (then |x.y| >= max |x_i y_i| >= 2^e_max). */
static double orc_lower(const int64_t *M, const uint8_t *C, int32_t e_max, double S, int64_t n,
                        int one_signed)
{
    double low = fabs(S) * (1.0 - 0x1p-52) - orc_guard_slack(M, C, e_max, S, n);
    if (one_signed && low < 1.0) low = 1.0;
    return low;
}

/* Thm 3.4 with E replaced by the certified E_lo = e_max + flexp(low) <=
 * flexp(x.y): relerr <= bound_rel 2^(e_max - E_lo) <= tol. */
static int orc_certified(double bound_rel, double low, double tol)
{
    return low > 0.0 && ldexp(bound_rel, -ilogb(low)) <= tol;
}

/* ------------------------------------------------------------------ */
/* qdot (Alg. 3)                                                         */
/* ------------------------------------------------------------------ */
static int qdot_core(const double *x, const double *y, int64_t n, double tol,
                     const int32_t *opt, int mu_single, orc_result *r, uint8_t *cls_out,
                     int32_t *key_out, int64_t *hist_out)
{
    memset(r, 0, sizeof *r);
    int32_t key_mode = opt ? opt[0] : 0;
    int32_t score_mode = opt ? opt[1] : 0;
    int32_t nonstrict = opt ? opt[2] : 0;
    int32_t accum_mode = opt ? opt[3] : 0;
    int32_t guard_mode = opt ? opt[4] : 0;
    int32_t bin_mode = opt ? opt[5] : 0;
    int32_t bin_param = opt ? opt[6] : 0;
    if (n < 0 || (n > 0 && (!x || !y)) || !(tol > 0.0) || !isfinite(tol) ||
        key_mode < 0 || key_mode > 1 || score_mode < 0 || score_mode > 1 ||
        nonstrict < 0 || nonstrict > 1 || accum_mode < 0 || accum_mode > 1 ||
        guard_mode < 0 || guard_mode > 1 ||
        (guard_mode == 1 && (key_mode != 0 || accum_mode != 0)) ||
        bin_mode < 0 || bin_mode > 2 ||
        (bin_mode == 1 && (bin_param < 1 || bin_param > ORC_W)) ||
        (bin_mode == 2 && (bin_param < 0 || bin_param > ORC_W)) ||
        (bin_mode != 0 && (accum_mode != 0 || guard_mode != 0))) {
        r->status = ORC_E_INVAL;
        r->value = NAN;
        return r->status;
    }
    for (int64_t i = 0; i < n; i++) {
        if (!isfinite(x[i]) || !isfinite(y[i])) {
            r->status = ORC_E_NONFINITE;
            r->value = NAN;
            return r->status;
        }
    }

    /* Alg. 2, exponent preprocessing and exact bins: the bin of key k holds
     * the components whose product has exponent k.  A zero product has no
     * exponent; it is perforated (it contributes exactly nothing) and kept
     * out of the bins, e_max, e_min and N_bins. */
    int64_t *M = (int64_t *)calloc(ORC_W, sizeof(int64_t));
    int32_t *key = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int pos_seen = 0, neg_seen = 0;
    for (int64_t i = 0; i < n; i++) {
        if (x[i] == 0.0 || y[i] == 0.0) {
            key[i] = INT32_MIN;
            r->n_zero++;
            continue;
        }
        key[i] = orc_key(x[i], y[i], key_mode);
        M[key[i] - ORC_KMIN]++;
        if ((x[i] < 0.0) != (y[i] < 0.0)) neg_seen = 1;
        else pos_seen = 1;
    }
    int32_t e_max = INT32_MIN, e_min = INT32_MAX, n_bins = 0;
    for (int32_t k = ORC_KMIN; k <= ORC_KMAX; k++) {
        if (M[k - ORC_KMIN] == 0) continue;
        if (k > e_max) e_max = k;
        if (k < e_min) e_min = k;
    }
    /* Alg. 2's bins: a partition of [e_min, e_max]; N_bins counts the
     * non-empty ones */
    orc_bin *bins = (orc_bin *)malloc(sizeof(orc_bin) * (ORC_W + 1));
    int nbins = e_max >= e_min ? orc_partition(M, e_min, e_max, bin_mode, bin_param, bins) : 0;
    for (int i = 0; i < nbins; i++) n_bins += bins[i].M > 0;
    if (hist_out) memcpy(hist_out, M, sizeof(int64_t) * ORC_W);
    if (key_out)
        for (int64_t i = 0; i < n; i++) key_out[i] = key[i];

    if (n_bins == 0) { /* every product is zero: exact answer +0 */
        r->value = 0.0;
        r->count[ORC_PERF] = n;
        r->flags = ORC_F_ALL_PERF | (guard_mode ? ORC_F_GUARANTEED : 0);
        if (cls_out)
            for (int64_t i = 0; i < n; i++) cls_out[i] = ORC_PERF;
        free(bins);
        free(M);
        free(key);
        return ORC_OK;
    }
    r->e_max = e_max;
    r->e_min = e_min;
    r->n_bins = n_bins;

    /* floor(log2 eps), with eps divided by N_bins in the default score */
    int32_t t = orc_t(score_mode == 0 ? n_bins : 1, tol);
    r->t = t;

    /* bin scores and precisions against e_max, then Alg. 1 */
    uint8_t *C = (uint8_t *)malloc(ORC_W);
    int32_t e_ref = e_max;
    orc_select(bins, nbins, e_max, e_min, e_ref, t, nonstrict, mu_single, r->n_zero, C, r);
    int kept = !(r->flags & ORC_F_ALL_PERF);
    double S = orc_compute(x, y, n, key, C, e_max, e_ref + t + 22, accum_mode, cls_out, r);
    r->passes = kept;

    if (guard_mode) {
        /* Guaranteed mode (Thm 3.4).  A certified lower bound of |x.y|
         * gives E_lo <= flexp(x.y); if the Thm 3.4 bound with E_lo does not
         * meet tol, the classes are selected again against E_lo (or all set
         * to the input precision when |x.y| is not bounded away from 0) and
         * Alg. 1 runs a second time. */
        const int one_signed = !(pos_seen && neg_seen);
        double low = orc_lower(M, C, e_max, S, n, one_signed);
        if (orc_certified(r->bound_rel, low, tol)) {
            r->flags |= ORC_F_GUARANTEED;
        } else {
            /* the most precise reselection: every bin at the input
             * precision, i.e. scoring >= m_single (double inputs) or
             * >= m_half (single inputs), one more in the non-strict reading */
            int32_t ref2 = low > 0.0 ? e_max + ilogb(low)
                                     : e_min - t - (mu_single ? M_HALF : M_SINGLE) + 1 - nonstrict;
            if (ref2 < e_max) {
                e_ref = ref2;
                orc_select(bins, nbins, e_max, e_min, e_ref, t, nonstrict, mu_single, r->n_zero,
                           C, r);
                int kept2 = !(r->flags & ORC_F_ALL_PERF);
                S = orc_compute(x, y, n, key, C, e_max, e_ref + t + 22, accum_mode, cls_out, r);
                double low2 = orc_lower(M, C, e_max, S, n, one_signed);
                if (low2 > low) low = low2;
                r->flags |= ORC_F_RESELECTED;
                if (orc_certified(r->bound_rel, low, tol)) r->flags |= ORC_F_GUARANTEED;
                r->passes = kept + kept2;
            }
        }
        r->lower = low > 0.0 ? ldexp(low, e_max) : 0.0;
    }
    r->e_ref = e_ref;

    free(C);
    free(bins);
    free(M);
    free(key);
    return ORC_OK;
}

int orc_qdot(const double *x, const double *y, int64_t n, double tol,
             const int32_t *opt, orc_result *r, uint8_t *cls_out,
             int32_t *key_out, int64_t *hist_out)
{
    return qdot_core(x, y, n, tol, opt, 0, r, cls_out, key_out, hist_out);
}

/* Single-precision inputs (mu = m_single in eq. (precision-def)): every
 * float is exactly a double, so the keys, the histogram and the leaves are
 * those of the same values given as doubles; only the precision table ends
 * at single. */
int orc_qdot_f32(const float *x, const float *y, int64_t n, double tol,
                 const int32_t *opt, orc_result *r, uint8_t *cls_out,
                 int32_t *key_out, int64_t *hist_out)
{
    if (n < 0 || (n > 0 && (!x || !y))) {
        memset(r, 0, sizeof *r);
        r->status = ORC_E_INVAL;
        r->value = NAN;
        return r->status;
    }
    double *xd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *yd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        xd[i] = (double)x[i];
        yd[i] = (double)y[i];
    }
    int st = qdot_core(xd, yd, n, tol, opt, 1, r, cls_out, key_out, hist_out);
    free(xd);
    free(yd);
    return st;
}

/* ------------------------------------------------------------------ */
/* Applications (Sec. 4.2 and 4.3)                                       */
/* ------------------------------------------------------------------ */
void orc_spmv(int64_t n, const int32_t *rowptr, const int32_t *col,
              const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int32_t j = rowptr[i]; j < rowptr[i + 1]; j++) {
            double p = val[j] * x[col[j]];
            s = s + p;
        }
        y[i] = s;
    }
}

static int inner(const double *a, const double *b, int64_t n, int use_qdot,
                 double qtol, const int32_t *opt, double *out, orc_result *rec)
{
    orc_result r;
    if (!use_qdot) {
        *out = orc_dot_exact(a, b, n);
        if (rec) {
            memset(rec, 0, sizeof *rec);
            rec->value = *out;
            rec->count[ORC_DOUBLE] = n;
        }
        return ORC_OK;
    }
    int st = orc_qdot(a, b, n, qtol, opt, &r, NULL, NULL, NULL);
    if (rec) *rec = r;
    *out = r.value;
    if (st != ORC_OK) return st;
    if (r.flags & ORC_F_ALL_PERF && r.n_bins > 0) return ORC_E_BREAKDOWN;
    return ORC_OK;
}

int orc_cg(int64_t n, const int32_t *rowptr, const int32_t *col,
           const double *val, const double *b, double *x, double rtol,
           double qtol, int32_t maxit, int32_t use_qdot, const int32_t *opt,
           int32_t *iters, double *relres_est, double *relres_true,
           orc_result *trace)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    int st = ORC_OK;
    int ntr = 0;
    /* r0 = b - A x0, p0 = r0 */
    orc_spmv(n, rowptr, col, val, x, q);
    for (int64_t i = 0; i < n; i++) {
        r[i] = b[i] - q[i];
        p[i] = r[i];
    }
    double bnorm = sqrt(orc_dot_exact(b, b, n));
    double c;
    st = inner(r, r, n, use_qdot, qtol, opt, &c, trace ? &trace[ntr] : NULL);
    ntr++;
    int32_t k = 0;
    while (st == ORC_OK && sqrt(c) > rtol * bnorm) {
        if (k >= maxit) {
            st = ORC_E_MAXIT;
            break;
        }
        orc_spmv(n, rowptr, col, val, p, q);
        double d;
        st = inner(p, q, n, use_qdot, qtol, opt, &d,
                   trace ? &trace[ntr] : NULL);
        ntr++;
        if (st != ORC_OK) break;
        if (!(d > 0.0) || !isfinite(d)) {
            st = ORC_E_BREAKDOWN;
            break;
        }
        double alpha = c / d;
        for (int64_t i = 0; i < n; i++) {
            double ap = alpha * p[i];
            x[i] = x[i] + ap;
            double aq = alpha * q[i];
            r[i] = r[i] - aq;
        }
        double cn;
        st = inner(r, r, n, use_qdot, qtol, opt, &cn,
                   trace ? &trace[ntr] : NULL);
        ntr++;
        if (st != ORC_OK) break;
        double beta = cn / c;
        for (int64_t i = 0; i < n; i++) {
            double bp = beta * p[i];
            p[i] = r[i] + bp;
        }
        c = cn;
        k++;
    }
    if (iters) *iters = k;
    if (relres_est) *relres_est = sqrt(c) / bnorm;
    if (relres_true) {
        orc_spmv(n, rowptr, col, val, x, q);
        for (int64_t i = 0; i < n; i++) q[i] = b[i] - q[i];
        *relres_true = sqrt(orc_dot_exact(q, q, n)) / bnorm;
    }
    free(r);
    free(p);
    free(q);
    return st;
}

int orc_power(int64_t n, const int32_t *rowptr, const int32_t *col,
              const double *val, double *x, int32_t iters, double qtol,
              int32_t use_qdot, const int32_t *opt, double *lambda,
              double *lambda_trace, orc_result *trace)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    int st = ORC_OK;
    double lam = 0.0;
    for (int32_t k = 0; k < iters; k++) {
        orc_spmv(n, rowptr, col, val, x, w);
        double c;
        st = inner(x, w, n, use_qdot, qtol, opt, &lam, trace ? &trace[2 * k] : NULL);
        if (st != ORC_OK) break;
        st = inner(w, w, n, use_qdot, qtol, opt, &c, trace ? &trace[2 * k + 1] : NULL);
        if (st != ORC_OK) break;
        if (!(c > 0.0) || !isfinite(c)) {
            st = ORC_E_BREAKDOWN;
            break;
        }
        double s = sqrt(c);
        for (int64_t i = 0; i < n; i++) x[i] = w[i] / s;
        if (lambda_trace) lambda_trace[k] = lam;
    }
    if (lambda) *lambda = lam;
    free(w);
    return st;
}
