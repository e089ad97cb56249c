/*
 * CPU oracle for exact hypercube convolution {0,1}^D x {0,1}^D -> 3^D
 * (Serang, "An exact, cache-localized algorithm for the sub-quadratic
 * convolution of hypercubes").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no code, header or table with the GPU path.
 *
 * Plain, slow, obviously correct C.  Built with -O2 -ffp-contract=off and no
 * fast-math, so every floating-point operation is a separately rounded IEEE
 * operation in the order written.
 *
 * Exported functions (per element type, suffix f64 / f32 / i64):
 *   hco_naive_*      Algorithm 1 (naive Cartesian product)
 *   hco_canonical_*  the method, per-axis form, full-size scratch
 *   hco_recursive_*  the method, three-subproblem recursion, memory-light
 *   hco_adjoint_*    transposed maps (gradient of sum(w * z))
 *   hco_carryfree_naive_*   carry-free 1-D convolution by its definition
 *   hco_difference_naive_*  distribution of X - Y by its definition
 *   hco_sum3_naive_*, hco_sum3_canonical_*  distribution of X1 + X2 + X3
 *                    by its definition and by the per-axis method extended
 *                    to three operands (hc_oracle_sum3.h)
 *   hco_ternary_naive_*, hco_ternary_canonical_*  convolution of two ternary
 *                    cubes {0,1,2}^D (the distribution of X1 + ... + X4 from
 *                    two pair sums) by its definition and by the six-product
 *                    per-axis method (hc_oracle_ternary.h)
 * plus fp64/long double helpers for pins: the max-convolution and its p-norm
 * estimate at single indices, the ternary index map, the direct
 * per-element definition sum, the direct correlation gradient and the
 * rounding-error bound.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

uint64_t hco_pow3(int n)
{
    uint64_t r = 1;
    for (int i = 0; i < n; ++i) r *= 3;
    return r;
}

/* Packed boolean index -> ternary index with the same digits (Introduction:
 * the D boolean coordinates fit one machine integer; Discussion: bit i of
 * the flat index is one axis).  Bit d (weight 2^d) becomes digit d (weight
 * 3^d); axis 0 is the most significant in both. */
void hco_tern_map(int D, uint64_t* out)
{
    const uint64_t n2 = (uint64_t)1 << D;
    for (uint64_t i = 0; i < n2; ++i) {
        uint64_t t = 0, p = 1;
        for (int d = 0; d < D; ++d) {
            if ((i >> d) & 1u) t += p;
            p *= 3;
        }
        out[i] = t;
    }
}

uint64_t hco_tern(uint64_t i)
{
    uint64_t t = 0, p = 1;
    while (i) {
        if (i & 1u) t += p;
        p *= 3;
        i >>= 1;
    }
    return t;
}

#define ELEM double
#define SFX f64
#define HCO_HALF(v) ((v) * 0.5)
#include "hc_oracle_impl.h"
#include "hc_oracle_sum3.h"
#include "hc_oracle_ternary.h"
#undef ELEM
#undef SFX
#undef HCO_HALF

#define ELEM float
#define SFX f32
#define HCO_HALF(v) ((v) * 0.5f)
#include "hc_oracle_impl.h"
#include "hc_oracle_sum3.h"
#include "hc_oracle_ternary.h"
#undef ELEM
#undef SFX
#undef HCO_HALF

#define ELEM uint64_t
#define SFX i64
#define HCO_HALF(v) ((uint64_t)((int64_t)(v) / 2))
#include "hc_oracle_impl.h"
#include "hc_oracle_sum3.h"
#include "hc_oracle_ternary.h"
#undef ELEM
#undef SFX
#undef HCO_HALF

/* Neumaier-compensated accumulation in long double. */
typedef struct { long double s, c; } hco_acc;
static void hco_acc_add(hco_acc* a, long double v)
{
    const long double t = a->s + v;
    if (fabsl(a->s) >= fabsl(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/* Definition of convolution (Introduction) evaluated at single output
 * indices: z[k] = sum over (i, j) with tern(i) + tern(j) = k of x[i]*y[j].
 * Digit 0 of k admits only bits (0,0), digit 2 only (1,1), digit 1 either
 * (0,1) or (1,0), so z[k] has 2^(number of 1 digits) terms; they are summed
 * with compensation in long double.  out[r] receives z[ks[r]]. */
void hco_direct_at_f64(const double* x, const double* y, int D,
                       const uint64_t* ks, int64_t n, double* out)
{
    for (int64_t r = 0; r < n; ++r) {
        uint64_t k = ks[r];
        uint64_t base_i = 0, base_j = 0;
        int ones_bits[64];
        int n_ones = 0;
        for (int d = 0; d < D; ++d) {
            const uint64_t digit = k % 3;
            k /= 3;
            if (digit == 2) { base_i |= (uint64_t)1 << d; base_j |= (uint64_t)1 << d; }
            else if (digit == 1) ones_bits[n_ones++] = d;
        }
        hco_acc acc = {0.0L, 0.0L};
        const uint64_t n_terms = (uint64_t)1 << n_ones;
        for (uint64_t m = 0; m < n_terms; ++m) {
            uint64_t i = base_i, j = base_j;
            for (int b = 0; b < n_ones; ++b) {
                if ((m >> b) & 1u) i |= (uint64_t)1 << ones_bits[b];
                else j |= (uint64_t)1 << ones_bits[b];
            }
            hco_acc_add(&acc, (long double)x[i] * (long double)y[j]);
        }
        out[r] = (double)(acc.s + acc.c);
    }
}

/* Same definition for int64 data with wrapping uint64 arithmetic. */
void hco_direct_at_i64(const uint64_t* x, const uint64_t* y, int D,
                       const uint64_t* ks, int64_t n, uint64_t* out)
{
    for (int64_t r = 0; r < n; ++r) {
        uint64_t k = ks[r];
        uint64_t base_i = 0, base_j = 0;
        int ones_bits[64];
        int n_ones = 0;
        for (int d = 0; d < D; ++d) {
            const uint64_t digit = k % 3;
            k /= 3;
            if (digit == 2) { base_i |= (uint64_t)1 << d; base_j |= (uint64_t)1 << d; }
            else if (digit == 1) ones_bits[n_ones++] = d;
        }
        uint64_t acc = 0;
        const uint64_t n_terms = (uint64_t)1 << n_ones;
        for (uint64_t m = 0; m < n_terms; ++m) {
            uint64_t i = base_i, j = base_j;
            for (int b = 0; b < n_ones; ++b) {
                if ((m >> b) & 1u) i |= (uint64_t)1 << ones_bits[b];
                else j |= (uint64_t)1 << ones_bits[b];
            }
            acc += x[i] * y[j];
        }
        out[r] = acc;
    }
}

/* Pairs (i, j) that meet at output k: digit 0 fixes bits (0,0), digit 2
 * fixes (1,1), digit 1 admits (0,1) and (1,0).  Fills base_i, base_j and the
 * bit positions of the 1 digits; returns their number. */
static int hco_pairs_of(uint64_t k, int D, uint64_t* base_i, uint64_t* base_j, int* ones_bits)
{
    int n_ones = 0;
    *base_i = *base_j = 0;
    for (int d = 0; d < D; ++d) {
        const uint64_t digit = k % 3;
        k /= 3;
        if (digit == 2) { *base_i |= (uint64_t)1 << d; *base_j |= (uint64_t)1 << d; }
        else if (digit == 1) ones_bits[n_ones++] = d;
    }
    return n_ones;
}

/* Max-convolution on the semiring (x, max) (Discussion), by its definition
 * at single output indices: z_max[k] = max over the pairs of k of x[i]*y[j]. */
void hco_maxconv_at_f64(const double* x, const double* y, int D, const uint64_t* ks, int64_t n, double* out)
{
    for (int64_t r = 0; r < n; ++r) {
        uint64_t bi, bj;
        int ones[64];
        const int s = hco_pairs_of(ks[r], D, &bi, &bj, ones);
        double m = -INFINITY;
        for (uint64_t q = 0; q < ((uint64_t)1 << s); ++q) {
            uint64_t i = bi, j = bj;
            for (int b = 0; b < s; ++b) {
                if ((q >> b) & 1u) i |= (uint64_t)1 << ones[b];
                else j |= (uint64_t)1 << ones[b];
            }
            const double v = x[i] * y[j];
            if (v > m) m = v;
        }
        out[r] = m;
    }
}

/* p-norm estimate of the max-convolution (Discussion: p-norm rings):
 *   z_p[k] = (sum over the pairs of k of (x[i] y[j])^p)^(1/p)
 * for nonnegative inputs.  Evaluated stably by factoring out the output's
 * largest term t_max (the max-convolution itself):
 *   z_p[k] = t_max (sum (t / t_max)^p)^(1/p),
 * with long double powers and a compensated sum, so no power under- or
 * overflows.  It brackets the maximum: z_max <= z_p <= 2^(s/p) z_max, with
 * s the number of 1 digits of k. */
void hco_pnorm_at_f64(const double* x, const double* y, int D, double p, const uint64_t* ks, int64_t n,
                      double* out)
{
    for (int64_t r = 0; r < n; ++r) {
        uint64_t bi, bj;
        int ones[64];
        const int s = hco_pairs_of(ks[r], D, &bi, &bj, ones);
        const uint64_t n_terms = (uint64_t)1 << s;
        long double tmax = 0.0L;
        for (int pass = 0; pass < 2; ++pass) {
            hco_acc acc = {0.0L, 0.0L};
            for (uint64_t q = 0; q < n_terms; ++q) {
                uint64_t i = bi, j = bj;
                for (int b = 0; b < s; ++b) {
                    if ((q >> b) & 1u) i |= (uint64_t)1 << ones[b];
                    else j |= (uint64_t)1 << ones[b];
                }
                const long double t = (long double)x[i] * (long double)y[j];
                if (pass == 0) {
                    if (t > tmax) tmax = t;
                } else if (tmax > 0.0L) {
                    hco_acc_add(&acc, powl(t / tmax, (long double)p));
                }
            }
            if (pass == 1) out[r] = (double)(tmax > 0.0L ? tmax * powl(acc.s + acc.c, 1.0L / (long double)p) : 0.0L);
        }
    }
}

/* Direct correlation gradient of L = sum_k w[k] z[k] at selected input
 * indices (derived from the definition: dz[tern(i)+tern(j)]/dx[i] = y[j]):
 *   gx[i] = sum_j w[tern(i) + tern(j)] * y[j]
 *   gy[j] = sum_i w[tern(i) + tern(j)] * x[i]
 * Compensated long double sums.  gx_out[r] = gx[idx[r]], gy_out[r] = gy[idx[r]]. */
void hco_correlation_at_f64(const double* x, const double* y, const double* w, int D,
                            const uint64_t* idx, int64_t n, double* gx_out, double* gy_out)
{
    const uint64_t n2 = (uint64_t)1 << D;
    uint64_t* t = (uint64_t*)malloc(n2 * sizeof(uint64_t));
    if (!t) abort();
    hco_tern_map(D, t);
    for (int64_t r = 0; r < n; ++r) {
        const uint64_t ti = t[idx[r]];
        hco_acc ax = {0.0L, 0.0L}, ay = {0.0L, 0.0L};
        for (uint64_t j = 0; j < n2; ++j) {
            hco_acc_add(&ax, (long double)w[ti + t[j]] * (long double)y[j]);
            hco_acc_add(&ay, (long double)w[t[j] + ti] * (long double)x[j]);
        }
        if (gx_out) gx_out[r] = (double)(ax.s + ax.c);
        if (gy_out) gy_out[r] = (double)(ay.s + ay.c);
    }
    free(t);
}

/* Magnitude that bounds the rounding error of the method (derived by
 * first-order rounding analysis; the paper states only that the result is
 * exact when (a + b) - a = b holds):
 *   B = |G|(F|x| . F|y|),  |G|: (p0, p1, p2) -> (p0, p0 + p1 + p2, p2)
 * computed with the same memory-light recursion as the method.  For the
 * per-axis method in precision u,  |z_computed - z_exact| <= (4D + 2) u B. */
static void hco_bound_rec(const double* x, const double* y, double* b, int D)
{
    if (D == 0) { b[0] = fabs(x[0]) * fabs(y[0]); return; }
    const uint64_t h = (uint64_t)1 << (D - 1);
    const uint64_t t = hco_pow3(D - 1);
    double* s = (double*)malloc(2 * h * sizeof(double));
    if (!s) abort();
    for (uint64_t i = 0; i < h; ++i) s[i] = fabs(x[i]) + fabs(x[h + i]);
    for (uint64_t i = 0; i < h; ++i) s[h + i] = fabs(y[i]) + fabs(y[h + i]);
    hco_bound_rec(x, y, b, D - 1);
    hco_bound_rec(x + h, y + h, b + 2 * t, D - 1);
    hco_bound_rec(s, s + h, b + t, D - 1);
    for (uint64_t k = 0; k < t; ++k) b[t + k] = (b[t + k] + b[k]) + b[2 * t + k];
    free(s);
}

int hco_bound_f64(const double* x, const double* y, double* b, int D)
{
    if (D < 0 || D > 20) return 1;
    hco_bound_rec(x, y, b, D);
    return 0;
}

/* The same bound at single output indices, for sizes where the whole array
 * would not fit.  B is a tensor product over the axes: where k has digit 0
 * (or 2) it selects bit 0 (or 1) of both inputs on that axis, so B[k] equals
 * the bound of the two sub-cubes spanned by the s axes where k has digit 1
 * (the other bits fixed), taken at that sub-cube's all-ones index.  Returns
 * 1 without writing when some index has more than 14 digits equal to 1. */
int hco_bound_at_f64(const double* x, const double* y, int D, const uint64_t* ks, int64_t n, double* out)
{
    if (D < 0 || D > 40) return 1;
    for (int64_t r = 0; r < n; ++r) {
        uint64_t k = ks[r];
        int s = 0;
        for (int d = 0; d < D; ++d, k /= 3) s += (k % 3 == 1);
        if (s > 14) return 1;
    }
    for (int64_t r = 0; r < n; ++r) {
        uint64_t k = ks[r];
        uint64_t base = 0;
        int ones_bits[64];
        int s = 0;
        for (int d = 0; d < D; ++d) {
            const uint64_t digit = k % 3;
            k /= 3;
            if (digit == 2) base |= (uint64_t)1 << d;
            else if (digit == 1) ones_bits[s++] = d;
        }
        /* sub-cube index: its bit s-1-b (axis b of the sub-cube, most
         * significant first) is the input bit ones_bits[s-1-b] */
        const uint64_t m = (uint64_t)1 << s;
        double* sx = (double*)malloc(2 * m * sizeof(double));
        double* b = (double*)malloc(hco_pow3(s) * sizeof(double));
        if (!sx || !b) abort();
        for (uint64_t q = 0; q < m; ++q) {
            uint64_t i = base;
            for (int c = 0; c < s; ++c)
                if ((q >> c) & 1u) i |= (uint64_t)1 << ones_bits[c];
            sx[q] = x[i];
            sx[m + q] = y[i];
        }
        hco_bound_rec(sx, sx + m, b, s);
        out[r] = b[(hco_pow3(s) - 1) / 2];
        free(sx);
        free(b);
    }
    return 0;
}

/* Magnitude bounding the rounding error of the transposed-map adjoint:
 *   Bx = |F^T|(|G^T| |w| . F|y|),  By = |F^T|(|G^T| |w| . F|x|)
 * with |G^T|: (w0, w1, w2) -> (w0 + w1, w1, w2 + w1); same axis orders as the
 * adjoint.  Either output may be NULL. */
int hco_adjoint_bound_f64(const double* x, const double* y, const double* w,
                          double* bx, double* by, int D)
{
    if (D < 0 || D > 20) return 1;
    const uint64_t n2 = (uint64_t)1 << D;
    double* xa = (double*)malloc(n2 * sizeof(double));
    double* ya = (double*)malloc(n2 * sizeof(double));
    const uint64_t n3 = hco_pow3(D);
    double* W = (double*)malloc(n3 * sizeof(double));
    double* F = (double*)malloc(n3 * sizeof(double));
    double* T = (double*)malloc(n3 * sizeof(double));
    double* A = (double*)malloc(n3 * sizeof(double));
    if (!xa || !ya || !W || !F || !T || !A) abort();
    for (uint64_t i = 0; i < n2; ++i) { xa[i] = fabs(x[i]); ya[i] = fabs(y[i]); }
    for (uint64_t k = 0; k < n3; ++k) W[k] = fabs(w[k]);
    for (int a = 0; a < D; ++a) {
        const uint64_t n_hi = hco_pow3(a);
        const uint64_t n_lo = hco_pow3(D - a - 1);
        for (uint64_t hi = 0; hi < n_hi; ++hi)
            for (uint64_t lo = 0; lo < n_lo; ++lo) {
                const double w0 = W[(hi * 3 + 0) * n_lo + lo];
                const double w1 = W[(hi * 3 + 1) * n_lo + lo];
                const double w2 = W[(hi * 3 + 2) * n_lo + lo];
                W[(hi * 3 + 0) * n_lo + lo] = w0 + w1;
                W[(hi * 3 + 2) * n_lo + lo] = w2 + w1;
            }
    }
    for (int which = 0; which < 2; ++which) {
        double* g = which == 0 ? bx : by;
        if (!g) continue;
        hco_forward_all_f64(which == 0 ? ya : xa, F, T, D);
        for (uint64_t k = 0; k < n3; ++k) A[k] = W[k] * F[k];
        for (int a = D - 1; a >= 0; --a) {
            const uint64_t n_hi = hco_pow3(a);
            const uint64_t n_lo = (uint64_t)1 << (D - a - 1);
            for (uint64_t hi = 0; hi < n_hi; ++hi)
                for (uint64_t lo = 0; lo < n_lo; ++lo) {
                    const double g0 = A[(hi * 3 + 0) * n_lo + lo];
                    const double g1 = A[(hi * 3 + 1) * n_lo + lo];
                    const double g2 = A[(hi * 3 + 2) * n_lo + lo];
                    T[(hi * 2 + 0) * n_lo + lo] = g0 + g1;
                    T[(hi * 2 + 1) * n_lo + lo] = g1 + g2;
                }
            double* s = A; A = T; T = s;
        }
        for (uint64_t i = 0; i < n2; ++i) g[i] = A[i];
    }
    free(xa); free(ya); free(W); free(F); free(T); free(A);
    return 0;
}

/* Distribution of X1 + X2 + X3 at single output indices, by its definition:
 * base-4 digit 0 of k admits bits (0,0,0) on that axis, digit 3 (1,1,1),
 * digits 1 and 2 the three bit triples with that sum.  The 3^s terms (s
 * digits equal to 1 or 2) are summed with compensation in long double. */
void hco_sum3_direct_at_f64(const double* x1, const double* x2, const double* x3, int D,
                            const uint64_t* ks, int64_t n, double* out)
{
    static const int trip[4][3][3] = {
        {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}},
        {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
        {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}},
        {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}},
    };
    for (int64_t r = 0; r < n; ++r) {
        int digit[64];
        int mid[64];
        int s = 0;
        uint64_t k = ks[r];
        for (int d = 0; d < D; ++d) {
            digit[d] = (int)(k & 3u);
            k >>= 2;
            if (digit[d] == 1 || digit[d] == 2) mid[s++] = d;
        }
        uint64_t n_terms = 1;
        for (int c = 0; c < s; ++c) n_terms *= 3;
        hco_acc acc = {0.0L, 0.0L};
        for (uint64_t m = 0; m < n_terms; ++m) {
            uint64_t i = 0, j = 0, l = 0, mm = m;
            int c = 0;
            for (int d = 0; d < D; ++d) {
                int choice = 0;
                if (c < s && mid[c] == d) { choice = (int)(mm % 3); mm /= 3; ++c; }
                const int* b = trip[digit[d]][choice];
                i |= (uint64_t)b[0] << d;
                j |= (uint64_t)b[1] << d;
                l |= (uint64_t)b[2] << d;
            }
            hco_acc_add(&acc, (long double)x1[i] * (long double)x2[j] * (long double)x3[l]);
        }
        out[r] = (double)(acc.s + acc.c);
    }
}

/* The convolution of two ternary cubes by its definition at chosen output
 * indices (base-5 digits), every pair of entries whose digits sum to the
 * output's, Neumaier-compensated in long double (float64 data). */
void hco_ternary_direct_at_f64(const double* a, const double* b, int D, const uint64_t* ks, int64_t n,
                               double* out)
{
    for (int64_t r = 0; r < n; ++r) {
        int digit[64];
        uint64_t k = ks[r];
        uint64_t n_terms = 1;
        for (int d = 0; d < D; ++d) {
            digit[d] = (int)(k % 5);
            k /= 5;
            /* pairs (i, j) in {0,1,2}^2 with i + j = digit: 1, 2, 3, 2, 1 */
            n_terms *= (uint64_t)(digit[d] <= 2 ? digit[d] + 1 : 5 - digit[d]);
        }
        hco_acc acc = {0.0L, 0.0L};
        for (uint64_t m = 0; m < n_terms; ++m) {
            uint64_t i = 0, j = 0, w = 1, mm = m;
            for (int d = 0; d < D; ++d) {
                const int s = digit[d];
                const int lo = s <= 2 ? 0 : s - 2;   /* smallest i on this axis */
                const int cnt = s <= 2 ? s + 1 : 5 - s;
                const int id = lo + (int)(mm % (uint64_t)cnt);
                mm /= (uint64_t)cnt;
                i += (uint64_t)id * w;
                j += (uint64_t)(s - id) * w;
                w *= 3;
            }
            hco_acc_add(&acc, (long double)a[i] * (long double)b[j]);
        }
        out[r] = (double)(acc.s + acc.c);
    }
}

/* Magnitude bounding the rounding error of the ternary convolution's
 * per-axis method (first-order rounding analysis, as for the other bounds):
 *   B = |U|(T|a| . T|b|),
 *   T:   (a0, a1, a2) -> (a0, a1, a2, a0 + a1, a1 + a2, a0 + a2)
 *   |U|: (p0, p1, p2, q01, q12, q02) -> (p0, q01 + p0 + p1,
 *         q02 + p0 + p2 + p1, q12 + p1 + p2, p2)
 * with |computed - exact| <= (5D + 1) u B: at most D roundings per forward
 * value, one per product and three per inverse step.  b receives 5^D
 * values (D <= 10). */
int hco_ternary_bound_f64(const double* a, const double* b, double* out, int D)
{
    if (D < 0 || D > 10) return 1;
    const uint64_t n3 = hco_pow3(D);
    uint64_t n6 = 1, n5 = 1;
    for (int d = 0; d < D; ++d) { n6 *= 6; n5 *= 5; }
    double* fa = (double*)malloc(n6 * sizeof(double));
    double* fb = (double*)malloc(n6 * sizeof(double));
    double* t = (double*)malloc(n6 * sizeof(double));
    if (!fa || !fb || !t) { free(fa); free(fb); free(t); return 2; }
    double* ops[2] = {fa, fb};
    const double* src[2] = {a, b};
    for (int o = 0; o < 2; ++o) {
        /* T on |x|, axes ascending, ping-pong so that the last axis lands in ops[o] */
        double* cur = (D % 2 == 0) ? ops[o] : t;
        double* nxt = (D % 2 == 0) ? t : ops[o];
        for (uint64_t i = 0; i < n3; ++i) cur[i] = fabs(src[o][i]);
        for (int ax = 0; ax < D; ++ax) {
            uint64_t n_hi = 1, n_lo = 1;
            for (int d = 0; d < ax; ++d) n_hi *= 6;
            for (int d = ax + 1; d < D; ++d) n_lo *= 3;
            for (uint64_t hi = 0; hi < n_hi; ++hi)
                for (uint64_t lo = 0; lo < n_lo; ++lo) {
                    const double a0 = cur[(hi * 3 + 0) * n_lo + lo];
                    const double a1 = cur[(hi * 3 + 1) * n_lo + lo];
                    const double a2 = cur[(hi * 3 + 2) * n_lo + lo];
                    nxt[(hi * 6 + 0) * n_lo + lo] = a0;
                    nxt[(hi * 6 + 1) * n_lo + lo] = a1;
                    nxt[(hi * 6 + 2) * n_lo + lo] = a2;
                    nxt[(hi * 6 + 3) * n_lo + lo] = a0 + a1;
                    nxt[(hi * 6 + 4) * n_lo + lo] = a1 + a2;
                    nxt[(hi * 6 + 5) * n_lo + lo] = a0 + a2;
                }
            double* s = cur; cur = nxt; nxt = s;
        }
    }
    for (uint64_t k = 0; k < n6; ++k) fa[k] = fa[k] * fb[k];
    double* cur = fa;
    double* nxt = t;
    for (int ax = D - 1; ax >= 0; --ax) {
        uint64_t n_hi = 1, n_lo = 1;
        for (int d = 0; d < ax; ++d) n_hi *= 6;
        for (int d = ax + 1; d < D; ++d) n_lo *= 5;
        for (uint64_t hi = 0; hi < n_hi; ++hi)
            for (uint64_t lo = 0; lo < n_lo; ++lo) {
                const double* p = cur + hi * 6 * n_lo + lo;
                double* c = nxt + hi * 5 * n_lo + lo;
                const double p0 = p[0], p1 = p[n_lo], p2 = p[2 * n_lo];
                const double q01 = p[3 * n_lo], q12 = p[4 * n_lo], q02 = p[5 * n_lo];
                c[0] = p0;
                c[n_lo] = q01 + p0 + p1;
                c[2 * n_lo] = q02 + p0 + p2 + p1;
                c[3 * n_lo] = q12 + p1 + p2;
                c[4 * n_lo] = p2;
            }
        double* s = cur; cur = nxt; nxt = s;
    }
    for (uint64_t k = 0; k < n5; ++k) out[k] = cur[k];
    free(fa);
    free(fb);
    free(t);
    return 0;
}

/* Magnitude bounding the rounding error of the three-operand method
 * (derived by first-order rounding analysis, like the two-operand bound):
 *   B = |G4|(F4a|x1| . F4a|x2| . F4a|x3|),
 *   F4a: (a0, a1) -> (a0, a0 + a1, a0 + a1, a1)
 *   |G4|: (p0, p1, pm, pi) -> (p0, (p1 + pm)/2 + pi, (p1 + pm)/2 + p0, pi)
 * with |computed - exact| <= (5D + 2) u B: at most D roundings per forward
 * value, two per product and two per inverse step. */
int hco_sum3_bound_f64(const double* x1, const double* x2, const double* x3, double* b, int D)
{
    if (D < 0 || D > 14) return 1;
    const uint64_t n2 = (uint64_t)1 << D;
    const uint64_t n4 = (uint64_t)1 << (2 * D);
    double* f = (double*)malloc(n4 * sizeof(double));
    double* t = (double*)malloc(n4 * sizeof(double));
    if (!f || !t) abort();
    const double* xs[3] = {x1, x2, x3};
    for (int op = 0; op < 3; ++op) {
        double* cur = (D % 2 == 0) ? f : t;
        double* nxt = (D % 2 == 0) ? t : f;
        for (uint64_t i = 0; i < n2; ++i) cur[i] = fabs(xs[op][i]);
        for (int a = 0; a < D; ++a) {
            const uint64_t n_hi = (uint64_t)1 << (2 * a);
            const uint64_t n_lo = (uint64_t)1 << (D - a - 1);
            for (uint64_t hi = 0; hi < n_hi; ++hi)
                for (uint64_t lo = 0; lo < n_lo; ++lo) {
                    const double a0 = cur[(hi * 2 + 0) * n_lo + lo];
                    const double a1 = cur[(hi * 2 + 1) * n_lo + lo];
                    nxt[(hi * 4 + 0) * n_lo + lo] = a0;
                    nxt[(hi * 4 + 1) * n_lo + lo] = a0 + a1;
                    nxt[(hi * 4 + 2) * n_lo + lo] = a0 + a1;
                    nxt[(hi * 4 + 3) * n_lo + lo] = a1;
                }
            double* sw = cur; cur = nxt; nxt = sw;
        }
        /* cur == f now */
        for (uint64_t k = 0; k < n4; ++k) b[k] = op == 0 ? f[k] : b[k] * f[k];
    }
    for (int a = D - 1; a >= 0; --a) {
        const uint64_t n_hi = (uint64_t)1 << (2 * a);
        const uint64_t n_lo = (uint64_t)1 << (2 * (D - a - 1));
        for (uint64_t hi = 0; hi < n_hi; ++hi)
            for (uint64_t lo = 0; lo < n_lo; ++lo) {
                double* p = b + hi * 4 * n_lo + lo;
                const double p0 = p[0], p1 = p[n_lo], pm = p[2 * n_lo], pi = p[3 * n_lo];
                p[n_lo] = 0.5 * (p1 + pm) + pi;
                p[2 * n_lo] = 0.5 * (p1 + pm) + p0;
            }
    }
    free(f);
    free(t);
    return 0;
}
