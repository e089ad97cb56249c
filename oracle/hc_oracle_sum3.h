/*
 * Type-generic oracle for the distribution of a sum of three independent
 * vectors whose axes are all Bernoulli (Introduction: sums of multiple
 * probability mass functions whose axes are Bernoulli variables).
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes, links or
 * calls anything in oracle/.
 *
 * Included once per element type by hc_oracle.c with ELEM, SFX and
 * HCO_HALF(v) (exact halving of a value that is even in exact arithmetic:
 * multiplication by 1/2 for floats, signed division by 2 for wrapping int64
 * data) defined.
 *
 * Layout: x1, x2, x3 hold 2^D values each (flat index = bit vector, axis 0 the
 * most significant bit).  z holds 4^D values; base-4 digit d of the flat
 * index (weight 4^d) is the coordinate on axis D-1-d, so the product
 * x1[i] x2[j] x3[l] belongs to z[quad(i) + quad(j) + quad(l)], quad(i) being
 * the bits of i read as base-4 digits (digit sums are at most 3: no carries).
 */

#define HCO_CAT2(a, b) a##b
#define HCO_CAT(a, b) HCO_CAT2(a, b)
#define HCO_FN(name) HCO_CAT(name, SFX)

/* The definition (Introduction: convolution of tensors, here of three
 * hypercubes): every triple of entries, i outer, then j, then l, each
 * product formed as (x1[i] * x2[j]) * x3[l]. */
int HCO_FN(hco_sum3_naive_)(const ELEM* x1, const ELEM* x2, const ELEM* x3, ELEM* z, int D)
{
    if (D < 0 || D > 12) return 1;
    const uint64_t n2 = (uint64_t)1 << D;
    const uint64_t n4 = (uint64_t)1 << (2 * D);
    uint64_t* q = (uint64_t*)malloc(n2 * sizeof(uint64_t));
    if (!q) return 2;
    for (uint64_t i = 0; i < n2; ++i) {
        uint64_t t = 0;
        for (int d = 0; d < D; ++d)
            if ((i >> d) & 1u) t += (uint64_t)1 << (2 * d);
        q[i] = t;
    }
    for (uint64_t k = 0; k < n4; ++k) z[k] = (ELEM)0;
    for (uint64_t i = 0; i < n2; ++i)
        for (uint64_t j = 0; j < n2; ++j)
            for (uint64_t l = 0; l < n2; ++l)
                z[q[i] + q[j] + q[l]] += (x1[i] * x2[j]) * x3[l];
    free(q);
    return 0;
}

/* The method extended to three operands, in per-axis form.  Along one axis
 * each operand is a linear polynomial a0 + a1 t (its two entries), the sum's
 * distribution along that axis is the product of three of them, a cubic
 * c0 + c1 t + c2 t^2 + c3 t^3, and c is recovered exactly from the values at
 * t = 0, 1, -1 and infinity (the Methods section's identity uses 0, 1 and
 * infinity for the product of two):
 *   forward  (a0, a1) -> (a0, a0 + a1, a0 - a1, a1)          axes 0..D-1
 *   product  (x1^ * x2^) * x3^                               elementwise
 *   inverse  (p0, p1, pm, pi) -> (p0, (p1 - pm)/2 - pi,
 *                                 (p1 + pm)/2 - p0, pi)       axes D-1..0
 * Halving is exact in binary floating point (outside the subnormal range)
 * and, for int64 data, whenever the true difference fits in int64. */
static void HCO_FN(hco_sum3_forward_axis_)(const ELEM* in, ELEM* out, int D, int a)
{
    const uint64_t n_hi = (uint64_t)1 << (2 * a);
    const uint64_t n_lo = (uint64_t)1 << (D - a - 1);
    for (uint64_t hi = 0; hi < n_hi; ++hi)
        for (uint64_t lo = 0; lo < n_lo; ++lo) {
            const ELEM a0 = in[(hi * 2 + 0) * n_lo + lo];
            const ELEM a1 = in[(hi * 2 + 1) * n_lo + lo];
            out[(hi * 4 + 0) * n_lo + lo] = a0;
            out[(hi * 4 + 1) * n_lo + lo] = a0 + a1;
            out[(hi * 4 + 2) * n_lo + lo] = a0 - a1;
            out[(hi * 4 + 3) * n_lo + lo] = a1;
        }
}

static void HCO_FN(hco_sum3_inverse_axis_)(ELEM* z, int D, int a)
{
    const uint64_t n_hi = (uint64_t)1 << (2 * a);
    const uint64_t n_lo = (uint64_t)1 << (2 * (D - a - 1));
    for (uint64_t hi = 0; hi < n_hi; ++hi)
        for (uint64_t lo = 0; lo < n_lo; ++lo) {
            ELEM* p = z + hi * 4 * n_lo + lo;
            const ELEM p0 = p[0], p1 = p[n_lo], pm = p[2 * n_lo], pi = p[3 * n_lo];
            const ELEM d = p1 - pm;
            const ELEM s = p1 + pm;
            p[n_lo] = HCO_HALF(d) - pi;
            p[2 * n_lo] = HCO_HALF(s) - p0;
        }
}

/* Forward maps of one operand on all axes: 2^D -> 4^D (out must hold 4^D,
 * tmp 4^D values). */
static void HCO_FN(hco_sum3_forward_all_)(const ELEM* x, ELEM* out, ELEM* tmp, int D)
{
    const uint64_t n2 = (uint64_t)1 << D;
    ELEM* cur = tmp;
    ELEM* nxt = out;
    /* the last axis must land in out: start in the buffer that makes it so */
    if (D % 2 == 0) { cur = out; nxt = tmp; }
    for (uint64_t i = 0; i < n2; ++i) cur[i] = x[i];
    for (int a = 0; a < D; ++a) {
        HCO_FN(hco_sum3_forward_axis_)(cur, nxt, D, a);
        ELEM* t = cur; cur = nxt; nxt = t;
    }
}

int HCO_FN(hco_sum3_canonical_)(const ELEM* x1, const ELEM* x2, const ELEM* x3, ELEM* z, int D)
{
    if (D < 0 || D > 14) return 1;
    const uint64_t n4 = (uint64_t)1 << (2 * D);
    ELEM* f = (ELEM*)malloc(n4 * sizeof(ELEM));
    ELEM* t = (ELEM*)malloc(n4 * sizeof(ELEM));
    if (!f || !t) { free(f); free(t); return 2; }
    HCO_FN(hco_sum3_forward_all_)(x1, z, t, D);
    HCO_FN(hco_sum3_forward_all_)(x2, f, t, D);
    for (uint64_t k = 0; k < n4; ++k) z[k] = z[k] * f[k];
    HCO_FN(hco_sum3_forward_all_)(x3, f, t, D);
    for (uint64_t k = 0; k < n4; ++k) z[k] = z[k] * f[k];
    for (int a = D - 1; a >= 0; --a) HCO_FN(hco_sum3_inverse_axis_)(z, D, a);
    free(f);
    free(t);
    return 0;
}

#undef HCO_FN
#undef HCO_CAT
#undef HCO_CAT2
