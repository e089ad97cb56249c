/*
 * Type-generic oracle for the convolution of two ternary cubes
 * {0,1,2}^D x {0,1,2}^D -> {0,...,4}^D, the next link of a chain of sums
 * (Introduction: sums of multiple probability mass functions whose axes are
 * Bernoulli variables): with A the distribution of X1 + X2 and B that of
 * X3 + X4 (each the hypercube convolution of a pair), A * B is the
 * distribution of X1 + X2 + X3 + X4.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes, links or
 * calls anything in oracle/.
 *
 * Included once per element type by hc_oracle.c with ELEM and SFX defined.
 *
 * Layout: a, b hold 3^D values each in the layout of the hypercube
 * convolution's output (ternary digit d of the flat index, weight 3^d, is
 * the coordinate on axis D-1-d).  z holds 5^D values; base-5 digit d of the
 * flat index (weight 5^d) is the coordinate on axis D-1-d, so a[i] b[j]
 * belongs to z[five(i) + five(j)], five(i) being the ternary digits of i
 * read as base-5 digits (digit sums are at most 4: no carries).
 */

#define HCO_CAT2(a, b) a##b
#define HCO_CAT(a, b) HCO_CAT2(a, b)
#define HCO_FN(name) HCO_CAT(name, SFX)

/* The definition (Introduction: convolution of tensors): every pair of
 * entries, i outer, then j. */
int HCO_FN(hco_ternary_naive_)(const ELEM* a, const ELEM* b, ELEM* z, int D)
{
    if (D < 0 || D > 8) return 1;
    const uint64_t n3 = hco_pow3(D);
    uint64_t n5 = 1;
    for (int d = 0; d < D; ++d) n5 *= 5;
    uint64_t* f = (uint64_t*)malloc(n3 * sizeof(uint64_t));
    if (!f) return 2;
    for (uint64_t i = 0; i < n3; ++i) {
        uint64_t t = 0, w = 1, r = i;
        for (int d = 0; d < D; ++d) {
            t += (r % 3) * w;
            r /= 3;
            w *= 5;
        }
        f[i] = t;
    }
    for (uint64_t k = 0; k < n5; ++k) z[k] = (ELEM)0;
    for (uint64_t i = 0; i < n3; ++i)
        for (uint64_t j = 0; j < n3; ++j) z[f[i] + f[j]] += a[i] * b[j];
    free(f);
    return 0;
}

/* The per-axis method, in the Karatsuba form of the Methods section taken to
 * lines of three.  Along one axis each operand is a quadratic a0 + a1 t +
 * a2 t^2; their product c0 + ... + c4 t^4 needs six products and no
 * division:
 *   forward  (a0, a1, a2) -> (a0, a1, a2, a0 + a1, a1 + a2, a0 + a2)
 *                                                           axes 0..D-1
 *   product  a^ * b^                                        elementwise
 *   inverse  (p0, p1, p2, q01, q12, q02) -> (p0, (q01 - p0) - p1,
 *            ((q02 - p0) - p2) + p1, (q12 - p1) - p2, p2)   axes D-1..0
 * (p_i = a_i b_i, q_ij = (a_i + a_j)(b_i + b_j)).  Before axis a is
 * inverted the array is [6^a][6][5^(D-a-1)]; afterwards [6^a][5][...]. */
static void HCO_FN(hco_ternary_forward_axis_)(const ELEM* in, ELEM* out, int D, int a)
{
    uint64_t n_hi = 1, n_lo = 1;
    for (int d = 0; d < a; ++d) n_hi *= 6;
    for (int d = a + 1; d < D; ++d) n_lo *= 3;
    for (uint64_t hi = 0; hi < n_hi; ++hi)
        for (uint64_t lo = 0; lo < n_lo; ++lo) {
            const ELEM a0 = in[(hi * 3 + 0) * n_lo + lo];
            const ELEM a1 = in[(hi * 3 + 1) * n_lo + lo];
            const ELEM a2 = in[(hi * 3 + 2) * n_lo + lo];
            out[(hi * 6 + 0) * n_lo + lo] = a0;
            out[(hi * 6 + 1) * n_lo + lo] = a1;
            out[(hi * 6 + 2) * n_lo + lo] = a2;
            out[(hi * 6 + 3) * n_lo + lo] = a0 + a1;
            out[(hi * 6 + 4) * n_lo + lo] = a1 + a2;
            out[(hi * 6 + 5) * n_lo + lo] = a0 + a2;
        }
}

static void HCO_FN(hco_ternary_inverse_axis_)(const ELEM* in, ELEM* out, int D, int a)
{
    uint64_t n_hi = 1, n_lo = 1;
    for (int d = 0; d < a; ++d) n_hi *= 6;
    for (int d = a + 1; d < D; ++d) n_lo *= 5;
    for (uint64_t hi = 0; hi < n_hi; ++hi)
        for (uint64_t lo = 0; lo < n_lo; ++lo) {
            const ELEM* p = in + hi * 6 * n_lo + lo;
            ELEM* c = out + hi * 5 * n_lo + lo;
            const ELEM p0 = p[0], p1 = p[n_lo], p2 = p[2 * n_lo];
            const ELEM q01 = p[3 * n_lo], q12 = p[4 * n_lo], q02 = p[5 * n_lo];
            c[0] = p0;
            c[n_lo] = (q01 - p0) - p1;
            c[2 * n_lo] = ((q02 - p0) - p2) + p1;
            c[3 * n_lo] = (q12 - p1) - p2;
            c[4 * n_lo] = p2;
        }
}

/* Forward maps of one operand on all axes: 3^D -> 6^D (out and tmp hold
 * 6^D values each). */
static void HCO_FN(hco_ternary_forward_all_)(const ELEM* x, ELEM* out, ELEM* tmp, int D)
{
    const uint64_t n3 = hco_pow3(D);
    ELEM* cur = tmp;
    ELEM* nxt = out;
    /* the last axis must land in out: start in the buffer that makes it so */
    if (D % 2 == 0) { cur = out; nxt = tmp; }
    for (uint64_t i = 0; i < n3; ++i) cur[i] = x[i];
    for (int a = 0; a < D; ++a) {
        HCO_FN(hco_ternary_forward_axis_)(cur, nxt, D, a);
        ELEM* t = cur; cur = nxt; nxt = t;
    }
}

int HCO_FN(hco_ternary_canonical_)(const ELEM* a, const ELEM* b, ELEM* z, int D)
{
    if (D < 0 || D > 10) return 1;
    uint64_t n6 = 1;
    for (int d = 0; d < D; ++d) n6 *= 6;
    ELEM* fa = (ELEM*)malloc(n6 * sizeof(ELEM));
    ELEM* fb = (ELEM*)malloc(n6 * sizeof(ELEM));
    ELEM* t = (ELEM*)malloc(n6 * sizeof(ELEM));
    if (!fa || !fb || !t) { free(fa); free(fb); free(t); return 2; }
    HCO_FN(hco_ternary_forward_all_)(a, fa, t, D);
    HCO_FN(hco_ternary_forward_all_)(b, fb, t, D);
    for (uint64_t k = 0; k < n6; ++k) fa[k] = fa[k] * fb[k];
    /* inverse, descending; the array shrinks by 6 -> 5 on each axis */
    ELEM* cur = fa;
    ELEM* nxt = t;
    for (int ax = D - 1; ax >= 0; --ax) {
        HCO_FN(hco_ternary_inverse_axis_)(cur, nxt, D, ax);
        ELEM* s = cur; cur = nxt; nxt = s;
    }
    uint64_t n5 = 1;
    for (int d = 0; d < D; ++d) n5 *= 5;
    for (uint64_t k = 0; k < n5; ++k) z[k] = cur[k];
    free(fa);
    free(fb);
    free(t);
    return 0;
}

#undef HCO_FN
#undef HCO_CAT
#undef HCO_CAT2
