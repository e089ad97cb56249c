/*
 * Type-generic body of the CPU oracle for hypercube convolution.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes, links or
 * calls anything in oracle/.  Only tests, the smoke check and the benchmark's
 * CPU baseline use it.
 *
 * This file is included once per element type by hc_oracle.c with
 *   ELEM  arithmetic type (double, float, or uint64_t for int64 data, so that
 *         overflow wraps modulo 2^64 instead of being undefined)
 *   SFX   suffix appended to every exported name (f64, f32, i64)
 *
 * Conventions (Methods section, row-major storage; Discussion, bits of a flat
 * index as the axes of a hypercube):
 *   x, y   2^D values, flat index i = bit vector, axis 0 = most significant bit
 *   z      3^D values, flat index k = ternary digits, axis 0 = most significant
 *   tern(i) maps the bits of i to the ternary number with the same digits, so
 *   x[i]*y[j] belongs to z[tern(i) + tern(j)] (digit sums are at most 2, so
 *   no digit carries).
 *
 * Floating-point evaluation order (the paper is silent on it; reading fixed
 * here and listed in the design notes):
 *   forward sums on axes 0, 1, ..., D-1 in that order, each new middle entry
 *   being a0 + a1; one multiply per entry; inverse on axes D-1, ..., 1, 0 in
 *   that order, each middle entry becoming (p1 - p0) - p2.  This is exactly the
 *   order the three-subproblem recursion of the Methods section produces.
 */

#define HCO_CAT2(a, b) a##b
#define HCO_CAT(a, b) HCO_CAT2(a, b)
#define HCO_FN(name) HCO_CAT(name, SFX)

/* Naive multidimensional convolution (Introduction, Algorithm 1) applied to
 * two hypercubes: every x[i] multiplies every y[j] and is added into
 * z[i + j], where i + j is the digit-wise (carry-free) sum of the two index
 * vectors.  i runs in the outer loop and j in the inner loop, as in the
 * algorithm's nested loops. */
int HCO_FN(hco_naive_)(const ELEM* x, const ELEM* y, ELEM* z, int D)
{
    if (D < 0 || D > 20) return 1;
    const uint64_t n2 = (uint64_t)1 << D;
    const uint64_t n3 = hco_pow3(D);
    uint64_t* t = (uint64_t*)malloc(n2 * sizeof(uint64_t));
    if (!t) return 2;
    hco_tern_map(D, t);
    for (uint64_t k = 0; k < n3; ++k) z[k] = (ELEM)0;
    for (uint64_t i = 0; i < n2; ++i)
        for (uint64_t j = 0; j < n2; ++j)
            z[t[i] + t[j]] += x[i] * y[j];
    free(t);
    return 0;
}

/* One forward step of the method on axis a: the state has shape
 * (3,)^a x (2,) x (2,)^(D-a-1); each pair (a0, a1) along axis a becomes the
 * triple (a0, a0 + a1, a1).  The middle entry is the marginal x[0] + x[1] of
 * the Methods section (three-subproblem recursion). */
static void HCO_FN(hco_forward_axis_)(const ELEM* in, ELEM* out, int D, int a)
{
    const uint64_t n_hi = hco_pow3(a);
    const uint64_t n_lo = (uint64_t)1 << (D - a - 1);
    for (uint64_t hi = 0; hi < n_hi; ++hi) {
        for (uint64_t lo = 0; lo < n_lo; ++lo) {
            const ELEM a0 = in[(hi * 2 + 0) * n_lo + lo];
            const ELEM a1 = in[(hi * 2 + 1) * n_lo + lo];
            out[(hi * 3 + 0) * n_lo + lo] = a0;
            out[(hi * 3 + 1) * n_lo + lo] = a0 + a1;
            out[(hi * 3 + 2) * n_lo + lo] = a1;
        }
    }
}

/* One inverse step on axis a of a (3,)^D state, in place: the middle entry of
 * every line becomes (p1 - p0) - p2, i.e. t - z[0] - z[2] = z[1] of the
 * Methods section, subtracting z[0] first and z[2] second. */
static void HCO_FN(hco_inverse_axis_)(ELEM* v, int D, int a)
{
    const uint64_t n_hi = hco_pow3(a);
    const uint64_t n_lo = hco_pow3(D - a - 1);
    for (uint64_t hi = 0; hi < n_hi; ++hi) {
        for (uint64_t lo = 0; lo < n_lo; ++lo) {
            const ELEM p0 = v[(hi * 3 + 0) * n_lo + lo];
            const ELEM p1 = v[(hi * 3 + 1) * n_lo + lo];
            const ELEM p2 = v[(hi * 3 + 2) * n_lo + lo];
            v[(hi * 3 + 1) * n_lo + lo] = (p1 - p0) - p2;
        }
    }
}

/* Forward map of one operand on all D axes, ascending: 2^D -> 3^D.
 * out and tmp each hold 3^D elements. */
static void HCO_FN(hco_forward_all_)(const ELEM* x, ELEM* out, ELEM* tmp, int D)
{
    const uint64_t n2 = (uint64_t)1 << D;
    ELEM* cur = (D % 2 == 0) ? out : tmp;   /* so that the last step lands in out */
    ELEM* nxt = (D % 2 == 0) ? tmp : out;
    for (uint64_t i = 0; i < n2; ++i) cur[i] = x[i];
    for (int a = 0; a < D; ++a) {
        HCO_FN(hco_forward_axis_)(cur, nxt, D, a);
        ELEM* s = cur; cur = nxt; nxt = s;
    }
}

/* The method in per-axis form (Methods section, three-subproblem recursion
 * unrolled over all axes): forward on axes 0..D-1, elementwise product, then
 * inverse on axes D-1..0.  Needs 3 * 3^D elements of scratch; used for D up to
 * about 16. */
int HCO_FN(hco_canonical_)(const ELEM* x, const ELEM* y, ELEM* z, int D)
{
    if (D < 0 || D > 20) return 1;
    const uint64_t n3 = hco_pow3(D);
    ELEM* X = (ELEM*)malloc(n3 * sizeof(ELEM));
    ELEM* Y = (ELEM*)malloc(n3 * sizeof(ELEM));
    ELEM* T = (ELEM*)malloc(n3 * sizeof(ELEM));
    if (!X || !Y || !T) { free(X); free(Y); free(T); return 2; }
    HCO_FN(hco_forward_all_)(x, X, T, D);
    HCO_FN(hco_forward_all_)(y, Y, T, D);
    for (uint64_t k = 0; k < n3; ++k) z[k] = X[k] * Y[k];
    for (int a = D - 1; a >= 0; --a) HCO_FN(hco_inverse_axis_)(z, D, a);
    free(X); free(Y); free(T);
    return 0;
}

/* The three-subproblem recursion of the Methods section, memory-light:
 *   z[0] = x[0] * y[0]
 *   z[2] = x[1] * y[1]
 *   t    = (x[0] + x[1]) * (y[0] + y[1])
 *   z[1] = (t - z[0]) - z[2]
 * with the marginals x[0] + x[1], y[0] + y[1] written to fresh scratch (the
 * caller's inputs are never modified), and the base case D = 0 a product of
 * scalars.  The three sub-convolutions are independent; at the top par_depth
 * levels they run as parallel tasks, which changes no arithmetic. */
static void HCO_FN(hco_rec_)(const ELEM* x, const ELEM* y, ELEM* z, int D, int par_depth)
{
    if (D == 0) { z[0] = x[0] * y[0]; return; }
    const uint64_t h = (uint64_t)1 << (D - 1);
    const uint64_t t = hco_pow3(D - 1);
    ELEM local[2 * 128];
    ELEM* s = (h <= 128) ? local : (ELEM*)malloc(2 * h * sizeof(ELEM));
    if (!s) abort();
    ELEM* sx = s;
    ELEM* sy = s + h;
    for (uint64_t i = 0; i < h; ++i) sx[i] = x[i] + x[h + i];
    for (uint64_t i = 0; i < h; ++i) sy[i] = y[i] + y[h + i];
    if (par_depth > 0) {
#pragma omp task
        HCO_FN(hco_rec_)(x, y, z, D - 1, par_depth - 1);
#pragma omp task
        HCO_FN(hco_rec_)(x + h, y + h, z + 2 * t, D - 1, par_depth - 1);
#pragma omp task
        HCO_FN(hco_rec_)(sx, sy, z + t, D - 1, par_depth - 1);
#pragma omp taskwait
    } else {
        HCO_FN(hco_rec_)(x, y, z, D - 1, 0);
        HCO_FN(hco_rec_)(x + h, y + h, z + 2 * t, D - 1, 0);
        HCO_FN(hco_rec_)(sx, sy, z + t, D - 1, 0);
    }
    for (uint64_t k = 0; k < t; ++k) z[t + k] = (z[t + k] - z[k]) - z[2 * t + k];
    if (s != local) free(s);
}

/* Entry point of the recursion; threads <= 1 runs it on the calling thread
 * only, otherwise the top levels fan out over that many OpenMP threads. */
int HCO_FN(hco_recursive_)(const ELEM* x, const ELEM* y, ELEM* z, int D, int threads)
{
    if (D < 0 || D > 21) return 1;
    if (threads <= 1) {
        HCO_FN(hco_rec_)(x, y, z, D, 0);
        return 0;
    }
    int depth = 0;
    while (depth < D && depth < 6 && hco_pow3(depth) < (uint64_t)threads * 4) ++depth;
#pragma omp parallel num_threads(threads)
    {
#pragma omp single
        HCO_FN(hco_rec_)(x, y, z, D, depth);
    }
    return 0;
}

/* Adjoint of the method by transposed maps, in the reverse of the forward
 * order (derived from z = G(Fx . Fy) being bilinear; the paper gives no
 * backward):
 *   w_hat = (G^T on axes 0..D-1) w,   G^T: (w0, w1, w2) -> (w0 - w1, w1, w2 - w1)
 *   gx    = (F^T on axes D-1..0)(w_hat . Fy),  F^T: (g0, g1, g2) -> (g0 + g1, g1 + g2)
 *   gy    = (F^T on axes D-1..0)(w_hat . Fx)
 * gx or gy may be NULL to skip that output. */
int HCO_FN(hco_adjoint_)(const ELEM* x, const ELEM* y, const ELEM* w,
                         ELEM* gx, ELEM* gy, int D)
{
    if (D < 0 || D > 20) return 1;
    const uint64_t n3 = hco_pow3(D);
    ELEM* W = (ELEM*)malloc(n3 * sizeof(ELEM));
    ELEM* F = (ELEM*)malloc(n3 * sizeof(ELEM));
    ELEM* T = (ELEM*)malloc(n3 * sizeof(ELEM));
    ELEM* A = (ELEM*)malloc(n3 * sizeof(ELEM));
    if (!W || !F || !T || !A) { free(W); free(F); free(T); free(A); return 2; }
    for (uint64_t k = 0; k < n3; ++k) W[k] = w[k];
    for (int a = 0; a < D; ++a) {
        const uint64_t n_hi = hco_pow3(a);
        const uint64_t n_lo = hco_pow3(D - a - 1);
        for (uint64_t hi = 0; hi < n_hi; ++hi)
            for (uint64_t lo = 0; lo < n_lo; ++lo) {
                const ELEM w0 = W[(hi * 3 + 0) * n_lo + lo];
                const ELEM w1 = W[(hi * 3 + 1) * n_lo + lo];
                const ELEM w2 = W[(hi * 3 + 2) * n_lo + lo];
                W[(hi * 3 + 0) * n_lo + lo] = w0 - w1;
                W[(hi * 3 + 2) * n_lo + lo] = w2 - w1;
            }
    }
    for (int which = 0; which < 2; ++which) {
        ELEM* g = which == 0 ? gx : gy;
        if (!g) continue;
        /* gx pairs w_hat with the transformed y, gy with the transformed x */
        HCO_FN(hco_forward_all_)(which == 0 ? y : x, F, T, D);
        for (uint64_t k = 0; k < n3; ++k) A[k] = W[k] * F[k];
        for (int a = D - 1; a >= 0; --a) {
            /* state: (3,)^(a+1) x (2,)^(D-a-1) -> (3,)^a x (2,)^(D-a) */
            const uint64_t n_hi = hco_pow3(a);
            const uint64_t n_lo = (uint64_t)1 << (D - a - 1);
            for (uint64_t hi = 0; hi < n_hi; ++hi)
                for (uint64_t lo = 0; lo < n_lo; ++lo) {
                    const ELEM g0 = A[(hi * 3 + 0) * n_lo + lo];
                    const ELEM g1 = A[(hi * 3 + 1) * n_lo + lo];
                    const ELEM g2 = A[(hi * 3 + 2) * n_lo + lo];
                    T[(hi * 2 + 0) * n_lo + lo] = g0 + g1;
                    T[(hi * 2 + 1) * n_lo + lo] = g1 + g2;
                }
            ELEM* s = A; A = T; T = s;
        }
        const uint64_t n2 = (uint64_t)1 << D;
        for (uint64_t i = 0; i < n2; ++i) g[i] = A[i];
    }
    free(W); free(F); free(T); free(A);
    return 0;
}

/* Carry-free convolution of two length-n vectors (Discussion): indices are
 * added bit by bit without carries, so x[i] * y[j] belongs to the output
 * whose base-3 digits are the digit-wise sums of the bits of i and j.  The
 * output has 3^D entries, D the number of bits of n - 1 (D = 0 for n = 1).
 * Written over the 1-D indices directly: i outer loop, j inner loop. */
int HCO_FN(hco_carryfree_naive_)(const ELEM* x, const ELEM* y, uint64_t n, ELEM* z)
{
    if (n == 0 || n > ((uint64_t)1 << 20)) return 1;
    int D = 0;
    while (((uint64_t)1 << D) < n) ++D;
    const uint64_t n3 = hco_pow3(D);
    for (uint64_t k = 0; k < n3; ++k) z[k] = (ELEM)0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t ti = hco_tern(i);
        for (uint64_t j = 0; j < n; ++j) z[ti + hco_tern(j)] += x[i] * y[j];
    }
    return 0;
}

/* Distribution of the difference of two random vectors with values in
 * {0,1}^D (Introduction: probability mass functions of sums and differences).
 * Output digit a holds bit_a(i) - bit_a(j) + 1 in {0, 1, 2}, i.e. x[i] * y[j]
 * belongs to z[tern(i) - tern(j) + (3^D - 1) / 2].  i outer, j inner. */
int HCO_FN(hco_difference_naive_)(const ELEM* x, const ELEM* y, ELEM* z, int D)
{
    if (D < 0 || D > 20) return 1;
    const uint64_t n2 = (uint64_t)1 << D;
    const uint64_t n3 = hco_pow3(D);
    const uint64_t mid = (n3 - 1) / 2;
    for (uint64_t k = 0; k < n3; ++k) z[k] = (ELEM)0;
    for (uint64_t i = 0; i < n2; ++i) {
        const uint64_t ti = hco_tern(i) + mid;
        for (uint64_t j = 0; j < n2; ++j) z[ti - hco_tern(j)] += x[i] * y[j];
    }
    return 0;
}

#undef HCO_FN
#undef HCO_CAT
#undef HCO_CAT2
