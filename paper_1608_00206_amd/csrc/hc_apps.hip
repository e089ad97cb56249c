// Applications of hypercube convolution built on the forward path:
//
//   carry-free 1-D convolution (Discussion): two length-n vectors are
//     embedded as hypercubes of D = ceil(log2 n) bits, zero-padded to 2^D,
//     and convolved; output index = digit-wise sum of the two index bit
//     vectors read in base 3.
//   distribution of a difference X - Y of random vectors with values in
//     {0,1}^D (Introduction: sums and differences of multidimensional
//     distributions; the sum is the convolution itself): reflecting y on
//     every axis maps bit b to 1 - b, so the convolution of x with the
//     reflected y puts x[i] y[j] at digits bit(i) + 1 - bit(j) = (X - Y) + 1.
//
//   p-norm estimate of the max-convolution (Discussion: p-norm rings): for
//     nonnegative x, y,  z[k] ~ max over the pairs of k of x[i] y[j], as
//     (sum (x[i] y[j])^p)^(1/p) = mx my (conv((x/mx)^p, (y/my)^p)[k])^(1/p),
//     mx, my the inputs' maxima; the convolution is exact up to rounding, so
//     larger p stay usable than with an FFT, until cancellation in the
//     inverse map (relative error ~ (4D+2) u B/z' of the powered result)
//     dominates.  Optionally rounded to integers.
//
// All three reuse the forward path unchanged; the new device work is a
// padding, reflecting or powering copy into the caller's workspace, and the
// root of the p-norm, which runs as the epilogue of the convolution's last
// inverse pass where that pass has an epilogue kernel, else in place on z.
#include <cmath>
#include <type_traits>

#include "hc.h"
#include "hc_internal.hpp"
#include "hc_kernels.hpp"

namespace hc {

constexpr int APP_NT = 256;

// dst[i] = src[i] for i < n, 0 for n <= i < n2
template <typename T>
__global__ __launch_bounds__(APP_NT) void k_pad(const T* __restrict__ src, T* __restrict__ dst, uint64_t n,
                                                uint64_t n2)
{
    for (uint64_t i = (uint64_t)blockIdx.x * APP_NT + threadIdx.x; i < n2; i += (uint64_t)gridDim.x * APP_NT)
        dst[i] = i < n ? src[i] : T(0);
}

// dst[b][j] = src[b][(n2 - 1) ^ j]: every axis reflected (bit b -> 1 - b)
template <typename T>
__global__ __launch_bounds__(APP_NT) void k_reflect(const T* __restrict__ src, T* __restrict__ dst, uint64_t n2)
{
    const uint64_t off = (uint64_t)blockIdx.y * n2;
    for (uint64_t j = (uint64_t)blockIdx.x * APP_NT + threadIdx.x; j < n2; j += (uint64_t)gridDim.x * APP_NT)
        dst[off + j] = src[off + ((n2 - 1) ^ j)];
}

static uint32_t copy_grid(uint64_t n, int cus)
{
    const uint64_t want = (n + APP_NT - 1) / APP_NT;
    const uint64_t cap = (uint64_t)cus * 32;
    return (uint32_t)(want < cap ? (want ? want : 1) : cap);
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename T>
static void launch_pad(const T* src, T* dst, uint64_t n, uint64_t n2, int cus, hipStream_t s)
{
    LaunchScope scope(s, (double)(n + n2) * sizeof(T), "pad<%s>", tname<T>());
    k_pad<T><<<copy_grid(n2, cus), APP_NT, 0, s>>>(src, dst, n, n2);
}

template <typename T>
static void launch_reflect(const T* src, T* dst, uint64_t n2, int batch, int cus, hipStream_t s)
{
    LaunchScope scope(s, 2.0 * batch * n2 * sizeof(T), "reflect<%s>", tname<T>());
    dim3 grid(copy_grid(n2, cus), batch, 1);
    k_reflect<T><<<grid, APP_NT, 0, s>>>(src, dst, n2);
}

// Per item and operand, the largest entry (negative entries and NaN count as
// 0), in two stages so that a single large pair spreads over the chip:
// k_maxscale_part reduces MAXSCALE_PARTS slices of each input to partial
// maxima, part[(op * batch + b) * MAXSCALE_PARTS + slice]; k_maxscale_final
// reduces those to scales[op * batch + b].
constexpr int MAXSCALE_PARTS = 64;
constexpr int MAX_NT = 256;

template <typename T>
__device__ __forceinline__ T block_max(T m, T* red)
{
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = MAX_NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h && red[threadIdx.x + h] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

// grid (MAXSCALE_PARTS, batch, 2): blockIdx.y = item, blockIdx.z = operand
template <typename T>
__global__ __launch_bounds__(MAX_NT) void k_maxscale_part(const T* __restrict__ x, const T* __restrict__ y,
                                                          uint64_t n2, T* __restrict__ part)
{
    __shared__ T red[MAX_NT];
    const T* src = (blockIdx.z ? y : x) + (uint64_t)blockIdx.y * n2;
    T m = T(0);
    for (uint64_t i = (uint64_t)blockIdx.x * MAX_NT + threadIdx.x; i < n2; i += (uint64_t)MAXSCALE_PARTS * MAX_NT) {
        const T v = src[i];
        m = v > m ? v : m;
    }
    m = block_max(m, red);
    if (threadIdx.x == 0)
        part[((uint64_t)blockIdx.z * gridDim.y + blockIdx.y) * MAXSCALE_PARTS + blockIdx.x] = m;
}

// grid (batch, 2)
template <typename T>
__global__ __launch_bounds__(MAX_NT) void k_maxscale_final(const T* __restrict__ part, T* __restrict__ scales)
{
    __shared__ T red[MAX_NT];
    const uint64_t row = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    T m = T(0);
    for (int i = threadIdx.x; i < MAXSCALE_PARTS; i += MAX_NT) {
        const T v = part[row * MAXSCALE_PARTS + i];
        m = v > m ? v : m;
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) scales[row] = m;
}

template <typename T>
__device__ __forceinline__ T pow_t(T a, T b)
{
    if constexpr (sizeof(T) == 4) return powf(a, b);
    else return pow(a, b);
}

// a^k for an integer k >= 1 by binary powering: the result accumulates the
// squares a, a^2, a^4, ... selected by the bits of k, low bits first (each
// product one IEEE multiplication in this order).
template <typename T>
__device__ __forceinline__ T int_pow(T a, int k)
{
    T A = T(1), b = a;
    for (;;) {
        if (k & 1) A *= b;
        k >>= 1;
        if (!k) break;
        b *= b;
    }
    return A;
}

// (xh + xl) <- (xh + xl)(yh + yl) on double-double values: the product's
// rounding error and the cross terms are gathered with fused multiply-adds,
// then renormalised (|e| is far below |p|, so the fast two-sum is exact).
__device__ __forceinline__ void dd_mul(double& xh, double& xl, double yh, double yl)
{
    const double p = xh * yh;
    double e = fma(xh, yh, -p);
    e = fma(xh, yl, e);
    e = fma(xl, yh, e);
    const double h = p + e;
    xl = e - (h - p);
    xh = h;
}

// q^k for an integer k >= 1 in float64 with one final rounding of a
// double-double result: binary powering (the squares q, q^2, q^4, ...
// selected by the bits of k, low bits first), every product by dd_mul.
// Relative error about u, about what a correctly rounded pow gives, in a
// fixed order of IEEE operations.
__device__ __forceinline__ double pow_dd(double q, int k)
{
    double Ah = 1.0, Al = 0.0, bh = q, bl = 0.0;
    for (;;) {
        if (k & 1) dd_mul(Ah, Al, bh, bl);
        k >>= 1;
        if (!k) break;
        dd_mul(bh, bl, bh, bl);
    }
    return Ah + Al;
}

// xp[b][i] = (x[b][i] / mx_b)^p, yp likewise (0 where the entry or the scale
// is not positive).  Integer p (ip > 0) take pow_dd on the quotient formed in
// float64 (rounded once to T at the end); other p take the device library's
// pow.  blockIdx.y = item, blockIdx.z = operand.
template <typename T>
__global__ __launch_bounds__(APP_NT) void k_power(const T* __restrict__ x, const T* __restrict__ y,
                                                  T* __restrict__ xp, T* __restrict__ yp,
                                                  const T* __restrict__ scales, uint64_t n2, T p, int ip)
{
    const int op = blockIdx.z;
    const uint64_t off = (uint64_t)blockIdx.y * n2;
    const T* src = (op ? y : x) + off;
    T* dst = (op ? yp : xp) + off;
    const T m = scales[(uint64_t)op * gridDim.y + blockIdx.y];
    for (uint64_t i = (uint64_t)blockIdx.x * APP_NT + threadIdx.x; i < n2; i += (uint64_t)gridDim.x * APP_NT) {
        const T v = src[i];
        T r = T(0);
        if (v > T(0) && m > T(0)) {
            if (ip > 0) r = (T)pow_dd((double)v / (double)m, ip);
            else r = pow_t<T>(v / m, p);
        }
        dst[i] = r;
    }
}

template <typename T>
__device__ __forceinline__ T exp_t(T a)
{
    if constexpr (sizeof(T) == 4) return expf(a);
    else return exp(a);
}

template <typename T>
__device__ __forceinline__ T log_t(T a)
{
    if constexpr (sizeof(T) == 4) return logf(a);
    else return log(a);
}

// Integer p up to this bound take the polished root below; other p take
// exp(log(v) / p).
constexpr int ROOT_INT_MAX = 1024;

// Coefficients of (1 + eps)^(1/p) = 1 + c1 eps + c2 eps^2 + c3 eps^3 + c4 eps^4 + ...
struct RootCoef {
    double c[4];
    float inv_pf;  // 1/p rounded to float, for the seed
    int log2p;     // log2(p) when p is a power of two
};

// v^(1/p) for finite v > 0 and integer 2 <= p <= ROOT_INT_MAX, in float64.
// With v = m 2^e (m in [1/2, 1)) and e = n p + rem (|rem| <= p/2 + 1),
// v^(1/p) = 2^n V^(1/p) for V = m 2^rem, which stays far inside the normal
// range.  A float seed a ~ V^(1/p) (hardware log2 and exp2, relative error
// ~1e-7) is polished with one step of the binomial series: A = a^p by binary
// powering (relative error below (p - 1) u, worth under u after the 1/p
// below), eps = V / A - 1 (V - A is exact, |eps| < 1e-3), and
// V^(1/p) = a (1 + eps)^(1/p), the series cut after eps^4.  The result is
// within 2 u of the exact root, with a margin of 10x on the seed's error.
__device__ __forceinline__ double root_int(double v, int p, const RootCoef& rc)
{
    int e;
    const double m = frexp(v, &e);
    const int n = (int)rintf((float)e * rc.inv_pf);
    const int rem = e - n * p;
    const float t = ((float)rem + __builtin_amdgcn_logf((float)m)) * rc.inv_pf;
    const double a = (double)__builtin_amdgcn_exp2f(t);
    const double A = int_pow<double>(a, p);
    const double V = ldexp(m, rem);
    double q = __builtin_amdgcn_rcp(A);
    q = fma(q, fma(-A, q, 1.0), q);
    const double eps = (V - A) * q;
    const double P = eps * (rc.c[0] + eps * (rc.c[1] + eps * (rc.c[2] + eps * rc.c[3])));
    return ldexp(fma(a, P, a), n);
}

// v^(1/p) for finite v > 0 and p = 2^L, L <= ROOT_POW2_MAX, in float64: the
// steps of root_int with the exponent split by shifts (n = floor((e + p/2) /
// p), |rem| <= p/2) and the L squarings unrolled.  The seed's error (t
// within 2^-24.8 absolute, a within 2^-22.5 relative) bounds |eps| by
// p 2^-22.5; for p <= 32 that is 2^-17.5, so the series stops after eps^2
// (the dropped c2 eps^3 + c3 eps^4 stay below u / 60); larger p keep the
// terms to eps^4, as root_int does.  Either way the result is within 2 u of
// the exact root.
constexpr int ROOT_POW2_MAX = 10;  // 2^10 = ROOT_INT_MAX
constexpr int ROOT_SHORT_SERIES_MAX = 5;

template <int L>
__device__ __forceinline__ double root_pow2(double v, const RootCoef& rc)
{
    static_assert(L >= 1 && L <= ROOT_POW2_MAX && (1 << ROOT_POW2_MAX) == ROOT_INT_MAX, "p = 2 ... ROOT_INT_MAX");
    constexpr int p = 1 << L;
    int e;
    const double m = frexp(v, &e);
    const int n = (e + p / 2) >> L;
    const int rem = e - n * p;
    const float t = ((float)rem + __builtin_amdgcn_logf((float)m)) * (1.0f / (float)p);
    const double a = (double)__builtin_amdgcn_exp2f(t);
    double A = a;
#pragma unroll
    for (int k = 0; k < L; ++k) A *= A;
    const double V = ldexp(m, rem);
    double q = __builtin_amdgcn_rcp(A);
    q = fma(q, fma(-A, q, 1.0), q);
    const double eps = (V - A) * q;
    double P;
    if constexpr (L <= ROOT_SHORT_SERIES_MAX) P = eps * (rc.c[0] + eps * rc.c[1]);
    else P = eps * (rc.c[0] + eps * (rc.c[1] + eps * (rc.c[2] + eps * rc.c[3])));
    return ldexp(fma(a, P, a), n);
}

// How k_root takes the root: p = 1 needs none; p = 2, 4, ..., 2^ROOT_POW2_MAX
// take root_pow2 (mode ROOT_POW2 + L); other integer p in [2, ROOT_INT_MAX]
// take root_int (in float64 for both types); other p take exp(log(v) / p),
// whose relative error is a few ulps times 1 + |ln v| / p.  Every error is
// far below the estimate's own 2^(s/p) bias.
enum RootMode { ROOT_NONE = 0, ROOT_INT = 1, ROOT_EXPLOG = 2, ROOT_POW2 = 3 };

// mx my max(v, 0)^(1/p) for one output (s = mx my), optionally rounded.
// The root is taken on every lane and the result selected (0 where v <= 0 or
// v is NaN, whose root arithmetic gives NaN), so that no lane waits for a
// branch around the arithmetic.
template <typename T, int MODE>
__device__ __forceinline__ T root_value(T v, T s, T inv_p, int ip, const RootCoef& rc, int round)
{
    const bool pos = v > T(0);
    T w;
    if constexpr (MODE == ROOT_NONE) w = v;
    else if constexpr (MODE == ROOT_INT) w = (T)root_int((double)v, ip, rc);
    else if constexpr (MODE > ROOT_POW2) w = (T)root_pow2<MODE - ROOT_POW2>((double)v, rc);
    else w = exp_t<T>(log_t<T>(v) * inv_p);
    const T sw = s * w;
    T r = pos ? sw : T(0);
    if (round) r = rint(r);
    return r;
}

constexpr int ROOT_U = 4;
constexpr uint64_t ROOT_SPAN = (uint64_t)ROOT_U * APP_NT;

// z[b][k] = mx_b my_b max(z[b][k], 0)^(1/p), optionally rounded to an integer.
// grid (ceil(n3 / ROOT_SPAN), batch).
template <typename T, int MODE>
__global__ __launch_bounds__(APP_NT) void k_root(T* __restrict__ z, const T* __restrict__ scales, uint64_t n3,
                                                 T inv_p, int ip, RootCoef rc, int round)
{
    const uint64_t off = (uint64_t)blockIdx.y * n3;
    const T s = scales[blockIdx.y] * scales[gridDim.y + blockIdx.y];
    // one workgroup per ROOT_SPAN consecutive elements, four per thread, all
    // loaded before any arithmetic (a grid-stride loop over the same data
    // streams 12% slower)
    const uint64_t k0 = (uint64_t)blockIdx.x * ROOT_SPAN + threadIdx.x;
    T v[ROOT_U];
#pragma unroll
    for (int q = 0; q < ROOT_U; ++q) {
        const uint64_t k = k0 + q * APP_NT;
        v[q] = k < n3 ? z[off + k] : T(0);
    }
#pragma unroll
    for (int q = 0; q < ROOT_U; ++q) {
        const uint64_t k = k0 + q * APP_NT;
        const T r = root_value<T, MODE>(v[q], s, inv_p, ip, rc, round);
        if (k < n3) z[off + k] = r;
    }
}

// The root as the epilogue of the convolution's last inverse pass: every
// entry of the pass's tile goes through root_value before it is stored, so
// the separate read and write of z by k_root disappear.  bind() fixes the
// batch item's scale.
template <typename T, int MODE>
struct RootEpilogue {
    const T* scales;
    int batch;
    T inv_p;
    int ip;
    RootCoef rc;
    int round;
    struct Bound {
        static constexpr bool ALL = true;
        T s, inv_p;
        int ip;
        RootCoef rc;
        int round;
        __device__ __forceinline__ T apply(T v) const { return root_value<T, MODE>(v, s, inv_p, ip, rc, round); }
    };
    __device__ __forceinline__ Bound bind(uint32_t b) const
    {
        return Bound{scales[b] * scales[batch + b], inv_p, ip, rc, round};
    }
};

// LastPass::launch for the root: passes of 3 or 4 register axes and 1 or 2
// wave axes (the last pass of default plans whose last group has 4 to 6
// axes) have an epilogue kernel; other shapes decline.
template <typename T, int MODE>
static int launch_root_pass(const LastPass& self, const InvPass& ip, void* z, BMap z_map, uint64_t L,
                            uint32_t n_hi, int batch, int cus, hipStream_t s)
{
    using EP = RootEpilogue<T, MODE>;
    const bool ok = (ip.mR == 3 || ip.mR == 4) && (ip.mW == 1 || ip.mW == 2);
    if (!ok) return HC_ERR_UNSUPPORTED;
    const EP& epi = *static_cast<const EP*>(self.ctx);
    const uint32_t tiles_per_hi = (uint32_t)((L + 63) / 64);
    const uint64_t n_tiles = (uint64_t)tiles_per_hi * n_hi;
    const dim3 grid(tile_grid(n_tiles, cus, 0), batch, 1);
    const int TM = (int)pow3u(ip.mR + ip.mW);
    LaunchScope scope(s, 2.0 * batch * n_hi * L * TM * sizeof(T), "inv_pass_root<%s,%d+%d>", tname<T>(), ip.mR,
                      ip.mW);
    T* zt = static_cast<T*>(z);
    const uint32_t nt = (uint32_t)n_tiles;
    if (ip.mR == 4 && ip.mW == 2)
        k_inv_pass_epi<T, 4, 2, EP><<<grid, 64 * 9, 0, s>>>(zt, z_map, L, tiles_per_hi, nt, epi);
    else if (ip.mR == 4)
        k_inv_pass_epi<T, 4, 1, EP><<<grid, 64 * 3, 0, s>>>(zt, z_map, L, tiles_per_hi, nt, epi);
    else if (ip.mW == 2)
        k_inv_pass_epi<T, 3, 2, EP><<<grid, 64 * 9, 0, s>>>(zt, z_map, L, tiles_per_hi, nt, epi);
    else
        k_inv_pass_epi<T, 3, 1, EP><<<grid, 64 * 3, 0, s>>>(zt, z_map, L, tiles_per_hi, nt, epi);
    return HC_OK;
}

// Scales (2 per item) followed by the partial maxima (2 * MAXSCALE_PARTS per item).
static size_t maxconv_scale_bytes(int batch, size_t es)
{
    return round256(2 * (size_t)batch * (1 + MAXSCALE_PARTS) * es);
}

template <typename T>
static int maxconv_t(const T* x, const T* y, T* z, int D, int batch, double p, bool round, bool separate_root,
                     char* ws, size_t ws_bytes, int cus, hipStream_t s)
{
    const uint64_t n2 = 1ull << D, n3 = pow3u(D);
    T* scales = reinterpret_cast<T*>(ws);
    const size_t sc_b = maxconv_scale_bytes(batch, sizeof(T));
    const size_t op_b = round256((size_t)batch * n2 * sizeof(T));
    T* part = scales + 2 * (size_t)batch;
    T* xp = reinterpret_cast<T*>(ws + sc_b);
    T* yp = reinterpret_cast<T*>(ws + sc_b + op_b);
    {
        LaunchScope scope(s, 2.0 * batch * n2 * sizeof(T), "maxscale<%s>", tname<T>());
        k_maxscale_part<T><<<dim3(MAXSCALE_PARTS, batch, 2), MAX_NT, 0, s>>>(x, y, n2, part);
        k_maxscale_final<T><<<dim3(batch, 2, 1), MAX_NT, 0, s>>>(part, scales);
    }
    const int ip = (p == std::floor(p) && p >= 2 && p <= ROOT_INT_MAX) ? (int)p : 0;
    {
        LaunchScope scope(s, 4.0 * batch * n2 * sizeof(T), "power<%s>", tname<T>());
        // p = 1 is the scaled value itself (pow_dd with k = 1)
        k_power<T><<<dim3(copy_grid(n2, cus), batch, 2), APP_NT, 0, s>>>(x, y, xp, yp, scales, n2, (T)p,
                                                                          p == 1 ? 1 : ip);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "max-convolution launch");
    RootCoef coef{};
    const double c1 = 1.0 / p;
    coef.c[0] = c1;
    coef.c[1] = coef.c[0] * (c1 - 1) / 2;
    coef.c[2] = coef.c[1] * (c1 - 2) / 3;
    coef.c[3] = coef.c[2] * (c1 - 3) / 4;
    coef.inv_pf = (float)c1;
    coef.log2p = 0;
    while (ip > 1 && (1 << (coef.log2p + 1)) <= ip) ++coef.log2p;
    const bool pow2 = ip >= 2 && (1 << coef.log2p) == ip;
    const T inv_p = (T)c1;
    const int rnd = round ? 1 : 0;
    const int mode = p == 1 ? ROOT_NONE
                            : (pow2 && coef.log2p <= ROOT_POW2_MAX ? ROOT_POW2 + coef.log2p
                                                                   : (ip ? ROOT_INT : ROOT_EXPLOG));
    // the root runs as the epilogue of the convolution's last inverse pass
    // where that pass has an epilogue kernel, else as its own kernel
    auto run = [&](auto mode_c) -> int {
        constexpr int M = decltype(mode_c)::value;
        const RootEpilogue<T, M> epi{scales, batch, inv_p, ip, coef, rnd};
        LastPass last;
        last.launch = launch_root_pass<T, M>;
        last.ctx = &epi;
        const int rc = convolve_batch_last(xp, yp, z, D, sizeof(T) == 4 ? HC_F32 : HC_F64, batch,
                                           ws + sc_b + 2 * op_b, ws_bytes - sc_b - 2 * op_b, s,
                                           separate_root ? nullptr : &last);
        if (rc != HC_OK) return rc;
        if (!last.taken) {
            LaunchScope scope(s, 2.0 * batch * n3 * sizeof(T), "root<%s>", tname<T>());
            const dim3 grid((uint32_t)((n3 + ROOT_SPAN - 1) / ROOT_SPAN), batch, 1);
            k_root<T, M><<<grid, APP_NT, 0, s>>>(z, scales, n3, inv_p, ip, coef, rnd);
        }
        return HC_OK;
    };
    using std::integral_constant;
    int rc;
    switch (mode) {
        case ROOT_NONE: rc = run(integral_constant<int, ROOT_NONE>{}); break;
        case ROOT_INT: rc = run(integral_constant<int, ROOT_INT>{}); break;
        case ROOT_POW2 + 1: rc = run(integral_constant<int, ROOT_POW2 + 1>{}); break;
        case ROOT_POW2 + 2: rc = run(integral_constant<int, ROOT_POW2 + 2>{}); break;
        case ROOT_POW2 + 3: rc = run(integral_constant<int, ROOT_POW2 + 3>{}); break;
        case ROOT_POW2 + 4: rc = run(integral_constant<int, ROOT_POW2 + 4>{}); break;
        case ROOT_POW2 + 5: rc = run(integral_constant<int, ROOT_POW2 + 5>{}); break;
        case ROOT_POW2 + 6: rc = run(integral_constant<int, ROOT_POW2 + 6>{}); break;
        case ROOT_POW2 + 7: rc = run(integral_constant<int, ROOT_POW2 + 7>{}); break;
        case ROOT_POW2 + 8: rc = run(integral_constant<int, ROOT_POW2 + 8>{}); break;
        case ROOT_POW2 + 9: rc = run(integral_constant<int, ROOT_POW2 + 9>{}); break;
        case ROOT_POW2 + 10: rc = run(integral_constant<int, ROOT_POW2 + 10>{}); break;
        default: rc = run(integral_constant<int, ROOT_EXPLOG>{}); break;
    }
    static_assert(ROOT_POW2_MAX == 10, "one case per power of two");
    if (rc != HC_OK) return rc;
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "max-convolution launch");
    return HC_OK;
}

static int carryfree_dim(uint64_t n)
{
    if (n == 0 || n > (1ull << HC_MAX_D)) return -1;
    int D = 0;
    while ((1ull << D) < n) ++D;
    return D;
}

}  // namespace hc

using namespace hc;

extern "C" {

int hc_carryfree_dim(uint64_t n) { return carryfree_dim(n); }

uint64_t hc_carryfree_index(uint64_t i, uint64_t j)
{
    uint64_t k = 0, w = 1;
    while (i | j) {
        k += ((i & 1u) + (j & 1u)) * w;
        i >>= 1;
        j >>= 1;
        w *= 3;
    }
    return k;
}

size_t hc_carryfree_workspace_bytes(uint64_t n, int dtype)
{
    const int D = carryfree_dim(n);
    const size_t es = dtype_size(dtype);
    if (D < 0 || es == 0) return (size_t)-1;
    const size_t conv = hc_workspace_bytes(D, dtype, 1);
    if (n == (1ull << D)) return conv;
    return round256(2 * ((size_t)1 << D) * es) + conv;
}

int hc_carryfree_convolve(const void* x, const void* y, uint64_t n, void* z, int dtype, void* workspace,
                          size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_carryfree_convolve n=%llu dtype=%d", (unsigned long long)n, dtype);
    if (!x || !y || !z) return fail(HC_ERR_INVALID_ARG, "x, y and z must be non-null");
    const int D = carryfree_dim(n);
    if (D < 0) return fail(HC_ERR_D_RANGE, "length %llu outside [1, 2^%d]", (unsigned long long)n, HC_MAX_D);
    const size_t es = dtype_size(dtype);
    if (es == 0) return fail(HC_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    const uint64_t n2 = 1ull << D;
    if (n == n2) return hc_convolve(x, y, z, D, dtype, workspace, workspace_bytes, stream);
    if (misaligned(x, es) || misaligned(y, es) || misaligned(z, es) || misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const size_t need = hc_carryfree_workspace_bytes(n, dtype);
    if (!workspace || workspace_bytes < need)
        return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                    workspace ? workspace_bytes : (size_t)0);
    const size_t out_b = (size_t)pow3u(D) * es;
    if (ranges_overlap(z, out_b, x, n * es) || ranges_overlap(z, out_b, y, n * es))
        return fail(HC_ERR_ALIAS, "z overlaps x or y");
    if (ranges_overlap(workspace, need, x, n * es) || ranges_overlap(workspace, need, y, n * es))
        return fail(HC_ERR_ALIAS, "workspace overlaps x or y");
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    char* ws = static_cast<char*>(workspace);
    void* xp = ws;
    void* yp = ws + n2 * es;
    const size_t pad_b = round256(2 * n2 * es);
    switch (dtype) {
        case HC_F64:
            launch_pad<double>((const double*)x, (double*)xp, n, n2, cus, stream);
            launch_pad<double>((const double*)y, (double*)yp, n, n2, cus, stream);
            break;
        case HC_F32:
            launch_pad<float>((const float*)x, (float*)xp, n, n2, cus, stream);
            launch_pad<float>((const float*)y, (float*)yp, n, n2, cus, stream);
            break;
        default:
            launch_pad<uint64_t>((const uint64_t*)x, (uint64_t*)xp, n, n2, cus, stream);
            launch_pad<uint64_t>((const uint64_t*)y, (uint64_t*)yp, n, n2, cus, stream);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pad launch");
    return hc_convolve(xp, yp, z, D, dtype, ws + pad_b, workspace_bytes - pad_b, stream);
}

size_t hc_difference_workspace_bytes(int D, int dtype, int batch)
{
    if (D < 0 || D > HC_MAX_D || dtype_size(dtype) == 0 || batch < 1) return (size_t)-1;
    return round256((size_t)batch * ((size_t)1 << D) * dtype_size(dtype)) + hc_workspace_bytes(D, dtype, batch);
}

int hc_difference_batch(const void* x, const void* y, void* z, int D, int dtype, int batch, void* workspace,
                        size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_difference_batch D=%d dtype=%d batch=%d", D, dtype, batch);
    if (!x || !y || !z) return fail(HC_ERR_INVALID_ARG, "x, y and z must be non-null");
    if (D < 0 || D > HC_MAX_D) return fail(HC_ERR_D_RANGE, "D=%d outside [0, %d]", D, HC_MAX_D);
    const size_t es = dtype_size(dtype);
    if (es == 0) return fail(HC_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (batch < 1 || batch > 65535) return fail(HC_ERR_INVALID_ARG, "batch=%d outside [1, 65535]", batch);
    if (misaligned(x, es) || misaligned(y, es) || misaligned(z, es) || misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const size_t need = hc_difference_workspace_bytes(D, dtype, batch);
    if (!workspace || workspace_bytes < need)
        return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                    workspace ? workspace_bytes : (size_t)0);
    const uint64_t n2 = 1ull << D;
    const size_t in_b = (size_t)batch * n2 * es;
    if (ranges_overlap(workspace, need, x, in_b) || ranges_overlap(workspace, need, y, in_b))
        return fail(HC_ERR_ALIAS, "workspace overlaps x or y");
    if (ranges_overlap(z, (size_t)batch * pow3u(D) * es, y, in_b)) return fail(HC_ERR_ALIAS, "z overlaps y");
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    char* ws = static_cast<char*>(workspace);
    switch (dtype) {
        case HC_F64: launch_reflect<double>((const double*)y, (double*)ws, n2, batch, cus, stream); break;
        case HC_F32: launch_reflect<float>((const float*)y, (float*)ws, n2, batch, cus, stream); break;
        default: launch_reflect<uint64_t>((const uint64_t*)y, (uint64_t*)ws, n2, batch, cus, stream); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reflect launch");
    const size_t r_b = round256(in_b);
    return hc_convolve_batch(x, ws, z, D, dtype, batch, ws + r_b, workspace_bytes - r_b, stream);
}

size_t hc_maxconv_workspace_bytes(int D, int dtype, int batch)
{
    if (D < 0 || D > HC_MAX_D || (dtype != HC_F64 && dtype != HC_F32) || batch < 1) return (size_t)-1;
    const size_t es = dtype_size(dtype);
    return maxconv_scale_bytes(batch, es) + 2 * round256((size_t)batch * ((size_t)1 << D) * es) +
           hc_workspace_bytes(D, dtype, batch);
}

int hc_maxconv_pnorm_batch(const void* x, const void* y, void* z, int D, int dtype, int batch, double p,
                           unsigned flags, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_maxconv_pnorm_batch D=%d dtype=%d batch=%d p=%g", D, dtype, batch, p);
    if (!x || !y || !z) return fail(HC_ERR_INVALID_ARG, "x, y and z must be non-null");
    if (D < 0 || D > HC_MAX_D) return fail(HC_ERR_D_RANGE, "D=%d outside [0, %d]", D, HC_MAX_D);
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_ERR_UNSUPPORTED, "the p-norm max-convolution supports float64 and float32 only");
    if (batch < 1 || batch > 65535) return fail(HC_ERR_INVALID_ARG, "batch=%d outside [1, 65535]", batch);
    if (!(p >= 1.0) || !(p <= 1e300)) return fail(HC_ERR_INVALID_ARG, "p must be a finite number >= 1");
    if (flags & ~(HC_MAXCONV_ROUND | HC_MAXCONV_SEPARATE_ROOT))
        return fail(HC_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const size_t es = dtype_size(dtype);
    if (misaligned(x, es) || misaligned(y, es) || misaligned(z, es) || misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const size_t need = hc_maxconv_workspace_bytes(D, dtype, batch);
    if (!workspace || workspace_bytes < need)
        return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                    workspace ? workspace_bytes : (size_t)0);
    const uint64_t n2 = 1ull << D;
    const size_t in_b = (size_t)batch * n2 * es, out_b = (size_t)batch * pow3u(D) * es;
    if (ranges_overlap(workspace, need, x, in_b) || ranges_overlap(workspace, need, y, in_b))
        return fail(HC_ERR_ALIAS, "workspace overlaps x or y");
    if (ranges_overlap(z, out_b, x, in_b) || ranges_overlap(z, out_b, y, in_b) ||
        ranges_overlap(z, out_b, workspace, need))
        return fail(HC_ERR_ALIAS, "z overlaps x, y or the workspace");
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    const bool round = (flags & HC_MAXCONV_ROUND) != 0;
    const bool separate = (flags & HC_MAXCONV_SEPARATE_ROOT) != 0;
    char* ws = static_cast<char*>(workspace);
    if (dtype == HC_F64)
        return maxconv_t<double>((const double*)x, (const double*)y, (double*)z, D, batch, p, round, separate, ws,
                                 workspace_bytes, cus, stream);
    return maxconv_t<float>((const float*)x, (const float*)y, (float*)z, D, batch, p, round, separate, ws,
                            workspace_bytes, cus, stream);
}

}  // extern "C"
