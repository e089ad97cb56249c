// Distribution of X1 + X2 + X3 for three independent random vectors whose D
// axes are all Bernoulli (Introduction: sums of multiple probability mass
// functions whose axes are Bernoulli variables).  The sum of two is the
// hypercube convolution itself; this file adds the next link of the chain.
//
// Along one axis each operand is a linear polynomial a0 + a1 t, and the
// sum's distribution along that axis is the product of three of them, a
// cubic c0 + c1 t + c2 t^2 + c3 t^3.  The Methods section recovers the
// product of two from its values at t = 0, 1 and infinity; the product of
// three needs one more point, and t = -1 keeps the recovery exact (its
// only division is by 2):
//   forward  F4: (a0, a1) -> (a0, a0 + a1, a0 - a1, a1)        axes 0..D-1
//   product  (x1^ * x2^) * x3^                                 elementwise
//   inverse  G4: (p0, p1, pm, pi) -> (p0, (p1 - pm)/2 - pi,
//                                     (p1 + pm)/2 - p0, pi)     axes D-1..0
// on 4^D values per operand.  Every floating-point operation is one IEEE
// operation in this order, so results are bitwise independent of tiling.
// int64 data wraps modulo 2^64; the halving divides the signed difference by
// 2, exact whenever the true intermediate fits in int64.
//
// Layout: x1, x2, x3 hold 2^D values (bit d of the flat index = axis D-1-d);
// z holds 4^D values, base-4 digit d of the flat index (weight 4^d) = axis
// D-1-d, so x1[i] x2[j] x3[l] lands at quad(i) + quad(j) + quad(l).
//
// GPU schedule, mirroring the two-operand path:
//   outer forward   F4 on axes 0..p-1 in groups of at most 3, for the three
//                   operands: 2^D -> 4^p x 2^K each              (k_s3_fwd)
//   fused inner     per outer index o: F4 on the K = 6 inner axes of the
//                   three rows, the product, G4 on the inner axes, one
//                   contiguous 4^K row of z, every step on two axes held
//                   in registers                                 (k_s3_tile6)
//                   (D < 6: one tile of D axes,      k_s3_fused_r / k_s3_fused)
//   outer inverse   G4 on axes p-1..0 in place: groups of 4 from axis p-1
//                   down, three axes in registers and the fourth across the
//                   workgroup's waves                          (k_s3_inv4w),
//                   then axes p mod 4 - 1 .. 0 in registers      (k_s3_inv)
#include "hc.h"

#include <hip/hip_runtime.h>

#include <type_traits>
#include <vector>

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int S3_MAX_D = 16;
constexpr int S3_GROUP = 3;
constexpr int S3_NT = 256;

template <typename T>
__device__ __forceinline__ T half_of(T v)
{
    if constexpr (std::is_same<T, uint64_t>::value) return (uint64_t)((int64_t)v / 2);
    else return v * T(0.5);
}

// G4 on one line of four values (in registers)
template <typename T>
__device__ __forceinline__ void g4(T& p0, T& p1, T& pm, T& pi)
{
    const T d = p1 - pm;
    const T s = p1 + pm;
    p1 = half_of(d) - pi;
    pm = half_of(s) - p0;
}

// F4 on M axes of 2^M values held by one thread, ascending (axis 0 of the
// group first): s has room for 4^M values; on entry s[0 .. 2^M) holds the
// group's binary sub-cube.
template <typename T, int M>
__device__ __forceinline__ void f4_group(T (&s)[1 << (2 * M)])
{
#pragma unroll
    for (int a = 0; a < M; ++a) {
        // state [4^a][2][2^(M-a-1)] -> [4^a][4][2^(M-a-1)], rewritten from the
        // top down so that no entry is overwritten before it is read
        const int lo_n = 1 << (M - a - 1);
        const int hi_n = 1 << (2 * a);
#pragma unroll
        for (int hi = hi_n - 1; hi >= 0; --hi)
#pragma unroll
            for (int lo = lo_n - 1; lo >= 0; --lo) {
                const T a0 = s[(hi * 2 + 0) * lo_n + lo];
                const T a1 = s[(hi * 2 + 1) * lo_n + lo];
                s[(hi * 4 + 3) * lo_n + lo] = a1;
                s[(hi * 4 + 2) * lo_n + lo] = a0 - a1;
                s[(hi * 4 + 1) * lo_n + lo] = a0 + a1;
                s[(hi * 4 + 0) * lo_n + lo] = a0;
            }
    }
}

// G4 on M axes of 4^M values held by one thread, descending (the group's
// innermost axis first).
template <typename T, int M>
__device__ __forceinline__ void g4_group(T (&v)[1 << (2 * M)])
{
#pragma unroll
    for (int a = M - 1; a >= 0; --a) {
        const int lo_n = 1 << (2 * (M - a - 1));
        const int hi_n = 1 << (2 * a);
#pragma unroll
        for (int hi = 0; hi < hi_n; ++hi)
#pragma unroll
            for (int lo = 0; lo < lo_n; ++lo) {
                T* p = v + hi * 4 * lo_n + lo;
                g4(p[0], p[lo_n], p[2 * lo_n], p[3 * lo_n]);
            }
    }
}

// a digit 1 or 2 (base 4) among the M digits of g: the entries G4 changes
__host__ __device__ constexpr bool has_mid_digit(int g, int M)
{
    for (int a = 0; a < M; ++a, g >>= 2)
        if ((g & 3) == 1 || (g & 3) == 2) return true;
    return false;
}

// Outer forward: F4 on M axes, out of place, for the three operands
// (blockIdx.z); in [n_hi][2^M][L] -> out [n_hi][4^M][L], L = 2^log2L; one
// thread per column, lanes along the contiguous index.
template <typename T, int M>
__global__ __launch_bounds__(S3_NT) void k_s3_fwd(const T* __restrict__ in0, const T* __restrict__ in1,
                                                  const T* __restrict__ in2, T* __restrict__ out0,
                                                  T* __restrict__ out1, T* __restrict__ out2, uint64_t in_bs,
                                                  uint64_t out_bs, uint64_t n_cols, uint32_t log2L)
{
    const T* in = blockIdx.z == 0 ? in0 : (blockIdx.z == 1 ? in1 : in2);
    T* out = blockIdx.z == 0 ? out0 : (blockIdx.z == 1 ? out1 : out2);
    const uint64_t c = (uint64_t)blockIdx.x * S3_NT + threadIdx.x;
    if (c >= n_cols) return;
    in += (uint64_t)blockIdx.y * in_bs;
    out += (uint64_t)blockIdx.y * out_bs;
    const uint64_t L = 1ull << log2L;
    const uint64_t hi = c >> log2L, lo = c & (L - 1);
    const T* src = in + (hi << M) * L + lo;
    T* dst = out + hi * (1ull << (2 * M)) * L + lo;
    T s[1 << (2 * M)];
#pragma unroll
    for (int b = 0; b < (1 << M); ++b) s[b] = src[(uint64_t)b * L];
    f4_group<T, M>(s);
#pragma unroll
    for (int t = 0; t < (1 << (2 * M)); ++t) dst[(uint64_t)t * L] = s[t];
}

// Outer inverse: G4 on M axes in place, z viewed as [n_hi][4^M][L],
// L = 4^(axes below); one thread per column; entries G4 leaves unchanged
// (no digit 1 or 2 among the group's digits) are not written back.
template <typename T, int M>
__global__ __launch_bounds__(S3_NT) void k_s3_inv(T* __restrict__ z, uint64_t z_bs, uint64_t n_cols,
                                                  uint32_t log2L)
{
    const uint64_t c = (uint64_t)blockIdx.x * S3_NT + threadIdx.x;
    if (c >= n_cols) return;
    z += (uint64_t)blockIdx.y * z_bs;
    const uint64_t L = 1ull << log2L;
    const uint64_t hi = c >> log2L, lo = c & (L - 1);
    T* p = z + hi * (1ull << (2 * M)) * L + lo;
    T v[1 << (2 * M)];
#pragma unroll
    for (int t = 0; t < (1 << (2 * M)); ++t) v[t] = p[(uint64_t)t * L];
    g4_group<T, M>(v);
#pragma unroll
    for (int t = 0; t < (1 << (2 * M)); ++t)
        if (has_mid_digit(t, M)) p[(uint64_t)t * L] = v[t];
}

// Outer inverse on four axes in place, waves across the outermost axis: z
// viewed as [n_hi][4^4][L], L a multiple of 64.  A workgroup of four waves
// takes 64 consecutive columns; wave w holds digit w of the group's
// outermost axis and its lanes' 64 registers the three inner axes (row
// 64 w + t for register index t), so every load and store moves one
// contiguous 64-column segment of a row.  G4 runs on the three inner axes in
// registers (descending), then on the outermost axis through LDS in four
// sub-rounds of 16 register indices: every wave writes its 16 values, and
// wave w then takes indices 4w .. 4w+3 with all four digits.  Entries G4
// leaves unchanged are not written back.
template <typename T>
__global__ __launch_bounds__(S3_NT) void k_s3_inv4w(T* __restrict__ z, uint64_t z_bs, uint32_t n_tiles,
                                                    uint32_t tiles_per_hi, uint32_t log2L)
{
    __shared__ T S[4 * 16 * 64];
    const uint32_t tile = blockIdx.x;
    if (tile >= n_tiles) return;  // the whole workgroup
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint64_t L = 1ull << log2L;
    const uint32_t hi = tile / tiles_per_hi, j = tile - hi * tiles_per_hi;
    char* tbase = reinterpret_cast<char*>(z + (uint64_t)blockIdx.y * z_bs + (uint64_t)hi * 256 * L + (uint64_t)j * 64);
    const uint64_t row = L * sizeof(T);
    const uint32_t off = (uint32_t)lane * (uint32_t)sizeof(T);
    constexpr uint32_t SEG = 64 * sizeof(T);
    T v[64];
    {
        const char* rp = tbase + (uint64_t)w * 64 * row;
#pragma unroll
        for (int t = 0; t < 64; ++t) v[t] = buf_load<T>(row_rsrc(rp + t * row, SEG), off);
    }
    g4_group<T, 3>(v);
    // the stores' resources are built from an opaque copy of the base, so
    // that the loads' 64 resources are not kept live in scalar registers
    char* wbase = tbase;
    asm volatile("" : "+s"(wbase));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r > 0) __syncthreads();  // the previous sub-round's reads are done
#pragma unroll
        for (int k = 0; k < 16; ++k) S[(w * 16 + k) * 64 + lane] = v[16 * r + k];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * w + q;
            const int t = 16 * r + k;
            T p0 = S[(0 * 16 + k) * 64 + lane], p1 = S[(1 * 16 + k) * 64 + lane];
            T pm = S[(2 * 16 + k) * 64 + lane], pi = S[(3 * 16 + k) * 64 + lane];
            g4(p0, p1, pm, pi);
            const bool t_mid = has_mid_digit(t, 3);
            if (t_mid) buf_store<T>(row_rsrc(wbase + (uint64_t)t * row, SEG), off, p0);
            buf_store<T>(row_rsrc(wbase + (uint64_t)(64 + t) * row, SEG), off, p1);
            buf_store<T>(row_rsrc(wbase + (uint64_t)(128 + t) * row, SEG), off, pm);
            if (t_mid) buf_store<T>(row_rsrc(wbase + (uint64_t)(192 + t) * row, SEG), off, pi);
        }
    }
}

// Fused inner tile: for outer index o, the three rows r_op[o] (2^K values
// each) -> F4 on the K inner axes (ascending) in LDS -> product -> G4 on the
// inner axes (descending) -> z[o] (4^K values, contiguous).
template <typename T, int K>
struct S3Tile {
    static constexpr int N2 = 1 << K, N4 = 1 << (2 * K);
};

template <typename T, int K>
__global__ __launch_bounds__(S3_NT) void k_s3_fused(const T* __restrict__ r0, const T* __restrict__ r1,
                                                    const T* __restrict__ r2, T* __restrict__ z, uint64_t r_bs,
                                                    uint64_t z_bs, uint32_t n_tiles)
{
    using C = S3Tile<T, K>;
    __shared__ T A[C::N4];
    __shared__ T B[C::N4];
    __shared__ T P[C::N4];
    const int tid = threadIdx.x;
    const uint64_t item = blockIdx.y;
    const TileWalk w = xcd_tile_walk(n_tiles);
    constexpr int RPT = (C::N2 + S3_NT - 1) / S3_NT;  // row entries per thread
    for (uint32_t o = w.first; o < w.end; o += w.step) {
        // the three rows' loads are issued together, before any LDS work
        T rv[3][RPT];
#pragma unroll
        for (int op = 0; op < 3; ++op) {
            const T* row = (op == 0 ? r0 : (op == 1 ? r1 : r2)) + item * r_bs + (uint64_t)o * C::N2;
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int i = tid + j * S3_NT;
                rv[op][j] = i < C::N2 ? row[i] : T(0);
            }
        }
#pragma unroll
        for (int op = 0; op < 3; ++op) {
            __syncthreads();  // the previous operand's product reads of its buffer are done
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int i = tid + j * S3_NT;
                if (i < C::N2) A[i] = rv[op][j];
            }
            __syncthreads();
            T* cur = A;
            T* nxt = B;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                // [4^a][2][2^(K-a-1)] -> [4^a][4][2^(K-a-1)]
                const int lo_n = 1 << (K - a - 1);
                const int n = (1 << (2 * a)) * lo_n;
                for (int idx = tid; idx < n; idx += S3_NT) {
                    const int hi = idx / lo_n, lo = idx - hi * lo_n;
                    const T a0 = cur[(hi * 2 + 0) * lo_n + lo];
                    const T a1 = cur[(hi * 2 + 1) * lo_n + lo];
                    nxt[(hi * 4 + 0) * lo_n + lo] = a0;
                    nxt[(hi * 4 + 1) * lo_n + lo] = a0 + a1;
                    nxt[(hi * 4 + 2) * lo_n + lo] = a0 - a1;
                    nxt[(hi * 4 + 3) * lo_n + lo] = a1;
                }
                __syncthreads();
                T* t = cur;
                cur = nxt;
                nxt = t;
            }
            // each thread multiplies the entries it owns (same index set per
            // operand, so no barrier is needed between the products)
            for (int i = tid; i < C::N4; i += S3_NT) P[i] = op == 0 ? cur[i] : P[i] * cur[i];
        }
        __syncthreads();
        // G4 on the inner axes, descending, in place on P
#pragma unroll
        for (int a = K - 1; a >= 0; --a) {
            const int lo_n = 1 << (2 * (K - a - 1));
            const int n = (1 << (2 * a)) * lo_n;
            for (int idx = tid; idx < n; idx += S3_NT) {
                const int hi = idx / lo_n, lo = idx - hi * lo_n;
                T* p = P + hi * 4 * lo_n + lo;
                T p0 = p[0], p1 = p[lo_n], pm = p[2 * lo_n], pi = p[3 * lo_n];
                g4(p0, p1, pm, pi);
                p[lo_n] = p1;
                p[2 * lo_n] = pm;
            }
            __syncthreads();
        }
        T* zr = z + item * z_bs + (uint64_t)o * C::N4;
        for (int i = tid; i < C::N4; i += S3_NT) zr[i] = P[i];
    }
}

// The same tile for K >= 2 with its two innermost axes in registers: the
// forward steps on axes 0..K-3 run in LDS for the three operands together;
// then one thread per (outer digits, digit of axis K-2) reads the 2 x 2
// binary sub-cube of each operand, applies F4 on axis K-2 (its own digit)
// and K-1, multiplies the operands, applies G4 on axis K-1 and writes four
// contiguous entries; G4 on axes K-2..0 then runs in LDS.  Every entry
// sees the same operations in the same order as in the tile above.
template <typename T>
__device__ __forceinline__ T f4_at(int g, T a0, T a1)
{
    const T s = a0 + a1;
    const T d = a0 - a1;
    return (g & 2) ? ((g & 1) ? a1 : d) : ((g & 1) ? s : a0);
}

template <typename T, int K>
__global__ __launch_bounds__(S3_NT) void k_s3_fused_r(const T* __restrict__ r0, const T* __restrict__ r1,
                                                      const T* __restrict__ r2, T* __restrict__ z, uint64_t r_bs,
                                                      uint64_t z_bs, uint32_t n_tiles)
{
    static_assert(K >= 2, "two register axes");
    constexpr int N2 = 1 << K, N4 = 1 << (2 * K);
    constexpr int NS = 1 << (2 * (K - 1));  // forward state after K-2 steps: 4^(K-2) x 2 x 2
    // LDS: region X (three operands at stride NS) and region Y (4 NS); the
    // forward steps alternate between them and end in X, so that the
    // product's 4^K entries go to Y while X is read
    __shared__ T S[7 * NS];
    T* const X = S;
    T* const Y = S + 3 * NS;
    T* const P = Y;
    const int tid = threadIdx.x;
    const uint64_t item = blockIdx.y;
    const TileWalk w = xcd_tile_walk(n_tiles);
    constexpr int RPT = (N2 + S3_NT - 1) / S3_NT;
    for (uint32_t o = w.first; o < w.end; o += w.step) {
        T rv[3][RPT];
#pragma unroll
        for (int op = 0; op < 3; ++op) {
            const T* row = (op == 0 ? r0 : (op == 1 ? r1 : r2)) + item * r_bs + (uint64_t)o * N2;
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int i = tid + j * S3_NT;
                rv[op][j] = i < N2 ? row[i] : T(0);
            }
        }
        __syncthreads();  // the previous tile's reads of P are done
#pragma unroll
        for (int op = 0; op < 3; ++op)
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int i = tid + j * S3_NT;
                if (i < N2) (((K - 2) & 1) ? Y : X)[op * NS + i] = rv[op][j];
            }
        __syncthreads();
        T* cur = ((K - 2) & 1) ? Y : X;
        T* nxt = ((K - 2) & 1) ? X : Y;
#pragma unroll
        for (int a = 0; a + 2 < K; ++a) {
            // per operand [4^a][2][2^(K-a-1)] -> [4^a][4][2^(K-a-1)]
            const int lo_n = 1 << (K - a - 1);
            const int n = (1 << (2 * a)) * lo_n;
            for (int idx = tid; idx < 3 * n; idx += S3_NT) {
                const int op = idx / n, r = idx - op * n;
                const int hi = r / lo_n, lo = r - hi * lo_n;
                const T* c = cur + op * NS;
                T* d = nxt + op * NS;
                const T a0 = c[(hi * 2 + 0) * lo_n + lo];
                const T a1 = c[(hi * 2 + 1) * lo_n + lo];
                d[(hi * 4 + 0) * lo_n + lo] = a0;
                d[(hi * 4 + 1) * lo_n + lo] = a0 + a1;
                d[(hi * 4 + 2) * lo_n + lo] = a0 - a1;
                d[(hi * 4 + 3) * lo_n + lo] = a1;
            }
            __syncthreads();
            T* t = cur;
            cur = nxt;
            nxt = t;
        }
        // registers: thread (hi, g) with g the digit of axis K-2
        for (int t = tid; t < NS; t += S3_NT) {
            const int hi = t >> 2, g = t & 3;
            T prod[4];
#pragma unroll
            for (int op = 0; op < 3; ++op) {
                const T* c = cur + op * NS + hi * 4;  // [b(K-2)][b(K-1)]
                const T v0 = f4_at<T>(g, c[0], c[2]);
                const T v1 = f4_at<T>(g, c[1], c[3]);
                const T f[4] = {v0, v0 + v1, v0 - v1, v1};
#pragma unroll
                for (int e = 0; e < 4; ++e) prod[e] = op == 0 ? f[e] : prod[e] * f[e];
            }
            g4(prod[0], prod[1], prod[2], prod[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) P[t * 4 + e] = prod[e];
        }
        __syncthreads();
        // G4 on axes K-2 .. 0, in place on P
#pragma unroll
        for (int a = K - 2; a >= 0; --a) {
            const int lo_n = 1 << (2 * (K - a - 1));
            const int n = (1 << (2 * a)) * lo_n;
            for (int idx = tid; idx < n; idx += S3_NT) {
                const int hi = idx / lo_n, lo = idx - hi * lo_n;
                T* p = P + hi * 4 * lo_n + lo;
                T p0 = p[0], p1 = p[lo_n], pm = p[2 * lo_n], pi = p[3 * lo_n];
                g4(p0, p1, pm, pi);
                p[lo_n] = p1;
                p[2 * lo_n] = pm;
            }
            __syncthreads();
        }
        T* zr = z + item * z_bs + (uint64_t)o * N4;
        for (int i = tid; i < N4; i += S3_NT) zr[i] = P[i];
    }
}

// F4 on one axis of a pair of values, all four outputs
template <typename T>
__device__ __forceinline__ void f4_pair(T a0, T a1, T& o0, T& o1, T& o2, T& o3)
{
    o0 = a0;
    o1 = a0 + a1;
    o2 = a0 - a1;
    o3 = a1;
}

// F4 on two axes of a 2 x 2 block held by one thread, the outer axis first:
// x[b * 2 + b'] -> y[g * 4 + g'] (g, g' the digits of the outer, inner axis)
template <typename T>
__device__ __forceinline__ void f4_two(const T (&x)[4], T (&y)[16])
{
    T u[4][2];
#pragma unroll
    for (int b1 = 0; b1 < 2; ++b1) f4_pair(x[b1], x[2 + b1], u[0][b1], u[1][b1], u[2][b1], u[3][b1]);
#pragma unroll
    for (int g0 = 0; g0 < 4; ++g0) f4_pair(u[g0][0], u[g0][1], y[g0 * 4 + 0], y[g0 * 4 + 1], y[g0 * 4 + 2], y[g0 * 4 + 3]);
}

// G4 on two axes of 16 values held by one thread (index g * 4 + g'), the
// inner axis first
template <typename T>
__device__ __forceinline__ void g4_two(T (&q)[16])
{
#pragma unroll
    for (int g0 = 0; g0 < 4; ++g0) g4(q[g0 * 4 + 0], q[g0 * 4 + 1], q[g0 * 4 + 2], q[g0 * 4 + 3]);
#pragma unroll
    for (int g1 = 0; g1 < 4; ++g1) g4(q[0 * 4 + g1], q[1 * 4 + g1], q[2 * 4 + g1], q[3 * 4 + g1]);
}

// Fused tile of six inner axes, 256 threads, every step on two axes at once.
// Tile digits: axes 0..5 of the tile with digits g0..g5; the output row is
// z[o][b * 256 + c * 16 + a] with b = (g0, g1), c = (g2, g3), a = (g4, g5)
// (each pair as 4 g + g').  Steps, each followed by a barrier:
//   forward on axes 0, 1   48 threads (operand, binary digits of axes 2..5)
//   forward on axes 2, 3   192 threads (operand, binary axes 4, 5, b)
//   forward on axes 4, 5, the product, G4 on axes 5, 4: thread (b, c)
//   G4 on axes 3, 2:       thread (a, b), in place
//   G4 on axes 1, 0:       thread (a, c), stored to z (coalesced)
// LDS holds 4096 values: the product array P[a][b][c] at
// a * 256 + (b ^ (c & 1)) * 16 + (c ^ a), a layout in which each of the
// three access patterns above meets 32 distinct 8-byte banks per 32 lanes;
// the forward states sit in the same memory ahead of it.
template <typename T>
__global__ __launch_bounds__(S3_NT) void k_s3_tile6(const T* __restrict__ r0, const T* __restrict__ r1,
                                                    const T* __restrict__ r2, T* __restrict__ z, uint64_t r_bs,
                                                    uint64_t z_bs, uint32_t n_tiles)
{
    static_assert(S3_NT == 256, "one thread per (b, c), (a, b) and (a, c)");
    __shared__ T S[4096];
    T* const A = S;          // input rows [op][64]                        (192)
    T* const C = S;          // after axes 0..3: [op][k][g01 * 16 + (g23 ^ g01)]  (3072)
    T* const B = S + 3072;   // after axes 0, 1: [op][g01 * 16 + (lo ^ g01)]      (768)
    T* const P = S;
    const int tid = threadIdx.x;
    const uint64_t item = blockIdx.y;
    const TileWalk w = xcd_tile_walk(n_tiles);
    for (uint32_t o = w.first; o < w.end; o += w.step) {
        T in = T(0);
        if (tid < 192) {
            const int op = tid >> 6;
            const T* row = (op == 0 ? r0 : (op == 1 ? r1 : r2)) + item * r_bs + (uint64_t)o * 64;
            in = row[tid & 63];
        }
        __syncthreads();  // the previous tile's reads of P are done
        if (tid < 192) A[tid] = in;
        __syncthreads();
        if (tid < 48) {
            // F4 on axes 0, 1 for binary digits lo of axes 2..5
            const int op = tid >> 4, lo = tid & 15;
            const T* a = A + op * 64;
            const T x[4] = {a[lo], a[16 + lo], a[32 + lo], a[48 + lo]};
            T y[16];
            f4_two(x, y);
            T* b = B + op * 256;
#pragma unroll
            for (int g01 = 0; g01 < 16; ++g01) b[g01 * 16 + (lo ^ g01)] = y[g01];
        }
        __syncthreads();
        if (tid < 192) {
            // F4 on axes 2, 3 for (b = g01, binary digits k of axes 4, 5)
            const int op = tid >> 6, k = (tid >> 4) & 3, g01 = tid & 15;
            const T* b = B + op * 256 + g01 * 16;
            const T x[4] = {b[(0 + k) ^ g01], b[(4 + k) ^ g01], b[(8 + k) ^ g01], b[(12 + k) ^ g01]};
            T y[16];
            f4_two(x, y);
            T* c = C + op * 1024 + k * 256 + g01 * 16;
#pragma unroll
            for (int e = 0; e < 16; ++e) c[e ^ g01] = y[e];
        }
        __syncthreads();
        {
            // thread (b, c): F4 on axes 4, 5, the product, G4 on axes 5, 4
            const int bb = tid >> 4, cc = tid & 15;
            T x[3][4];
#pragma unroll
            for (int op = 0; op < 3; ++op)
#pragma unroll
                for (int k = 0; k < 4; ++k) x[op][k] = C[op * 1024 + k * 256 + bb * 16 + (cc ^ bb)];
            __syncthreads();  // P overwrites C
            T prod[16];
            f4_two(x[0], prod);
#pragma unroll
            for (int op = 1; op < 3; ++op) {
                T f[16];
                f4_two(x[op], f);
#pragma unroll
                for (int e = 0; e < 16; ++e) prod[e] = prod[e] * f[e];
            }
            g4_two(prod);
#pragma unroll
            for (int aa = 0; aa < 16; ++aa) P[aa * 256 + (bb ^ (cc & 1)) * 16 + (cc ^ aa)] = prod[aa];
        }
        __syncthreads();
        {
            // thread (a, b): G4 on axes 3, 2
            const int aa = tid & 15, bb = tid >> 4;
            T q[16];
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) q[cc] = P[aa * 256 + (bb ^ (cc & 1)) * 16 + (cc ^ aa)];
            g4_two(q);
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                if (has_mid_digit(cc, 2)) P[aa * 256 + (bb ^ (cc & 1)) * 16 + (cc ^ aa)] = q[cc];
        }
        __syncthreads();
        {
            // thread (a, c): G4 on axes 1, 0 and the stores
            const int aa = tid & 15, cc = tid >> 4;
            T q[16];
#pragma unroll
            for (int bb = 0; bb < 16; ++bb) q[bb] = P[aa * 256 + (bb ^ (cc & 1)) * 16 + (cc ^ aa)];
            g4_two(q);
            T* zr = z + item * z_bs + (uint64_t)o * 4096 + tid;
#pragma unroll
            for (int bb = 0; bb < 16; ++bb) zr[bb * 256] = q[bb];
        }
    }
}

// Inner axes per fused tile (k_s3_tile6 for six; fewer only when D < 6)
int fused_depth(int D) { return D < 6 ? D : 6; }

struct S3Plan {
    int D = 0, K = 0, p = 0;
    uint64_t n2 = 0, n4 = 0;
    uint64_t stage = 0;  // elements of one forward staging buffer per operand and item
    std::vector<int> groups;      // forward: outer axes per group, ascending from axis 0
    std::vector<int> inv_groups;  // inverse: p mod 4 axes first, then groups of 4
};

S3Plan make_s3_plan(int D, size_t es)
{
    S3Plan P;
    P.D = D;
    P.K = fused_depth(D);
    P.p = D - P.K;
    P.n2 = 1ull << D;
    P.n4 = 1ull << (2 * D);
    for (int left = P.p; left > 0;) {
        const int m = left < S3_GROUP ? left : S3_GROUP;
        P.groups.push_back(m);
        left -= m;
    }
    if (P.p % 4) P.inv_groups.push_back(P.p % 4);
    for (int i = 0; i < P.p / 4; ++i) P.inv_groups.push_back(4);
    // intermediate after a outer axes: 4^a 2^(D-a) = 2^(D+a) elements
    P.stage = P.p > 0 ? (1ull << (D + P.p)) : 0;
    return P;
}

size_t s3_ws_bytes(const S3Plan& P, int batch, size_t es) { return (size_t)batch * 6 * P.stage * es; }

template <typename T, int M>
void launch_fwd(const T* i0, const T* i1, const T* i2, T* o0, T* o1, T* o2, uint64_t in_bs, uint64_t out_bs,
                uint64_t n_cols, uint32_t log2L, int batch, hipStream_t s)
{
    dim3 grid((uint32_t)((n_cols + S3_NT - 1) / S3_NT), batch, 3);
    LaunchScope scope(s, 3.0 * batch * n_cols * ((1 << M) + (1 << (2 * M))) * sizeof(T), "s3_fwd<%s,M=%d>",
                      tname<T>(), M);
    k_s3_fwd<T, M><<<grid, S3_NT, 0, s>>>(i0, i1, i2, o0, o1, o2, in_bs, out_bs, n_cols, log2L);
}

template <typename T, int M>
void launch_inv(T* z, uint64_t z_bs, uint64_t n_cols, uint32_t log2L, int batch, hipStream_t s)
{
    dim3 grid((uint32_t)((n_cols + S3_NT - 1) / S3_NT), batch, 1);
    const double T4 = 1 << (2 * M), T2 = 1 << M;
    LaunchScope scope(s, (double)batch * n_cols * (T4 + T4 - T2) * sizeof(T), "s3_inv<%s,M=%d>", tname<T>(), M);
    k_s3_inv<T, M><<<grid, S3_NT, 0, s>>>(z, z_bs, n_cols, log2L);
}

template <typename T>
void launch_inv4(T* z, uint64_t z_bs, uint64_t n_cols, uint32_t log2L, int batch, hipStream_t s)
{
    const uint32_t tiles_per_hi = (uint32_t)((1ull << log2L) / 64);
    const uint32_t n_tiles = (uint32_t)(n_cols / 64);
    dim3 grid(n_tiles, batch, 1);
    LaunchScope scope(s, (double)batch * n_cols * (256.0 + 240.0) * sizeof(T), "s3_inv<%s,M=4>", tname<T>());
    k_s3_inv4w<T><<<grid, S3_NT, 0, s>>>(z, z_bs, n_tiles, tiles_per_hi, log2L);
}

template <typename T, int K>
void launch_fused(const T* r0, const T* r1, const T* r2, T* z, uint64_t r_bs, uint64_t z_bs, uint32_t n_tiles,
                  int batch, int cus, hipStream_t s)
{
    dim3 grid(tile_grid(n_tiles, cus, 0), batch, 1);
    LaunchScope scope(s, (double)batch * n_tiles * (3.0 * (1 << K) + (1 << (2 * K))) * sizeof(T),
                      "s3_fused<%s,K=%d>", tname<T>(), K);
    if constexpr (K == 6)
        k_s3_tile6<T><<<grid, S3_NT, 0, s>>>(r0, r1, r2, z, r_bs, z_bs, n_tiles);
    else if constexpr (K >= 2)
        k_s3_fused_r<T, K><<<grid, S3_NT, 0, s>>>(r0, r1, r2, z, r_bs, z_bs, n_tiles);
    else
        k_s3_fused<T, K><<<grid, S3_NT, 0, s>>>(r0, r1, r2, z, r_bs, z_bs, n_tiles);
}

template <typename T>
int run_s3(const S3Plan& P, const T* x1, const T* x2, const T* x3, T* z, int batch, T* ws, int cus, hipStream_t s)
{
    const int D = P.D;
    const T* c0 = x1;
    const T* c1 = x2;
    const T* c2 = x3;
    uint64_t c_bs = P.n2;
    int a = 0;
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const int M = P.groups[gi];
        T* base = ws + (gi & 1) * 3 * (uint64_t)batch * P.stage;
        T* o0 = base;
        T* o1 = base + (uint64_t)batch * P.stage;
        T* o2 = base + 2 * (uint64_t)batch * P.stage;
        const uint32_t log2L = (uint32_t)(D - a - M);
        const uint64_t n_cols = (1ull << (2 * a)) << log2L;
        switch (M) {
            case 1: launch_fwd<T, 1>(c0, c1, c2, o0, o1, o2, c_bs, P.stage, n_cols, log2L, batch, s); break;
            case 2: launch_fwd<T, 2>(c0, c1, c2, o0, o1, o2, c_bs, P.stage, n_cols, log2L, batch, s); break;
            default: launch_fwd<T, 3>(c0, c1, c2, o0, o1, o2, c_bs, P.stage, n_cols, log2L, batch, s); break;
        }
        c0 = o0;
        c1 = o1;
        c2 = o2;
        c_bs = P.stage;
        a += M;
    }
    const uint32_t n_tiles = (uint32_t)(1ull << (2 * P.p));
    switch (P.K) {
        case 0: launch_fused<T, 0>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        case 1: launch_fused<T, 1>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        case 2: launch_fused<T, 2>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        case 3: launch_fused<T, 3>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        case 4: launch_fused<T, 4>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        case 5: launch_fused<T, 5>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        case 6: launch_fused<T, 6>(c0, c1, c2, z, c_bs, P.n4, n_tiles, batch, cus, s); break;
        default: return fail(HC_ERR_UNSUPPORTED, "no three-operand tile of %d axes", P.K);
    }
    // outer inverse: groups descending from the innermost outer axis
    int top = P.p;
    for (int gi = (int)P.inv_groups.size() - 1; gi >= 0; --gi) {
        const int M = P.inv_groups[gi];
        const int a0 = top - M;
        const uint32_t log2L = (uint32_t)(2 * (D - top));
        const uint64_t n_cols = (1ull << (2 * a0)) << log2L;
        switch (M) {
            case 1: launch_inv<T, 1>(z, P.n4, n_cols, log2L, batch, s); break;
            case 2: launch_inv<T, 2>(z, P.n4, n_cols, log2L, batch, s); break;
            case 3: launch_inv<T, 3>(z, P.n4, n_cols, log2L, batch, s); break;
            default: launch_inv4<T>(z, P.n4, n_cols, log2L, batch, s); break;
        }
        top = a0;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return HC_OK;
}

}  // namespace
}  // namespace hc

using namespace hc;

extern "C" {

size_t hc_sum3_workspace_bytes(int D, int dtype, int batch)
{
    const size_t es = dtype_size(dtype);
    if (D < 0 || D > S3_MAX_D || es == 0 || batch < 1 || batch > 65535) return (size_t)-1;
    return s3_ws_bytes(make_s3_plan(D, es), batch, es);
}

int hc_sum3_batch(const void* x1, const void* x2, const void* x3, void* z, int D, int dtype, int batch,
                  void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_sum3_batch D=%d dtype=%d batch=%d", D, dtype, batch);
    if (!x1 || !x2 || !x3 || !z) return fail(HC_ERR_INVALID_ARG, "x1, x2, x3 and z must be non-null");
    if (D < 0 || D > S3_MAX_D) return fail(HC_ERR_D_RANGE, "D=%d outside [0, %d]", D, S3_MAX_D);
    const size_t es = dtype_size(dtype);
    if (es == 0) return fail(HC_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (batch < 1 || batch > 65535) return fail(HC_ERR_INVALID_ARG, "batch=%d outside [1, 65535]", batch);
    if (misaligned(x1, es) || misaligned(x2, es) || misaligned(x3, es) || misaligned(z, es) ||
        misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const S3Plan P = make_s3_plan(D, es);
    const size_t in_b = (size_t)batch * P.n2 * es, out_b = (size_t)batch * P.n4 * es;
    if (ranges_overlap(z, out_b, x1, in_b) || ranges_overlap(z, out_b, x2, in_b) ||
        ranges_overlap(z, out_b, x3, in_b))
        return fail(HC_ERR_ALIAS, "z overlaps an input");
    const size_t need = s3_ws_bytes(P, batch, es);
    if (need > 0) {
        if (!workspace || workspace_bytes < need)
            return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                        workspace ? workspace_bytes : (size_t)0);
        if (ranges_overlap(workspace, need, z, out_b) || ranges_overlap(workspace, need, x1, in_b) ||
            ranges_overlap(workspace, need, x2, in_b) || ranges_overlap(workspace, need, x3, in_b))
            return fail(HC_ERR_ALIAS, "workspace overlaps a data buffer");
    }
    int cus = 0;
    const int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    switch (dtype) {
        case HC_F64:
            return run_s3<double>(P, (const double*)x1, (const double*)x2, (const double*)x3, (double*)z, batch,
                                  (double*)workspace, cus, stream);
        case HC_F32:
            return run_s3<float>(P, (const float*)x1, (const float*)x2, (const float*)x3, (float*)z, batch,
                                 (float*)workspace, cus, stream);
        default:
            return run_s3<uint64_t>(P, (const uint64_t*)x1, (const uint64_t*)x2, (const uint64_t*)x3, (uint64_t*)z,
                                    batch, (uint64_t*)workspace, cus, stream);
    }
}

}  // extern "C"
