// Convolution of two ternary cubes {0,1,2}^D x {0,1,2}^D -> {0,...,4}^D, the
// next link of a chain of sums (Introduction: sums of multiple probability
// mass functions whose axes are Bernoulli variables): with A = X1 + X2 and
// B = X3 + X4 (each a hypercube convolution), A * B is the distribution of
// X1 + X2 + X3 + X4.
//
// The Methods section's Karatsuba identity, taken to lines of three: along
// one axis each operand is a quadratic a0 + a1 t + a2 t^2, and their product
// c0 + ... + c4 t^4 needs six products and no division:
//   forward  T: (a0, a1, a2) -> (a0, a1, a2, a0 + a1, a1 + a2, a0 + a2)
//                                                          axes 0..D-1
//   product  a^ * b^                                       elementwise
//   inverse  U: (p0, p1, p2, q01, q12, q02) -> (p0, (q01 - p0) - p1,
//            ((q02 - p0) - p2) + p1, (q12 - p1) - p2, p2)  axes D-1..0
// on 6^D values per operand.  Every floating-point operation is one IEEE
// operation in this order, so results are bitwise independent of tiling;
// int64 data wraps modulo 2^64 (exact: no division).
//
// Layout: a, b hold 3^D values (ternary digit d of the flat index, weight
// 3^d, is the coordinate on axis D-1-d: the layout of the hypercube
// convolution's output); z holds 5^D values, base-5 digit d = axis D-1-d.
//
// GPU schedule (K = min(D, 4) inner axes, p = D - K outer axes):
//   outer forward   T on the outer axes, ascending, both operands, in
//                   groups of at most 2:
//                   [6^a][3^M][L] -> [6^a][6^M][L]             (k_tn_fwd)
//   fused inner     per outer index o: T on the K inner axes of the two
//                   rows, the product, U on the inner axes, a contiguous
//                   5^K row of [6^p][5^K]; K = 4 two axes at a time in
//                   registers, seven tiles per workgroup       (k_tn_tile4)
//                   (D < 4: one all-LDS tile of D axes          k_tn_fused)
//   outer inverse   U on the outer axes, descending, out of place:
//                   [6^a][6^M][L] -> [6^a][5^M][L], the last pass into z;
//                   groups of 3 with the outermost axis across waves
//                   (k_tn_inv3w), then p mod 3 axes in registers (k_tn_inv)
#include "hc.h"

#include <hip/hip_runtime.h>

#include <vector>

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int TN_MAX_D = 12;
constexpr int TN_K = 4;
constexpr int TN_GROUP = 2;
constexpr int TN_NT = 256;

__host__ __device__ constexpr uint64_t powc(uint64_t b, int n) { return n == 0 ? 1 : b * powc(b, n - 1); }

// T on M axes of one line held by one thread: s[0 .. 3^M) in, s[0 .. 6^M)
// out, the group's first axis first.
template <typename T, int M>
__device__ __forceinline__ void t_group(T (&s)[powc(6, M)])
{
#pragma unroll
    for (int j = 0; j < M; ++j) {
        // [6^j][3][3^(M-j-1)] -> [6^j][6][3^(M-j-1)], rewritten from the top
        // down so that no entry is overwritten before it is read
        const int lo_n = (int)powc(3, M - j - 1);
        const int hi_n = (int)powc(6, j);
#pragma unroll
        for (int hi = hi_n - 1; hi >= 0; --hi)
#pragma unroll
            for (int lo = lo_n - 1; lo >= 0; --lo) {
                const T a0 = s[(hi * 3 + 0) * lo_n + lo];
                const T a1 = s[(hi * 3 + 1) * lo_n + lo];
                const T a2 = s[(hi * 3 + 2) * lo_n + lo];
                s[(hi * 6 + 5) * lo_n + lo] = a0 + a2;
                s[(hi * 6 + 4) * lo_n + lo] = a1 + a2;
                s[(hi * 6 + 3) * lo_n + lo] = a0 + a1;
                s[(hi * 6 + 2) * lo_n + lo] = a2;
                s[(hi * 6 + 1) * lo_n + lo] = a1;
                s[(hi * 6 + 0) * lo_n + lo] = a0;
            }
    }
}

// U on one line of six values, written as five
template <typename T>
__device__ __forceinline__ void u_line(const T& p0, const T& p1, const T& p2, const T& q01, const T& q12,
                                       const T& q02, T& c0, T& c1, T& c2, T& c3, T& c4)
{
    c0 = p0;
    c1 = (q01 - p0) - p1;
    c2 = ((q02 - p0) - p2) + p1;
    c3 = (q12 - p1) - p2;
    c4 = p2;
}

// U on M axes of one line held by one thread: s[0 .. 6^M) in, s[0 .. 5^M)
// out, the group's last axis first.
template <typename T, int M>
__device__ __forceinline__ void u_group(T (&s)[powc(6, M)])
{
#pragma unroll
    for (int j = M - 1; j >= 0; --j) {
        // [6^j][6][5^(M-j-1)] -> [6^j][5][5^(M-j-1)], rewritten from the
        // bottom up (every output index is at most its inputs' indices)
        const int lo_n = (int)powc(5, M - j - 1);
        const int hi_n = (int)powc(6, j);
#pragma unroll
        for (int hi = 0; hi < hi_n; ++hi)
#pragma unroll
            for (int lo = 0; lo < lo_n; ++lo) {
                const T* p = s + hi * 6 * lo_n + lo;
                T c0, c1, c2, c3, c4;
                u_line(p[0], p[lo_n], p[2 * lo_n], p[3 * lo_n], p[4 * lo_n], p[5 * lo_n], c0, c1, c2, c3, c4);
                T* c = s + hi * 5 * lo_n + lo;
                c[0] = c0;
                c[lo_n] = c1;
                c[2 * lo_n] = c2;
                c[3 * lo_n] = c3;
                c[4 * lo_n] = c4;
            }
    }
}

// Outer forward: T on M axes for both operands (blockIdx.z), out of place;
// in [n_hi][3^M][L] -> out [n_hi][6^M][L]; one thread per column.
template <typename T, int M>
__global__ __launch_bounds__(TN_NT) void k_tn_fwd(const T* __restrict__ in0, const T* __restrict__ in1,
                                                  T* __restrict__ out0, T* __restrict__ out1, uint64_t in_bs,
                                                  uint64_t out_bs, uint64_t n_cols, uint64_t L)
{
    const TileWalk wk = xcd_tile_walk((uint32_t)((n_cols + TN_NT - 1) / TN_NT));
    if (wk.first >= wk.end) return;
    const uint64_t c = (uint64_t)wk.first * TN_NT + threadIdx.x;
    if (c >= n_cols) return;
    const T* in = (blockIdx.z == 0 ? in0 : in1) + (uint64_t)blockIdx.y * in_bs;
    T* out = (blockIdx.z == 0 ? out0 : out1) + (uint64_t)blockIdx.y * out_bs;
    const uint64_t hi = c / L, lo = c - hi * L;
    const T* src = in + hi * powc(3, M) * L + lo;
    T* dst = out + hi * powc(6, M) * L + lo;
    T s[powc(6, M)];
#pragma unroll
    for (int t = 0; t < (int)powc(3, M); ++t) s[t] = src[(uint64_t)t * L];
    t_group<T, M>(s);
#pragma unroll
    for (int t = 0; t < (int)powc(6, M); ++t) dst[(uint64_t)t * L] = s[t];
}

// Outer inverse: U on M axes, out of place; in [n_hi][6^M][L] -> out
// [n_hi][5^M][L]; one thread per column.
template <typename T, int M>
__global__ __launch_bounds__(TN_NT) void k_tn_inv(const T* __restrict__ in, T* __restrict__ out, uint64_t in_bs,
                                                  uint64_t out_bs, uint64_t n_cols, uint64_t L)
{
    const TileWalk wk = xcd_tile_walk((uint32_t)((n_cols + TN_NT - 1) / TN_NT));
    if (wk.first >= wk.end) return;
    const uint64_t c = (uint64_t)wk.first * TN_NT + threadIdx.x;
    if (c >= n_cols) return;
    in += (uint64_t)blockIdx.y * in_bs;
    out += (uint64_t)blockIdx.y * out_bs;
    const uint64_t hi = c / L, lo = c - hi * L;
    const T* src = in + hi * powc(6, M) * L + lo;
    T* dst = out + hi * powc(5, M) * L + lo;
    T s[powc(6, M)];
#pragma unroll
    for (int t = 0; t < (int)powc(6, M); ++t) s[t] = src[(uint64_t)t * L];
    u_group<T, M>(s);
#pragma unroll
    for (int t = 0; t < (int)powc(5, M); ++t) dst[(uint64_t)t * L] = s[t];
}

// Fused inner tile: for outer index o, the rows a[o], b[o] (3^K values
// each) -> T on the K inner axes (ascending) in LDS -> product -> U on the
// inner axes (descending) -> y[o] (5^K values, contiguous).  LDS: two
// buffers of 6^K values per operand.
template <typename T, int K>
__global__ __launch_bounds__(TN_NT) void k_tn_fused(const T* __restrict__ a, const T* __restrict__ b,
                                                    T* __restrict__ y, uint64_t in_bs, uint64_t y_bs,
                                                    uint32_t n_tiles)
{
    constexpr int N3 = (int)powc(3, K), N5 = (int)powc(5, K), N6 = (int)powc(6, K);
    __shared__ T S[4 * N6];
    const int tid = threadIdx.x;
    const uint64_t item = blockIdx.y;
    const TileWalk w = xcd_tile_walk(n_tiles);
    for (uint32_t o = w.first; o < w.end; o += w.step) {
        __syncthreads();  // the previous tile's reads of S are done
        const T* ar = a + item * in_bs + (uint64_t)o * N3;
        const T* br = b + item * in_bs + (uint64_t)o * N3;
        for (int i = tid; i < N3; i += TN_NT) {
            S[i] = ar[i];
            S[2 * N6 + i] = br[i];
        }
        __syncthreads();
        int cur = 0;  // operand op's current buffer: S + (2 op + cur) N6
#pragma unroll
        for (int j = 0; j < K; ++j) {
            // per operand [6^j][3][3^(K-j-1)] -> [6^j][6][3^(K-j-1)]
            const int lo_n = (int)powc(3, K - j - 1);
            const int n = (int)powc(6, j) * lo_n;
            for (int idx = tid; idx < 2 * n; idx += TN_NT) {
                const int op = idx / n, r = idx - op * n;
                const int hi = r / lo_n, lo = r - hi * lo_n;
                const T* src = S + (2 * op + cur) * N6;
                T* dst = S + (2 * op + (cur ^ 1)) * N6;
                const T a0 = src[(hi * 3 + 0) * lo_n + lo];
                const T a1 = src[(hi * 3 + 1) * lo_n + lo];
                const T a2 = src[(hi * 3 + 2) * lo_n + lo];
                dst[(hi * 6 + 0) * lo_n + lo] = a0;
                dst[(hi * 6 + 1) * lo_n + lo] = a1;
                dst[(hi * 6 + 2) * lo_n + lo] = a2;
                dst[(hi * 6 + 3) * lo_n + lo] = a0 + a1;
                dst[(hi * 6 + 4) * lo_n + lo] = a1 + a2;
                dst[(hi * 6 + 5) * lo_n + lo] = a0 + a2;
            }
            __syncthreads();
            cur ^= 1;
        }
        // the product, into operand 0's current buffer
        {
            T* pa = S + cur * N6;
            const T* pb = S + (2 + cur) * N6;
            for (int i = tid; i < N6; i += TN_NT) pa[i] = pa[i] * pb[i];
        }
        __syncthreads();
        // U on the inner axes, descending, between operand 0's two buffers
#pragma unroll
        for (int j = K - 1; j >= 0; --j) {
            // [6^j][6][5^(K-j-1)] -> [6^j][5][5^(K-j-1)]
            const int lo_n = (int)powc(5, K - j - 1);
            const int n = (int)powc(6, j) * lo_n;
            const T* src = S + cur * N6;
            T* dst = S + (cur ^ 1) * N6;
            for (int idx = tid; idx < n; idx += TN_NT) {
                const int hi = idx / lo_n, lo = idx - hi * lo_n;
                const T* p = src + hi * 6 * lo_n + lo;
                T* c = dst + hi * 5 * lo_n + lo;
                T c0, c1, c2, c3, c4;
                u_line(p[0], p[lo_n], p[2 * lo_n], p[3 * lo_n], p[4 * lo_n], p[5 * lo_n], c0, c1, c2, c3, c4);
                c[0] = c0;
                c[lo_n] = c1;
                c[2 * lo_n] = c2;
                c[3 * lo_n] = c3;
                c[4 * lo_n] = c4;
            }
            __syncthreads();
            cur ^= 1;
        }
        const T* res = S + cur * N6;
        T* yr = y + item * y_bs + (uint64_t)o * N5;
        for (int i = tid; i < N5; i += TN_NT) yr[i] = res[i];
    }
}

// T on two axes of a 3 x 3 block held by one thread, the outer axis first:
// x[b * 3 + b'] -> y[g * 6 + g']
template <typename T>
__device__ __forceinline__ void t_two(const T (&x)[9], T (&y)[36])
{
    T u[6][3];
#pragma unroll
    for (int b1 = 0; b1 < 3; ++b1) {
        const T a0 = x[b1], a1 = x[3 + b1], a2 = x[6 + b1];
        u[0][b1] = a0;
        u[1][b1] = a1;
        u[2][b1] = a2;
        u[3][b1] = a0 + a1;
        u[4][b1] = a1 + a2;
        u[5][b1] = a0 + a2;
    }
#pragma unroll
    for (int g0 = 0; g0 < 6; ++g0) {
        const T a0 = u[g0][0], a1 = u[g0][1], a2 = u[g0][2];
        y[g0 * 6 + 0] = a0;
        y[g0 * 6 + 1] = a1;
        y[g0 * 6 + 2] = a2;
        y[g0 * 6 + 3] = a0 + a1;
        y[g0 * 6 + 4] = a1 + a2;
        y[g0 * 6 + 5] = a0 + a2;
    }
}

// U on two axes of a 6 x 6 block held by one thread, the inner axis first:
// p[g * 6 + g'] -> c[k * 5 + k']
template <typename T>
__device__ __forceinline__ void u_two(const T (&p)[36], T (&c)[25])
{
    T v[6][5];
#pragma unroll
    for (int g0 = 0; g0 < 6; ++g0)
        u_line(p[g0 * 6 + 0], p[g0 * 6 + 1], p[g0 * 6 + 2], p[g0 * 6 + 3], p[g0 * 6 + 4], p[g0 * 6 + 5], v[g0][0],
               v[g0][1], v[g0][2], v[g0][3], v[g0][4]);
#pragma unroll
    for (int k1 = 0; k1 < 5; ++k1)
        u_line(v[0][k1], v[1][k1], v[2][k1], v[3][k1], v[4][k1], v[5][k1], c[0 * 5 + k1], c[1 * 5 + k1],
               c[2 * 5 + k1], c[3 * 5 + k1], c[4 * 5 + k1]);
}

// Outer inverse on three axes, out of place, with the group's outermost
// axis across the workgroup's six waves: in [n_hi][6^3][L] -> out
// [n_hi][5^3][L].  A workgroup takes 64 consecutive columns (lanes past L
// take part in the barrier only); wave w holds digit w of the outermost axis
// and its lanes' 36 registers the two inner axes (row 36 w + t).  U runs on
// the two inner axes in registers (36 -> 25 values), then on the outermost
// axis through LDS in five sub-rounds of five register indices: every wave
// writes its five values, and wave w < 5 then takes index k = 5 r + w with
// all six digits and stores rows 25 c + k.
constexpr int TN_INV3_NT = 384;

template <typename T>
__global__ __launch_bounds__(TN_INV3_NT) void k_tn_inv3w(const T* __restrict__ in, T* __restrict__ out,
                                                         uint64_t in_bs, uint64_t out_bs, uint64_t L,
                                                         uint32_t tiles_per_hi, uint32_t n_tiles)
{
    __shared__ T S[6 * 5 * 64];
    const TileWalk wk = xcd_tile_walk(n_tiles);
    if (wk.first >= wk.end) return;  // the whole workgroup
    const uint32_t tile = wk.first;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t hi = tile / tiles_per_hi, j = tile - hi * tiles_per_hi;
    const uint64_t col = (uint64_t)j * 64 + lane;
    const bool act = col < L;
    const T* src = in + (uint64_t)blockIdx.y * in_bs + (uint64_t)hi * 216 * L + col;
    T* dst = out + (uint64_t)blockIdx.y * out_bs + (uint64_t)hi * 125 * L + col;
    T v[36];
#pragma unroll
    for (int t = 0; t < 36; ++t) v[t] = act ? src[(uint64_t)(w * 36 + t) * L] : T(0);
    T c[25];
    u_two(v, c);
    // five sub-rounds of five register indices: every wave writes its five
    // values, then wave w < 5 takes index 5 r + w with all six digits
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        if (r > 0) __syncthreads();  // the previous sub-round's reads are done
#pragma unroll
        for (int i = 0; i < 5; ++i) S[(w * 5 + i) * 64 + lane] = c[5 * r + i];
        __syncthreads();
        if (w < 5) {
            const int k = 5 * r + w;
            T r0, r1, r2, r3, r4;
            u_line(S[(0 * 5 + w) * 64 + lane], S[(1 * 5 + w) * 64 + lane], S[(2 * 5 + w) * 64 + lane],
                   S[(3 * 5 + w) * 64 + lane], S[(4 * 5 + w) * 64 + lane], S[(5 * 5 + w) * 64 + lane], r0, r1, r2,
                   r3, r4);
            if (act) {
                dst[(uint64_t)(0 * 25 + k) * L] = r0;
                dst[(uint64_t)(1 * 25 + k) * L] = r1;
                dst[(uint64_t)(2 * 25 + k) * L] = r2;
                dst[(uint64_t)(3 * 25 + k) * L] = r3;
                dst[(uint64_t)(4 * 25 + k) * L] = r4;
            }
        }
    }
}

// The fused tile for K = 4, every step on two axes held in one thread's
// registers; a workgroup takes TN_TPB tiles at once (36 threads each).
// Tile digits: axes 0..3 with ternary digits b0..b3 (inputs) and six-slot
// digits g0..g3; per tile, in LDS:
//   load     both 81-entry rows                                  -> IN
//   F01      18 threads (operand, b2 b3): T on axes 0, 1          -> F[op][g0 g1][b2 b3]
//   main     36 threads (g0 g1): T on axes 2, 3 for both operands,
//            the product, U on axes 3, 2                         -> P[g0 g1][c2 c3]
//   U01      25 threads (c2 c3): U on axes 1, 0, stored to z (a 25-entry
//            run per output digit pair c0 c1)
// P takes the memory of IN and F (after a barrier).  A group's rows are
// loaded into registers, every load in flight at once, and stored to LDS
// after the barrier; when a workgroup runs several groups, the next group's
// loads are issued while the current group computes.
constexpr int TN_TPB = 7;
constexpr int TN_TILE_LDS = 900;  // 36 x 25 (P) >= 162 (IN) + 648 (F)

// Held to three waves per SIMD (three workgroups per CU, as the 50 KB of LDS
// allow): the row registers cost a few spills in 8-byte types, which
// measured faster than two workgroups per CU.
template <typename T>
__global__ __launch_bounds__(TN_NT) __attribute__((amdgpu_waves_per_eu(3))) void k_tn_tile4(const T* __restrict__ a, const T* __restrict__ b,
                                                    T* __restrict__ y, uint64_t in_bs, uint64_t y_bs,
                                                    uint32_t n_tiles)
{
    static_assert(TN_TPB * 36 <= TN_NT, "36 threads per tile");
    __shared__ T S[TN_TPB * TN_TILE_LDS];
    const int tid = threadIdx.x;
    const int ts = tid / 36, l = tid - ts * 36;  // tile slot, thread within the tile
    const uint64_t item = blockIdx.y;
    const uint32_t n_groups = (n_tiles + TN_TPB - 1) / TN_TPB;
    const TileWalk w = xcd_tile_walk(n_groups);
    const T* ai = a + item * in_bs;
    const T* bi = b + item * in_bs;
    T* yi = y + item * y_bs;
    // a group's rows in registers (LPT per thread)
    constexpr int LPT = (TN_TPB * 162 + TN_NT - 1) / TN_NT;
    T pre[LPT];
    auto load_group = [&](uint32_t o0) {
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int idx = tid + j * TN_NT;
            T v = T(0);
            if (idx < TN_TPB * 162) {
                const int slot = idx / 162, r = idx - slot * 162;
                const int op = r / 81, i = r - op * 81;
                const uint32_t o = o0 + slot;
                if (o < n_tiles) v = (op ? bi : ai)[(uint64_t)o * 81 + i];
            }
            pre[j] = v;
        }
    };
    if (w.first < w.end) load_group(w.first * TN_TPB);
    for (uint32_t grp = w.first; grp < w.end; grp += w.step) {
        const uint32_t o0 = grp * TN_TPB;
        __syncthreads();  // the previous group's reads of S are done
        // IN[slot][op][81] from the registers, then the next group's loads
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int idx = tid + j * TN_NT;
            if (idx < TN_TPB * 162) {
                const int slot = idx / 162, r = idx - slot * 162;
                S[slot * TN_TILE_LDS + r] = pre[j];
            }
        }
        if (grp + w.step < w.end) load_group((grp + w.step) * TN_TPB);
        __syncthreads();
        T* tile = S + (ts < TN_TPB ? ts : 0) * TN_TILE_LDS;
        if (ts < TN_TPB && l < 18) {
            const int op = l / 9, lo = l - op * 9;
            const T* in = tile + op * 81;
            T x[9];
#pragma unroll
            for (int bb = 0; bb < 9; ++bb) x[bb] = in[bb * 9 + lo];
            T yv[36];
            t_two(x, yv);
            T* f = tile + 162 + op * 324;
#pragma unroll
            for (int g = 0; g < 36; ++g) f[g * 9 + lo] = yv[g];
        }
        __syncthreads();
        T res[25];
        if (ts < TN_TPB) {
            const int g01 = l;
            T xa[9], xb[9];
#pragma unroll
            for (int bb = 0; bb < 9; ++bb) {
                xa[bb] = tile[162 + g01 * 9 + bb];
                xb[bb] = tile[162 + 324 + g01 * 9 + bb];
            }
            T fa[36], fb[36];
            t_two(xa, fa);
            t_two(xb, fb);
#pragma unroll
            for (int g = 0; g < 36; ++g) fa[g] = fa[g] * fb[g];
            u_two(fa, res);
        }
        __syncthreads();  // P overwrites IN and F
        if (ts < TN_TPB) {
#pragma unroll
            for (int c = 0; c < 25; ++c) tile[l * 25 + c] = res[c];
        }
        __syncthreads();
        if (ts < TN_TPB && l < 25 && o0 + ts < n_tiles) {
            const int c23 = l;
            T pv[36];
#pragma unroll
            for (int g = 0; g < 36; ++g) pv[g] = tile[g * 25 + c23];
            T cv[25];
            u_two(pv, cv);
            T* zr = yi + (uint64_t)(o0 + ts) * 625 + c23;
#pragma unroll
            for (int c = 0; c < 25; ++c) zr[c * 25] = cv[c];
        }
    }
}

struct TnPlan {
    int D = 0, K = 0, p = 0;
    uint64_t n3 = 0, n5 = 0;
    uint64_t fwd_stage = 0;  // 6^p 3^K: elements of a forward staging buffer per operand and item
    uint64_t inv_stage = 0;  // 6^p 5^K: elements of an inverse staging buffer per item
    std::vector<int> groups;      // forward: outer axes per group (at most 2), ascending from axis 0
    std::vector<int> inv_groups;  // inverse: p mod 3 axes first, then groups of 3
};

TnPlan make_tn_plan(int D)
{
    TnPlan P;
    P.D = D;
    P.K = D < TN_K ? D : TN_K;
    P.p = D - P.K;
    P.n3 = powc(3, D);
    P.n5 = powc(5, D);
    for (int left = P.p; left > 0;) {
        const int m = left < TN_GROUP ? left : TN_GROUP;
        P.groups.push_back(m);
        left -= m;
    }
    if (P.p % 3) P.inv_groups.push_back(P.p % 3);
    for (int i = 0; i < P.p / 3; ++i) P.inv_groups.push_back(3);
    P.fwd_stage = P.p > 0 ? powc(6, P.p) * powc(3, P.K) : 0;
    P.inv_stage = P.p > 0 ? powc(6, P.p) * powc(5, P.K) : 0;
    return P;
}

// four forward staging buffers (two per operand) and two inverse ones
size_t tn_ws_bytes(const TnPlan& P, int batch, size_t es)
{
    return (size_t)batch * (4 * P.fwd_stage + 2 * P.inv_stage) * es;
}

template <typename T, int M>
void launch_tn_fwd(const T* i0, const T* i1, T* o0, T* o1, uint64_t in_bs, uint64_t out_bs, uint64_t n_cols,
                   uint64_t L, int batch, hipStream_t s)
{
    const uint32_t nb = (uint32_t)((n_cols + TN_NT - 1) / TN_NT);
    dim3 grid(nb >= 8 ? (nb + 7) & ~7u : nb, batch, 2);
    LaunchScope scope(s, 2.0 * batch * n_cols * (powc(3, M) + powc(6, M)) * sizeof(T), "tn_fwd<%s,M=%d>",
                      tname<T>(), M);
    k_tn_fwd<T, M><<<grid, TN_NT, 0, s>>>(i0, i1, o0, o1, in_bs, out_bs, n_cols, L);
}

template <typename T, int M>
void launch_tn_inv(const T* in, T* out, uint64_t in_bs, uint64_t out_bs, uint64_t n_cols, uint64_t L, int batch,
                   hipStream_t s)
{
    const uint32_t nb = (uint32_t)((n_cols + TN_NT - 1) / TN_NT);
    dim3 grid(nb >= 8 ? (nb + 7) & ~7u : nb, batch, 1);
    LaunchScope scope(s, (double)batch * n_cols * (powc(6, M) + powc(5, M)) * sizeof(T), "tn_inv<%s,M=%d>",
                      tname<T>(), M);
    k_tn_inv<T, M><<<grid, TN_NT, 0, s>>>(in, out, in_bs, out_bs, n_cols, L);
}

template <typename T>
void launch_tn_inv3(const T* in, T* out, uint64_t in_bs, uint64_t out_bs, uint64_t n_hi, uint64_t L, int batch,
                    hipStream_t s)
{
    const uint32_t tiles_per_hi = (uint32_t)((L + 63) / 64);
    const uint32_t n_tiles = (uint32_t)(n_hi * tiles_per_hi);
    dim3 grid(n_tiles >= 8 ? (n_tiles + 7) & ~7u : n_tiles, batch, 1);
    LaunchScope scope(s, (double)batch * n_hi * L * (216.0 + 125.0) * sizeof(T), "tn_inv<%s,M=3>", tname<T>());
    k_tn_inv3w<T><<<grid, TN_INV3_NT, 0, s>>>(in, out, in_bs, out_bs, L, tiles_per_hi, n_tiles);
}

template <typename T, int K>
void launch_tn_fused(const T* a, const T* b, T* y, uint64_t in_bs, uint64_t y_bs, uint32_t n_tiles, int batch,
                     int cus, hipStream_t s)
{
    LaunchScope scope(s, (double)batch * n_tiles * (2.0 * powc(3, K) + powc(5, K)) * sizeof(T), "tn_fused<%s,K=%d>",
                      tname<T>(), K);
    if constexpr (K == 4) {
        const uint32_t n_groups = (n_tiles + TN_TPB - 1) / TN_TPB;
        dim3 grid(tile_grid(n_groups, cus, 0), batch, 1);
        k_tn_tile4<T><<<grid, TN_NT, 0, s>>>(a, b, y, in_bs, y_bs, n_tiles);
    } else {
        dim3 grid(tile_grid(n_tiles, cus, 0), batch, 1);
        k_tn_fused<T, K><<<grid, TN_NT, 0, s>>>(a, b, y, in_bs, y_bs, n_tiles);
    }
}

template <typename T>
int run_tn(const TnPlan& P, const T* a, const T* b, T* z, int batch, T* ws, int cus, hipStream_t s)
{
    const int D = P.D;
    const uint64_t bf = (uint64_t)batch * P.fwd_stage;
    T* fa[2] = {ws, ws + bf};
    T* fb[2] = {ws + 2 * bf, ws + 3 * bf};
    T* iv[2] = {ws + 4 * bf, ws + 4 * bf + (uint64_t)batch * P.inv_stage};
    // outer forward, ascending
    const T* ca = a;
    const T* cb = b;
    uint64_t c_bs = P.n3;
    int ax = 0;
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const int M = P.groups[gi];
        const uint64_t L = powc(3, D - ax - M);
        const uint64_t n_cols = powc(6, ax) * L;
        T* oa = fa[gi & 1];
        T* ob = fb[gi & 1];
        if (M == 1) launch_tn_fwd<T, 1>(ca, cb, oa, ob, c_bs, P.fwd_stage, n_cols, L, batch, s);
        else launch_tn_fwd<T, 2>(ca, cb, oa, ob, c_bs, P.fwd_stage, n_cols, L, batch, s);
        ca = oa;
        cb = ob;
        c_bs = P.fwd_stage;
        ax += M;
    }
    // fused inner tiles: into z when there are no outer axes
    const uint32_t n_tiles = (uint32_t)powc(6, P.p);
    T* y = P.p > 0 ? iv[0] : z;
    const uint64_t y_bs = P.p > 0 ? P.inv_stage : P.n5;
    switch (P.K) {
        case 0: launch_tn_fused<T, 0>(ca, cb, y, c_bs, y_bs, n_tiles, batch, cus, s); break;
        case 1: launch_tn_fused<T, 1>(ca, cb, y, c_bs, y_bs, n_tiles, batch, cus, s); break;
        case 2: launch_tn_fused<T, 2>(ca, cb, y, c_bs, y_bs, n_tiles, batch, cus, s); break;
        case 3: launch_tn_fused<T, 3>(ca, cb, y, c_bs, y_bs, n_tiles, batch, cus, s); break;
        case 4: launch_tn_fused<T, 4>(ca, cb, y, c_bs, y_bs, n_tiles, batch, cus, s); break;
        default: return fail(HC_ERR_UNSUPPORTED, "no ternary tile of %d axes", P.K);
    }
    // outer inverse, descending, out of place; the last pass writes z
    int top = P.p;
    int buf = 0;
    for (int gi = (int)P.inv_groups.size() - 1; gi >= 0; --gi) {
        const int M = P.inv_groups[gi];
        const int a0 = top - M;
        const uint64_t L = powc(5, D - top);
        const uint64_t n_cols = powc(6, a0) * L;
        const bool last = gi == 0;
        T* out = last ? z : iv[buf ^ 1];
        const uint64_t out_bs = last ? P.n5 : P.inv_stage;
        if (M == 1) launch_tn_inv<T, 1>(iv[buf], out, P.inv_stage, out_bs, n_cols, L, batch, s);
        else if (M == 2) launch_tn_inv<T, 2>(iv[buf], out, P.inv_stage, out_bs, n_cols, L, batch, s);
        else launch_tn_inv3<T>(iv[buf], out, P.inv_stage, out_bs, powc(6, a0), L, batch, s);
        buf ^= 1;
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

size_t hc_ternary_workspace_bytes(int D, int dtype, int batch)
{
    const size_t es = dtype_size(dtype);
    if (D < 0 || D > TN_MAX_D || es == 0 || batch < 1 || batch > 65535) return (size_t)-1;
    return tn_ws_bytes(make_tn_plan(D), batch, es);
}

int hc_ternary_convolve_batch(const void* a, const void* b, void* z, int D, int dtype, int batch, void* workspace,
                              size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_ternary_convolve_batch D=%d dtype=%d batch=%d", D, dtype, batch);
    if (!a || !b || !z) return fail(HC_ERR_INVALID_ARG, "a, b and z must be non-null");
    if (D < 0 || D > TN_MAX_D) return fail(HC_ERR_D_RANGE, "D=%d outside [0, %d]", D, TN_MAX_D);
    const size_t es = dtype_size(dtype);
    if (es == 0) return fail(HC_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (batch < 1 || batch > 65535) return fail(HC_ERR_INVALID_ARG, "batch=%d outside [1, 65535]", batch);
    if (misaligned(a, es) || misaligned(b, es) || misaligned(z, es) || misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const TnPlan P = make_tn_plan(D);
    const size_t in_b = (size_t)batch * P.n3 * es, out_b = (size_t)batch * P.n5 * es;
    if (ranges_overlap(z, out_b, a, in_b) || ranges_overlap(z, out_b, b, in_b))
        return fail(HC_ERR_ALIAS, "z overlaps an input");
    const size_t need = tn_ws_bytes(P, batch, es);
    if (need > 0) {
        if (!workspace || workspace_bytes < need)
            return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                        workspace ? workspace_bytes : (size_t)0);
        if (ranges_overlap(workspace, need, z, out_b) || ranges_overlap(workspace, need, a, in_b) ||
            ranges_overlap(workspace, need, b, in_b))
            return fail(HC_ERR_ALIAS, "workspace overlaps a data buffer");
    }
    int cus = 0;
    const int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    switch (dtype) {
        case HC_F64:
            return run_tn<double>(P, (const double*)a, (const double*)b, (double*)z, batch, (double*)workspace, cus,
                                  stream);
        case HC_F32:
            return run_tn<float>(P, (const float*)a, (const float*)b, (float*)z, batch, (float*)workspace, cus,
                                 stream);
        default:
            return run_tn<uint64_t>(P, (const uint64_t*)a, (const uint64_t*)b, (uint64_t*)z, batch,
                                    (uint64_t*)workspace, cus, stream);
    }
}

}  // extern "C"
