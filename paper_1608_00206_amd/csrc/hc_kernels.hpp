// Kernels of the hypercube-convolution path (forward and backward).
//
// Layout (Methods section: row-major tensors; axis 0 = most significant):
//   x, y   2^D values, bit d of the flat index (weight 2^d) = axis D-1-d
//   z      3^D values, ternary digit of weight 3^d = axis D-1-d
// The D axes are split into p = D - K outer axes and K inner axes.  The
// forward path is
//   outer forward   F on axes 0..p-1           x: 2^D -> 3^p x 2^K   (k_fwd_pass)
//   fused inner     per outer index o: F on axes p..D-1, product, G on axes
//                   D-1..p, one contiguous 3^K row of z            (k_fused_inner)
//   outer inverse   G on axes p-1..0 in groups, in place on z      (k_inv_pass)
// which applies every map in exactly the canonical axis order, so the result
// is bitwise independent of K, of the grouping and of the tiling.
//
// The backward path (gradient of sum(w * z)) mirrors it with the transposed
// maps: k_inv_adj_pass (G^T on outer axes, ascending), k_fused_inner_adj,
// k_fwd_adj_pass (F^T on outer axes, descending).
#pragma once

#include "hc_device.hpp"

namespace hc {

// =========================================================================
// Outer forward pass: F on M consecutive binary axes, out of place.
//   in  [n_hi][2^M][L]   ->   out [n_hi][3^M][L],   L = 2^log2L
// One thread per (hi, lo) column; lanes take consecutive lo, so every load and
// store of a wave is one contiguous run.  blockIdx.y = batch item,
// blockIdx.z = operand (0: x, 1: y).
// =========================================================================
template <typename T, int M, int NT>
__global__ __launch_bounds__(NT) void k_fwd_pass(const T* __restrict__ in0, const T* __restrict__ in1,
                                                 T* __restrict__ out0, T* __restrict__ out1,
                                                 uint64_t in_bstride, uint64_t out_bstride,
                                                 uint32_t n_cols, uint32_t log2L)
{
    const T* in = blockIdx.z ? in1 : in0;
    T* out = blockIdx.z ? out1 : out0;
    in += (uint64_t)blockIdx.y * in_bstride;
    out += (uint64_t)blockIdx.y * out_bstride;
    const uint32_t c = blockIdx.x * NT + threadIdx.x;
    if (c >= n_cols) return;
    const uint64_t L = 1ull << log2L;
    const uint64_t hi = c >> log2L;
    const uint64_t lo = c & (L - 1);
    const T* src = in + ((hi << M) * L) + lo;
    T* dst = out + hi * (uint64_t)pow3c(M) * L + lo;
    T s[pow3c(M)];
#pragma unroll
    for (int b = 0; b < (1 << M); ++b) s[b] = src[(uint64_t)b * L];
    fwd_group<T, M>(s);
#pragma unroll
    for (int t = 0; t < pow3c(M); ++t) dst[(uint64_t)t * L] = s[t];
}

// =========================================================================
// Fused inner tile: everything on the K least significant axes for one outer
// index o.  Inner axes are split into groups C (outermost, kC axes), B (kB)
// and A (innermost, kA); each phase holds one group in registers and LDS
// carries the sub-cube between phases:
//   P0  load rows x~[o], y~[o] (2^K each)                         -> R0
//   P1  F on group C  (thread per (bB, bA))                      R0 -> R1
//   P2  F on group B  (thread per (gC, bA))                      R1 -> R2
//   P3  F on group A for x and y, product, G on group A
//       (thread per (gC, gB))                                    R2 -> Z
//   P4  G on group B  (thread per (gC, gA))                       Z -> Z
//   P5  G on group C  (thread per (gB, gA)), contiguous store of z[o]
// =========================================================================
template <int K>
struct FusedCfg {
    static constexpr int kA = cmin(K, 3);
    static constexpr int kB = cmin(K - kA, 3);
    static constexpr int kC = K - kA - kB;
    static constexpr int nA = 1 << kA, nB = 1 << kB, nC = 1 << kC;
    static constexpr int tA = pow3c(kA), tB = pow3c(kB), tC = pow3c(kC);
    static constexpr int N2 = 1 << K, N3 = pow3c(K);
    static constexpr int R0h = N2;              // per operand
    static constexpr int R1h = tC * nB * nA;    // per operand
    static constexpr int R2h = nA * tC * tB;    // per operand
    static constexpr int FWD_LDS = 2 * (R0h + R1h + R2h);
    static constexpr int LDS = cmax(N3, FWD_LDS);
    // backward: R2 (x, y) stays live next to the w_hat tile
    static constexpr int ADJ_LDS = 2 * R2h + cmax(N3, 2 * (R0h + R1h));
};

// Forward half shared by the fused forward and the fused adjoint: loads the
// two rows and applies F on groups C and B, leaving x and y in R2 with layout
// [bA][gC][gB] (so that P3's reads are consecutive across lanes).
template <typename T, int K, int NT>
__device__ __forceinline__ void fused_forward_cb(const T* __restrict__ xr, const T* __restrict__ yr,
                                                 T* R0, T* R1, T* R2)
{
    using C = FusedCfg<K>;
    const int tid = threadIdx.x;
    for (int i = tid; i < C::N2; i += NT) {
        R0[i] = xr[i];
        R0[C::R0h + i] = yr[i];
    }
    lds_barrier();
    // P1: F on group C
    for (int it = tid; it < 2 * C::nB * C::nA; it += NT) {
        const int op = it / (C::nB * C::nA);
        const int r = it - op * (C::nB * C::nA);
        T s[pow3c(C::kC)];
#pragma unroll
        for (int bC = 0; bC < C::nC; ++bC) s[bC] = R0[op * C::R0h + bC * (C::nB * C::nA) + r];
        fwd_group<T, C::kC>(s);
#pragma unroll
        for (int gC = 0; gC < C::tC; ++gC) R1[op * C::R1h + gC * (C::nB * C::nA) + r] = s[gC];
    }
    lds_barrier();
    // P2: F on group B
    for (int it = tid; it < 2 * C::tC * C::nA; it += NT) {
        const int op = it / (C::tC * C::nA);
        const int r = it - op * (C::tC * C::nA);
        const int gC = r / C::nA;
        const int bA = r - gC * C::nA;
        T s[pow3c(C::kB)];
#pragma unroll
        for (int bB = 0; bB < C::nB; ++bB) s[bB] = R1[op * C::R1h + (gC * C::nB + bB) * C::nA + bA];
        fwd_group<T, C::kB>(s);
#pragma unroll
        for (int gB = 0; gB < C::tB; ++gB) R2[op * C::R2h + (bA * C::tC + gC) * C::tB + gB] = s[gB];
    }
    lds_barrier();
}

template <typename T, int K, int NT>
__global__ __launch_bounds__(NT) void k_fused_inner(const T* __restrict__ xt, const T* __restrict__ yt,
                                                    T* __restrict__ z, uint64_t in_bstride,
                                                    uint64_t z_bstride, uint32_t n_tiles)
{
    using C = FusedCfg<K>;
    __shared__ T lds[C::LDS];
    T* R0 = lds;
    T* R1 = R0 + 2 * C::R0h;
    T* R2 = R1 + 2 * C::R1h;
    T* Z = lds;  // aliases R0..R2; written only after R2 has been read
    constexpr int N3I = C::tC * C::tB;                 // P3 items
    constexpr int IPT = (N3I + NT - 1) / NT;
    const int tid = threadIdx.x;
    xt += (uint64_t)blockIdx.y * in_bstride;
    yt += (uint64_t)blockIdx.y * in_bstride;
    z += (uint64_t)blockIdx.y * z_bstride;

    const TileWalk w = xcd_tile_walk(n_tiles);
    for (uint32_t o = w.first; o < w.end; o += w.step) {
        lds_barrier();  // the previous tile's P5 reads of Z are done
        fused_forward_cb<T, K, NT>(xt + (uint64_t)o * C::N2, yt + (uint64_t)o * C::N2, R0, R1, R2);

        // P3: registers take this thread's R2 columns, then Z may overwrite R2
        T xa[IPT][C::nA], ya[IPT][C::nA];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int it = tid + j * NT;
            if (it < N3I) {
#pragma unroll
                for (int bA = 0; bA < C::nA; ++bA) {
                    xa[j][bA] = R2[bA * N3I + it];
                    ya[j][bA] = R2[C::R2h + bA * N3I + it];
                }
            }
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int it = tid + j * NT;
            if (it < N3I) {
                T xs[pow3c(C::kA)], ys[pow3c(C::kA)];
#pragma unroll
                for (int bA = 0; bA < C::nA; ++bA) {
                    xs[bA] = xa[j][bA];
                    ys[bA] = ya[j][bA];
                }
                fwd_group<T, C::kA>(xs);
                fwd_group<T, C::kA>(ys);
#pragma unroll
                for (int g = 0; g < C::tA; ++g) xs[g] = xs[g] * ys[g];
                inv_group<T, C::kA>(xs);
#pragma unroll
                for (int g = 0; g < C::tA; ++g) Z[it * C::tA + g] = xs[g];
            }
        }
        lds_barrier();
        // P4: G on group B
        if constexpr (C::kB > 0) {
            for (int it = tid; it < C::tC * C::tA; it += NT) {
                const int gC = it / C::tA;
                const int gA = it - gC * C::tA;
                T v[pow3c(C::kB)];
#pragma unroll
                for (int gB = 0; gB < C::tB; ++gB) v[gB] = Z[(gC * C::tB + gB) * C::tA + gA];
                inv_group<T, C::kB>(v);
#pragma unroll
                for (int gB = 0; gB < C::tB; ++gB)
                    if (has_digit_one(gB, C::kB)) Z[(gC * C::tB + gB) * C::tA + gA] = v[gB];
            }
            lds_barrier();
        }
        // P5: G on group C and the contiguous store of row o
        T* zr = z + (uint64_t)o * C::N3;
        for (int it = tid; it < C::tB * C::tA; it += NT) {
            T v[pow3c(C::kC)];
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC) v[gC] = Z[gC * (C::tB * C::tA) + it];
            inv_group<T, C::kC>(v);
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC) zr[gC * (C::tB * C::tA) + it] = v[gC];
        }
    }
}

// =========================================================================
// Outer inverse pass: G on m = mB + mA consecutive axes, in place.
//   z viewed as [n_hi][3^mB][3^mA][L],  L = 3^(axes below the group)
// Group A (the group's inner mA axes) comes first in the descending order,
// then group B.  A tile is C consecutive columns of one hi.
//   mB == 0:  one thread per column, all 3^mA values in registers.
//   mB >  0:  phase 1 thread per (gB, column) does G on A in registers and
//             parks the tile in LDS; phase 2 thread per (gA, column) does G
//             on B and stores.  Entries whose group digits contain no 1 are
//             unchanged by G and are not written back.
// =========================================================================
template <typename T, int mA, int mB, int C, int NT>
__global__ __launch_bounds__(NT) void k_inv_pass(T* __restrict__ z, uint64_t z_bstride, uint64_t L,
                                                 uint32_t tiles_per_hi, uint32_t n_tiles)
{
    constexpr int tA = pow3c(mA), tB = pow3c(mB), TM = tA * tB;
    z += (uint64_t)blockIdx.y * z_bstride;
    const int tid = threadIdx.x;
    const TileWalk w = xcd_tile_walk(n_tiles);
    if constexpr (mB == 0) {
        for (uint32_t t = w.first; t < w.end; t += w.step) {
            const uint32_t hi = t / tiles_per_hi;
            const uint32_t j = t - hi * tiles_per_hi;
            const uint64_t lo = (uint64_t)j * NT + tid;
            if (lo < L) {
                T* base = z + (uint64_t)hi * TM * L + lo;
                T v[tA];
#pragma unroll
                for (int g = 0; g < tA; ++g) v[g] = base[(uint64_t)g * L];
                inv_group<T, mA>(v);
#pragma unroll
                for (int g = 0; g < tA; ++g)
                    if (has_digit_one(g, mA)) base[(uint64_t)g * L] = v[g];
            }
        }
    } else {
        __shared__ T S[TM * C];
        for (uint32_t t = w.first; t < w.end; t += w.step) {
            const uint32_t hi = t / tiles_per_hi;
            const uint32_t j = t - hi * tiles_per_hi;
            const uint64_t lo0 = (uint64_t)j * C;
            T* base = z + (uint64_t)hi * TM * L + lo0;
            lds_barrier();
            for (int it = tid; it < tB * C; it += NT) {
                const int gB = it / C;
                const int cl = it - gB * C;
                const bool ok = lo0 + cl < L;
                T v[tA];
#pragma unroll
                for (int gA = 0; gA < tA; ++gA)
                    v[gA] = ok ? base[(uint64_t)(gB * tA + gA) * L + cl] : T(0);
                inv_group<T, mA>(v);
#pragma unroll
                for (int gA = 0; gA < tA; ++gA) S[(gB * tA + gA) * C + cl] = v[gA];
            }
            lds_barrier();
            for (int it = tid; it < tA * C; it += NT) {
                const int gA = it / C;
                const int cl = it - gA * C;
                if (lo0 + cl < L) {
                    T v[tB];
#pragma unroll
                    for (int gB = 0; gB < tB; ++gB) v[gB] = S[(gB * tA + gA) * C + cl];
                    inv_group<T, mB>(v);
                    bool a_one = false;
                    int g = gA;
#pragma unroll
                    for (int d = 0; d < mA; ++d) {
                        a_one |= (g % 3 == 1);
                        g /= 3;
                    }
#pragma unroll
                    for (int gB = 0; gB < tB; ++gB)
                        if (has_digit_one(gB, mB) || a_one) base[(uint64_t)(gB * tA + gA) * L + cl] = v[gB];
                }
            }
        }
    }
}

// =========================================================================
// Backward: G^T on m = mB + mA consecutive axes (ascending: group B, the
// group's outer axes, first).  src -> dst, which may be the same buffer.
//   mB == 0:  one thread per column.
//   mB >  0:  phase 1 thread per (gA, column) does G^T on B, parks in LDS;
//             phase 2 thread per (gB, column) does G^T on A and stores.
// Entries whose group digits are all 1 are unchanged by G^T; in place they
// are not written back.
// =========================================================================
template <typename T, int mA, int mB, int C, int NT>
__global__ __launch_bounds__(NT) void k_inv_adj_pass(const T* src, T* dst, uint64_t src_bstride,
                                                     uint64_t dst_bstride, uint64_t L,
                                                     uint32_t tiles_per_hi, uint32_t n_tiles)
{
    constexpr int tA = pow3c(mA), tB = pow3c(mB), TM = tA * tB;
    src += (uint64_t)blockIdx.y * src_bstride;
    dst += (uint64_t)blockIdx.y * dst_bstride;
    const bool in_place = (src == dst);
    const int tid = threadIdx.x;
    const TileWalk w = xcd_tile_walk(n_tiles);
    if constexpr (mB == 0) {
        for (uint32_t t = w.first; t < w.end; t += w.step) {
            const uint32_t hi = t / tiles_per_hi;
            const uint32_t j = t - hi * tiles_per_hi;
            const uint64_t lo = (uint64_t)j * NT + tid;
            if (lo < L) {
                const uint64_t off = (uint64_t)hi * TM * L + lo;
                T v[tA];
#pragma unroll
                for (int g = 0; g < tA; ++g) v[g] = src[off + (uint64_t)g * L];
                inv_adj_group<T, mA>(v);
#pragma unroll
                for (int g = 0; g < tA; ++g)
                    if (!in_place || !all_digits_one(g, mA)) dst[off + (uint64_t)g * L] = v[g];
            }
        }
    } else {
        __shared__ T S[TM * C];
        for (uint32_t t = w.first; t < w.end; t += w.step) {
            const uint32_t hi = t / tiles_per_hi;
            const uint32_t j = t - hi * tiles_per_hi;
            const uint64_t lo0 = (uint64_t)j * C;
            const uint64_t off = (uint64_t)hi * TM * L + lo0;
            lds_barrier();
            for (int it = tid; it < tA * C; it += NT) {
                const int gA = it / C;
                const int cl = it - gA * C;
                const bool ok = lo0 + cl < L;
                T v[tB];
#pragma unroll
                for (int gB = 0; gB < tB; ++gB)
                    v[gB] = ok ? src[off + (uint64_t)(gB * tA + gA) * L + cl] : T(0);
                inv_adj_group<T, mB>(v);
#pragma unroll
                for (int gB = 0; gB < tB; ++gB) S[(gB * tA + gA) * C + cl] = v[gB];
            }
            lds_barrier();
            for (int it = tid; it < tB * C; it += NT) {
                const int gB = it / C;
                const int cl = it - gB * C;
                if (lo0 + cl < L) {
                    T v[tA];
#pragma unroll
                    for (int gA = 0; gA < tA; ++gA) v[gA] = S[(gB * tA + gA) * C + cl];
                    inv_adj_group<T, mA>(v);
                    bool b_all_one = true;
                    int g = gB;
#pragma unroll
                    for (int d = 0; d < mB; ++d) {
                        b_all_one &= (g % 3 == 1);
                        g /= 3;
                    }
#pragma unroll
                    for (int gA = 0; gA < tA; ++gA)
                        if (!in_place || !(b_all_one && all_digits_one(gA, mA)))
                            dst[off + (uint64_t)(gB * tA + gA) * L + cl] = v[gA];
                }
            }
        }
    }
}

// =========================================================================
// Backward: F^T on M consecutive axes (descending), out of place.
//   in [n_hi][3^M][L]  ->  out [n_hi][2^M][L],   L = 2^log2L
// blockIdx.y = batch item, blockIdx.z = operand.
// =========================================================================
template <typename T, int M, int NT>
__global__ __launch_bounds__(NT) void k_fwd_adj_pass(const T* __restrict__ in0, const T* __restrict__ in1,
                                                     T* __restrict__ out0, T* __restrict__ out1,
                                                     uint64_t in_bstride, uint64_t out_bstride,
                                                     uint32_t n_cols, uint32_t log2L)
{
    const T* in = blockIdx.z ? in1 : in0;
    T* out = blockIdx.z ? out1 : out0;
    if (out == nullptr) return;
    in += (uint64_t)blockIdx.y * in_bstride;
    out += (uint64_t)blockIdx.y * out_bstride;
    const uint32_t c = blockIdx.x * NT + threadIdx.x;
    if (c >= n_cols) return;
    const uint64_t L = 1ull << log2L;
    const uint64_t hi = c >> log2L;
    const uint64_t lo = c & (L - 1);
    const T* src = in + hi * (uint64_t)pow3c(M) * L + lo;
    T* dst = out + ((hi << M) * L) + lo;
    T s[pow3c(M)];
#pragma unroll
    for (int t = 0; t < pow3c(M); ++t) s[t] = src[(uint64_t)t * L];
    fwd_adj_group<T, M>(s);
#pragma unroll
    for (int b = 0; b < (1 << M); ++b) dst[(uint64_t)b * L] = s[b];
}

// =========================================================================
// Fused inner tile of the backward pass, for one outer index o:
//   Q0  x~[o], y~[o] -> F on groups C, B (shared with the forward)      -> R2
//   Q1  G^T on group C of w_hat[o] (thread per (gB, gA)), from global    -> W
//   Q2  G^T on group B (thread per (gC, gA))                             W -> W
//   Q3  G^T on group A; F on group A of x and y; gx_hat = w.y_hat,
//       gy_hat = w.x_hat; F^T on group A  (thread per (gC, gB))         -> R2
//   Q4  F^T on group B (thread per (gC, bA))                          R2 -> R1
//   Q5  F^T on group C (thread per (bB, bA)), contiguous store of the
//       2^K-entry rows gx~[o], gy~[o]
// Either gradient output may be null (not requested).
// =========================================================================
template <typename T, int K, int NT>
__global__ __launch_bounds__(NT) void k_fused_inner_adj(const T* __restrict__ xt, const T* __restrict__ yt,
                                                        const T* __restrict__ w, T* __restrict__ gxt,
                                                        T* __restrict__ gyt, uint64_t in_bstride,
                                                        uint64_t w_bstride, uint64_t g_bstride,
                                                        uint32_t n_tiles)
{
    using C = FusedCfg<K>;
    __shared__ T lds[C::ADJ_LDS];
    T* R2 = lds;                       // x2, y2, later gx2, gy2
    T* U = lds + 2 * C::R2h;           // R0 + R1 during Q0, W from Q1, R1' in Q4
    T* R0 = U;
    T* R1 = U + 2 * C::R0h;
    T* W = U;
    constexpr int N3I = C::tC * C::tB;
    constexpr int IPT = (N3I + NT - 1) / NT;
    const int tid = threadIdx.x;
    xt += (uint64_t)blockIdx.y * in_bstride;
    yt += (uint64_t)blockIdx.y * in_bstride;
    w += (uint64_t)blockIdx.y * w_bstride;
    if (gxt) gxt += (uint64_t)blockIdx.y * g_bstride;
    if (gyt) gyt += (uint64_t)blockIdx.y * g_bstride;

    const TileWalk walk = xcd_tile_walk(n_tiles);
    for (uint32_t o = walk.first; o < walk.end; o += walk.step) {
        lds_barrier();
        fused_forward_cb<T, K, NT>(xt + (uint64_t)o * C::N2, yt + (uint64_t)o * C::N2, R0, R1, R2);
        // Q1: G^T on group C, straight from global memory
        const T* wr = w + (uint64_t)o * C::N3;
        for (int it = tid; it < C::tB * C::tA; it += NT) {
            T v[pow3c(C::kC)];
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC) v[gC] = wr[gC * (C::tB * C::tA) + it];
            inv_adj_group<T, C::kC>(v);
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC) W[gC * (C::tB * C::tA) + it] = v[gC];
        }
        lds_barrier();
        // Q2: G^T on group B
        if constexpr (C::kB > 0) {
            for (int it = tid; it < C::tC * C::tA; it += NT) {
                const int gC = it / C::tA;
                const int gA = it - gC * C::tA;
                T v[pow3c(C::kB)];
#pragma unroll
                for (int gB = 0; gB < C::tB; ++gB) v[gB] = W[(gC * C::tB + gB) * C::tA + gA];
                inv_adj_group<T, C::kB>(v);
#pragma unroll
                for (int gB = 0; gB < C::tB; ++gB)
                    if (!all_digits_one(gB, C::kB)) W[(gC * C::tB + gB) * C::tA + gA] = v[gB];
            }
            lds_barrier();
        }
        // Q3: registers take this thread's W row and R2 columns; then R2 is reused
        T wa[IPT][pow3c(C::kA)], xa[IPT][C::nA], ya[IPT][C::nA];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int it = tid + j * NT;
            if (it < N3I) {
#pragma unroll
                for (int g = 0; g < C::tA; ++g) wa[j][g] = W[it * C::tA + g];
#pragma unroll
                for (int bA = 0; bA < C::nA; ++bA) {
                    xa[j][bA] = R2[bA * N3I + it];
                    ya[j][bA] = R2[C::R2h + bA * N3I + it];
                }
            }
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int it = tid + j * NT;
            if (it < N3I) {
                inv_adj_group<T, C::kA>(wa[j]);
                if (gyt) {
                    T s[pow3c(C::kA)];
#pragma unroll
                    for (int bA = 0; bA < C::nA; ++bA) s[bA] = xa[j][bA];
                    fwd_group<T, C::kA>(s);
#pragma unroll
                    for (int g = 0; g < C::tA; ++g) s[g] = wa[j][g] * s[g];
                    fwd_adj_group<T, C::kA>(s);
#pragma unroll
                    for (int bA = 0; bA < C::nA; ++bA) R2[C::R2h + bA * N3I + it] = s[bA];
                }
                if (gxt) {
                    T s[pow3c(C::kA)];
#pragma unroll
                    for (int bA = 0; bA < C::nA; ++bA) s[bA] = ya[j][bA];
                    fwd_group<T, C::kA>(s);
#pragma unroll
                    for (int g = 0; g < C::tA; ++g) s[g] = wa[j][g] * s[g];
                    fwd_adj_group<T, C::kA>(s);
#pragma unroll
                    for (int bA = 0; bA < C::nA; ++bA) R2[bA * N3I + it] = s[bA];
                }
            }
        }
        lds_barrier();
        // Q4: F^T on group B: R2 [bA][gC][gB] -> R1 [gC][bB][bA]
        for (int it = tid; it < 2 * C::tC * C::nA; it += NT) {
            const int op = it / (C::tC * C::nA);
            if ((op == 0 && !gxt) || (op == 1 && !gyt)) continue;
            const int r = it - op * (C::tC * C::nA);
            const int gC = r / C::nA;
            const int bA = r - gC * C::nA;
            T s[pow3c(C::kB)];
#pragma unroll
            for (int gB = 0; gB < C::tB; ++gB) s[gB] = R2[op * C::R2h + (bA * C::tC + gC) * C::tB + gB];
            fwd_adj_group<T, C::kB>(s);
#pragma unroll
            for (int bB = 0; bB < C::nB; ++bB) R1[op * C::R1h + (gC * C::nB + bB) * C::nA + bA] = s[bB];
        }
        lds_barrier();
        // Q5: F^T on group C and the contiguous stores of the two rows
        for (int it = tid; it < 2 * C::nB * C::nA; it += NT) {
            const int op = it / (C::nB * C::nA);
            T* g = op == 0 ? gxt : gyt;
            if (!g) continue;
            const int r = it - op * (C::nB * C::nA);
            T s[pow3c(C::kC)];
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC) s[gC] = R1[op * C::R1h + gC * (C::nB * C::nA) + r];
            fwd_adj_group<T, C::kC>(s);
            T* gr = g + (uint64_t)o * C::N2;
#pragma unroll
            for (int bC = 0; bC < C::nC; ++bC) gr[bC * (C::nB * C::nA) + r] = s[bC];
        }
    }
}

}  // namespace hc
