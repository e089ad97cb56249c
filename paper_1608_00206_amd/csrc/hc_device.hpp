// Device building blocks for exact hypercube convolution on gfx950.
//
// The method (Methods section, three-subproblem recursion) in per-axis form:
//   forward  F on every axis:  (a0, a1)     -> (a0, a0 + a1, a1)
//   product  elementwise x_hat * y_hat
//   inverse  G on every axis:  (p0, p1, p2) -> (p0, (p1 - p0) - p2, p2)
// Floating-point order (fixed so that every tiling produces identical bits):
// forward on axes in ascending order (axis 0 = most significant index digit),
// inverse in descending order, middle entries evaluated exactly as written
// above.  This is the order the recursion itself produces.
//
// Backward (gradient of sum(w * z), derived by transposing the maps):
//   G^T: (w0, w1, w2) -> (w0 - w1, w1, w2 - w1), axes ascending
//   F^T: (g0, g1, g2) -> (g0 + g1, g1 + g2),     axes descending
//
// Every helper here works on a register array whose indices are compile-time
// constants after unrolling; nothing is ever indexed dynamically.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hc {

__host__ __device__ constexpr int pow3c(int n) { return n <= 0 ? 1 : 3 * pow3c(n - 1); }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// True when some ternary digit (of `digits` digits) of g equals 1.
__host__ __device__ constexpr bool has_digit_one(int g, int digits)
{
    return digits <= 0 ? false : (g % 3 == 1) || has_digit_one(g / 3, digits - 1);
}
// True when every ternary digit of g equals 1.
__host__ __device__ constexpr bool all_digits_one(int g, int digits)
{
    return digits <= 0 ? true : (g % 3 == 1) && all_digits_one(g / 3, digits - 1);
}

// Workgroup barrier that orders LDS traffic only.  Outstanding global stores
// keep draining while the workgroup moves on (a full __syncthreads would wait
// for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- forward F
// State of M group axes after J forward steps: shape [3^J][2^(M-J)] stored
// row-major in s[0 .. 3^J * 2^(M-J)).  Step J maps axis J from 2 to 3 entries.
template <typename T, int M, int J>
__device__ __forceinline__ void fwd_steps(T (&s)[pow3c(M)])
{
    if constexpr (J < M) {
        constexpr int hi_n = pow3c(J);
        constexpr int lo_n = 1 << (M - J - 1);
        T n[pow3c(M)];
#pragma unroll
        for (int hi = 0; hi < hi_n; ++hi) {
#pragma unroll
            for (int lo = 0; lo < lo_n; ++lo) {
                const T a0 = s[(hi * 2 + 0) * lo_n + lo];
                const T a1 = s[(hi * 2 + 1) * lo_n + lo];
                n[(hi * 3 + 0) * lo_n + lo] = a0;
                n[(hi * 3 + 1) * lo_n + lo] = a0 + a1;
                n[(hi * 3 + 2) * lo_n + lo] = a1;
            }
        }
#pragma unroll
        for (int i = 0; i < hi_n * 3 * lo_n; ++i) s[i] = n[i];
        fwd_steps<T, M, J + 1>(s);
    }
}

// F on M axes, ascending: s[0 .. 2^M) holds the binary sub-cube on entry
// (bit M-1-j of the index = group axis j); s[0 .. 3^M) holds the ternary
// sub-cube on exit.
template <typename T, int M>
__device__ __forceinline__ void fwd_group(T (&s)[pow3c(M)])
{
    fwd_steps<T, M, 0>(s);
}

// ---------------------------------------------------------------- inverse G
template <typename T, int M, int J>
__device__ __forceinline__ void inv_steps(T (&v)[pow3c(M)])
{
    if constexpr (J >= 0) {
        constexpr int hi_n = pow3c(J);
        constexpr int lo_n = pow3c(M - J - 1);
#pragma unroll
        for (int hi = 0; hi < hi_n; ++hi) {
#pragma unroll
            for (int lo = 0; lo < lo_n; ++lo) {
                const T p0 = v[(hi * 3 + 0) * lo_n + lo];
                const T p1 = v[(hi * 3 + 1) * lo_n + lo];
                const T p2 = v[(hi * 3 + 2) * lo_n + lo];
                v[(hi * 3 + 1) * lo_n + lo] = (p1 - p0) - p2;
            }
        }
        inv_steps<T, M, J - 1>(v);
    }
}

// G on M axes (of a [3^M] sub-cube), descending: axis M-1 first, axis 0 last.
template <typename T, int M>
__device__ __forceinline__ void inv_group(T (&v)[pow3c(M)])
{
    inv_steps<T, M, M - 1>(v);
}

// ------------------------------------------------------- adjoint of inverse
template <typename T, int M, int J>
__device__ __forceinline__ void inv_adj_steps(T (&v)[pow3c(M)])
{
    if constexpr (J < M) {
        constexpr int hi_n = pow3c(J);
        constexpr int lo_n = pow3c(M - J - 1);
#pragma unroll
        for (int hi = 0; hi < hi_n; ++hi) {
#pragma unroll
            for (int lo = 0; lo < lo_n; ++lo) {
                const T w0 = v[(hi * 3 + 0) * lo_n + lo];
                const T w1 = v[(hi * 3 + 1) * lo_n + lo];
                const T w2 = v[(hi * 3 + 2) * lo_n + lo];
                v[(hi * 3 + 0) * lo_n + lo] = w0 - w1;
                v[(hi * 3 + 2) * lo_n + lo] = w2 - w1;
            }
        }
        inv_adj_steps<T, M, J + 1>(v);
    }
}

// G^T on M axes, ascending: axis 0 first.
template <typename T, int M>
__device__ __forceinline__ void inv_adj_group(T (&v)[pow3c(M)])
{
    inv_adj_steps<T, M, 0>(v);
}

// ------------------------------------------------------- adjoint of forward
// State before step J (descending): shape [3^(J+1)][2^(M-J-1)]; after: [3^J][2^(M-J)].
template <typename T, int M, int J>
__device__ __forceinline__ void fwd_adj_steps(T (&s)[pow3c(M)])
{
    if constexpr (J >= 0) {
        constexpr int hi_n = pow3c(J);
        constexpr int lo_n = 1 << (M - J - 1);
        T n[pow3c(M)];
#pragma unroll
        for (int hi = 0; hi < hi_n; ++hi) {
#pragma unroll
            for (int lo = 0; lo < lo_n; ++lo) {
                const T g0 = s[(hi * 3 + 0) * lo_n + lo];
                const T g1 = s[(hi * 3 + 1) * lo_n + lo];
                const T g2 = s[(hi * 3 + 2) * lo_n + lo];
                n[(hi * 2 + 0) * lo_n + lo] = g0 + g1;
                n[(hi * 2 + 1) * lo_n + lo] = g1 + g2;
            }
        }
#pragma unroll
        for (int i = 0; i < hi_n * 2 * lo_n; ++i) s[i] = n[i];
        fwd_adj_steps<T, M, J - 1>(s);
    }
}

// F^T on M axes, descending: s[0 .. 3^M) on entry, s[0 .. 2^M) on exit.
template <typename T, int M>
__device__ __forceinline__ void fwd_adj_group(T (&s)[pow3c(M)])
{
    fwd_adj_steps<T, M, M - 1>(s);
}

// ------------------------------------------------------- buffer accesses
// A row segment addressed through a buffer resource: the wave-uniform base
// address and byte bound live in scalar registers, each lane supplies a
// 32-bit byte offset.  This keeps per-row addressing out of the vector
// register file, and the hardware bound check turns accesses at or past
// `bytes` into loads of zero and dropped stores (the ragged column tail).
// Word 3 = 0x00020000: raw (untyped) 32-bit data access on gfx9-family parts.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(sizeof(T) == 8 || sizeof(T) == 4, "8- or 4-byte elements");
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, T v)
{
    if constexpr (sizeof(T) == 8) {
        using V2 = unsigned int __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
    }
}

// A per-lane value the compiler must take as given at this point: it keeps
// one register for it and folds constant offsets into the instructions that
// use it, instead of materialising one address per access.
__device__ __forceinline__ uint32_t opaque_u32(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// --------------------------------------------------------- batch items
// Element offset of batch item b in one buffer: a uniform stride, or a
// per-item table (device memory) when the items are packed unevenly.
struct BMap {
    uint64_t stride = 0;
    const uint64_t* table = nullptr;
    __host__ __device__ BMap(uint64_t s = 0, const uint64_t* t = nullptr) : stride(s), table(t) {}
    __device__ __forceinline__ uint64_t at(uint32_t b) const { return table ? table[b] : (uint64_t)b * stride; }
};

// -------------------------------------------------------- tile scheduling
// Map a workgroup to its first tile so that each XCD (workgroups are handed
// to the 8 XCDs round-robin) walks one contiguous chunk of tiles: neighbouring
// tiles, which share cache lines at their edges, then meet in the same L2.
struct TileWalk {
    uint32_t first, step, end;
};

__device__ __forceinline__ TileWalk xcd_tile_walk(uint32_t n_tiles)
{
    const uint32_t G = gridDim.x;
    const uint32_t b = blockIdx.x;
    if (G < 8 || (G & 7u) != 0) return {b, G, n_tiles};
    const uint32_t per_xcd = G >> 3;
    const uint32_t xcd = b & 7u;
    const uint32_t local = b >> 3;
    const uint32_t chunk = (n_tiles + 7u) >> 3;
    const uint32_t begin = xcd * chunk;
    uint32_t end = begin + chunk;
    if (end > n_tiles) end = n_tiles;
    return {begin + local, per_xcd, end};
}

}  // namespace hc
