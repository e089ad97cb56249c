// Kernels of the hypercube-convolution path (forward and backward).
//
// Layout (Methods section: row-major tensors; axis 0 = most significant):
//   x, y   2^D values, bit d of the flat index (weight 2^d) = axis D-1-d
//   z      3^D values, ternary digit of weight 3^d = axis D-1-d
// The D axes are split into p = D - K outer axes and K inner axes.  The
// forward path is
//   outer forward   F on axes 0..p-1           x: 2^D -> 3^p x 2^K   (fwd_column)
//   fused inner     per outer index o: F on axes p..D-1, product, G on axes
//                   D-1..p, one contiguous 3^K row of z            (fused_tile)
//   outer inverse   G on axes p-1..0 in groups, in place on z
//                                                     (inv_tile, inv_tile_r4)
// which applies every map in exactly the canonical axis order, so the result
// is bitwise independent of K, of the grouping and of the tiling.
//
// The backward path (gradient of sum(w * z)) mirrors it with the transposed
// maps: inv_tile<ADJ> (G^T on outer axes, ascending), fused_tile_adj,
// fwd_adj_column (F^T on outer axes, descending).
//
// Each step is a device function working on one tile or column, called by
// the kernels below; a batch item (a uniform batch or one pair of a batched
// plan) is selected by blockIdx.y through per-item offset maps (BMap).
#pragma once

#include "hc_device.hpp"

namespace hc {

// =========================================================================
// Outer forward pass: F on M consecutive binary axes, out of place.
//   in  [n_hi][2^M][L]   ->   out [n_hi][3^M][L],   L = 2^log2L
// One thread per (hi, lo) column c; lanes take consecutive lo, so every load
// and store of a wave is one contiguous run.
// =========================================================================
template <typename T, int M>
__device__ __forceinline__ void fwd_column(const T* __restrict__ in, T* __restrict__ out, uint32_t c,
                                           uint32_t log2L)
{
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

// blockIdx.y = batch item, blockIdx.z = operand (0: x, 1: y).
template <typename T, int M, int NT>
__global__ __launch_bounds__(NT) void k_fwd_pass(const T* __restrict__ in0, const T* __restrict__ in1,
                                                 T* __restrict__ out0, T* __restrict__ out1,
                                                 BMap in_map, BMap out_map, uint32_t n_cols, uint32_t log2L)
{
    const T* in = blockIdx.z ? in1 : in0;
    T* out = blockIdx.z ? out1 : out0;
    const uint32_t c = blockIdx.x * NT + threadIdx.x;
    if (c >= n_cols) return;
    fwd_column<T, M>(in + in_map.at(blockIdx.y), out + out_map.at(blockIdx.y), c, log2L);
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
};

// Forward half shared by the fused forward and the fused adjoint: takes the
// two rows from registers and applies F on groups C and B, leaving x and y in
// R2 with layout [bA][gC][gB] (so that P3's reads are consecutive across
// lanes).
// Rows held in registers (entries tid, tid + NT, ... of each): the adjoint
// tile loads them before its w row, so that both loads are in flight at once.
// `tid` is the thread's index among the NT threads that share the tile
// (threadIdx.x unless a workgroup splits into several tile groups).
template <typename T, int K, int NT>
struct RowRegs {
    static constexpr int N = (FusedCfg<K>::N2 + NT - 1) / NT;
    T x[N], y[N];
    __device__ __forceinline__ void load(const T* __restrict__ xr, const T* __restrict__ yr,
                                         int tid = (int)threadIdx.x)
    {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int i = tid + j * NT;
            if (i < FusedCfg<K>::N2) {
                x[j] = xr[i];
                y[j] = yr[i];
            }
        }
    }
};

template <typename T, int K, int NT>
__device__ __forceinline__ void fused_forward_cb_from(const RowRegs<T, K, NT>& rows, T* R0, T* R1, T* R2,
                                                      int tid = (int)threadIdx.x)
{
    using C = FusedCfg<K>;
#pragma unroll
    for (int j = 0; j < RowRegs<T, K, NT>::N; ++j) {
        const int i = tid + j * NT;
        if (i < C::N2) {
            R0[i] = rows.x[j];
            R0[C::R0h + i] = rows.y[j];
        }
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

// One fused tile from rows already loaded into registers -> zr (3^K).  lds
// holds FusedCfg<K>::LDS elements; the caller separates two tiles that reuse
// it by an lds_barrier().  NT threads take part, `tid` = 0 .. NT-1 among them.
template <typename T, int K, int NT>
__device__ __forceinline__ void fused_tile_from(const RowRegs<T, K, NT>& rows, T* __restrict__ zr, T* lds,
                                                int tid)
{
    using C = FusedCfg<K>;
    T* R0 = lds;
    T* R1 = R0 + 2 * C::R0h;
    T* R2 = R1 + 2 * C::R1h;
    T* Z = lds;  // aliases R0..R2; written only after R2 has been read
    constexpr int N3I = C::tC * C::tB;  // P3 items
    constexpr int IPT = (N3I + NT - 1) / NT;
    fused_forward_cb_from<T, K, NT>(rows, R0, R1, R2, tid);
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
    // P5: G on group C and the contiguous store of the row
    for (int it = tid; it < C::tB * C::tA; it += NT) {
        T v[pow3c(C::kC)];
#pragma unroll
        for (int gC = 0; gC < C::tC; ++gC) v[gC] = Z[gC * (C::tB * C::tA) + it];
        inv_group<T, C::kC>(v);
#pragma unroll
        for (int gC = 0; gC < C::tC; ++gC) zr[gC * (C::tB * C::tA) + it] = v[gC];
    }
}

// One fused tile: rows xr, yr (2^K each) -> zr (3^K), all NT threads of the
// workgroup taking part.
template <typename T, int K, int NT>
__device__ __forceinline__ void fused_tile(const T* __restrict__ xr, const T* __restrict__ yr, T* __restrict__ zr,
                                           T* lds)
{
    RowRegs<T, K, NT> rows;
    rows.load(xr, yr);
    fused_tile_from<T, K, NT>(rows, zr, lds, (int)threadIdx.x);
}

template <typename T, int K, int NT>
__global__ __launch_bounds__(NT) void k_fused_inner(const T* __restrict__ xt, const T* __restrict__ yt,
                                                    T* __restrict__ z, BMap in_map, BMap z_map,
                                                    uint32_t n_tiles)
{
    using C = FusedCfg<K>;
    __shared__ T lds[C::LDS];
    xt += in_map.at(blockIdx.y);
    yt += in_map.at(blockIdx.y);
    z += z_map.at(blockIdx.y);
    const TileWalk w = xcd_tile_walk(n_tiles);
    for (uint32_t o = w.first; o < w.end; o += w.step) {
        lds_barrier();  // the previous tile's P5 reads of Z are done
        fused_tile<T, K, NT>(xt + (uint64_t)o * C::N2, yt + (uint64_t)o * C::N2, z + (uint64_t)o * C::N3, lds);
    }
}

// =========================================================================
// Outer inverse pass (forward path: G, axes descending) and its adjoint
// (backward path: G^T, axes ascending) on one group of m = mR + mW
// consecutive axes, with z viewed as [n_hi][3^m][L], L = 3^(axes below).
//
// A tile is 64*CW consecutive columns lo of one hi and all 3^m rows.  The
// group splits into a register part R (mR axes, 3^mR values per lane) and a
// wave part W (mW axes, one wave per digit vector gW):
//   phase 1   wave (cg, gW), lane l loads the 3^mR rows of its (gW, column)
//             line and applies the map on R in registers.  Row bases are the
//             same for all lanes of a wave, so each load is one 512 B run.
//   phase 2   (mW > 0) the values cross to a per-gR layout through LDS in
//             sub-rounds of S_GA register indices (double-buffered, one
//             barrier each); wave w applies the map on W for its gR and stores.
// Axis order: the forward inverse takes R = the group's inner axes (G runs
// from the innermost axis out); the adjoint takes R = the group's outer axes
// (G^T runs from the outermost axis in).  Row of (gOuter, gInner) =
// gOuter * 3^(inner axes) + gInner in both cases.
// Entries the map leaves unchanged are not stored when src == dst:
//   G   changes entries with a 1 among the group digits,
//   G^T changes entries whose group digits are not all 1.
// Rows are addressed through buffer resources (row_rsrc) whose byte bound
// ends at column L: lanes past L load zeros and their stores are dropped, and
// a wave whose 64 columns all lie past L does nothing.
// =========================================================================
// Epilogue of a final inverse pass: NoEpilogue stores the entries the map
// changes, as above.  An epilogue with ALL = true maps every entry of the
// tile through apply() and stores them all (used to fuse an elementwise step
// that follows the convolution into its last pass).
struct NoEpilogue {
    static constexpr bool ALL = false;
    template <typename T>
    __device__ __forceinline__ T apply(T v) const { return v; }
};

template <int mR, int mW, int CW>
struct PassCfg {
    static_assert(mW == 0 || CW == 1, "several column groups only without the wave part");
    static constexpr int tR = pow3c(mR), tW = pow3c(mW);
    static constexpr int WAVES = tW * CW;
    static constexpr int NT = 64 * WAVES;
    static constexpr int COLS = 64 * CW;
    static constexpr int S_GA = tR < 9 ? tR : 9;          // register indices per sub-round
    static constexpr int NSUB = (tR + S_GA - 1) / S_GA;
    static constexpr int Q = (S_GA + tW - 1) / tW;        // register indices per wave per sub-round
    // mR = 4 with a wave part streams thirds (inv_tile_r4): three sub-round
    // buffers hold one third of the register indices at once
    static constexpr bool THIRDS = mR == 4 && mW > 0;
    static constexpr int LDS = mW == 0 ? 0 : (THIRDS ? 3 : 2) * tW * S_GA * 64;  // elements
};

// One tile of an inverse pass, run by a workgroup of exactly PassCfg::WAVES
// waves; `wave` must be wave-uniform.  S holds PassCfg::LDS elements when
// mW > 0.  With a wave part every wave is active (the tile's first column
// j * 64 is below L); without one, a wave whose 64 columns all lie past L
// skips its work.
template <typename T, int mR, int mW, int CW, bool ADJ, bool IN_PLACE, class E = NoEpilogue>
__device__ __forceinline__ void inv_tile(const T* src, T* dst, uint64_t L, uint32_t hi, uint32_t j, int wave, T* S,
                                         const E& epi = E{})
{
    using P = PassCfg<mR, mW, CW>;
    constexpr int tR = P::tR, tW = P::tW, TM = tR * tW;
    constexpr int tInner = ADJ ? tW : tR;  // rows per step of the group's outer part
    const int lane = threadIdx.x & 63;
    const int cg = wave / tW;
    const int gW1 = wave - cg * tW;
    const uint64_t lo_w = (uint64_t)j * P::COLS + (uint64_t)cg * 64;  // this wave's first column
    const bool active = mW > 0 || lo_w < L;
    const uint32_t col_off = (uint32_t)lane * (uint32_t)sizeof(T);
    const uint32_t seg_bytes = (uint32_t)((L - lo_w < 64 ? L - lo_w : 64) * sizeof(T));  // when active
    const uint64_t row_bytes = L * sizeof(T);
    const uint64_t tile_off = ((uint64_t)hi * TM * L + lo_w) * sizeof(T);
    const char* s_tile = reinterpret_cast<const char*>(src) + tile_off;
    char* d_tile = reinterpret_cast<char*>(dst) + tile_off;
    T v[tR];
    if (active) {
        // phase 1: rows wave*tR + gR (forward) or gR*tW + wave (adjoint)
        const uint64_t step = (ADJ ? (uint64_t)tInner : 1ull) * row_bytes;
        const char* rp = s_tile + (uint64_t)(ADJ ? gW1 : gW1 * tInner) * row_bytes;
#pragma unroll
        for (int gR = 0; gR < tR; ++gR) {
            v[gR] = buf_load<T>(row_rsrc(rp, seg_bytes), col_off);
            rp += step;
        }
        if constexpr (ADJ) inv_adj_group<T, mR>(v);
        else inv_group<T, mR>(v);
        if constexpr (mW == 0) {
            char* wp = d_tile;
#pragma unroll
            for (int gR = 0; gR < tR; ++gR) {
                const bool changed = ADJ ? !all_digits_one(gR, mR) : has_digit_one(gR, mR);
                if constexpr (E::ALL) buf_store<T>(row_rsrc(wp, seg_bytes), col_off, epi.apply(v[gR]));
                else if (changed || !IN_PLACE) buf_store<T>(row_rsrc(wp, seg_bytes), col_off, v[gR]);
                wp += row_bytes;
            }
        }
    }
    if constexpr (mW > 0) {
        // S viewed as [2][tW][S_GA][64]
#pragma unroll
        for (int r = 0; r < P::NSUB; ++r) {
            T* Sb = S + (r & 1) * (tW * P::S_GA * 64);
            if (active) {
#pragma unroll
                for (int k = 0; k < P::S_GA; ++k)
                    if (r * P::S_GA + k < tR) Sb[(gW1 * P::S_GA + k) * 64 + lane] = v[r * P::S_GA + k];
            }
            lds_barrier();
#pragma unroll
            for (int q = 0; q < P::Q; ++q) {
                const int k = gW1 * P::Q + q;
                const int gR = r * P::S_GA + k;
                if (active && k < P::S_GA && gR < tR) {
                    T u[tW];
#pragma unroll
                    for (int gW = 0; gW < tW; ++gW) u[gW] = Sb[(gW * P::S_GA + k) * 64 + lane];
                    if constexpr (ADJ) inv_adj_group<T, mW>(u);
                    else inv_group<T, mW>(u);
                    // G: some digit of gR is 1; G^T: every digit of gR is 1
                    bool r_flag = ADJ;
                    int g = gR;
#pragma unroll
                    for (int d = 0; d < mR; ++d) {
                        if (ADJ) r_flag = r_flag && (g % 3 == 1);
                        else r_flag = r_flag || (g % 3 == 1);
                        g /= 3;
                    }
                    // forward: rows gW*tR + gR; adjoint: rows gR*tW + gW
                    const uint64_t step = (ADJ ? 1ull : (uint64_t)tInner) * row_bytes;
                    char* wp = d_tile + (uint64_t)(ADJ ? gR * tInner : gR) * row_bytes;
#pragma unroll
                    for (int gW = 0; gW < tW; ++gW) {
                        const bool changed = ADJ ? !(r_flag && all_digits_one(gW, mW))
                                                 : (r_flag || has_digit_one(gW, mW));
                        if constexpr (E::ALL) buf_store<T>(row_rsrc(wp, seg_bytes), col_off, epi.apply(u[gW]));
                        else if (changed || !IN_PLACE) buf_store<T>(row_rsrc(wp, seg_bytes), col_off, u[gW]);
                        wp += step;
                    }
                }
            }
        }
    }
}

// One tile of an inverse pass with mR = 4 and a wave part (CW = 1, every wave
// active).  The 81 register values of a lane would not fit the register budget
// of a 3^mW-wave workgroup, so the register sub-cube is streamed in thirds of
// its outermost register axis d0 (register index gR = d0*27 + rest):
//   G   (descending): thirds d0 = 0 and 2 need only the three inner register
//       axes, after which they are final; third 1 then takes
//       (p1 - p0) - p2 across the thirds, reading third 0 back from LDS.
//   G^T (ascending):  d0 comes first: thirds 0 and 2 subtract third 1, then
//       every third takes the three inner register axes.
// Each third crosses to the wave part through three LDS sub-round buffers
// ([3][tW][9][64]); third 1 is loaded while the first third is being stored.
// Every entry sees the same operations in the same order as in inv_tile.
template <typename T, int mW, bool ADJ, bool IN_PLACE, class E = NoEpilogue>
__device__ __forceinline__ void inv_tile_r4(const T* src, T* dst, uint64_t L, uint32_t hi, uint32_t j, int wave,
                                            T* S, const E& epi = E{})
{
    constexpr int tR = 81, TH = 27, tW = pow3c(mW), TM = tR * tW;
    constexpr int SG = 9;                       // register indices per sub-round
    constexpr int Q = (SG + tW - 1) / tW;       // register indices per wave per sub-round
    constexpr int BUF = tW * SG * 64;           // elements per sub-round buffer
    const int lane = threadIdx.x & 63;
    const int gW1 = wave;
    const uint64_t lo_w = (uint64_t)j * 64;
    const uint32_t col_off = (uint32_t)lane * (uint32_t)sizeof(T);
    const uint32_t seg_bytes = (uint32_t)((L - lo_w < 64 ? L - lo_w : 64) * sizeof(T));
    const uint64_t row_bytes = L * sizeof(T);
    const uint64_t tile_off = ((uint64_t)hi * TM * L + lo_w) * sizeof(T);
    const char* s_tile = reinterpret_cast<const char*>(src) + tile_off;
    char* d_tile = reinterpret_cast<char*>(dst) + tile_off;
    // phase-1 rows of this wave: forward gW1*tR + gR, adjoint gR*tW + gW1
    const char* s_wave = s_tile + (uint64_t)(ADJ ? gW1 : gW1 * tR) * row_bytes;
    const uint64_t s_step = (ADJ ? (uint64_t)tW : 1ull) * row_bytes;
    // LDS byte offsets; each base is opaque so that the accesses from it use
    // immediate offsets (at most 64 KiB past the base)
    char* Sc = reinterpret_cast<char*>(S);
    auto lds_at = [&](uint32_t base, uint32_t off) -> T& { return *reinterpret_cast<T*>(Sc + base + off); };

    auto load_third = [&](T (&t)[TH], int d0) {
        const char* rp = s_wave + (uint64_t)(d0 * TH) * s_step;
#pragma unroll
        for (int i = 0; i < TH; ++i) {
            t[i] = buf_load<T>(row_rsrc(rp, seg_bytes), col_off);
            rp += s_step;
        }
    };
    // register index d0*27 + i goes to buffer i / 9, entry (gW1*9 + i%9)
    auto own_base = [&](int buf) {
        return opaque_u32((uint32_t)((buf * BUF + gW1 * SG * 64 + lane) * sizeof(T)));
    };
    auto put_third = [&](const T (&t)[TH]) {
        const uint32_t b01 = own_base(0), b2 = own_base(2);
#pragma unroll
        for (int i = 0; i < TH; ++i) {
            const uint32_t o = (uint32_t)(((i / SG) % 2 * BUF + (i % SG) * 64) * sizeof(T));
            lds_at(i / SG == 2 ? b2 : b01, o) = t[i];
        }
    };
    // the wave part for the third d0 held in the buffers, then the stores
    auto wave_part = [&](auto d0c) {
        constexpr int d0 = decltype(d0c)::value;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = gW1 * Q + q;  // register index within a sub-round: digits d2 d3
            if (k < SG) {
                const bool k_one = (k % 3 == 1) || (k / 3 == 1);
                const bool k_all = (k % 3 == 1) && (k / 3 == 1);
#pragma unroll
                for (int sr = 0; sr < 3; ++sr) {  // digit d1
                    const uint32_t rb = opaque_u32((uint32_t)((sr * BUF + k * 64 + lane) * sizeof(T)));
                    T u[tW];
#pragma unroll
                    for (int gW = 0; gW < tW; ++gW) u[gW] = lds_at(rb, (uint32_t)(gW * SG * 64 * sizeof(T)));
                    if constexpr (ADJ) inv_adj_group<T, mW>(u);
                    else inv_group<T, mW>(u);
                    const int gR = d0 * TH + sr * SG + k;
                    char* wp = d_tile + (uint64_t)(ADJ ? gR * tW : gR) * row_bytes;
                    const uint64_t step = (ADJ ? 1ull : (uint64_t)tR) * row_bytes;
#pragma unroll
                    for (int gW = 0; gW < tW; ++gW) {
                        bool changed;
                        if constexpr (ADJ)
                            changed = !(d0 == 1 && sr == 1 && k_all && all_digits_one(gW, mW));
                        else
                            changed = d0 == 1 || sr == 1 || k_one || has_digit_one(gW, mW);
                        if constexpr (E::ALL) buf_store<T>(row_rsrc(wp, seg_bytes), col_off, epi.apply(u[gW]));
                        else if (changed || !IN_PLACE) buf_store<T>(row_rsrc(wp, seg_bytes), col_off, u[gW]);
                        wp += step;
                    }
                }
            }
        }
    };
    using D0 = std::integral_constant<int, 0>;
    using D1 = std::integral_constant<int, 1>;
    using D2 = std::integral_constant<int, 2>;

    if constexpr (!ADJ) {
        T a[TH], c[TH];
        load_third(a, 0);
        load_third(c, 2);
        inv_group<T, 3>(a);
        inv_group<T, 3>(c);
        put_third(a);
        // the third load may not move above the first third's arithmetic:
        // three live thirds would not fit the register budget
        __builtin_amdgcn_sched_barrier(0);
        T b[TH];
        load_third(b, 1);
        lds_barrier();
        wave_part(D0{});
        inv_group<T, 3>(b);
        {
            const uint32_t b01 = own_base(0), b2 = own_base(2);
#pragma unroll
            for (int i = 0; i < TH; ++i) {
                const uint32_t o = (uint32_t)(((i / SG) % 2 * BUF + (i % SG) * 64) * sizeof(T));
                b[i] = (b[i] - lds_at(i / SG == 2 ? b2 : b01, o)) - c[i];
            }
        }
        lds_barrier();
        put_third(b);
        lds_barrier();
        wave_part(D1{});
        lds_barrier();
        put_third(c);
        lds_barrier();
        wave_part(D2{});
    } else {
        T a[TH], b[TH];
        load_third(a, 0);
        load_third(b, 1);
#pragma unroll
        for (int i = 0; i < TH; ++i) a[i] = a[i] - b[i];
        inv_adj_group<T, 3>(a);
        put_third(a);
        // the third load may not move above the first third's arithmetic:
        // three live thirds would not fit the register budget
        __builtin_amdgcn_sched_barrier(0);
        T c[TH];
        load_third(c, 2);
        lds_barrier();
        wave_part(D0{});
#pragma unroll
        for (int i = 0; i < TH; ++i) c[i] = c[i] - b[i];
        inv_adj_group<T, 3>(b);
        inv_adj_group<T, 3>(c);
        lds_barrier();
        put_third(b);
        lds_barrier();
        wave_part(D1{});
        lds_barrier();
        put_third(c);
        lds_barrier();
        wave_part(D2{});
    }
}

template <typename T, int mR, int mW, int CW, bool ADJ, bool IN_PLACE>
__global__ __launch_bounds__(64 * pow3c(mW) * CW) void k_inv_pass(const T* src, T* dst, BMap src_map,
                                                                 BMap dst_map, uint64_t L, uint32_t tiles_per_hi,
                                                                 uint32_t n_tiles)
{
    using P = PassCfg<mR, mW, CW>;
    __shared__ T S[P::LDS > 0 ? P::LDS : 1];
    src += src_map.at(blockIdx.y);
    dst += dst_map.at(blockIdx.y);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileWalk walk = xcd_tile_walk(n_tiles);
    if constexpr (P::THIRDS) {
        // launched with one tile per workgroup: no loop, so nothing tile-
        // invariant is kept live across the register-heavy body
        if (walk.first < walk.end) {
            const uint32_t hi = walk.first / tiles_per_hi;
            inv_tile_r4<T, mW, ADJ, IN_PLACE>(src, dst, L, hi, walk.first - hi * tiles_per_hi, wave, S);
        }
    } else {
        for (uint32_t t = walk.first; t < walk.end; t += walk.step) {
            const uint32_t hi = t / tiles_per_hi;
            const uint32_t j = t - hi * tiles_per_hi;
            if constexpr (mW > 0) lds_barrier();  // the previous tile's phase-2 reads are done
            inv_tile<T, mR, mW, CW, ADJ, IN_PLACE>(src, dst, L, hi, j, wave, S);
        }
    }
}

// The last inverse pass of a forward run with an epilogue: in place, every
// entry mapped through epi.bind(item).apply() and stored.  Launched like
// k_inv_pass with the same tile counts (one tile per workgroup for the
// streamed-thirds tile).
template <typename T, int mR, int mW, class EP>
__global__ __launch_bounds__(64 * pow3c(mW)) void k_inv_pass_epi(T* z, BMap z_map, uint64_t L,
                                                                 uint32_t tiles_per_hi, uint32_t n_tiles, EP epi)
{
    using P = PassCfg<mR, mW, 1>;
    static_assert(mW > 0, "epilogue passes have a wave part");
    __shared__ T S[P::LDS];
    z += z_map.at(blockIdx.y);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileWalk walk = xcd_tile_walk(n_tiles);
    const auto e = epi.bind(blockIdx.y);
    if constexpr (P::THIRDS) {
        if (walk.first < walk.end) {
            const uint32_t hi = walk.first / tiles_per_hi;
            inv_tile_r4<T, mW, false, true>(z, z, L, hi, walk.first - hi * tiles_per_hi, wave, S, e);
        }
    } else {
        for (uint32_t t = walk.first; t < walk.end; t += walk.step) {
            const uint32_t hi = t / tiles_per_hi;
            lds_barrier();
            inv_tile<T, mR, mW, 1, false, true>(z, z, L, hi, t - hi * tiles_per_hi, wave, S, e);
        }
    }
}

// =========================================================================
// Backward: F^T on M consecutive axes (descending), out of place.
//   in [n_hi][3^M][L]  ->  out [n_hi][2^M][L],   L = 2^log2L
// =========================================================================
template <typename T, int M>
__device__ __forceinline__ void fwd_adj_column(const T* __restrict__ in, T* __restrict__ out, uint32_t c,
                                               uint32_t log2L)
{
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

// blockIdx.y = batch item, blockIdx.z = operand; a null output skips it.
template <typename T, int M, int NT>
__global__ __launch_bounds__(NT) void k_fwd_adj_pass(const T* __restrict__ in0, const T* __restrict__ in1,
                                                     T* __restrict__ out0, T* __restrict__ out1,
                                                     BMap in_map, BMap out_map, uint32_t n_cols, uint32_t log2L)
{
    const T* in = blockIdx.z ? in1 : in0;
    T* out = blockIdx.z ? out1 : out0;
    if (out == nullptr) return;
    const uint32_t c = blockIdx.x * NT + threadIdx.x;
    if (c >= n_cols) return;
    fwd_adj_column<T, M>(in + in_map.at(blockIdx.y), out + out_map.at(blockIdx.y), c, log2L);
}

// =========================================================================
// Fused inner tile of the backward pass, for one outer index o:
//   Q1  G^T on the tail outer axes and on group C of w_hat[o] (thread per
//       (gB, gA)), from global                                           -> W
//   Q2  G^T on group B (thread per (gC, gA))                             W -> W
//   Q3  registers take this thread's W row (3^kA values); W is released
//   Q0  x~[o], y~[o] -> F on groups C, B (shared with the forward)      -> R2
//   Q3' G^T on group A; F on group A of x and y; gx_hat = w.y_hat,
//       gy_hat = w.x_hat; F^T on group A  (thread per (gC, gB))         -> R2
//   Q4  F^T on group B (thread per (gC, bA))                          R2 -> R1
//   Q5  F^T on group C (thread per (bB, bA)), contiguous store of the
//       2^K-entry rows gx~[o], gy~[o]
// The w_hat tile and the x, y stages never share LDS at the same time, so
// the tile needs no more LDS than the forward one (FusedCfg<K>::LDS).
// Either gradient row may be null (not requested).
// =========================================================================
// Value of G^T on the TAIL last outer axes at one entry of row o, read from
// the untransformed rows of the tile's siblings along those axes (rows
// o + (e - d) * 3^(axes below) for digits e the map combines, each row
// `rs` elements long).  dA is o's digit on the first tail axis, dB on the
// second; the first axis is transformed before the second, as G^T runs
// ascending.  Per axis: digit 1 keeps w1, digits 0 and 2 give w0 - w1 and
// w2 - w1.
// Every operand is loaded unconditionally (a digit 1 makes two of the
// addresses coincide) and the result is selected, so that the loads of many
// entries are in flight together instead of waiting behind branches.
template <typename T, int TAIL>
__device__ __forceinline__ T tail_adj(const T* __restrict__ p, int dA, int dB, int64_t rs)
{
    if constexpr (TAIL == 0) {
        return p[0];
    } else if constexpr (TAIL == 1) {
        const T own = p[0];
        const T w1 = p[(int64_t)(1 - dA) * rs];
        const T diff = own - w1;
        return dA == 1 ? w1 : diff;
    } else {
        const T a = p[0];                                           // (dA, dB)
        const T b = p[(int64_t)(1 - dA) * 3 * rs];                  // (1, dB)
        const T c = p[(int64_t)(1 - dB) * rs];                      // (dA, 1)
        const T d = p[((int64_t)(1 - dA) * 3 + (1 - dB)) * rs];     // (1, 1)
        // axis A: u(e) = w[dA, e] - w[1, e], or w[1, e] when dA = 1
        const T uab = a - b, ucd = c - d;
        const T uB = dA == 1 ? b : uab;
        const T u1 = dA == 1 ? d : ucd;
        // axis B
        const T diff = uB - u1;
        return dB == 1 ? u1 : diff;
    }
}

template <typename T, int K, int NT, int TAIL>
__device__ __forceinline__ void fused_tile_adj(const T* __restrict__ xr, const T* __restrict__ yr,
                                               const T* __restrict__ wr, T* __restrict__ gxr,
                                               T* __restrict__ gyr, T* lds, int dA, int dB)
{
    using C = FusedCfg<K>;
    T* W = lds;
    T* R0 = lds;
    T* R1 = R0 + 2 * C::R0h;
    T* R2 = R1 + 2 * C::R1h;           // x2, y2, later gx2, gy2
    constexpr int N3I = C::tC * C::tB;
    constexpr int IPT = (N3I + NT - 1) / NT;
    const int tid = threadIdx.x;
    // the x~, y~ rows are loaded first and held in registers until Q0
    RowRegs<T, K, NT> rows;
    rows.load(xr, yr);
    // Q1: G^T on the tail axes (if any) and on group C, from global memory;
    // unrolled over this thread's items so that their loads are in flight
    // together
    constexpr int NQ1 = C::tB * C::tA;
#pragma unroll
    for (int j = 0; j < (NQ1 + NT - 1) / NT; ++j) {
        const int it = tid + j * NT;
        if (it < NQ1) {
            T v[pow3c(C::kC)];
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC)
                v[gC] = tail_adj<T, TAIL>(wr + gC * NQ1 + it, dA, dB, C::N3);
            inv_adj_group<T, C::kC>(v);
#pragma unroll
            for (int gC = 0; gC < C::tC; ++gC) W[gC * NQ1 + it] = v[gC];
        }
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
    // Q3: registers take this thread's W row; then the forward half reuses W
    T wa[IPT][pow3c(C::kA)];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int it = tid + j * NT;
        if (it < N3I) {
#pragma unroll
            for (int g = 0; g < C::tA; ++g) wa[j][g] = W[it * C::tA + g];
        }
    }
    lds_barrier();
    fused_forward_cb_from<T, K, NT>(rows, R0, R1, R2);
    // Q3': each thread's R2 columns are read and rewritten by that thread only
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int it = tid + j * NT;
        if (it < N3I) {
            T xa[C::nA], ya[C::nA];
#pragma unroll
            for (int bA = 0; bA < C::nA; ++bA) {
                xa[bA] = R2[bA * N3I + it];
                ya[bA] = R2[C::R2h + bA * N3I + it];
            }
            inv_adj_group<T, C::kA>(wa[j]);
            if (gyr) {
                T s[pow3c(C::kA)];
#pragma unroll
                for (int bA = 0; bA < C::nA; ++bA) s[bA] = xa[bA];
                fwd_group<T, C::kA>(s);
#pragma unroll
                for (int g = 0; g < C::tA; ++g) s[g] = wa[j][g] * s[g];
                fwd_adj_group<T, C::kA>(s);
#pragma unroll
                for (int bA = 0; bA < C::nA; ++bA) R2[C::R2h + bA * N3I + it] = s[bA];
            }
            if (gxr) {
                T s[pow3c(C::kA)];
#pragma unroll
                for (int bA = 0; bA < C::nA; ++bA) s[bA] = ya[bA];
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
        if ((op == 0 && !gxr) || (op == 1 && !gyr)) continue;
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
        T* g = op == 0 ? gxr : gyr;
        if (!g) continue;
        const int r = it - op * (C::nB * C::nA);
        T s[pow3c(C::kC)];
#pragma unroll
        for (int gC = 0; gC < C::tC; ++gC) s[gC] = R1[op * C::R1h + gC * (C::nB * C::nA) + r];
        fwd_adj_group<T, C::kC>(s);
#pragma unroll
        for (int bC = 0; bC < C::nC; ++bC) g[bC * (C::nB * C::nA) + r] = s[bC];
    }
}

// TAIL (0, 1 or 2): the last TAIL outer axes get G^T inside the tile, from
// w rows that have had G^T on the outer axes above them only (or none).
template <typename T, int K, int NT, int TAIL>
__global__ __launch_bounds__(NT, 3) void k_fused_inner_adj(const T* __restrict__ xt, const T* __restrict__ yt,
                                                        const T* __restrict__ w, T* __restrict__ gxt,
                                                        T* __restrict__ gyt, BMap in_map, BMap w_map,
                                                        BMap g_map, uint32_t n_tiles)
{
    using C = FusedCfg<K>;
    __shared__ T lds[C::LDS];
    xt += in_map.at(blockIdx.y);
    yt += in_map.at(blockIdx.y);
    w += w_map.at(blockIdx.y);
    if (gxt) gxt += g_map.at(blockIdx.y);
    if (gyt) gyt += g_map.at(blockIdx.y);
    const TileWalk walk = xcd_tile_walk(n_tiles);
    for (uint32_t o = walk.first; o < walk.end; o += walk.step) {
        lds_barrier();
        const int dB = TAIL == 2 ? (int)(o % 3u) : 0;
        const int dA = TAIL == 2 ? (int)((o / 3u) % 3u) : (TAIL == 1 ? (int)(o % 3u) : 0);
        fused_tile_adj<T, K, NT, TAIL>(xt + (uint64_t)o * C::N2, yt + (uint64_t)o * C::N2,
                                       w + (uint64_t)o * C::N3, gxt ? gxt + (uint64_t)o * C::N2 : nullptr,
                                       gyt ? gyt + (uint64_t)o * C::N2 : nullptr, lds, dA, dB);
    }
}

}  // namespace hc
