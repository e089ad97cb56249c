// Persistent batched kernel: every pair of a batched plan in one launch.
//
// The single-pair path of the Methods section (outer forward F, fused inner
// tiles, outer inverse G) runs here once per pair, by one workgroup:
//   * a workgroup takes pairs by ticket, an atomic counter over a task list
//     sorted by decreasing D (the longest pairs start first, the short ones
//     fill in behind them);
//   * it runs every step of its pair itself: the outer forward groups into its
//     own workspace slot, the fused tiles one after another, the outer inverse
//     passes in place on the pair's z;
//   * a full workgroup barrier separates the steps, which makes the global
//     stores of one step visible to every wave of the workgroup in the next.
// A pair never spans workgroups, so no workgroup ever waits for another: the
// phase of a pair is simply where its workgroup is in this program, and the
// grid drains once the ticket counter has passed the last pair.  The last
// workgroup to leave resets the two counters for the next launch.
//
// Every step calls the same tile functions as the single-pair kernels, in
// the same axis order, so each pair's z is bitwise that of hc_convolve.
#include <hip/hip_runtime.h>

#include "hc.h"
#include "hc_internal.hpp"
#include "hc_kernels.hpp"

namespace hc {

template <typename T>
struct PersistCfg {
    static constexpr int NT = PAIR_NT;
    static constexpr int WAVES = NT / 64;
    static constexpr int KMAX = pair_kmax(sizeof(T));
    // 8-byte elements: the fused stage of a pair with outer axes runs three
    // tiles of 3^8 at once, one per group of three waves (its 3^p tiles split
    // evenly into three runs).  4-byte elements: one tile of 3^9 at a time
    // by all nine waves, and two workgroups per CU.
    static constexpr int GROUPS = sizeof(T) == 4 ? 1 : 3, GNT = NT / GROUPS;
    static constexpr int TILE_LDS = FusedCfg<KMAX>::LDS;
    // one LDS buffer serves the fused tiles of all groups and the two-axis
    // wave passes
    static constexpr int LDS = cmax(GROUPS * TILE_LDS, cmax(PassCfg<4, 2, 1>::LDS, PassCfg<3, 2, 1>::LDS));
    static_assert(PassCfg<4, 2, 1>::WAVES == WAVES && PassCfg<2, 2, 1>::LDS <= LDS, "pass shapes");
    static_assert(GNT % 64 == 0, "tile groups of whole waves");
};

__device__ __forceinline__ uint64_t pow3d(int n)
{
    uint64_t r = 1;
    for (int i = 0; i < n; ++i) r *= 3;
    return r;
}

// Full workgroup barrier: orders global memory as well as LDS.
__device__ __forceinline__ void wg_barrier() { __syncthreads(); }

// The fused tile of a pair with no outer axes (K = D).  A function of its
// own (not inlined): its shapes K = 0 .. KMAX would otherwise add to the
// register pressure of the kernel's large-pair path.
template <typename T>
__device__ __attribute__((noinline)) void single_tile(int K, const T* x, const T* y, T* z, T* S)
{
    constexpr int NT = PersistCfg<T>::NT;
    switch (K) {
        case 0: fused_tile<T, 0, NT>(x, y, z, S); break;
        case 1: fused_tile<T, 1, NT>(x, y, z, S); break;
        case 2: fused_tile<T, 2, NT>(x, y, z, S); break;
        case 3: fused_tile<T, 3, NT>(x, y, z, S); break;
        case 4: fused_tile<T, 4, NT>(x, y, z, S); break;
        case 5: fused_tile<T, 5, NT>(x, y, z, S); break;
        case 6: fused_tile<T, 6, NT>(x, y, z, S); break;
        case 7: fused_tile<T, 7, NT>(x, y, z, S); break;
        case 8: fused_tile<T, 8, NT>(x, y, z, S); break;
        default:
            if constexpr (PersistCfg<T>::KMAX >= 9) fused_tile<T, 9, NT>(x, y, z, S);
            break;
    }
}

// The fused stage of a pair with p >= 1 outer axes: tile group g (the
// WAVES / GROUPS waves from g * WAVES / GROUPS on) runs the tiles
// [g, g + 1) * 3^p / GROUPS one after another, with the next tile's rows
// loaded while the current tile is computed.  The groups run the same number
// of tiles with the same code, so they meet at every barrier.
template <typename T>
__device__ __forceinline__ void fused_stage(const T* xt, const T* yt, T* z, int p, int wave, T* S)
{
    using C = PersistCfg<T>;
    constexpr int K = C::KMAX, GNT = C::GNT;
    const int grp = wave / (C::WAVES / C::GROUPS);
    const int gtid = (int)threadIdx.x - grp * GNT;
    T* Sg = S + grp * C::TILE_LDS;
    const uint32_t per = (uint32_t)(pow3d(p) / C::GROUPS);
    uint32_t o = (uint32_t)grp * per;
    const uint32_t end = o + per;
    RowRegs<T, K, GNT> next;
    next.load(xt + ((uint64_t)o << K), yt + ((uint64_t)o << K), gtid);
    for (; o < end; ++o) {
        const RowRegs<T, K, GNT> cur = next;
        if (o + 1 < end) next.load(xt + ((uint64_t)(o + 1) << K), yt + ((uint64_t)(o + 1) << K), gtid);
        lds_barrier();  // the previous tile's reads of S are done
        fused_tile_from<T, K, GNT>(cur, z + (uint64_t)o * pow3c(K), Sg, gtid);
    }
}

// Outer forward group of M <= 3 axes for both operands, every column by this
// workgroup: in [n_hi][2^M][L] -> out [n_hi][3^M][L].  (Groups stay at three
// axes: the 81 values of a four-axis column would not fit the register
// budget that the wave passes leave.)
template <typename T>
__device__ __forceinline__ void fwd_group_all(int M, const T* x, const T* y, T* ox, T* oy, uint32_t n_cols,
                                              uint32_t log2L)
{
    constexpr int NT = PersistCfg<T>::NT;
    for (uint32_t it = threadIdx.x; it < 2 * n_cols; it += NT) {
        const bool op = it >= n_cols;
        const uint32_t c = op ? it - n_cols : it;
        const T* in = op ? y : x;
        T* out = op ? oy : ox;
        switch (M) {
            case 1: fwd_column<T, 1>(in, out, c, log2L); break;
            case 2: fwd_column<T, 2>(in, out, c, log2L); break;
            default: fwd_column<T, 3>(in, out, c, log2L); break;
        }
    }
}

// One outer inverse pass over the pair's z, in place.  Register-only passes
// (mW = 0): each wave takes its own 64-column tiles.  Passes with two wave
// axes: the nine waves take the tiles one after another together.
template <typename T>
__device__ __forceinline__ void inverse_pass(int mR, int mW, T* z, uint64_t L, uint32_t n_hi, int wave, T* S)
{
    constexpr int WAVES = PersistCfg<T>::WAVES;
    const uint32_t tph = (uint32_t)((L + 63) / 64);
    const uint32_t n_t = n_hi * tph;
    if (mW == 0) {
        for (uint32_t t = (uint32_t)wave; t < n_t; t += WAVES) {
            const uint32_t hi = t / tph;
            const uint32_t j = t - hi * tph;
            switch (mR) {
                case 1: inv_tile<T, 1, 0, 1, false, true>(z, z, L, hi, j, 0, nullptr); break;
                case 2: inv_tile<T, 2, 0, 1, false, true>(z, z, L, hi, j, 0, nullptr); break;
                default: inv_tile<T, 3, 0, 1, false, true>(z, z, L, hi, j, 0, nullptr); break;
            }
        }
    } else {
        for (uint32_t t = 0; t < n_t; ++t) {
            const uint32_t hi = t / tph;
            const uint32_t j = t - hi * tph;
            lds_barrier();  // the previous tile's reads of S are done
            switch (mR) {
                case 2: inv_tile<T, 2, 2, 1, false, true>(z, z, L, hi, j, wave, S); break;
                case 3: inv_tile<T, 3, 2, 1, false, true>(z, z, L, hi, j, wave, S); break;
                default: inv_tile_r4<T, 2, false, true>(z, z, L, hi, j, wave, S); break;
            }
        }
    }
}

// The whole single-pair path of one pair by this workgroup.
template <typename T>
__device__ __forceinline__ void run_pair(const PairPlan& pp, int D, const T* x, const T* y, T* z, T* slot, T* S)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (pp.p == 0) {
        single_tile<T>(pp.K, x, y, z, S);
        return;
    }
    // outer forward groups, ascending; the last lands in x~ / y~
    T* xt = slot;
    T* yt = xt + pp.xt_elems;
    T* xtmp = yt + pp.xt_elems;
    T* ytmp = xtmp + pp.tmp_elems;
    const T* cx = x;
    const T* cy = y;
    int a = 0;
    for (int i = 0; i < pp.n_fwd; ++i) {
        const int M = pp.fwd[i];
        const bool to_xt = ((pp.n_fwd - 1 - i) & 1) == 0;
        T* ox = to_xt ? xt : xtmp;
        T* oy = to_xt ? yt : ytmp;
        const uint32_t log2L = (uint32_t)(D - a - M);
        fwd_group_all<T>(M, cx, cy, ox, oy, (uint32_t)(pow3d(a) << log2L), log2L);
        wg_barrier();
        cx = ox;
        cy = oy;
        a += M;
    }
    // fused inner tiles (a pair with outer axes has K = KMAX)
    fused_stage<T>(xt, yt, z, pp.p, wave, S);
    wg_barrier();
    // outer inverse passes, in place
    for (int i = 0; i < pp.n_inv; ++i) {
        const int ia = pp.inv_a[i], mR = pp.inv_r[i], mW = pp.inv_w[i];
        inverse_pass<T>(mR, mW, z, pow3d(D - ia - mR - mW), (uint32_t)pow3d(ia), wave, S);
        wg_barrier();
    }
}

// 4-byte elements: at most 96 registers, so that two workgroups share a CU.
template <typename T>
__global__ __launch_bounds__(PAIR_NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1)))
void k_pairs_persistent(const T* __restrict__ x, const T* __restrict__ y, T* z, T* ws, uint64_t slot_elems,
                        const PairTask* __restrict__ tasks, const PairPlan* __restrict__ plans, uint32_t n_pairs,
                        uint32_t* counters)
{
    __shared__ T S[PersistCfg<T>::LDS];
    __shared__ uint32_t s_ticket;
    T* slot = ws + (uint64_t)blockIdx.x * slot_elems;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = atomicAdd(&counters[0], 1u);
        wg_barrier();
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
        if (t >= n_pairs) break;  // uniform: every wave leaves together
        const PairTask task = tasks[t];
        run_pair<T>(plans[task.D], (int)task.D, x + task.x_off, y + task.x_off, z + task.z_off, slot, S);
        wg_barrier();  // this pair's stores are done before the slot and S are reused
    }
    if (threadIdx.x == 0) {
        // each workgroup counts itself out once, after its last ticket; the
        // last one to do so resets both counters for the next launch
        const uint32_t out = atomicAdd(&counters[1], 1u);
        if (out + 1 == gridDim.x) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

// ------------------------------------------------------------------ host
PairPlan pair_plan(int D, int dtype, int fwd_max, int inv_max)
{
    PairPlan pp;
    const int kmax = pair_kmax(dtype_size(dtype));
    const int K = D < kmax ? D : kmax;
    fwd_max = fwd_max < 2 ? 2 : (fwd_max > 3 ? 3 : fwd_max);
    inv_max = inv_max < 2 ? 2 : (inv_max > 6 ? 6 : inv_max);
    pp.K = (uint8_t)K;
    pp.p = (uint8_t)(D - K);
    if (pp.p == 0) return pp;
    // outer forward groups of at most fwd_max axes, balanced; stage i lands
    // in x~ when an even number of stages follow it, else in the staging region
    const int n = (pp.p + fwd_max - 1) / fwd_max;
    int left = pp.p, done = 0;
    for (int i = 0; i < n; ++i) {
        const int M = (left + (n - i) - 1) / (n - i);
        pp.fwd[i] = (uint8_t)M;
        done += M;
        left -= M;
        const uint64_t e = pow3u(done) << (D - done);
        if (((n - 1 - i) & 1) == 1 && e > pp.tmp_elems) pp.tmp_elems = (uint32_t)e;
    }
    pp.n_fwd = (uint8_t)n;
    pp.xt_elems = (uint32_t)(pow3u(pp.p) << K);
    // inverse groups of at most inv_max axes from the top: six axes as 4 + 2
    // (streamed thirds), five as 3 + 2, four as 2 + 2, up to three in
    // registers only
    int top = pp.p;
    while (top > 0) {
        const int m = top < inv_max ? top : inv_max;
        const int base = top - m;
        const int r = m == 6 ? 4 : (m == 5 ? 3 : (m == 4 ? 2 : m));
        pp.inv_a[pp.n_inv] = (uint8_t)base;
        pp.inv_r[pp.n_inv] = (uint8_t)r;
        pp.inv_w[pp.n_inv] = (uint8_t)(m - r);
        ++pp.n_inv;
        top = base;
    }
    return pp;
}

uint64_t pair_slot_elems(const PairPlan& pp) { return pp.p == 0 ? 0 : 2ull * (pp.xt_elems + pp.tmp_elems); }

double pair_alg_bytes(const PairPlan& pp, int D, size_t es)
{
    const double e = (double)es;
    if (pp.p == 0) return (2.0 * (1ull << D) + (double)pow3u(D)) * e;
    double b = 0;
    int a = 0;
    for (int i = 0; i < pp.n_fwd; ++i) {
        const int M = pp.fwd[i];
        const double cols = (double)pow3u(a) * (double)(1ull << (D - a - M));
        b += 2.0 * cols * ((1 << M) + pow3c(M)) * e;
        a += M;
    }
    b += (double)pow3u(pp.p) * (2.0 * (1 << pp.K) + pow3c(pp.K)) * e;
    for (int i = 0; i < pp.n_inv; ++i) {
        const int m = pp.inv_r[i] + pp.inv_w[i];
        const double TM = pow3c(m);
        b += (double)pow3u(D) / TM * (TM + TM - (1 << m)) * e;
    }
    return b;
}

template <typename T>
static const void* pairs_kernel()
{
    return reinterpret_cast<const void*>(&k_pairs_persistent<T>);
}

static const void* kernel_for(int dtype)
{
    switch (dtype) {
        case HC_F64: return pairs_kernel<double>();
        case HC_F32: return pairs_kernel<float>();
        default: return pairs_kernel<uint64_t>();
    }
}

int pairs_per_cu(int dtype, int* per_cu)
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel_for(dtype), PAIR_NT, 0);
    if (e != hipSuccess) return hip_fail(e, "persistent kernel occupancy");
    *per_cu = n > 0 ? n : 1;
    return HC_OK;
}

int launch_pairs_persistent(int dtype, const void* x, const void* y, void* z, void* ws, uint64_t slot_elems,
                            const PairTask* tasks, const PairPlan* plans, uint32_t n_pairs, uint32_t* counters,
                            uint32_t grid, hipStream_t s)
{
    switch (dtype) {
        case HC_F64:
            k_pairs_persistent<double><<<grid, PAIR_NT, 0, s>>>((const double*)x, (const double*)y, (double*)z,
                                                               (double*)ws, slot_elems, tasks, plans, n_pairs,
                                                               counters);
            break;
        case HC_F32:
            k_pairs_persistent<float><<<grid, PAIR_NT, 0, s>>>((const float*)x, (const float*)y, (float*)z,
                                                              (float*)ws, slot_elems, tasks, plans, n_pairs,
                                                              counters);
            break;
        default:
            k_pairs_persistent<uint64_t><<<grid, PAIR_NT, 0, s>>>((const uint64_t*)x, (const uint64_t*)y,
                                                                 (uint64_t*)z, (uint64_t*)ws, slot_elems, tasks,
                                                                 plans, n_pairs, counters);
            break;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HC_OK : hip_fail(e, "persistent kernel launch");
}

}  // namespace hc
