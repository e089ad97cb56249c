// Host side of libhc: argument validation, planning (fused depth, axis
// groups), workspace layout and kernel launches.  See include/hc.h for the
// contract of every entry point.
#include "hc.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "hc_internal.hpp"
#include "hc_kernels.hpp"

namespace hc {

// ------------------------------------------------------- logging, ranges
bool log_on()
{
    static const bool on = [] {
        const char* s = getenv("HC_LOG");
        return s && *s && strcmp(s, "0") != 0;
    }();
    return on;
}

void hc_log(const char* fmt, ...)
{
    if (!log_on()) return;
    char buf[8192];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    fprintf(stderr, "[hc] %s\n", buf);
}

TraceRange::TraceRange(const char* fmt, ...)
{
    char buf[160];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    roctxRangePushA(buf);
}

TraceRange::~TraceRange() { roctxRangePop(); }

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(HC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

uint64_t pow3u(int n)
{
    uint64_t r = 1;
    for (int i = 0; i < n; ++i) r *= 3;
    return r;
}

size_t dtype_size(int dtype)
{
    switch (dtype) {
        case HC_F64: return 8;
        case HC_F32: return 4;
        case HC_I64: return 8;
        default: return 0;
    }
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb)
{
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

bool misaligned(const void* p, size_t align)
{
    return p && ((uintptr_t)p & (align - 1)) != 0;
}

// ------------------------------------------------------------------ device
static std::mutex g_dev_mu;
static int g_cu_count[64];

int device_cus(int* cus)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(HC_ERR_NO_DEVICE, "no HIP device available");
    }
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (dev < 0 || dev >= 64) return fail(HC_ERR_NO_DEVICE, "device index %d unsupported", dev);
    if (g_cu_count[dev] == 0) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        g_cu_count[dev] = v > 0 ? v : 1;
    }
    *cus = g_cu_count[dev];
    return HC_OK;
}


// ---------------------------------------------------------------- profiler
// While enabled, each launch is bracketed by two events on its stream and
// tagged with a name and its algorithmic bytes.
struct ProfRec {
    char name[48];
    double bytes;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static std::atomic<bool> g_prof_on{false};
static thread_local int g_quiet = 0;  // > 0 inside a CaptureScope

CaptureScope::CaptureScope() { ++g_quiet; }
CaptureScope::~CaptureScope() { --g_quiet; }
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t pooled_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

LaunchScope::LaunchScope(hipStream_t s, double bytes, const char* fmt, ...) : stream_(s), on_(false), idx_(0)
{
    if (!g_prof_on || g_quiet > 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    ProfRec r;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(r.name, sizeof(r.name), fmt, ap);
    va_end(ap);
    r.bytes = bytes;
    r.a = pooled_event();
    r.b = pooled_event();
    if (!r.a || !r.b) {
        if (r.a) g_event_pool.push_back(r.a);
        if (r.b) g_event_pool.push_back(r.b);
        return;
    }
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    g_prof.push_back(r);
    idx_ = g_prof.size() - 1;
    on_ = true;
}

LaunchScope::~LaunchScope()
{
    if (!on_) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (idx_ < g_prof.size()) (void)hipEventRecord(g_prof[idx_].b, stream_);
}

// ------------------------------------------------------------------ plans
int max_fused_depth(int dtype)
{
    // One fused tile of 3^K elements must fit LDS with room for two or more
    // workgroups per CU: 3^8 x 8 B = 52.5 KB, 3^9 x 4 B = 78.7 KB.
    return dtype_size(dtype) == 4 ? 9 : 8;
}

// Default fused depth.  4-byte elements allow K = 9, but the K = 8 tile runs
// at a higher occupancy and is faster, unless K = 9 saves a whole outer pass
// or K = 8 would leave a last pass of 5 axes (measured slower than the K = 9
// plan at D = 13; even at D = 19).
static int default_depth(int D, int dtype)
{
    const int kmax = max_fused_depth(dtype);
    if (kmax != 9 || D < 9) return kmax;
    const int p8 = D - 8, p9 = D - 9;
    if ((p9 + 5) / 6 < (p8 + 5) / 6 || p8 % 6 == 5) return 9;
    return 8;
}

// Groups of the outer axes [0, top) for inverse passes, in the forward
// inverse's execution order (descending): groups of at most max_m axes,
// filled from the top, of which at most reg in registers.
static std::vector<InvPass> inverse_groups(int top, int reg, int max_m)
{
    std::vector<InvPass> out;
    while (top > 0) {
        const int m = top < max_m ? top : max_m;
        const int a = top - m;
        InvPass ip;
        ip.a = a;
        ip.mR = m < reg ? m : reg;
        ip.mW = m - ip.mR;
        // four and five axes run faster as 3 register axes plus 1 or 2 wave
        // axes than as 4 + 0 and 4 + 1
        if ((m == 4 || m == 5) && ip.mR == 4) {
            ip.mR = 3;
            ip.mW = m - 3;
        }
        out.push_back(ip);
        top = a;
    }
    return out;
}

Plan make_plan(int D, int dtype, const PlanOpts& o)
{
    Plan P;
    P.D = D;
    P.dtype = dtype;
    P.esize = dtype_size(dtype);
    const int kmax = max_fused_depth(dtype);
    int K = o.fused_depth > 0 ? o.fused_depth : default_depth(D, dtype);
    if (K > kmax) K = kmax;
    if (K > D) K = D;
    P.K = K;
    P.p = D - K;
    P.grid_per_cu = o.grid_per_cu;
    P.fused_nt = o.fused_nt == 512 ? 512 : 256;
    P.reg_cw = (o.reg_cw == 1 || o.reg_cw == 2) ? o.reg_cw : 4;
    P.n2 = 1ull << D;
    P.n3 = pow3u(D);
    // outer forward groups (ascending), at most 4 axes each, balanced
    if (P.p > 0) {
        const int n = (P.p + 3) / 4;
        int left = P.p;
        for (int i = 0; i < n; ++i) {
            const int m = (left + (n - i) - 1) / (n - i);
            P.k1.push_back(m);
            left -= m;
        }
    }
    // outer inverse passes (descending), groups of at most max_m axes, of
    // which at most reg axes in registers and at most 2 across waves
    const int reg = o.inv_reg > 0 ? cmin(o.inv_reg, 4) : 4;
    const int max_m = cmin(o.inv_group_max > 0 ? o.inv_group_max : 6, reg + 2);
    P.inv = inverse_groups(P.p, reg, max_m);
    // backward: the last bwd_tail outer axes get G^T inside the fused
    // adjoint tile; the passes cover the axes above them
    P.bwd_tail = P.p < 2 ? P.p : 2;
    if (o.bwd_tail >= 0 && o.bwd_tail < P.bwd_tail) P.bwd_tail = o.bwd_tail;
    P.inv_bwd = inverse_groups(P.p - P.bwd_tail, reg, max_m);
    // workspace: K1 stages ping-pong between the x~ region and a staging region
    P.xt_elems = P.p > 0 ? pow3u(P.p) << K : 0;
    P.tmp_elems = 0;
    {
        const int n = (int)P.k1.size();
        int a = 0;
        for (int i = 0; i < n; ++i) {
            a += P.k1[i];
            const uint64_t e = pow3u(a) << (D - a);
            if (((n - 1 - i) & 1) == 1 && e > P.tmp_elems) P.tmp_elems = e;
        }
    }
    return P;
}

PlanOpts default_opts()
{
    PlanOpts o;
    if (const char* s = getenv("HC_FUSED_K")) o.fused_depth = atoi(s);
    if (const char* s = getenv("HC_INV_MAXM")) o.inv_group_max = atoi(s);
    if (const char* s = getenv("HC_INV_REG")) o.inv_reg = atoi(s);
    if (const char* s = getenv("HC_GRID_PER_CU")) o.grid_per_cu = atoi(s);
    if (const char* s = getenv("HC_BWD_TAIL")) o.bwd_tail = atoi(s);
    if (const char* s = getenv("HC_FUSED_NT")) o.fused_nt = atoi(s);
    if (const char* s = getenv("HC_REG_CW")) o.reg_cw = atoi(s);
    return o;
}

size_t plan_ws_bytes(const Plan& P, int batch)
{
    if (P.p == 0) return 0;
    return (size_t)batch * 2 * (P.xt_elems + P.tmp_elems) * P.esize;
}

// Backward workspace per item: W (3^D), x~, y~ and staging, gx~, gy~ and the
// F^T staging (largest intermediate after the first F^T group).
size_t plan_bwd_ws_elems(const Plan& P, uint64_t* w_e, uint64_t* gtmp_e)
{
    *w_e = P.p > 0 ? P.n3 : 0;
    *gtmp_e = 0;
    if (P.p > 0 && P.k1.size() > 1) {
        // F^T groups run in the reverse order of the forward groups
        const int m_last = P.k1.back();
        const int a = P.p - m_last;
        *gtmp_e = pow3u(a) << (P.D - a);
    }
    return 0;
}

size_t plan_bwd_ws_bytes(const Plan& P, int batch)
{
    if (P.p == 0) return 0;
    uint64_t w_e, g_e;
    plan_bwd_ws_elems(P, &w_e, &g_e);
    const uint64_t per = w_e + 2 * (P.xt_elems + P.tmp_elems) + 2 * (P.xt_elems + g_e);
    return (size_t)batch * per * P.esize;
}

// ------------------------------------------------------------- launches
template <typename T, int M>
static void launch_fwd_pass_m(const T* in0, const T* in1, T* out0, T* out1, BMap in_bs, BMap out_bs,
                              uint32_t n_cols, uint32_t log2L, int batch, int ops, hipStream_t s)
{
    constexpr int NT = 256;
    dim3 grid((n_cols + NT - 1) / NT, batch, ops);
    const double bytes = (double)ops * batch * n_cols * ((1 << M) + pow3c(M)) * sizeof(T);
    LaunchScope scope(s, bytes, "fwd_pass<%s,M=%d>", tname<T>(), M);
    k_fwd_pass<T, M, NT><<<grid, NT, 0, s>>>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L);
}

template <typename T>
int launch_fwd_pass(int M, const T* in0, const T* in1, T* out0, T* out1, BMap in_bs, BMap out_bs,
                     uint32_t n_cols, uint32_t log2L, int batch, int ops, hipStream_t s)
{
    switch (M) {
        case 1: launch_fwd_pass_m<T, 1>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, ops, s); break;
        case 2: launch_fwd_pass_m<T, 2>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, ops, s); break;
        case 3: launch_fwd_pass_m<T, 3>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, ops, s); break;
        case 4: launch_fwd_pass_m<T, 4>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, ops, s); break;
        default: return fail(HC_ERR_UNSUPPORTED, "no forward pass for %d axes", M);
    }
    return HC_OK;
}

template <typename T, int M>
static void launch_fwd_adj_pass_m(const T* in0, const T* in1, T* out0, T* out1, BMap in_bs, BMap out_bs,
                                  uint32_t n_cols, uint32_t log2L, int batch, hipStream_t s)
{
    constexpr int NT = 256;
    dim3 grid((n_cols + NT - 1) / NT, batch, 2);
    const int ops = (out0 ? 1 : 0) + (out1 ? 1 : 0);
    const double bytes = (double)ops * batch * n_cols * ((1 << M) + pow3c(M)) * sizeof(T);
    LaunchScope scope(s, bytes, "fwd_adj_pass<%s,M=%d>", tname<T>(), M);
    k_fwd_adj_pass<T, M, NT><<<grid, NT, 0, s>>>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L);
}

template <typename T>
int launch_fwd_adj_pass(int M, const T* in0, const T* in1, T* out0, T* out1, BMap in_bs, BMap out_bs,
                         uint32_t n_cols, uint32_t log2L, int batch, hipStream_t s)
{
    switch (M) {
        case 1: launch_fwd_adj_pass_m<T, 1>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, s); break;
        case 2: launch_fwd_adj_pass_m<T, 2>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, s); break;
        case 3: launch_fwd_adj_pass_m<T, 3>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, s); break;
        case 4: launch_fwd_adj_pass_m<T, 4>(in0, in1, out0, out1, in_bs, out_bs, n_cols, log2L, batch, s); break;
        default: return fail(HC_ERR_UNSUPPORTED, "no adjoint forward pass for %d axes", M);
    }
    return HC_OK;
}

// Workgroups for n_tiles tiles.  per_cu == 0: one tile per workgroup (short
// workgroups that stream one tile and exit keep HBM busiest); the count is
// rounded up to a multiple of 8 so that the XCD-aware walk hands every XCD
// one contiguous chunk.  per_cu > 0: a persistent grid of at most that many
// workgroups per CU, each looping over tiles.
uint32_t tile_grid(uint64_t n_tiles, int cus, int per_cu)
{
    uint64_t g = n_tiles;
    if (per_cu > 0) {
        const uint64_t cap = (uint64_t)cus * per_cu;
        if (g > cap) g = cap;
        if (g >= 8) g &= ~7ull;
    } else if (g >= 8) {
        g = (g + 7) & ~7ull;
    }
    return (uint32_t)(g ? g : 1);
}

template <typename T, int K, int NT>
static void launch_fused_k(const T* xt, const T* yt, T* z, BMap in_bs, BMap z_bs, uint32_t n_tiles,
                           int batch, int cus, int per_cu, hipStream_t s)
{
    dim3 grid(tile_grid(n_tiles, cus, per_cu), batch, 1);
    const double bytes = (double)batch * n_tiles * (2.0 * (1 << K) + pow3c(K)) * sizeof(T);
    LaunchScope scope(s, bytes, "fused_inner<%s,K=%d>", tname<T>(), K);
    k_fused_inner<T, K, NT><<<grid, NT, 0, s>>>(xt, yt, z, in_bs, z_bs, n_tiles);
}

template <typename T, int K>
static int launch_fused_nt(int nt, const T* xt, const T* yt, T* z, BMap in_bs, BMap z_bs, uint32_t n_tiles,
                           int batch, int cus, int per_cu, hipStream_t s)
{
    if (nt == 256) launch_fused_k<T, K, 256>(xt, yt, z, in_bs, z_bs, n_tiles, batch, cus, per_cu, s);
    else if (nt == 512) launch_fused_k<T, K, 512>(xt, yt, z, in_bs, z_bs, n_tiles, batch, cus, per_cu, s);
    else return fail(HC_ERR_UNSUPPORTED, "no fused tile with %d threads", nt);
    return HC_OK;
}

template <typename T>
int launch_fused(int K, int nt, const T* xt, const T* yt, T* z, BMap in_bs, BMap z_bs, uint32_t n_tiles,
                 int batch, int cus, int per_cu, hipStream_t s)
{
#define HC_FUSED(KK) \
    case KK: return launch_fused_nt<T, KK>(nt, xt, yt, z, in_bs, z_bs, n_tiles, batch, cus, per_cu, s);
    switch (K) {
        HC_FUSED(0) HC_FUSED(1) HC_FUSED(2) HC_FUSED(3) HC_FUSED(4) HC_FUSED(5) HC_FUSED(6) HC_FUSED(7)
        HC_FUSED(8)
        case 9:
            if constexpr (sizeof(T) == 4)
                return launch_fused_nt<T, 9>(nt, xt, yt, z, in_bs, z_bs, n_tiles, batch, cus, per_cu, s);
            return fail(HC_ERR_UNSUPPORTED, "no fused tile of 9 axes for 8-byte elements");
        default: return fail(HC_ERR_UNSUPPORTED, "no fused tile of %d axes", K);
    }
#undef HC_FUSED
}

template <typename T, int K, int TAIL>
static void launch_fused_adj_k(const T* xt, const T* yt, const T* w, T* gxt, T* gyt, BMap in_bs,
                               BMap w_bs, BMap g_bs, uint32_t n_tiles, int batch, int cus, int per_cu,
                               hipStream_t s)
{
    constexpr int NT = 256;
    dim3 grid(tile_grid(n_tiles, cus, per_cu), batch, 1);
    const int ops = (gxt ? 1 : 0) + (gyt ? 1 : 0);
    // every w row is counted once: the sibling rows the tail axes combine
    // are the rows of neighbouring tiles (the same data, re-read from cache)
    const double bytes = (double)batch * n_tiles * ((2.0 + ops) * (1 << K) + pow3c(K)) * sizeof(T);
    LaunchScope scope(s, bytes, "fused_inner_adj<%s,K=%d,t=%d>", tname<T>(), K, TAIL);
    k_fused_inner_adj<T, K, NT, TAIL><<<grid, NT, 0, s>>>(xt, yt, w, gxt, gyt, in_bs, w_bs, g_bs, n_tiles);
}

template <typename T, int K>
static int launch_fused_adj_t(int tail, const T* xt, const T* yt, const T* w, T* gxt, T* gyt, BMap in_bs,
                              BMap w_bs, BMap g_bs, uint32_t n_tiles, int batch, int cus, int per_cu,
                              hipStream_t s)
{
    switch (tail) {
        case 0: launch_fused_adj_k<T, K, 0>(xt, yt, w, gxt, gyt, in_bs, w_bs, g_bs, n_tiles, batch, cus, per_cu, s); break;
        case 1: launch_fused_adj_k<T, K, 1>(xt, yt, w, gxt, gyt, in_bs, w_bs, g_bs, n_tiles, batch, cus, per_cu, s); break;
        case 2: launch_fused_adj_k<T, K, 2>(xt, yt, w, gxt, gyt, in_bs, w_bs, g_bs, n_tiles, batch, cus, per_cu, s); break;
        default: return fail(HC_ERR_UNSUPPORTED, "no adjoint fused tile with %d tail axes", tail);
    }
    return HC_OK;
}

template <typename T>
int launch_fused_adj(int K, int tail, const T* xt, const T* yt, const T* w, T* gxt, T* gyt, BMap in_bs,
                     BMap w_bs, BMap g_bs, uint32_t n_tiles, int batch, int cus, int per_cu, hipStream_t s)
{
#define HC_ADJ(KK) \
    case KK: return launch_fused_adj_t<T, KK>(tail, xt, yt, w, gxt, gyt, in_bs, w_bs, g_bs, n_tiles, batch, cus, per_cu, s);
    switch (K) {
        HC_ADJ(0) HC_ADJ(1) HC_ADJ(2) HC_ADJ(3) HC_ADJ(4) HC_ADJ(5) HC_ADJ(6) HC_ADJ(7) HC_ADJ(8)
        case 9:
            if constexpr (sizeof(T) == 4)
                return launch_fused_adj_t<T, 9>(tail, xt, yt, w, gxt, gyt, in_bs, w_bs, g_bs, n_tiles, batch, cus,
                                                per_cu, s);
            return fail(HC_ERR_UNSUPPORTED, "no adjoint fused tile of 9 axes for 8-byte elements");
        default: return fail(HC_ERR_UNSUPPORTED, "no adjoint fused tile of %d axes", K);
    }
#undef HC_ADJ
}

template <typename T, int mR, int mW, int CW, bool ADJ>
static void launch_pass_v(const T* src, T* dst, BMap src_bs, BMap dst_bs, uint64_t L, uint32_t n_hi,
                          int batch, int cus, int per_cu, hipStream_t s)
{
    // register-only passes take CW waves x 64 columns per workgroup; passes
    // with a wave part take one wave per digit vector of that part
    using PC = PassCfg<mR, mW, CW>;
    const uint32_t tiles_per_hi = (uint32_t)((L + PC::COLS - 1) / PC::COLS);
    const uint64_t n_tiles = (uint64_t)tiles_per_hi * n_hi;
    // the streamed-thirds tile runs one tile per workgroup
    dim3 grid(tile_grid(n_tiles, cus, PC::THIRDS ? 0 : per_cu), batch, 1);
    // reads every entry; writes the entries the map changes (all if out of place)
    constexpr int TM = pow3c(mR + mW);
    const double n_cols = (double)batch * n_hi * L;
    const double writes = src != dst ? TM : (ADJ ? TM - 1 : TM - (1 << (mR + mW)));
    const double bytes = n_cols * (TM + writes) * sizeof(T);
    LaunchScope scope(s, bytes, "%s<%s,%d+%d>", ADJ ? "inv_adj_pass" : "inv_pass", tname<T>(), mR, mW);
    // in place (the same buffer and the same per-item offsets): entries the
    // map leaves unchanged are not written back
    if (src == dst && src_bs.stride == dst_bs.stride && src_bs.table == dst_bs.table)
        k_inv_pass<T, mR, mW, CW, ADJ, true><<<grid, PC::NT, 0, s>>>(src, dst, src_bs, dst_bs, L, tiles_per_hi,
                                                                     (uint32_t)n_tiles);
    else
        k_inv_pass<T, mR, mW, CW, ADJ, false><<<grid, PC::NT, 0, s>>>(src, dst, src_bs, dst_bs, L, tiles_per_hi,
                                                                      (uint32_t)n_tiles);
}

// cw: 64-column groups per workgroup of a register-only pass (1, 2 or 4);
// passes with a wave part always take one.
template <typename T, bool ADJ>
int launch_pass(const InvPass& ip, int cw, const T* src, T* dst, BMap src_bs, BMap dst_bs, uint64_t L,
                uint32_t n_hi, int batch, int cus, int per_cu, hipStream_t s)
{
#define HC_PASS(R, W, C) \
    if (ip.mR == R && ip.mW == W && (W > 0 || cw == C)) { \
        launch_pass_v<T, R, W, C, ADJ>(src, dst, src_bs, dst_bs, L, n_hi, batch, cus, per_cu, s); \
        return HC_OK; \
    }
    HC_PASS(1, 0, 4) HC_PASS(2, 0, 4) HC_PASS(3, 0, 4) HC_PASS(4, 0, 4)
    HC_PASS(1, 0, 2) HC_PASS(2, 0, 2) HC_PASS(3, 0, 2) HC_PASS(4, 0, 2)
    HC_PASS(1, 0, 1) HC_PASS(2, 0, 1) HC_PASS(3, 0, 1) HC_PASS(4, 0, 1)
    HC_PASS(1, 1, 1) HC_PASS(2, 1, 1) HC_PASS(3, 1, 1) HC_PASS(4, 1, 1)
    HC_PASS(1, 2, 1) HC_PASS(2, 2, 1) HC_PASS(3, 2, 1) HC_PASS(4, 2, 1)
#undef HC_PASS
    return fail(HC_ERR_UNSUPPORTED, "no inverse pass with %d register and %d wave axes (%d column groups)", ip.mR,
                ip.mW, cw);
}

// ------------------------------------------------------------ forward run
template <typename T>
int run_forward(const Plan& P, const T* x, const T* y, T* z, int batch, T* ws, int cus, hipStream_t s, BMap x_map,
                BMap z_map, const LastPass* last)
{
    const int D = P.D, K = P.K;
    int rc = HC_OK;
    if (P.p == 0) {
        rc = launch_fused<T>(K, P.fused_nt, x, y, z, x_map, z_map, 1, batch, cus, P.grid_per_cu, s);
        if (rc != HC_OK) return rc;
    } else {
        T* xt = ws;
        T* yt = xt + (uint64_t)batch * P.xt_elems;
        T* xtmp = yt + (uint64_t)batch * P.xt_elems;
        T* ytmp = xtmp + (uint64_t)batch * P.tmp_elems;
        // outer forward, ascending groups; the last group lands in x~ / y~
        const int n = (int)P.k1.size();
        const T* cx = x;
        const T* cy = y;
        BMap c_bs = x_map;
        int a = 0;
        for (int i = 0; i < n; ++i) {
            const int M = P.k1[i];
            const bool to_xt = ((n - 1 - i) & 1) == 0;
            T* ox = to_xt ? xt : xtmp;
            T* oy = to_xt ? yt : ytmp;
            const uint64_t o_bs = to_xt ? P.xt_elems : P.tmp_elems;
            const int log2L = D - a - M;
            const uint64_t n_cols = pow3u(a) << log2L;
            rc = launch_fwd_pass<T>(M, cx, cy, ox, oy, c_bs, o_bs, (uint32_t)n_cols, (uint32_t)log2L, batch, 2, s);
            if (rc != HC_OK) return rc;
            cx = ox;
            cy = oy;
            c_bs = o_bs;
            a += M;
        }
        rc = launch_fused<T>(K, P.fused_nt, xt, yt, z, P.xt_elems, z_map, (uint32_t)pow3u(P.p), batch, cus,
                             P.grid_per_cu, s);
        if (rc != HC_OK) return rc;
        for (size_t i = 0; i < P.inv.size(); ++i) {
            const InvPass& ip = P.inv[i];
            const int m = ip.mR + ip.mW;
            const uint64_t L = pow3u(D - ip.a - m);
            const uint32_t n_hi = (uint32_t)pow3u(ip.a);
            if (last && i + 1 == P.inv.size()) {
                rc = last->launch(*last, ip, z, z_map, L, n_hi, batch, cus, s);
                if (rc == HC_OK) {
                    last->taken = true;
                    continue;
                }
                if (rc != HC_ERR_UNSUPPORTED) return rc;
            }
            rc = launch_pass<T, false>(ip, P.reg_cw, z, z, z_map, z_map, L, n_hi, batch, cus, P.grid_per_cu, s);
            if (rc != HC_OK) return rc;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return HC_OK;
}

// ----------------------------------------------------------- backward run
template <typename T>
int run_backward(const Plan& P, const T* x, const T* y, const T* gz, uint64_t gz_bs, T* gx, T* gy, int batch,
                 T* ws, int cus, hipStream_t s)
{
    const int D = P.D, K = P.K;
    int rc = HC_OK;
    if (P.p == 0) {
        rc = launch_fused_adj<T>(K, 0, x, y, gz, gx, gy, P.n2, gz_bs, P.n2, 1, batch, cus, P.grid_per_cu, s);
        if (rc != HC_OK) return rc;
    } else {
        uint64_t w_e, g_e;
        plan_bwd_ws_elems(P, &w_e, &g_e);
        T* W = ws;
        T* xt = W + (uint64_t)batch * w_e;
        T* yt = xt + (uint64_t)batch * P.xt_elems;
        T* xtmp = yt + (uint64_t)batch * P.xt_elems;
        T* ytmp = xtmp + (uint64_t)batch * P.tmp_elems;
        T* gxt = ytmp + (uint64_t)batch * P.tmp_elems;
        T* gyt = gxt + (uint64_t)batch * P.xt_elems;
        T* gxtmp = gyt + (uint64_t)batch * P.xt_elems;
        T* gytmp = gxtmp + (uint64_t)batch * g_e;
        // 1. G^T on the outer axes above the tail, ascending; the first pass
        // reads grad_z.  Without such passes the fused tiles read grad_z
        // itself.  A broadcast grad_z (batch stride 0) gives every item the
        // same W: it is computed once, on all outer axes (no tail), and the
        // tiles of all items read it.
        const bool shared = gz_bs == 0;
        const int tail = shared ? 0 : P.bwd_tail;
        const std::vector<InvPass>& groups = shared ? P.inv : P.inv_bwd;
        const int w_items = shared ? 1 : batch;
        const T* src = gz;
        uint64_t src_bs = gz_bs;
        for (int i = (int)groups.size() - 1; i >= 0; --i) {
            const InvPass& ip = groups[i];
            const int m = ip.mR + ip.mW;
            const uint64_t L = pow3u(D - ip.a - m);
            const uint32_t n_hi = (uint32_t)pow3u(ip.a);
            rc = launch_pass<T, true>(ip, P.reg_cw, src, W, src_bs, P.n3, L, n_hi, w_items, cus, P.grid_per_cu, s);
            if (rc != HC_OK) return rc;
            src = W;
            src_bs = P.n3;
        }
        // 2. outer forward of x and y (recomputed, as in the forward)
        const int n = (int)P.k1.size();
        const T* cx = x;
        const T* cy = y;
        uint64_t c_bs = P.n2;
        int a = 0;
        for (int i = 0; i < n; ++i) {
            const int M = P.k1[i];
            const bool to_xt = ((n - 1 - i) & 1) == 0;
            T* ox = to_xt ? xt : xtmp;
            T* oy = to_xt ? yt : ytmp;
            const uint64_t o_bs = to_xt ? P.xt_elems : P.tmp_elems;
            const int log2L = D - a - M;
            const uint64_t n_cols = pow3u(a) << log2L;
            rc = launch_fwd_pass<T>(M, cx, cy, ox, oy, c_bs, o_bs, (uint32_t)n_cols, (uint32_t)log2L, batch, 2, s);
            if (rc != HC_OK) return rc;
            cx = ox;
            cy = oy;
            c_bs = o_bs;
            a += M;
        }
        // 3. fused inner adjoint (G^T on the tail axes and the inner axes):
        // w rows -> gx~, gy~ rows
        const uint64_t w_bs = shared ? 0 : src_bs;
        rc = launch_fused_adj<T>(K, tail, xt, yt, src, gx ? gxt : nullptr, gy ? gyt : nullptr, P.xt_elems,
                                 w_bs, P.xt_elems, (uint32_t)pow3u(P.p), batch, cus, P.grid_per_cu, s);
        if (rc != HC_OK) return rc;
        // 4. F^T on the outer axes, descending groups (reverse of the forward)
        const T* ix = gxt;
        const T* iy = gyt;
        uint64_t i_bs = P.xt_elems;
        int top = P.p;
        for (int i = n - 1; i >= 0; --i) {
            const int M = P.k1[i];
            const int a0 = top - M;  // group [a0, top)
            T* ox;
            T* oy;
            uint64_t o_bs;
            if (i == 0) {
                ox = gx;
                oy = gy;
                o_bs = P.n2;
            } else if (((n - 1 - i) & 1) == 0) {
                ox = gxtmp;
                oy = gytmp;
                o_bs = g_e;
            } else {
                ox = gxt;
                oy = gyt;
                o_bs = P.xt_elems;
            }
            const int log2L = D - top;
            const uint64_t n_cols = pow3u(a0) << log2L;
            rc = launch_fwd_adj_pass<T>(M, gx ? ix : nullptr, gy ? iy : nullptr, gx ? ox : nullptr,
                                        gy ? oy : nullptr, i_bs, o_bs, (uint32_t)n_cols, (uint32_t)log2L, batch, s);
            if (rc != HC_OK) return rc;
            ix = ox;
            iy = oy;
            i_bs = o_bs;
            top = a0;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return HC_OK;
}

template int run_forward<double>(const Plan&, const double*, const double*, double*, int, double*, int, hipStream_t,
                                 BMap, BMap, const LastPass*);
template int run_forward<float>(const Plan&, const float*, const float*, float*, int, float*, int, hipStream_t, BMap,
                                BMap, const LastPass*);
template int run_forward<uint64_t>(const Plan&, const uint64_t*, const uint64_t*, uint64_t*, int, uint64_t*, int,
                                   hipStream_t, BMap, BMap, const LastPass*);
template int run_backward<double>(const Plan&, const double*, const double*, const double*, uint64_t, double*,
                                  double*, int, double*, int, hipStream_t);
template int run_backward<float>(const Plan&, const float*, const float*, const float*, uint64_t, float*, float*,
                                 int, float*, int, hipStream_t);

}  // namespace hc

using namespace hc;

// =================================================================== C ABI
extern "C" {

int hc_abi_version(void) { return HC_ABI_VERSION; }

const char* hc_status_string(int status)
{
    switch (status) {
        case HC_OK: return "ok";
        case HC_ERR_INVALID_ARG: return "invalid argument";
        case HC_ERR_D_RANGE: return "D out of range";
        case HC_ERR_UNSUPPORTED: return "unsupported dtype or configuration";
        case HC_ERR_ALIAS: return "output overlaps an input or the workspace";
        case HC_ERR_MISALIGNED: return "pointer misaligned (data to its element size, workspaces to 16 bytes)";
        case HC_ERR_WORKSPACE: return "workspace missing or too small";
        case HC_ERR_NO_DEVICE: return "no HIP device";
        case HC_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* hc_last_error(void) { return g_last_error.c_str(); }

size_t hc_dtype_size(int dtype) { return dtype_size(dtype); }

uint64_t hc_output_count(int D) { return (D < 0 || D > HC_MAX_D) ? 0 : pow3u(D); }

size_t hc_workspace_bytes(int D, int dtype, int batch)
{
    if (D < 0 || D > HC_MAX_D || dtype_size(dtype) == 0 || batch < 1) return (size_t)-1;
    return plan_ws_bytes(make_plan(D, dtype, default_opts()), batch);
}

size_t hc_backward_workspace_bytes(int D, int dtype, int batch)
{
    if (D < 0 || D > HC_MAX_D || dtype_size(dtype) == 0 || batch < 1) return (size_t)-1;
    return plan_bwd_ws_bytes(make_plan(D, dtype, default_opts()), batch);
}

int hc_convolve_batch(const void* x, const void* y, void* z, int D, int dtype, int batch, void* workspace,
                      size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_convolve_batch D=%d dtype=%d batch=%d", D, dtype, batch);
    return convolve_batch_last(x, y, z, D, dtype, batch, workspace, workspace_bytes, stream, nullptr);
}

}  // extern "C"

int hc::convolve_batch_last(const void* x, const void* y, void* z, int D, int dtype, int batch, void* workspace,
                            size_t workspace_bytes, hipStream_t stream, const LastPass* last)
{
    g_last_error.clear();
    if (!x || !y || !z) return fail(HC_ERR_INVALID_ARG, "x, y and z must be non-null");
    if (D < 0 || D > HC_MAX_D) return fail(HC_ERR_D_RANGE, "D=%d outside [0, %d]", D, HC_MAX_D);
    const size_t es = dtype_size(dtype);
    if (es == 0) return fail(HC_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (batch < 1 || batch > 65535) return fail(HC_ERR_INVALID_ARG, "batch=%d outside [1, 65535]", batch);
    if (misaligned(x, es) || misaligned(y, es) || misaligned(z, es) || misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const Plan P = make_plan(D, dtype, default_opts());
    const size_t in_b = (size_t)batch * P.n2 * es, out_b = (size_t)batch * P.n3 * es;
    const size_t need = plan_ws_bytes(P, batch);
    if (ranges_overlap(z, out_b, x, in_b) || ranges_overlap(z, out_b, y, in_b))
        return fail(HC_ERR_ALIAS, "z overlaps x or y");
    if (need > 0) {
        if (!workspace || workspace_bytes < need)
            return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                        workspace ? workspace_bytes : (size_t)0);
        if (ranges_overlap(z, out_b, workspace, need)) return fail(HC_ERR_ALIAS, "z overlaps the workspace");
        if (ranges_overlap(workspace, need, x, in_b) || ranges_overlap(workspace, need, y, in_b))
            return fail(HC_ERR_ALIAS, "workspace overlaps x or y");
    }
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    switch (dtype) {
        case HC_F64:
            return run_forward<double>(P, (const double*)x, (const double*)y, (double*)z, batch, (double*)workspace,
                                       cus, stream, P.n2, P.n3, last);
        case HC_F32:
            return run_forward<float>(P, (const float*)x, (const float*)y, (float*)z, batch, (float*)workspace, cus,
                                      stream, P.n2, P.n3, last);
        default:
            return run_forward<uint64_t>(P, (const uint64_t*)x, (const uint64_t*)y, (uint64_t*)z, batch,
                                         (uint64_t*)workspace, cus, stream, P.n2, P.n3, last);
    }
}

extern "C" {

int hc_convolve(const void* x, const void* y, void* z, int D, int dtype, void* workspace, size_t workspace_bytes,
                hipStream_t stream)
{
    return hc_convolve_batch(x, y, z, D, dtype, 1, workspace, workspace_bytes, stream);
}

int hc_convolve_backward_batch(const void* x, const void* y, const void* grad_z, int64_t grad_z_stride,
                               void* grad_x, void* grad_y, int D, int dtype, int batch, void* workspace,
                               size_t workspace_bytes, hipStream_t stream)
{
    TraceRange range("hc_convolve_backward_batch D=%d dtype=%d batch=%d", D, dtype, batch);
    g_last_error.clear();
    if (!x || !y || !grad_z) return fail(HC_ERR_INVALID_ARG, "x, y and grad_z must be non-null");
    if (!grad_x && !grad_y) return fail(HC_ERR_INVALID_ARG, "at least one of grad_x, grad_y is required");
    if (D < 0 || D > HC_MAX_D) return fail(HC_ERR_D_RANGE, "D=%d outside [0, %d]", D, HC_MAX_D);
    const size_t es = dtype_size(dtype);
    if (es == 0) return fail(HC_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (dtype == HC_I64) return fail(HC_ERR_UNSUPPORTED, "the backward pass supports float64 and float32 only");
    if (batch < 1 || batch > 65535) return fail(HC_ERR_INVALID_ARG, "batch=%d outside [1, 65535]", batch);
    const Plan P = make_plan(D, dtype, default_opts());
    if (grad_z_stride != 0 && (grad_z_stride < 0 || (uint64_t)grad_z_stride < P.n3))
        return fail(HC_ERR_INVALID_ARG, "grad_z_stride must be 0 or at least 3^D");
    if (misaligned(x, es) || misaligned(y, es) || misaligned(grad_z, es) || misaligned(grad_x, es) ||
        misaligned(grad_y, es) || misaligned(workspace, 16))
        return fail(HC_ERR_MISALIGNED, "data must be aligned to the element size, the workspace to 16 bytes");
    const size_t in_b = (size_t)batch * P.n2 * es;
    const size_t gz_b = (grad_z_stride == 0 ? P.n3 : (size_t)grad_z_stride * (batch - 1) + P.n3) * es;
    const size_t need = plan_bwd_ws_bytes(P, batch);
    const void* ins[3] = {x, y, grad_z};
    const size_t ins_b[3] = {in_b, in_b, gz_b};
    void* outs[2] = {grad_x, grad_y};
    for (void* o : outs) {
        if (!o) continue;
        for (int i = 0; i < 3; ++i)
            if (ranges_overlap(o, in_b, ins[i], ins_b[i])) return fail(HC_ERR_ALIAS, "a gradient overlaps an input");
        if (need && ranges_overlap(o, in_b, workspace, need))
            return fail(HC_ERR_ALIAS, "a gradient overlaps the workspace");
    }
    if (grad_x && grad_y && ranges_overlap(grad_x, in_b, grad_y, in_b))
        return fail(HC_ERR_ALIAS, "grad_x overlaps grad_y");
    if (need > 0) {
        if (!workspace || workspace_bytes < need)
            return fail(HC_ERR_WORKSPACE, "workspace of %zu bytes required, %zu given", need,
                        workspace ? workspace_bytes : (size_t)0);
        for (int i = 0; i < 3; ++i)
            if (ranges_overlap(workspace, need, ins[i], ins_b[i]))
                return fail(HC_ERR_ALIAS, "workspace overlaps an input");
    }
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != HC_OK) return rc;
    if (dtype == HC_F64)
        return run_backward<double>(P, (const double*)x, (const double*)y, (const double*)grad_z,
                                    (uint64_t)grad_z_stride, (double*)grad_x, (double*)grad_y, batch,
                                    (double*)workspace, cus, stream);
    return run_backward<float>(P, (const float*)x, (const float*)y, (const float*)grad_z, (uint64_t)grad_z_stride,
                               (float*)grad_x, (float*)grad_y, batch, (float*)workspace, cus, stream);
}

int hc_convolve_backward(const void* x, const void* y, const void* grad_z, void* grad_x, void* grad_y, int D,
                         int dtype, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    return hc_convolve_backward_batch(x, y, grad_z, 0, grad_x, grad_y, D, dtype, 1, workspace, workspace_bytes,
                                      stream);
}

int hc_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return HC_OK;
}

int hc_profile_collect(hc_kernel_stat* out, int capacity, int* count)
{
    g_last_error.clear();
    if (!count || (capacity > 0 && !out)) return fail(HC_ERR_INVALID_ARG, "count and out are required");
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof);
    }
    std::vector<hc_kernel_stat> agg;
    int rc = HC_OK;
    for (ProfRec& r : recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && rc == HC_OK) rc = hip_fail(e, "profiler events");
        hc_kernel_stat* st = nullptr;
        for (hc_kernel_stat& a : agg)
            if (strncmp(a.name, r.name, sizeof(a.name)) == 0) st = &a;
        if (!st) {
            agg.push_back(hc_kernel_stat{});
            st = &agg.back();
            snprintf(st->name, sizeof(st->name), "%s", r.name);
        }
        st->launches += 1;
        st->total_ms += ms;
        st->alg_bytes += r.bytes;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (ProfRec& r : recs) {
            g_event_pool.push_back(r.a);
            g_event_pool.push_back(r.b);
        }
    }
    const int n = (int)agg.size() < capacity ? (int)agg.size() : capacity;
    for (int i = 0; i < n; ++i) out[i] = agg[i];
    *count = n;
    return rc;
}

}  // extern "C"
