// Internal host-side declarations shared by the libhc translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

#include "hc_device.hpp"

namespace hc {

// One outer inverse pass over the axes [a, a + mR + mW): mR axes held in
// registers, mW axes across waves.  In the forward inverse (G, descending)
// the register part is the group's inner axes; in the adjoint (G^T,
// ascending) it is the group's outer axes.
struct InvPass {
    int a = 0, mR = 0, mW = 0;
};

// Tuning knobs; zero means "use the default".
struct PlanOpts {
    int fused_depth = 0;     // K: inner axes fused in one tile
    int inv_group_max = 0;   // largest outer inverse group (at most 6)
    int inv_reg = 0;         // axes of a group held in registers (at most 4)
    int grid_per_cu = 0;     // 0: one tile per workgroup; else at most this many workgroups per CU
    int bwd_tail = -1;       // backward: outer axes whose G^T runs in the fused tile (-1: 2)
    int fused_nt = 0;        // threads per fused-tile workgroup (256 or 512; 0: 256)
    int reg_cw = 0;          // 64-column groups per register-only pass workgroup (1, 2, 4; 0: 4)
};

struct Plan {
    int D = 0, dtype = 0;
    size_t esize = 0;
    int K = 0, p = 0;                 // fused inner depth, outer axes
    std::vector<int> k1;              // outer forward groups, ascending from axis 0
    std::vector<InvPass> inv;         // outer inverse passes in execution order
    int bwd_tail = 0;                 // backward: last outer axes transformed in the fused tile
    std::vector<InvPass> inv_bwd;     // backward: groups of the outer axes above the tail
    uint64_t n2 = 0, n3 = 0;
    uint64_t xt_elems = 0;            // 3^p * 2^K per operand and batch item
    uint64_t tmp_elems = 0;           // largest outer-forward staging stage
    int grid_per_cu = 0;              // launch policy, see PlanOpts
    int fused_nt = 256;               // threads per fused-tile workgroup
    int reg_cw = 4;                   // column groups per register-only pass workgroup
};

// Brackets one kernel launch with profiler events when profiling is on.
class LaunchScope {
  public:
    LaunchScope(hipStream_t s, double alg_bytes, const char* fmt, ...);
    ~LaunchScope();
    LaunchScope(const LaunchScope&) = delete;
    LaunchScope& operator=(const LaunchScope&) = delete;

  private:
    hipStream_t stream_;
    bool on_;
    size_t idx_;
};

// While alive, LaunchScope records nothing on this thread (used while a
// graph is captured and while the autotuner times candidates).
class CaptureScope {
  public:
    CaptureScope();
    ~CaptureScope();
    CaptureScope(const CaptureScope&) = delete;
    CaptureScope& operator=(const CaptureScope&) = delete;
};

// A roctx range around one entry point (shown by rocprofv3 --marker-trace;
// a plain call when no tool listens).
class TraceRange {
  public:
    explicit TraceRange(const char* fmt, ...);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Plan and autotuner decisions on stderr when the environment variable
// HC_LOG is set (to anything but 0).
bool log_on();
void hc_log(const char* fmt, ...);

// Short element-type name for profiler labels.
template <typename T>
const char* tname()
{
    return sizeof(T) == 4 ? "f32" : (std::is_same<T, double>::value ? "f64" : "i64");
}

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
uint64_t pow3u(int n);
size_t dtype_size(int dtype);
bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb);
bool misaligned(const void* p, size_t align);
int device_cus(int* cus);
int max_fused_depth(int dtype);
Plan make_plan(int D, int dtype, const PlanOpts& o);
PlanOpts default_opts();
size_t plan_ws_bytes(const Plan& P, int batch);
size_t plan_bwd_ws_bytes(const Plan& P, int batch);

// Workgroups for n_tiles tiles (one per tile when per_cu == 0, else a
// persistent grid of at most per_cu workgroups per CU).
uint32_t tile_grid(uint64_t n_tiles, int cus, int per_cu);

// A replacement for the last outer inverse pass of a forward run that fuses
// an elementwise step into it.  launch() either enqueues that pass and
// returns HC_OK, or returns HC_ERR_UNSUPPORTED for a pass shape it has no
// kernel for, and the plain pass runs instead; `taken` records which.  A
// plan without outer passes never calls it.
struct LastPass {
    int (*launch)(const LastPass& self, const InvPass& ip, void* z, BMap z_map, uint64_t L, uint32_t n_hi,
                  int batch, int cus, hipStream_t s) = nullptr;
    const void* ctx = nullptr;
    mutable bool taken = false;
};

// Forward path for `batch` items of one D; x_map / z_map give each item's
// element offset in x, y and z (uniform strides or per-item tables).
template <typename T>
int run_forward(const Plan& P, const T* x, const T* y, T* z, int batch, T* ws, int cus, hipStream_t s, BMap x_map,
                BMap z_map, const LastPass* last = nullptr);

// hc_convolve_batch with an optional replacement of its last inverse pass.
int convolve_batch_last(const void* x, const void* y, void* z, int D, int dtype, int batch, void* workspace,
                        size_t workspace_bytes, hipStream_t stream, const LastPass* last);
template <typename T>
int run_backward(const Plan& P, const T* x, const T* y, const T* gz, uint64_t gz_bs, T* gx, T* gy, int batch,
                 T* ws, int cus, hipStream_t s);

// ---------------------------------------------- persistent batched kernel
// Threads per workgroup: nine waves, one per digit pair of the two wave
// axes of its LDS passes.
constexpr int PAIR_NT = 576;
// Largest fused depth of its tiles: 9 for 4-byte elements (one 3^9 tile in
// LDS), 8 for 8-byte elements (three 3^8 tiles side by side in LDS).
__host__ __device__ constexpr int pair_kmax(size_t elem_size) { return elem_size == 4 ? 9 : 8; }

// Schedule of one pair of dimension D in the persistent kernel: fused depth
// K = min(D, pair_kmax), p = D - K outer axes, the outer forward groups
// (ascending) and the outer inverse passes in execution order (axes
// [inv_a, inv_a + inv_r + inv_w), inv_r of them in registers).
struct PairPlan {
    uint8_t K = 0, p = 0, n_fwd = 0, n_inv = 0;
    uint8_t fwd[4] = {0, 0, 0, 0};
    uint8_t inv_a[4] = {0, 0, 0, 0}, inv_r[4] = {0, 0, 0, 0}, inv_w[4] = {0, 0, 0, 0};
    uint32_t xt_elems = 0, tmp_elems = 0;  // per operand: x~ and the forward staging
};

// One entry of the ticket-ordered task list: a pair's dimension and element
// offsets into the packed x / y and z.
struct PairTask {
    uint64_t x_off = 0, z_off = 0;
    uint32_t D = 0, pad = 0;
};

// The default schedule takes forward groups of at most 3 axes and inverse
// groups of at most 6; the autotuner also tries smaller groups (fwd_max in
// {2, 3}, inv_max in 2..6).
PairPlan pair_plan(int D, int dtype, int fwd_max = 3, int inv_max = 6);
uint64_t pair_slot_elems(const PairPlan& pp);  // workspace elements per workgroup
double pair_alg_bytes(const PairPlan& pp, int D, size_t es);
int pairs_per_cu(int dtype, int* per_cu);      // resident workgroups per CU
int launch_pairs_persistent(int dtype, const void* x, const void* y, void* z, void* ws, uint64_t slot_elems,
                            const PairTask* tasks, const PairPlan* plans, uint32_t n_pairs, uint32_t* counters,
                            uint32_t grid, hipStream_t s);

}  // namespace hc
