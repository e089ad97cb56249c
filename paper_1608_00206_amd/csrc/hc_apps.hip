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
// Both reuse hc_convolve_batch unchanged; the only new device work is one
// padding or reflecting copy into the caller's workspace.
#include "hc.h"
#include "hc_internal.hpp"

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
    const uint64_t cap = (uint64_t)cus * 8;
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

}  // extern "C"
