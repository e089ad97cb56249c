/*
 * hc.h -- C ABI of libhc, exact convolution of hypercubes on AMD gfx950.
 *
 * The operation (Serang, "An exact, cache-localized algorithm for the
 * sub-quadratic convolution of hypercubes"; Introduction, definition of
 * tensor convolution, specialised to hypercubes {0,1}^D):
 *
 *     z[k] = sum over i, j in {0,1}^D with i + j = k of x[i] * y[j],
 *
 * where i + j adds the index vectors digit by digit, so every digit of k is
 * 0, 1 or 2 and z has 3^D entries.  It is computed with the method of the
 * Methods section (the three-subproblem recursion z[1] = t - z[0] - z[2],
 * t the convolution of the marginals x[0] + x[1] and y[0] + y[1]) in its
 * per-axis form:
 *     forward  (a0, a1)     -> (a0, a0 + a1, a1)      on axes 0, 1, ..., D-1
 *     product  elementwise
 *     inverse  (p0, p1, p2) -> (p0, (p1 - p0) - p2, p2)  on axes D-1, ..., 1, 0
 * Every floating-point operation is one IEEE operation in exactly this order
 * (no contraction into fused multiply-adds, no reassociation), so results are
 * bitwise reproducible and independent of tiling and tuning.  int64 data is
 * computed in wrapping 64-bit arithmetic, which is exact whenever the true
 * result fits in int64 (the method's identities hold in any ring).
 *
 * Memory layout (Methods section: tensors stored row-major):
 *   x, y  2^D contiguous elements; bit d of the flat index (weight 2^d) is
 *         the coordinate on axis D-1-d, so axis 0 is the most significant bit.
 *   z     3^D contiguous elements; ternary digit d of the flat index (weight
 *         3^d) is the coordinate on axis D-1-d.
 *   x[i] * y[j] therefore contributes to z[tern(i) + tern(j)], tern(i) being
 *   i's bits read as ternary digits (Discussion: carry-free convolution).
 *
 * Conventions for every entry point:
 *   - Data pointers are DEVICE pointers (memory of the current HIP device);
 *     the caller owns all buffers, including the workspace.  Nothing on the
 *     hot path allocates; plans allocate their own small tables when created.
 *   - Inputs are read-only (unlike the paper's listing, which overwrites x
 *     and y).  Outputs must not overlap inputs or the workspace.
 *   - Data pointers must be aligned to their element size (8 bytes for
 *     HC_F64/HC_I64, 4 for HC_F32); workspaces to 16 bytes.
 *   - Work is enqueued on `stream` (0 = the null stream); nothing synchronises.
 *   - Argument errors are detected on the host before anything is enqueued.
 *     Faults inside kernels surface asynchronously, as HC_ERR_HIP from a
 *     later call or from the caller's own synchronisation.
 *   - Return value: HC_OK or one of the hc_status codes below;
 *     hc_last_error() gives a message for the calling thread's last failure.
 */
#ifndef HC_H
#define HC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HC_ABI_VERSION 1
/* Largest D accepted; 3^21 float64 outputs are 84 GB. */
#define HC_MAX_D 21

typedef enum hc_dtype {
    HC_F64 = 0, /* IEEE binary64 */
    HC_F32 = 1, /* IEEE binary32 */
    HC_I64 = 2  /* two's complement int64, wrapping arithmetic */
} hc_dtype;

typedef enum hc_status {
    HC_OK = 0,
    HC_ERR_INVALID_ARG = 1, /* null pointer, bad count, bad flag */
    HC_ERR_D_RANGE = 2,     /* D < 0 or D > HC_MAX_D */
    HC_ERR_UNSUPPORTED = 3, /* dtype not supported by this entry point */
    HC_ERR_ALIAS = 4,       /* an output overlaps an input or the workspace */
    HC_ERR_MISALIGNED = 5,  /* data not aligned to its element size, a workspace not to 16 bytes */
    HC_ERR_WORKSPACE = 6,   /* workspace missing or smaller than required */
    HC_ERR_NO_DEVICE = 7,   /* no usable HIP device */
    HC_ERR_HIP = 8          /* a HIP runtime call failed */
} hc_status;

/* ABI version of the loaded library (HC_ABI_VERSION at build time). */
int hc_abi_version(void);

/* Static message for a status code. */
const char* hc_status_string(int status);

/* Message describing the calling thread's most recent failure ("" if none). */
const char* hc_last_error(void);

/* Size in bytes of one element of `dtype`, or 0 if the dtype is unknown. */
size_t hc_dtype_size(int dtype);

/* Number of outputs 3^D (0 if D is out of range). */
uint64_t hc_output_count(int D);

/*
 * Workspace for hc_convolve_batch (batch items of the same D), in bytes.
 * It holds the outer-forward images of x and y (3^(D-K) x 2^K each per batch
 * item, K the fused inner depth) and their staging.  Returns 0 when the
 * whole problem fits one fused tile (then no workspace is needed), and
 * (size_t)-1 for invalid arguments.
 */
size_t hc_workspace_bytes(int D, int dtype, int batch);

/*
 * Single convolution z = x * y of two D-dimensional hypercubes.
 *   x, y        device, 2^D elements of `dtype` each (read only)
 *   z           device, 3^D elements (written)
 *   workspace   device, at least hc_workspace_bytes(D, dtype, 1) bytes
 *               (may be NULL when that is 0)
 * Errors: HC_ERR_INVALID_ARG (null x/y/z), HC_ERR_D_RANGE, HC_ERR_UNSUPPORTED
 * (unknown dtype), HC_ERR_ALIAS (z overlaps x, y or workspace),
 * HC_ERR_MISALIGNED, HC_ERR_WORKSPACE, HC_ERR_NO_DEVICE, HC_ERR_HIP.
 */
int hc_convolve(const void* x, const void* y, void* z, int D, int dtype,
                void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * `batch` independent convolutions of the same D:
 *   z[b] = x[b] * y[b],  x[b] = x + b * 2^D elements, z[b] = z + b * 3^D.
 * Same buffers, errors and workspace rules as hc_convolve with
 * hc_workspace_bytes(D, dtype, batch).  1 <= batch <= 65535.
 */
int hc_convolve_batch(const void* x, const void* y, void* z, int D, int dtype, int batch,
                      void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Distribution of a sum of three independent random vectors X1 + X2 + X3
 * whose D axes are all Bernoulli (Introduction: sums of multiple probability
 * mass functions whose axes are Bernoulli variables; the sum of two is
 * hc_convolve itself):
 *   z[k] = sum over i, j, l in {0,1}^D with i + j + l = k of
 *          (x1[i] * x2[j]) * x3[l],
 * every digit of k in {0, 1, 2, 3}.  Computed by the Methods section's
 * per-axis method extended to three operands: along one axis each operand is
 * a linear polynomial a0 + a1 t and their product a cubic, recovered from its
 * values at t = 0, 1, -1 and infinity (the only division is by 2, exact in
 * binary floating point outside the subnormal range):
 *   forward  (a0, a1) -> (a0, a0 + a1, a0 - a1, a1)              axes 0..D-1
 *   product  (x1^ * x2^) * x3^                                   elementwise
 *   inverse  (p0, p1, pm, pi) -> (p0, (p1 - pm)/2 - pi,
 *                                 (p1 + pm)/2 - p0, pi)           axes D-1..0
 * each one IEEE operation in this order.  int64 data wraps modulo 2^64 and
 * halves by signed division; exact whenever every intermediate fits in int64.
 *   x1, x2, x3   device, batch x 2^D elements each (read only; layout as x)
 *   z            device, batch x 4^D elements (written); base-4 digit d of
 *                the flat index (weight 4^d) is the coordinate on axis D-1-d
 *   workspace    hc_sum3_workspace_bytes(D, dtype, batch) bytes
 * 0 <= D <= 16, 1 <= batch <= 65535.
 * Errors: as hc_convolve_batch (HC_ERR_D_RANGE above D = 16).
 */
size_t hc_sum3_workspace_bytes(int D, int dtype, int batch);  /* (size_t)-1 if invalid */
int hc_sum3_batch(const void* x1, const void* x2, const void* x3, void* z, int D, int dtype, int batch,
                  void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Convolution of two ternary cubes {0,1,2}^D x {0,1,2}^D -> {0,...,4}^D, the
 * next link of a chain of sums (Introduction: sums of multiple probability
 * mass functions whose axes are Bernoulli variables): with a the output of
 * hc_convolve for X1, X2 and b that for X3, X4, z is the distribution of
 * X1 + X2 + X3 + X4:
 *   z[k] = sum over i, j in {0,1,2}^D with i + j = k of a[i] * b[j],
 * every digit of k in {0, ..., 4}.  Computed by the Methods section's
 * Karatsuba identity taken to lines of three: along one axis each operand
 * is a quadratic, and the quartic product needs six products and no
 * division:
 *   forward  (a0, a1, a2) -> (a0, a1, a2, a0 + a1, a1 + a2, a0 + a2)
 *                                                            axes 0..D-1
 *   product  a^ * b^                                         elementwise
 *   inverse  (p0, p1, p2, q01, q12, q02) -> (p0, (q01 - p0) - p1,
 *            ((q02 - p0) - p2) + p1, (q12 - p1) - p2, p2)    axes D-1..0
 * each one IEEE operation in this order.  int64 data wraps modulo 2^64
 * (exact: there is no division).
 *   a, b        device, batch x 3^D elements each (read only; layout as the
 *               z of hc_convolve: ternary digit d, weight 3^d, is the
 *               coordinate on axis D-1-d)
 *   z           device, batch x 5^D elements (written); base-5 digit d of
 *               the flat index (weight 5^d) is the coordinate on axis D-1-d
 *   workspace   hc_ternary_workspace_bytes(D, dtype, batch) bytes
 * 0 <= D <= 12, 1 <= batch <= 65535.
 * Errors: as hc_convolve_batch (HC_ERR_D_RANGE above D = 12).
 */
size_t hc_ternary_workspace_bytes(int D, int dtype, int batch);  /* (size_t)-1 if invalid */
int hc_ternary_convolve_batch(const void* a, const void* b, void* z, int D, int dtype, int batch,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * hc_convolve_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same operation, arguments, kernels and results (bitwise) as
 * hc_convolve_batch, but the workspace is not passed: it is a device array
 * of HC_NOALLOC_SCRATCH_BYTES inside the library, present on every GPU the
 * library is loaded on until the process ends.  The call allocates nothing;
 * its first call on a device looks the array's address up on that device.
 *   x, y, z, D, dtype, batch, stream   as hc_convolve_batch
 * Limits: hc_workspace_bytes(D, dtype, batch) must not exceed
 * HC_NOALLOC_SCRATCH_BYTES (float64 and int64: D <= 16 for one item, float32:
 * D <= 17), else HC_ERR_WORKSPACE before anything is enqueued.
 * Concurrency: every call on one GPU uses that GPU's one array, so calls
 * whose executions overlap on one GPU (different streams, or different host
 * threads without ordering) race and give wrong results; calls ordered on
 * one stream are safe.  The array needs no clearing: each call writes every
 * workspace element it reads.
 * Errors: as hc_convolve_batch (HC_ERR_WORKSPACE as above).
 */
#define HC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hc_convolve_batch_noalloc(const void* x, const void* y, void* z, int D, int dtype, int batch,
                              hipStream_t stream);

/*
 * Workspace for hc_convolve_backward_batch, in bytes ((size_t)-1 if invalid).
 */
size_t hc_backward_workspace_bytes(int D, int dtype, int batch);

/*
 * Gradient of L = sum_b sum_k w[b][k] z[b][k] with z[b] = x[b] * y[b]:
 *   grad_x[b][i] = sum_j w[b][tern(i) + tern(j)] * y[b][j]
 *   grad_y[b][j] = sum_i w[b][tern(i) + tern(j)] * x[b][i]
 * computed by the transposed maps in reverse order (derived: z is bilinear
 * in x and y, so dL/dx = F^T (G^T w . F y)):
 *   G^T: (w0, w1, w2) -> (w0 - w1, w1, w2 - w1)   on axes 0, 1, ..., D-1
 *   F^T: (g0, g1, g2) -> (g0 + g1, g1 + g2)       on axes D-1, ..., 0
 *   x, y          device, batch x 2^D (read only)
 *   grad_z        device, 3^D elements per batch item at stride
 *                 grad_z_stride elements; stride 0 broadcasts one w to every
 *                 item, whose G^T transform is then computed once for all
 *                 items (read only)
 *   grad_x/grad_y device, batch x 2^D (written); either may be NULL
 *   workspace     at least hc_backward_workspace_bytes(D, dtype, batch)
 * Supported dtypes: HC_F64, HC_F32 (HC_I64 returns HC_ERR_UNSUPPORTED).
 * Errors as hc_convolve; HC_ERR_INVALID_ARG also when both grads are NULL or
 * grad_z_stride is neither 0 nor >= 3^D.
 */
int hc_convolve_backward_batch(const void* x, const void* y, const void* grad_z,
                               int64_t grad_z_stride, void* grad_x, void* grad_y,
                               int D, int dtype, int batch,
                               void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Single-pair form of hc_convolve_backward_batch (batch 1). */
int hc_convolve_backward(const void* x, const void* y, const void* grad_z,
                         void* grad_x, void* grad_y, int D, int dtype,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Batched plans: many independent pairs of uneven D in one graph launch.
 *
 * The pairs are packed: pair i's x (and y) occupy 2^D_i elements at element
 * offset x_off[i] = sum_{j<i} 2^D_j, and its z occupies 3^D_i elements at
 * z_off[i] = sum_{j<i} 3^D_j (hc_plan_layout returns both arrays).
 *
 * A plan groups the pairs by D; each group runs the single-pair path for all
 * its items at once (outer forward passes, fused inner tiles, outer inverse
 * passes), reading and writing every item in place in the packed buffers.
 * The groups are independent branches of one HIP graph, captured on the
 * first execution (and again whenever the buffers change) and replayed.
 * Results are bitwise those of hc_convolve on each pair.
 *
 * With HC_PLAN_PERSISTENT_PAIRS the graph holds one kernel launch instead: a
 * persistent grid (as many workgroups as stay resident, at most one per
 * pair) whose workgroups take pairs by ticket from a list sorted by
 * decreasing D and each run the whole single-pair path of their pair (outer
 * forward, fused tiles, outer inverse), separated by workgroup barriers.  No
 * workgroup waits for another.  The default schedule per D takes the
 * largest fused tile (3^9 for float32, else 3^8), outer forward groups of at
 * most three axes and outer inverse groups of six axes as 4 + 2 (then 3 + 2,
 * 2 + 2 or up to three register axes); with HC_PLAN_TUNE the autotuner times
 * smaller groups per D as persistent launches over that D's pairs and keeps
 * the fastest.  The workspace holds one slot per workgroup.  Results are
 * again bitwise those of hc_convolve.  Launches of one plan must not overlap
 * in time (they share the plan's ticket counters as well as its workspace).
 */
typedef struct hc_plan hc_plan;

/* Plan flags */
#define HC_PLAN_TUNE 1u        /* time candidate schedules per D at creation, keep the fastest */
#define HC_PLAN_PERSISTENT 2u  /* split pairs gated by phase counters: disabled, returns HC_ERR_UNSUPPORTED */
#define HC_PLAN_PERSISTENT_PAIRS 4u  /* one persistent kernel launch, a workgroup per pair (above) */

/*
 * Create a plan for n_pairs pairs with dimensions Ds[0..n_pairs) (host
 * array, 0 <= D <= 16) of `dtype`.  Allocates the plan's device tables and
 * streams on the current device.  With HC_PLAN_TUNE it also allocates
 * temporary buffers (outputs of at most 8 GiB: a D whose pairs need more is
 * timed on part of them) and times candidate schedules (this synchronises
 * the device); with the environment variable HC_TUNE_CACHE naming a file,
 * tuned choices are read from and appended to that file.
 * Errors: HC_ERR_INVALID_ARG (null Ds/out, n_pairs < 1, unknown flag,
 * HC_PLAN_PERSISTENT with HC_PLAN_PERSISTENT_PAIRS), HC_ERR_D_RANGE,
 * HC_ERR_UNSUPPORTED, HC_ERR_NO_DEVICE, HC_ERR_HIP.
 */
int hc_plan_create_batched(const int* Ds, int n_pairs, int dtype, unsigned flags, hc_plan** out);

/* Release the plan's device tables, streams and graph.  NULL is ignored. */
int hc_plan_destroy(hc_plan* plan);

/* Workspace bytes hc_plan_execute needs ((size_t)-1 for a null plan). */
size_t hc_plan_workspace_bytes(const hc_plan* plan);

/*
 * Packed layout: x_offsets and z_offsets (host arrays of n_pairs + 1
 * elements, either may be NULL) receive the element offsets of every pair
 * and, last, the total element counts.
 */
int hc_plan_layout(const hc_plan* plan, uint64_t* x_offsets, uint64_t* z_offsets);

/*
 * Run the plan: z = x * y for every pair of the packed buffers.  x, y, z and
 * the workspace follow the conventions above (device, aligned, z disjoint
 * from the others).  Enqueued on `stream` as one graph launch.  A call with
 * buffers other than the previous call's captures the graph again, so calls
 * on one plan must not overlap in time from several host threads; launches
 * of one plan on several streams share its workspace and must be ordered
 * by the caller.
 * Errors: HC_ERR_INVALID_ARG, HC_ERR_ALIAS, HC_ERR_MISALIGNED,
 * HC_ERR_WORKSPACE, HC_ERR_HIP.
 */
int hc_plan_execute(hc_plan* plan, const void* x, const void* y, void* z, void* workspace,
                    size_t workspace_bytes, hipStream_t stream);

/* Synchronise the device and report any asynchronous error: HC_OK or HC_ERR_HIP. */
int hc_plan_check(hc_plan* plan);

/* JSON description of the plan's schedule (groups, fused depth, inverse groups). */
int hc_plan_describe(const hc_plan* plan, char* buf, size_t len);

/*
 * Host-only view of the groups a plan for these pairs would use with the
 * default schedule (no device needed; HC_PLAN_TUNE is ignored).  For each
 * group `info` receives 6 values: D, number of pairs, first pair index,
 * fused depth K, number of outer forward passes, number of outer inverse
 * passes; at most `capacity` groups are written and *n_groups receives the
 * total.  Errors as hc_plan_create_batched for the arguments.
 */
int hc_plan_inspect(const int* Ds, int n_pairs, int dtype, unsigned flags, int64_t* info, int64_t capacity,
                    int64_t* n_groups);

/*
 * Carry-free convolution of two vectors (Discussion: embedding a 1-D
 * problem in a hypercube).  With D = ceil(log2 n) bits per index, x[i] * y[j]
 * is added to z[k] where k's base-3 digits are the digit-wise sums of the
 * bits of i and j (no carries): k = hc_carryfree_index(i, j).  Entries of the
 * vectors past n are taken as zero (the hypercubes are zero-padded to 2^D).
 *   x, y        device, n elements each (read only), 1 <= n <= 2^HC_MAX_D
 *   z           device, 3^D elements (written); D = hc_carryfree_dim(n)
 *   workspace   hc_carryfree_workspace_bytes(n, dtype) bytes: the padded
 *               copies (when n is not a power of two) and the convolution's
 *               own workspace
 * Results are bitwise those of hc_convolve on the zero-padded vectors.
 * Errors: as hc_convolve; HC_ERR_D_RANGE for n outside the range.
 */
int hc_carryfree_dim(uint64_t n);                       /* -1 if n is out of range */
uint64_t hc_carryfree_index(uint64_t i, uint64_t j);    /* output index of x[i] * y[j] */
size_t hc_carryfree_workspace_bytes(uint64_t n, int dtype);  /* (size_t)-1 if invalid */
int hc_carryfree_convolve(const void* x, const void* y, uint64_t n, void* z, int dtype, void* workspace,
                          size_t workspace_bytes, hipStream_t stream);

/*
 * Distribution of the difference X - Y of independent random vectors with
 * values in {0,1}^D (Introduction: distributions of sums and differences;
 * the sum X + Y is hc_convolve itself), for `batch` pairs:
 *   z[b][k] = sum over i, j with bit_a(i) - bit_a(j) = digit_a(k) - 1 on
 *             every axis a of x[b][i] * y[b][j]
 * so digit 0, 1, 2 of k stands for a difference of -1, 0, +1 on that axis.
 * Computed as the convolution of x with y reflected on every axis (each bit
 * b replaced by 1 - b), which the workspace holds.
 *   x, y        device, batch x 2^D elements (read only)
 *   z           device, batch x 3^D elements (written)
 *   workspace   hc_difference_workspace_bytes(D, dtype, batch) bytes
 * Results are bitwise those of hc_convolve_batch on (x, reflected y).
 * Errors: as hc_convolve_batch.
 */
size_t hc_difference_workspace_bytes(int D, int dtype, int batch);  /* (size_t)-1 if invalid */
int hc_difference_batch(const void* x, const void* y, void* z, int D, int dtype, int batch, void* workspace,
                        size_t workspace_bytes, hipStream_t stream);

/*
 * p-norm estimate of the max-convolution on the semiring (x, max)
 * (Discussion: p-norm rings): for nonnegative inputs and each batch item,
 *   z[k] = (sum over the pairs (i, j) of output k of (x[i] y[j])^p)^(1/p)
 * which lies between max_{pairs} x[i] y[j] and 2^(s/p) times it (s = number
 * of digits of k equal to 1).  Computed as mx my (conv((x/mx)^p, (y/my)^p))^(1/p)
 * with mx, my each input's maximum and the convolution of this library;
 * negative entries count as 0.  Integer p in [1, 1024] form (x/mx)^p from the
 * quotient in float64 by binary powering on double-double values (the
 * squares of x/mx selected by the bits of p, low bits first, each product
 * kept to about twice float64 precision with fused multiply-adds), rounded
 * once to the data type: a relative error of about one rounding, in a fixed
 * order of operations; other p use the device library's pow.
 * Limits: powers below the smallest float
 * vanish (outputs below about mx my * 2^(-1074/p) for float64 read 0), and the
 * inverse map's cancellation leaves a relative error of about
 * (4D+2) u B/(p z'), B the method's rounding bound of the powered inputs, so
 * very large p lose the small outputs (see the design notes for measurements).
 * The root itself is within 2 ulps of exact for integer p in [2, 1024]
 * (float64 polishing of a float seed, for both dtypes) and within a few ulps
 * times 1 + |ln z'|/p for other p (computed as exp(log(z')/p)).
 * With HC_MAXCONV_ROUND every estimate is rounded to the nearest integer,
 * which gives the exact max-convolution of small integers where both the
 * 2^(s/p) factor and the rounding error stay below one half.
 *   x, y        device, batch x 2^D elements (read only), float64 or float32
 *   z           device, batch x 3^D elements (written)
 *   p           finite, >= 1 (p = 1 is the ordinary convolution)
 *   workspace   hc_maxconv_workspace_bytes(D, dtype, batch) bytes
 * Errors: as hc_convolve_batch; HC_ERR_UNSUPPORTED for int64,
 * HC_ERR_INVALID_ARG for p or unknown flags.
 */
#define HC_MAXCONV_ROUND 1u
/* Run the root as a kernel of its own after the convolution instead of in
 * the convolution's last inverse pass (same results, bit for bit; for
 * testing and measurement). */
#define HC_MAXCONV_SEPARATE_ROOT 2u
size_t hc_maxconv_workspace_bytes(int D, int dtype, int batch);  /* (size_t)-1 if invalid */
int hc_maxconv_pnorm_batch(const void* x, const void* y, void* z, int D, int dtype, int batch, double p,
                           unsigned flags, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Kernel profiler (measurement support; not part of the method).
 * While enabled, every kernel launch of the calling process is bracketed by
 * a pair of HIP events recorded on the launch stream, and tagged with the
 * kernel's name and its algorithmic traffic (bytes the kernel must read and
 * write by definition of its step, not counting re-reads).  Not to be used
 * during stream capture.
 */
typedef struct hc_kernel_stat {
    char name[48];       /* kernel and template configuration */
    int64_t launches;    /* launches recorded */
    double total_ms;     /* summed event-to-event time of those launches */
    double alg_bytes;    /* summed algorithmic bytes of those launches */
} hc_kernel_stat;

/* Start (on != 0) or stop recording.  Returns HC_OK. */
int hc_profile_enable(int on);

/*
 * Wait for every recorded event, aggregate by kernel name into `out`
 * (at most `capacity` entries, *count receives the number written) and
 * clear the record.  Call it while no other thread is launching work through
 * this library.  Errors: HC_ERR_INVALID_ARG (null count or out with
 * capacity > 0), HC_ERR_HIP.
 */
int hc_profile_collect(hc_kernel_stat* out, int capacity, int* count);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
