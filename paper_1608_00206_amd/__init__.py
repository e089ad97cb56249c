"""Exact convolution of hypercubes {0,1}^D on AMD MI355X (gfx950).

Implements the sub-quadratic method of Serang's "An exact, cache-localized
algorithm for the sub-quadratic convolution of hypercubes" (Methods section:
three sub-convolutions per axis, z[1] = t - z[0] - z[2]) with hand-written
HIP kernels behind the C ABI in ``include/hc.h``.  PyTorch only supplies
device memory and the current stream; every step of the computation runs in
libhc's kernels.

    import torch, paper_1608_00206_amd as hc
    x = torch.rand(2 ** 16, dtype=torch.float64, device="cuda")
    y = torch.rand(2 ** 16, dtype=torch.float64, device="cuda")
    z = hc.convolve(x, y)            # 3^16 outputs, row-major ternary index
    z = hc.HypercubeConv.apply(x, y) # differentiable

Layouts: x and y hold 2^D values whose flat index bits are the axes (axis 0
the most significant bit); z holds 3^D values whose ternary digits are the
axes.  Batches are (B, 2^D) -> (B, 3^D).
"""
from __future__ import annotations

import torch

from . import _abi
from ._abi import HCError

__all__ = ["convolve", "convolve_batch", "convolve_backward", "HypercubeConv", "HCError", "BatchedPlan",
           "workspace_bytes", "backward_workspace_bytes", "dim_of", "DTYPES",
           "carryfree_convolve", "carryfree_index", "carryfree_dim", "difference", "difference_batch",
           "maxconv_pnorm", "maxconv_pnorm_batch"]

DTYPES = {torch.float64: _abi.HC_F64, torch.float32: _abi.HC_F32, torch.int64: _abi.HC_I64}


def dim_of(n: int) -> int:
    D = int(n).bit_length() - 1
    if n <= 0 or (1 << D) != n:
        raise ValueError(f"a hypercube has 2^D entries, got {n}")
    return D


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}; use float64, float32 or int64") from None


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_device(*ts: torch.Tensor) -> None:
    dev = ts[0].device
    if dev.type != "cuda":
        raise ValueError("tensors must be on a HIP device (device='cuda')")
    for t in ts[1:]:
        if t.device != dev:
            raise ValueError("all tensors must be on the same device")


def workspace_bytes(D: int, dtype: torch.dtype, batch: int = 1) -> int:
    n = _abi.hc_workspace_bytes(D, DTYPES[dtype], batch)
    if n == _abi.SIZE_MAX:
        raise ValueError("invalid D, dtype or batch")
    return n


def backward_workspace_bytes(D: int, dtype: torch.dtype, batch: int = 1) -> int:
    n = _abi.hc_backward_workspace_bytes(D, DTYPES[dtype], batch)
    if n == _abi.SIZE_MAX:
        raise ValueError("invalid D, dtype or batch")
    return n


def _launch(device: torch.device, fn, *args) -> None:
    """Calls a libhc entry point with `device` current (the library works on
    the current HIP device) and raises HCError on failure."""
    with torch.cuda.device(device):
        _abi.check(fn(*args))


def _workspace(nbytes: int, device, workspace):
    if nbytes == 0:
        return None
    if workspace is not None:
        if (workspace.device != device or not workspace.is_contiguous()
                or workspace.numel() * workspace.element_size() < nbytes):
            raise ValueError(f"workspace must be a contiguous tensor of at least {nbytes} bytes on {device}")
        return workspace
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def convolve_batch(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None) -> torch.Tensor:
    """z[b] = x[b] * y[b] for x, y of shape (B, 2^D); returns (B, 3^D)."""
    if x.dim() != 2 or x.shape != y.shape:
        raise ValueError("x and y must both have shape (B, 2^D)")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    _check_device(x, y)
    B, n = x.shape
    D = dim_of(n)
    code = _dtype_code(x)
    x = x.contiguous()
    y = y.contiguous()
    if out is None:
        out = torch.empty((B, 3 ** D), dtype=x.dtype, device=x.device)
    elif out.shape != (B, 3 ** D) or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must be a contiguous (B, 3^D) tensor of the input dtype")
    nbytes = workspace_bytes(D, x.dtype, B)
    ws = _workspace(nbytes, x.device, workspace)
    _launch(x.device, _abi.hc_convolve_batch, x.data_ptr(), y.data_ptr(), out.data_ptr(), D, code, B,
            ws.data_ptr() if ws is not None else 0, nbytes, _stream(x.device))
    return out


def convolve_batch_noalloc(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """convolve_batch through the library's allocation-free entry point: the
    caller passes the output, and the workspace is the library's own
    fixed-size device array (hc_convolve_batch_noalloc in include/hc.h)."""
    if x.dim() != 2 or x.shape != y.shape:
        raise ValueError("x and y must both have shape (B, 2^D)")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    _check_device(x, y, out)
    B, n = x.shape
    D = dim_of(n)
    code = _dtype_code(x)
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("x and y must be contiguous")
    if out.shape != (B, 3 ** D) or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous (B, 3^D) tensor of the input dtype")
    _launch(x.device, _abi.hc_convolve_batch_noalloc, x.data_ptr(), y.data_ptr(), out.data_ptr(), D, code, B,
            _stream(x.device))
    return out


def convolve(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None) -> torch.Tensor:
    """z = x * y for one pair of hypercubes.

    x, y: shape (2^D,) or (2,)*D.  Returns shape (3^D,) or (3,)*D to match.
    """
    if x.shape != y.shape:
        raise ValueError("x and y must have the same shape")
    n = x.numel()
    D = dim_of(n)
    if x.dim() >= 2 and any(s != 2 for s in x.shape):
        raise ValueError("a multi-dimensional input must have shape (2,)*D")
    flat_out = out.view(1, 3 ** D) if out is not None else None
    z = convolve_batch(x.reshape(1, n), y.reshape(1, n), out=flat_out, workspace=workspace)
    return z.view((3,) * D) if x.dim() >= 2 else z.view(3 ** D)


def convolve_backward(x: torch.Tensor, y: torch.Tensor, grad_z: torch.Tensor, need_x: bool = True,
                      need_y: bool = True, workspace: torch.Tensor | None = None):
    """Gradients of sum(grad_z * z) with respect to x and y.

    x, y: (B, 2^D); grad_z: (B, 3^D), or (3^D,) / an expanded (B, 3^D) view
    with batch stride 0 to share one weight vector across the batch.
    Returns (grad_x or None, grad_y or None).
    """
    if x.dim() != 2 or x.shape != y.shape:
        raise ValueError("x and y must both have shape (B, 2^D)")
    _check_device(x, y, grad_z)
    B, n = x.shape
    D = dim_of(n)
    code = _dtype_code(x)
    if grad_z.dtype != x.dtype:
        raise TypeError("grad_z must have the dtype of x")
    x = x.contiguous()
    y = y.contiguous()
    n3 = 3 ** D
    if grad_z.dim() == 1:
        if grad_z.numel() != n3:
            raise ValueError("grad_z must have 3^D entries")
        gz, gz_stride = grad_z.contiguous(), 0
    else:
        if grad_z.shape != (B, n3):
            raise ValueError("grad_z must have shape (B, 3^D)")
        if B > 1 and grad_z.stride(0) == 0 and grad_z.stride(1) == 1:
            gz, gz_stride = grad_z, 0
        else:
            gz = grad_z.contiguous()
            gz_stride = n3
    gx = torch.empty_like(x) if need_x else None
    gy = torch.empty_like(y) if need_y else None
    nbytes = backward_workspace_bytes(D, x.dtype, B)
    ws = _workspace(nbytes, x.device, workspace)
    _launch(x.device, _abi.hc_convolve_backward_batch, x.data_ptr(), y.data_ptr(), gz.data_ptr(), gz_stride,
            gx.data_ptr() if gx is not None else 0, gy.data_ptr() if gy is not None else 0,
            D, code, B, ws.data_ptr() if ws is not None else 0, nbytes, _stream(x.device))
    return gx, gy


def carryfree_dim(n: int) -> int:
    """Bits per index (ceil(log2 n)) of the carry-free convolution of length-n vectors."""
    D = _abi.hc_carryfree_dim(int(n))
    if D < 0:
        raise ValueError(f"length {n} out of range")
    return D


def carryfree_index(i: int, j: int) -> int:
    """Output index of x[i] * y[j] in the carry-free convolution: the base-3
    number whose digits are the bit-wise sums of i and j."""
    return int(_abi.hc_carryfree_index(int(i), int(j)))


def carryfree_convolve(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
                       workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Carry-free convolution of two 1-D tensors of equal length n (any n >= 1):
    x[i] * y[j] is added to z[carryfree_index(i, j)]; returns 3^D values,
    D = carryfree_dim(n)."""
    if x.dim() != 1 or x.shape != y.shape:
        raise ValueError("x and y must be 1-D tensors of the same length")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    _check_device(x, y)
    n = x.numel()
    D = carryfree_dim(n)
    code = _dtype_code(x)
    x = x.contiguous()
    y = y.contiguous()
    if out is None:
        out = torch.empty(3 ** D, dtype=x.dtype, device=x.device)
    elif out.numel() != 3 ** D or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must be a contiguous tensor of 3^D elements of the input dtype")
    nbytes = _abi.hc_carryfree_workspace_bytes(n, code)
    ws = _workspace(nbytes, x.device, workspace)
    _launch(x.device, _abi.hc_carryfree_convolve, x.data_ptr(), y.data_ptr(), n, out.data_ptr(), code,
            ws.data_ptr() if ws is not None else 0, nbytes, _stream(x.device))
    return out


def difference_batch(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
                     workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Distribution of X - Y for (B, 2^D) distributions x of X and y of Y
    over {0,1}^D: digit 0, 1, 2 of an output index stands for a difference
    of -1, 0, +1 on that axis.  Returns (B, 3^D)."""
    if x.dim() != 2 or x.shape != y.shape:
        raise ValueError("x and y must both have shape (B, 2^D)")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    _check_device(x, y)
    B, n = x.shape
    D = dim_of(n)
    code = _dtype_code(x)
    x = x.contiguous()
    y = y.contiguous()
    if out is None:
        out = torch.empty((B, 3 ** D), dtype=x.dtype, device=x.device)
    elif out.shape != (B, 3 ** D) or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must be a contiguous (B, 3^D) tensor of the input dtype")
    nbytes = _abi.hc_difference_workspace_bytes(D, code, B)
    ws = _workspace(nbytes, x.device, workspace)
    _launch(x.device, _abi.hc_difference_batch, x.data_ptr(), y.data_ptr(), out.data_ptr(), D, code, B,
            ws.data_ptr() if ws is not None else 0, nbytes, _stream(x.device))
    return out


def sum3_batch(x1: torch.Tensor, x2: torch.Tensor, x3: torch.Tensor, out: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Distribution of X1 + X2 + X3 for (B, 2^D) distributions over {0,1}^D:
    base-4 digit d of an output index is the sum of the three coordinates on
    axis D-1-d.  Returns (B, 4^D)."""
    if x1.dim() != 2 or x1.shape != x2.shape or x1.shape != x3.shape:
        raise ValueError("x1, x2 and x3 must all have shape (B, 2^D)")
    if not (x1.dtype == x2.dtype == x3.dtype):
        raise TypeError("x1, x2 and x3 must have the same dtype")
    _check_device(x1, x2, x3)
    B, n = x1.shape
    D = dim_of(n)
    code = _dtype_code(x1)
    x1, x2, x3 = x1.contiguous(), x2.contiguous(), x3.contiguous()
    if out is None:
        out = torch.empty((B, 4 ** D), dtype=x1.dtype, device=x1.device)
    elif out.shape != (B, 4 ** D) or out.dtype != x1.dtype or not out.is_contiguous() or out.device != x1.device:
        raise ValueError("out must be a contiguous (B, 4^D) tensor of the input dtype")
    nbytes = _abi.hc_sum3_workspace_bytes(D, code, B)
    if nbytes == _abi.SIZE_MAX:
        raise ValueError("invalid D, dtype or batch for sum3")
    ws = _workspace(nbytes, x1.device, workspace)
    _launch(x1.device, _abi.hc_sum3_batch, x1.data_ptr(), x2.data_ptr(), x3.data_ptr(), out.data_ptr(), D, code, B,
            ws.data_ptr() if ws is not None else 0, nbytes, _stream(x1.device))
    return out


def sum3(x1: torch.Tensor, x2: torch.Tensor, x3: torch.Tensor, out: torch.Tensor | None = None,
         workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Single-triple form of sum3_batch: (2^D,) inputs, (4^D,) output."""
    if x1.dim() != 1:
        raise ValueError("x1, x2 and x3 must be 1-D tensors of length 2^D")
    n = x1.numel()
    flat = out.view(1, -1) if out is not None else None
    return sum3_batch(x1.view(1, n), x2.view(1, n), x3.view(1, n), out=flat, workspace=workspace).view(-1)


def ternary_dim_of(n: int) -> int:
    D = 0
    while 3 ** D < n:
        D += 1
    if n <= 0 or 3 ** D != n:
        raise ValueError(f"a ternary cube has 3^D entries, got {n}")
    return D


def ternary_convolve_batch(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
                           workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Convolution of two ternary cubes {0,1,2}^D, (B, 3^D) each (the layout
    of convolve's output), into (B, 5^D): base-5 digit d of an output index
    is the sum of the two ternary digits on axis D-1-d."""
    if a.dim() != 2 or a.shape != b.shape:
        raise ValueError("a and b must both have shape (B, 3^D)")
    if a.dtype != b.dtype:
        raise TypeError("a and b must have the same dtype")
    _check_device(a, b)
    B, n = a.shape
    D = ternary_dim_of(n)
    code = _dtype_code(a)
    a, b = a.contiguous(), b.contiguous()
    if out is None:
        out = torch.empty((B, 5 ** D), dtype=a.dtype, device=a.device)
    elif out.shape != (B, 5 ** D) or out.dtype != a.dtype or not out.is_contiguous() or out.device != a.device:
        raise ValueError("out must be a contiguous (B, 5^D) tensor of the input dtype")
    nbytes = _abi.hc_ternary_workspace_bytes(D, code, B)
    if nbytes == _abi.SIZE_MAX:
        raise ValueError("invalid D, dtype or batch for ternary_convolve")
    ws = _workspace(nbytes, a.device, workspace)
    _launch(a.device, _abi.hc_ternary_convolve_batch, a.data_ptr(), b.data_ptr(), out.data_ptr(), D, code, B,
            ws.data_ptr() if ws is not None else 0, nbytes, _stream(a.device))
    return out


def ternary_convolve(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
                     workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Single-pair form of ternary_convolve_batch: (3^D,) inputs, (5^D,) output."""
    if a.dim() != 1:
        raise ValueError("a and b must be 1-D tensors of length 3^D")
    n = a.numel()
    flat = out.view(1, -1) if out is not None else None
    return ternary_convolve_batch(a.view(1, n), b.view(1, n), out=flat, workspace=workspace).view(-1)


def sum4_batch(x1: torch.Tensor, x2: torch.Tensor, x3: torch.Tensor, x4: torch.Tensor) -> torch.Tensor:
    """Distribution of X1 + X2 + X3 + X4 for (B, 2^D) distributions over
    {0,1}^D: the pair sums by convolve_batch, then their ternary
    convolution.  Returns (B, 5^D), base-5 digit = the sum of the four
    coordinates."""
    return ternary_convolve_batch(convolve_batch(x1, x2), convolve_batch(x3, x4))


def sum4(x1: torch.Tensor, x2: torch.Tensor, x3: torch.Tensor, x4: torch.Tensor) -> torch.Tensor:
    """Single form of sum4_batch: (2^D,) inputs, (5^D,) output."""
    if x1.dim() != 1:
        raise ValueError("x1 ... x4 must be 1-D tensors of length 2^D")
    n = x1.numel()
    return sum4_batch(*(x.view(1, n) for x in (x1, x2, x3, x4))).view(-1)


def difference(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Single-pair form of difference_batch: (2^D,) inputs, (3^D,) output."""
    if x.dim() != 1 or x.shape != y.shape:
        raise ValueError("x and y must be 1-D tensors of the same length 2^D")
    D = dim_of(x.numel())
    flat = out.view(1, 3 ** D) if out is not None else None
    return difference_batch(x.view(1, -1), y.view(1, -1), out=flat, workspace=workspace).view(3 ** D)


def maxconv_pnorm_batch(x: torch.Tensor, y: torch.Tensor, p: float, round: bool = False,
                        out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                        separate_root: bool = False) -> torch.Tensor:
    """p-norm estimate of the max-convolution max x[i] y[j] of nonnegative
    (B, 2^D) float64/float32 inputs: (sum (x[i] y[j])^p)^(1/p) per output;
    round=True rounds the estimates to integers.  separate_root=True runs the
    root as its own kernel rather than in the convolution's last pass (same
    bits).  Returns (B, 3^D)."""
    if x.dim() != 2 or x.shape != y.shape:
        raise ValueError("x and y must both have shape (B, 2^D)")
    if x.dtype != y.dtype:
        raise TypeError("x and y must have the same dtype")
    _check_device(x, y)
    B, n = x.shape
    D = dim_of(n)
    code = _dtype_code(x)
    x = x.contiguous()
    y = y.contiguous()
    if out is None:
        out = torch.empty((B, 3 ** D), dtype=x.dtype, device=x.device)
    elif out.shape != (B, 3 ** D) or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must be a contiguous (B, 3^D) tensor of the input dtype")
    nbytes = _abi.hc_maxconv_workspace_bytes(D, code, B)
    if nbytes == _abi.SIZE_MAX:
        raise TypeError("the p-norm max-convolution supports float64 and float32")
    ws = _workspace(nbytes, x.device, workspace)
    _launch(x.device, _abi.hc_maxconv_pnorm_batch, x.data_ptr(), y.data_ptr(), out.data_ptr(), D, code, B, float(p),
            (_abi.HC_MAXCONV_ROUND if round else 0) | (_abi.HC_MAXCONV_SEPARATE_ROOT if separate_root else 0),
            ws.data_ptr(), nbytes,
            _stream(x.device))
    return out


def maxconv_pnorm(x: torch.Tensor, y: torch.Tensor, p: float, round: bool = False,
                  out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                  separate_root: bool = False) -> torch.Tensor:
    """Single-pair form of maxconv_pnorm_batch: (2^D,) inputs, (3^D,) output."""
    if x.dim() != 1 or x.shape != y.shape:
        raise ValueError("x and y must be 1-D tensors of the same length 2^D")
    D = dim_of(x.numel())
    flat = out.view(1, 3 ** D) if out is not None else None
    return maxconv_pnorm_batch(x.view(1, -1), y.view(1, -1), p, round=round, out=flat, workspace=workspace,
                               separate_root=separate_root).view(3 ** D)


class HypercubeConv(torch.autograd.Function):
    """Differentiable z = x * y.  Accepts (2^D,) or (B, 2^D) inputs; saves
    only x and y (the forward transforms are recomputed in the backward)."""

    @staticmethod
    def forward(ctx, x, y):
        ctx.save_for_backward(x, y)
        if x.dim() == 1:
            return convolve_batch(x.unsqueeze(0), y.unsqueeze(0)).squeeze(0)
        return convolve_batch(x, y)

    @staticmethod
    def backward(ctx, grad_z):
        x, y = ctx.saved_tensors
        single = x.dim() == 1
        if single:
            x, y, grad_z = x.unsqueeze(0), y.unsqueeze(0), grad_z.unsqueeze(0)
        gx, gy = convolve_backward(x, y, grad_z, need_x=ctx.needs_input_grad[0],
                                   need_y=ctx.needs_input_grad[1])
        if single:
            gx = gx.squeeze(0) if gx is not None else None
            gy = gy.squeeze(0) if gy is not None else None
        return gx, gy


class BatchedPlan:
    """Many independent pairs of uneven D in one launch of a HIP graph
    (hc_plan_* in include/hc.h): pairs grouped by D, each group one batched
    run of the single-pair kernels, the groups parallel graph branches.

    Ds: the pairs' dimensions (0..16).  Inputs are packed: pair i's x and y
    occupy x_offsets[i]:x_offsets[i+1] of x_packed / y_packed, its z occupies
    z_offsets[i]:z_offsets[i+1] of the output.
    tune=True times candidate schedules per D at creation and keeps the
    fastest; persistent_pairs=True runs every pair in one persistent kernel
    launch instead (a workgroup per pair, pairs taken by ticket in decreasing
    D); persistent=True asks for the dependency-gated persistent kernel over
    split pairs, which is disabled (HCError HC_ERR_UNSUPPORTED).
    """

    def __init__(self, Ds, dtype: torch.dtype = torch.float64, tune: bool = False, persistent: bool = False,
                 persistent_pairs: bool = False):
        import json
        self._h = None
        self._ws = None  # the plan's own workspace when the caller passes none
        self.Ds = [int(d) for d in Ds]
        self.dtype = dtype
        flags = ((_abi.HC_PLAN_TUNE if tune else 0) | (_abi.HC_PLAN_PERSISTENT if persistent else 0)
                 | (_abi.HC_PLAN_PERSISTENT_PAIRS if persistent_pairs else 0))
        self._h = _abi.hc_plan_create_batched(self.Ds, DTYPES[dtype], flags)
        self.x_offsets, self.z_offsets = _abi.hc_plan_layout(self._h, len(self.Ds))
        self.workspace_bytes = _abi.hc_plan_workspace_bytes(self._h)
        self.schedule = json.loads(_abi.hc_plan_describe(self._h))

    @property
    def n_inputs(self) -> int:
        return self.x_offsets[-1]

    @property
    def n_outputs(self) -> int:
        return self.z_offsets[-1]

    def run(self, x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None) -> torch.Tensor:
        if self._h is None:
            raise RuntimeError("plan closed")
        if x.dtype != self.dtype or y.dtype != self.dtype:
            raise TypeError("inputs must have the plan's dtype")
        if x.numel() != self.n_inputs or y.numel() != self.n_inputs:
            raise ValueError(f"packed inputs must have {self.n_inputs} elements")
        _check_device(x, y)
        x = x.contiguous()
        y = y.contiguous()
        if out is None:
            out = torch.empty(self.n_outputs, dtype=self.dtype, device=x.device)
        elif (out.numel() != self.n_outputs or out.dtype != self.dtype or not out.is_contiguous()
              or out.device != x.device):
            raise ValueError("out must be a contiguous tensor of n_outputs elements on the inputs' device")
        if workspace is None and self.workspace_bytes > 0:
            # kept across calls: the same buffers replay the captured graph
            # instead of capturing it again
            if self._ws is None or self._ws.device != x.device:
                self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=x.device)
            workspace = self._ws
        ws = _workspace(self.workspace_bytes, x.device, workspace)
        _launch(x.device, _abi.hc_plan_execute, self._h, x.data_ptr(), y.data_ptr(), out.data_ptr(),
                ws.data_ptr() if ws is not None else 0, self.workspace_bytes,
                _stream(x.device))
        return out

    def check(self) -> None:
        """Synchronise and raise on an asynchronous device error."""
        _abi.check(_abi.hc_plan_check(self._h))

    def close(self) -> None:
        if self._h is not None:
            _abi.hc_plan_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
