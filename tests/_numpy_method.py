"""A numpy transcription of the per-axis method with switches that plant
plausible mistakes, used only to show that the pins catch them.  Test helper;
never used as a reference."""
from __future__ import annotations

import numpy as np


def per_axis(x, y, *, forward_order="asc", inverse_order="desc", assoc="left",
             sign=-1, drop_p2=False, forward_mid="sum", lsb_first=False):
    D = int(x.size).bit_length() - 1
    X = x.copy()
    Y = y.copy()
    if lsb_first:
        X = X.reshape((2,) * D).transpose(tuple(range(D))[::-1]).reshape(-1).copy() if D else X
        Y = Y.reshape((2,) * D).transpose(tuple(range(D))[::-1]).reshape(-1).copy() if D else Y
    axes = list(range(D)) if forward_order == "asc" else list(range(D))[::-1]
    shape = [2] * D
    for a in axes:
        def fwd(V):
            v = V.reshape(int(np.prod(shape[:a], dtype=np.int64)), 2, -1)
            mid = v[:, 0] + v[:, 1] if forward_mid == "sum" else v[:, 0].copy()
            return np.stack([v[:, 0], mid, v[:, 1]], axis=1).reshape(-1)
        X, Y = fwd(X), fwd(Y)
        shape[a] = 3
    Z = X * Y
    inv_axes = list(range(D))[::-1] if inverse_order == "desc" else list(range(D))
    for a in inv_axes:
        v = Z.reshape(3 ** a, 3, -1)
        p0, p1, p2 = v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()
        if drop_p2:
            v[:, 1] = p1 - p0
        elif assoc == "left":
            v[:, 1] = (p1 - p0) + sign * p2
        else:
            v[:, 1] = p1 - (p0 + p2)
        Z = v.reshape(-1)
    return Z


def sum3_per_axis(x1, x2, x3, *, minus_point=True, halve=True, inverse_order="desc", forward_order="asc",
                  keep_pi=False, assoc="left"):
    """numpy transcription of the three-operand per-axis method (values at
    0, 1, -1, infinity) with switches that plant mistakes."""
    D = int(x1.size).bit_length() - 1
    ops = [x1.copy(), x2.copy(), x3.copy()]
    axes = list(range(D)) if forward_order == "asc" else list(range(D))[::-1]
    out = []
    for X in ops:
        shape = [2] * D
        for a in axes:
            v = X.reshape(int(np.prod(shape[:a], dtype=np.int64)), 2, -1)
            m = v[:, 0] - v[:, 1] if minus_point else v[:, 0] + v[:, 1]
            X = np.stack([v[:, 0], v[:, 0] + v[:, 1], m, v[:, 1]], axis=1).reshape(-1)
            shape[a] = 4
        out.append(X)
    Z = (out[0] * out[1]) * out[2] if assoc == "left" else out[0] * (out[1] * out[2])
    inv_axes = list(range(D))[::-1] if inverse_order == "desc" else list(range(D))
    two = Z.dtype.type(2) if Z.dtype.kind == "f" else 2
    for a in inv_axes:
        v = Z.reshape(4 ** a, 4, -1)
        p0, p1, pm, pi = (v[:, i].copy() for i in range(4))
        d, s = p1 - pm, p1 + pm
        if halve:
            d = d / two if Z.dtype.kind == "f" else d // 2
            s = s / two if Z.dtype.kind == "f" else s // 2
        v[:, 1] = d if keep_pi else d - pi
        v[:, 2] = s - p0
        Z = v.reshape(-1)
    return Z


def ternary_per_axis(a, b, *, forward_order="asc", inverse_order="desc", q02_sign=1, keep_p1=True,
                     c1_drop_p1=False, slot_swap=False):
    """numpy transcription of the six-product per-axis method for two ternary
    cubes with switches that plant mistakes."""
    n = int(a.size)
    D = 0
    while 3 ** D < n:
        D += 1
    ops = []
    axes = list(range(D)) if forward_order == "asc" else list(range(D))[::-1]
    for X in (a.copy(), b.copy()):
        shape = [3] * D
        for ax in axes:
            v = X.reshape(int(np.prod(shape[:ax], dtype=np.int64)), 3, -1)
            a0, a1, a2 = v[:, 0], v[:, 1], v[:, 2]
            s02 = a0 + a2 if q02_sign > 0 else a0 - a2
            slots = [a0, a1, a2, a0 + a1, a1 + a2, s02]
            if slot_swap:
                slots[3], slots[4] = slots[4], slots[3]
            X = np.stack(slots, axis=1).reshape(-1)
            shape[ax] = 6
        ops.append(X)
    Z = ops[0] * ops[1]
    shape = [6] * D
    inv_axes = list(range(D))[::-1] if inverse_order == "desc" else list(range(D))
    for ax in inv_axes:
        v = Z.reshape(int(np.prod(shape[:ax], dtype=np.int64)), 6, -1)
        p0, p1, p2, q01, q12, q02 = (v[:, i] for i in range(6))
        c1 = (q01 - p0) if c1_drop_p1 else (q01 - p0) - p1
        c2 = ((q02 - p0) - p2) + p1 if keep_p1 else (q02 - p0) - p2
        c3 = (q12 - p1) - p2
        Z = np.stack([p0, c1, c2, c3, p2], axis=1).reshape(-1)
        shape[ax] = 5
    return Z
