"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration the benchmark times (default plans, tuned batched plans).

  D=16 int64     every output bitwise against Algorithm 1 (the naive
                 Cartesian product) and the recursion
  D=16 float64   every output bitwise against the canonical per-axis method;
                 sampled outputs within the derived rounding bound of the
                 compensated definition sum
  D=20 float64   every output (3^20 = 3.49e9) bitwise against the canonical
                 method (the recursion on 16 host threads), compared in
                 chunks; sampled outputs within the bound of the definition
  D=17, 19 float64, D=19, 20 float32, D=18 int64
                 every output bitwise against the recursion (the other
                 default plans at large D)
  batched        4096 pairs, D uniform in {6..14}, float64 and float32, tuned
                 plans: every pair bitwise against the oracle and against
                 single-pair calls
  backward       64 pairs at D=16, loss sum(w * z): every pair bitwise
                 against the transposed maps, sampled coordinates within the
                 bound of the direct correlation, central differences on x
                 and y coordinates and one random direction per pair
  D=21 float64   every output (84 GB) bitwise against the recursion
"""
import sys
import time

import numpy as np
import pytest
import torch

import hc_inputs
import oracle
import paper_1608_00206_amd as hc
from tests import pins

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = torch.device("cuda:0")
U64 = 2.0 ** -53


def say(msg):
    print(f"[fullsize] {msg}", file=sys.stderr, flush=True)


def on_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def sample_indices(D, n, seed, max_ones=14):
    """n distinct output indices, uniform over 3^D, keeping those with at most
    max_ones digits equal to 1 (the per-index bound's limit; at D = 20 that
    drops about 0.2% of a uniform sample), plus the two corners."""
    g = np.random.default_rng([hc_inputs.SEED, 77, seed, D])
    ks = g.integers(0, 3 ** D, 4 * n, dtype=np.uint64)
    keep = [int(k) for k in ks if sum(d == 1 for d in pins.ternary_digits(int(k), D)) <= max_ones]
    out = np.unique(np.array(keep[:n] + [0, 3 ** D - 1], dtype=np.uint64))
    return out


def check_against_definition(x, y, z_at, ks, D):
    """|z - definition| <= (4D+2) u B at the sampled indices (plus the
    compensated sum's own rounding)."""
    ref = oracle.direct_at(x, y, ks)
    B = oracle.bound_at(x, y, ks)
    tol = (4 * D + 2) * U64 * B + 2.0 ** -60 * np.abs(ref)
    err = np.abs(z_at - ref)
    assert np.all(err <= tol), f"max err/tol {np.max(err / np.maximum(tol, 1e-300))}"
    r = float(np.max(err / np.maximum(B, 1e-300)) / U64)
    pins.error_ratio_band(r, D)
    return r


def test_d16_int64_matches_algorithm1():
    D = 16
    x, y = hc_inputs.pair_ints(D, hc_inputs.W_D16)
    say("D=16 int64: GPU")
    z = hc.convolve(on_gpu(x), on_gpu(y))
    torch.cuda.synchronize(DEV)
    z = z.cpu().numpy()
    t0 = time.time()
    ref = oracle.naive(x, y)
    say(f"D=16 int64: Algorithm 1 on the host in {time.time() - t0:.1f} s")
    pins.assert_bitwise(z, ref, "D=16 int64 vs Algorithm 1")
    pins.assert_bitwise(z, oracle.recursive(x, y, threads=16), "D=16 int64 vs recursion")


def test_d16_f64_matches_canonical_and_definition():
    D = 16
    x, y = hc_inputs.pair_masses(D, hc_inputs.W_D16)
    z = hc.convolve(on_gpu(x), on_gpu(y))
    torch.cuda.synchronize(DEV)
    z = z.cpu().numpy()
    pins.assert_bitwise(z, oracle.canonical(x, y), "D=16 float64 vs canonical")
    ks = sample_indices(D, 4096, 1)
    r = check_against_definition(x, y, z[ks.astype(np.int64)], ks, D)
    say(f"D=16 float64: max |err|/(u B) over {ks.size} sampled outputs = {r:.2f}")


def test_d20_f64_every_output_bitwise():
    D = 20
    n3 = 3 ** D
    x, y = hc_inputs.pair_masses(D, hc_inputs.W_D20_F64)
    say("D=20 float64: GPU")
    z_gpu = hc.convolve(on_gpu(x), on_gpu(y))
    torch.cuda.synchronize(DEV)
    t0 = time.time()
    ref = oracle.recursive(x, y, threads=16)
    say(f"D=20 float64: oracle recursion in {time.time() - t0:.1f} s; comparing")
    chunk = 1 << 28
    mismatches = 0
    for c0 in range(0, n3, chunk):
        c1 = min(n3, c0 + chunk)
        part = z_gpu[c0:c1].cpu().numpy()
        mismatches += int(np.count_nonzero(part.view(np.uint64) != ref[c0:c1].view(np.uint64)))
    say(f"D=20 float64: {mismatches} of {n3} outputs differ")
    assert mismatches == 0
    ks = sample_indices(D, 256, 2)
    z_at = z_gpu[torch.from_numpy(ks.astype(np.int64)).to(DEV)].cpu().numpy()
    r = check_against_definition(x, y, z_at, ks, D)
    say(f"D=20 float64: max |err|/(u B) over {ks.size} sampled outputs = {r:.2f}")
    del z_gpu, ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("D,dtype", [(17, np.float64), (19, np.float64), (19, np.float32), (20, np.float32),
                                     (18, np.int64)])
def test_large_plans_every_output_bitwise(D, dtype):
    """The default plans of the other large shapes (float32 with fused depth
    9 at D = 19 and 8 at D = 20, 5- and 6-axis pass pairs for float64, int64
    wrapping arithmetic), every output bitwise against the recursion on 16
    host threads."""
    n3 = 3 ** D
    if np.dtype(dtype) == np.int64:
        x, y = hc_inputs.pair_ints(D, hc_inputs.W_D16)
    else:
        x, y = hc_inputs.pair_masses(D, hc_inputs.W_D20_F64)
        x, y = x.astype(dtype), y.astype(dtype)
    name = f"D={D} {np.dtype(dtype).name}"
    say(f"{name}: GPU")
    z_gpu = hc.convolve(on_gpu(x), on_gpu(y))
    torch.cuda.synchronize(DEV)
    ref = oracle.recursive(x, y, threads=16)
    view = np.uint32 if np.dtype(dtype).itemsize == 4 else np.uint64
    chunk = 1 << 28
    mismatches = 0
    for c0 in range(0, n3, chunk):
        c1 = min(n3, c0 + chunk)
        part = z_gpu[c0:c1].cpu().numpy()
        mismatches += int(np.count_nonzero(part.view(view) != ref[c0:c1].view(view)))
    say(f"{name}: {mismatches} of {n3} outputs differ")
    assert mismatches == 0
    del z_gpu, ref
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def batched_config():
    Ds = [int(d) for d in hc_inputs.batched_dims(4096)]
    return Ds


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_4096_pairs(batched_config, dtype):
    Ds = batched_config
    npdt = np.float64 if dtype == torch.float64 else np.float32
    say(f"batched {dtype}: tuning a plan for {len(Ds)} pairs")
    with hc.BatchedPlan(Ds, dtype=dtype, tune=True) as plan:
        xs, ys = [], []
        for p, D in enumerate(Ds):
            x, y = hc_inputs.pair_masses(D, hc_inputs.W_BATCHED, p, dtype=npdt)
            xs.append(x)
            ys.append(y)
        X = on_gpu(np.concatenate(xs))
        Y = on_gpu(np.concatenate(ys))
        Z = plan.run(X, Y)
        plan.check()
        xo, zo = plan.x_offsets, plan.z_offsets
        iv = torch.int64 if npdt == np.float64 else torch.int32
        # the same batch as one persistent launch (tuned): the same bits
        say(f"batched {dtype}: tuning the persistent plan")
        with hc.BatchedPlan(Ds, dtype=dtype, tune=True, persistent_pairs=True) as pplan:
            Zp = pplan.run(X, Y)
            pplan.check()
            assert torch.equal(Zp.view(iv), Z.view(iv)), "the persistent launch differs from the graph"
            del Zp
        # every pair against the single-pair entry point
        for p in range(len(Ds)):
            zs = hc.convolve(X[xo[p]:xo[p + 1]], Y[xo[p]:xo[p + 1]])
            if not torch.equal(zs.view(torch.int64 if npdt == np.float64 else torch.int32),
                               Z[zo[p]:zo[p + 1]].view(torch.int64 if npdt == np.float64 else torch.int32)):
                raise AssertionError(f"pair {p} (D={Ds[p]}) differs from the single-pair call")
        torch.cuda.synchronize(DEV)
        # every pair against the oracle (8 host threads); float32 also
        # reports its error against the float64 oracle on 3 pairs per D
        from concurrent.futures import ThreadPoolExecutor
        Zh = Z.cpu().numpy()

        def host_check(p):
            pins.assert_bitwise(Zh[zo[p]:zo[p + 1]], oracle.recursive(xs[p], ys[p]), f"pair {p} D={Ds[p]}")
            return p

        t0 = time.time()
        with ThreadPoolExecutor(8) as ex:
            assert list(ex.map(host_check, range(len(Ds)))) == list(range(len(Ds)))
        say(f"batched {dtype}: every pair bitwise against the oracle ({time.time() - t0:.1f} s)")
        if npdt == np.float32:
            by_d = {}
            for p, D in enumerate(Ds):
                by_d.setdefault(D, []).append(p)
            worst = 0.0
            for p in sorted(q for D in by_d for q in by_d[D][:3]):
                z = Zh[zo[p]:zo[p + 1]]
                z64 = oracle.canonical(xs[p].astype(np.float64), ys[p].astype(np.float64))
                worst = max(worst, float(np.max(np.abs(z - z64)) / np.max(np.abs(z64))))
            # reported, not gated: float32 against the float64 oracle
            say(f"batched float32 vs float64 oracle: max error / max|z| = {worst:.3g}")


def test_backward_64_pairs_d16():
    """Every one of the 64 pairs: grad_x and grad_y bitwise against the
    transposed maps (on 8 host threads), 256 coordinates per pair within the
    bound of the direct correlation, central differences of L = sum(w * z)
    on 32 coordinates of x and 32 of y per pair and along one random
    direction (x and y together) per pair.  L is bilinear, so a central
    difference has no truncation error, only rounding."""
    from concurrent.futures import ThreadPoolExecutor
    D, B = 16, 64
    xs = np.stack([hc_inputs.pair_masses(D, hc_inputs.W_BACKWARD, p)[0] for p in range(B)])
    ys = np.stack([hc_inputs.pair_masses(D, hc_inputs.W_BACKWARD, p)[1] for p in range(B)])
    X, Y = on_gpu(xs), on_gpu(ys)
    W = torch.empty((B, 3 ** D), dtype=torch.float64, device=DEV)
    for p in range(B):
        W[p] = on_gpu(hc_inputs.loss_weights(D, hc_inputs.W_BACKWARD, p))
    say("backward 64xD16: GPU")
    gx, gy = hc.convolve_backward(X, Y, W)
    torch.cuda.synchronize(DEV)
    gx, gy = gx.cpu().numpy(), gy.cpu().numpy()

    def host_check(p):
        w = hc_inputs.loss_weights(D, hc_inputs.W_BACKWARD, p)
        ox, oy = oracle.adjoint(xs[p], ys[p], w)
        pins.assert_bitwise(gx[p], ox, f"grad_x pair {p}")
        pins.assert_bitwise(gy[p], oy, f"grad_y pair {p}")
        idx = np.random.default_rng([hc_inputs.SEED, 78, p]).integers(0, 1 << D, 256).astype(np.uint64)
        cx, cy = oracle.correlation_at(xs[p], ys[p], w, idx)
        bx, by = oracle.adjoint_bound(xs[p], ys[p], w)
        ii = idx.astype(np.int64)
        tol = (4 * D + 2) * U64
        assert np.all(np.abs(gx[p][ii] - cx) <= tol * bx[ii] + 2.0 ** -60 * np.abs(cx)), f"pair {p} x"
        assert np.all(np.abs(gy[p][ii] - cy) <= tol * by[ii] + 2.0 ** -60 * np.abs(cy)), f"pair {p} y"
        return p

    t0 = time.time()
    with ThreadPoolExecutor(8) as ex:
        done = list(ex.map(host_check, range(B)))
    assert done == list(range(B))
    say(f"backward 64xD16: all pairs bitwise against the transposed maps ({time.time() - t0:.1f} s)")

    h = 1e-6

    def loss(a, b, p):
        return torch.dot(hc.convolve(a, b), W[p])

    t0 = time.time()
    for p in range(B):
        g = np.random.default_rng([hc_inputs.SEED, 79, p])
        ix = g.integers(0, 1 << D, 32)
        iy = g.integers(0, 1 << D, 32)
        x0, y0 = X[p], Y[p]
        fds = []
        for i in ix:
            xp = x0.clone(); xp[i] += h
            xm = x0.clone(); xm[i] -= h
            fds.append((loss(xp, y0, p) - loss(xm, y0, p)) / (2 * h))
        for i in iy:
            yp = y0.clone(); yp[i] += h
            ym = y0.clone(); ym[i] -= h
            fds.append((loss(x0, yp, p) - loss(x0, ym, p)) / (2 * h))
        vx = torch.from_numpy(g.standard_normal(1 << D)).to(DEV)
        vy = torch.from_numpy(g.standard_normal(1 << D)).to(DEV)
        fds.append((loss(x0 + h * vx, y0 + h * vy, p) - loss(x0 - h * vx, y0 - h * vy, p)) / (2 * h))
        fd = torch.stack(fds).cpu().numpy()
        sx, sy = float(np.max(np.abs(gx[p]))), float(np.max(np.abs(gy[p])))
        assert np.all(np.abs(fd[:32] - gx[p][ix]) <= 1e-6 * sx), f"pair {p}: x coordinates"
        assert np.all(np.abs(fd[32:64] - gy[p][iy]) <= 1e-6 * sy), f"pair {p}: y coordinates"
        vxh, vyh = vx.cpu().numpy(), vy.cpu().numpy()
        dd = float(gx[p] @ vxh + gy[p] @ vyh)
        scale = float(np.linalg.norm(gx[p]) * np.linalg.norm(vxh) + np.linalg.norm(gy[p]) * np.linalg.norm(vyh))
        assert abs(fd[64] - dd) <= 1e-9 * scale, f"pair {p}: direction {fd[64]} vs {dd}"
    say(f"backward 64xD16: central differences on every pair ({time.time() - t0:.1f} s)")


def test_d21_f64_every_output_bitwise():
    """D = 21, the largest D accepted (84 GB of float64 output): every output
    bitwise against the recursion on 16 host threads, compared in chunks;
    sampled outputs within the certified bound of the definition, and the
    total mass."""
    D = 21
    n3 = 3 ** D
    g = np.random.default_rng([hc_inputs.SEED, 80, D])
    x = g.random(1 << D)
    x /= x.sum()
    y = g.random(1 << D)
    y /= y.sum()
    say("D=21 float64: GPU")
    z = hc.convolve(on_gpu(x), on_gpu(y))
    torch.cuda.synchronize(DEV)
    assert z.numel() == n3
    t0 = time.time()
    ref = oracle.recursive(x, y, threads=16)
    say(f"D=21 float64: oracle recursion in {time.time() - t0:.1f} s; comparing")
    chunk = 1 << 28
    mismatches = 0
    for c0 in range(0, n3, chunk):
        c1 = min(n3, c0 + chunk)
        part = z[c0:c1].cpu().numpy()
        mismatches += int(np.count_nonzero(part.view(np.uint64) != ref[c0:c1].view(np.uint64)))
    say(f"D=21 float64: {mismatches} of {n3} outputs differ")
    assert mismatches == 0
    del ref
    ks = sample_indices(D, 256, 3)
    z_at = z[torch.from_numpy(ks.astype(np.int64)).to(DEV)].cpu().numpy()
    r = check_against_definition(x, y, z_at, ks, D)
    total = float(z.sum().item())
    assert abs(total - float(x.sum()) * float(y.sum())) < 1e-12
    say(f"D=21 float64: max |err|/(u B) over {ks.size} sampled outputs = {r:.2f}; sum z - 1 = {total - 1:.2e}")
    del z
    torch.cuda.empty_cache()


def test_maxconv_d20_root_in_last_pass():
    """The benchmark's p-norm max-convolution (D = 20 float64, p = 32, the
    root in the last inverse pass): bitwise equal to the separate root kernel
    on the GPU, and sampled outputs within the error model's tolerance of the
    oracle's p-norm."""
    from tests.test_gpu_apps import pnorm_tolerance
    D, p = 20, 32.0
    x, y = hc_inputs.pair_masses(D, hc_inputs.W_D20_F64)
    tx, ty = on_gpu(x), on_gpu(y)
    say("D=20 max-convolution: GPU, root in the last pass and separate")
    za = hc.maxconv_pnorm(tx, ty, p)
    zb = hc.maxconv_pnorm(tx, ty, p, separate_root=True)
    torch.cuda.synchronize(DEV)
    assert torch.equal(za.view(torch.int64), zb.view(torch.int64))
    del zb
    ks = sample_indices(D, 200, 3)
    z_at = za[torch.from_numpy(ks.astype(np.int64)).to(DEV)].cpu().numpy()
    ref = oracle.pnorm_at(x, y, p, ks)
    tol, _ = pnorm_tolerance(x, y, p, D, ref, np.float64, ks=ks)
    err = np.abs(z_at - ref)
    say(f"D=20 max-convolution: max err/tol over {ks.size} samples = {np.max(err / tol):.3g}")
    assert np.all(err <= tol)
    del za
    torch.cuda.empty_cache()
