#!/usr/bin/env python3
"""Benchmark of exact hypercube convolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload d20]

A step is one full pass of the method (outer forward, fused inner tiles,
outer inverse passes) over the workload, with inputs already resident in HBM.
Prints ONE JSON line: output elements per second for the workload, the
roofline of the dominant kernel (algorithmic bytes per launch over its
HIP-event-timed duration on the launch stream, against the 8 TB/s HBM peak),
and the CPU oracle timed on a bounded sample of the same workload.

Workloads (inputs from hc_inputs, seeded and synthetic):
  all       (default) d20 as the headline value, plus d10, d16-f64,
            d16-i64 (each with every output compared to the oracle),
            batched, backward and apps measured after it and reported under
            "secondary"
  d20       one pair, D=20, float64 masses (3^20 outputs)
  d20-f32   the same pair in float32
  d16-f64   one pair, D=16, float64 masses
  d16-i64   one pair, D=16, int64 values in [0, 15]
  d10       one pair, D=10, float64 masses
  batched   4096 pairs, D uniform in {6..14}, masses, float64 and float32
  backward  64 pairs at D=16 float64, forward + backward of sum(w * z)
  apps      carry-free convolution of two length-10^6 vectors, the
            distribution of X - Y and the p-norm max-convolution (p = 32),
            both at D=20 (float64), and the distribution of X1 + X2 + X3
            at D=14 (float64, 4^14 outputs)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3^D output elems/sec + % HBM peak, D=20 fp64; batched pairs/s; fwd+bwd time"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1608_00206_amd", "csrc", f)
                  for f in ("hc_device.hpp", "hc_kernels.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` in `workload` from committed rocprofv3
    counter runs (FETCH_SIZE and WRITE_SIZE, scaled by a copy-kernel
    calibration), or None when none were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    k = t.get("workloads", {}).get(workload, {}).get(kernel)
    if not k:
        return None
    return (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"]) * 1024.0


COPY_CAL_BYTES = 1 << 31  # read once and written once by the calibration copy


def copy_calibration(torch) -> None:
    """One plain copy kernel over a known number of bytes (torch's elementwise
    negation: every element read once, written once), run before the
    workload so that a rocprofv3 counter pass sees it beside the kernels."""
    n = COPY_CAL_BYTES // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    log(f"copy calibration: {COPY_CAL_BYTES} bytes read, {COPY_CAL_BYTES} bytes written")


_DT = {"double": "f64", "float": "f32", "long": "i64", "long long": "i64"}


def profiler_name(demangled: str):
    """The library profiler's name for a kernel from its demangled symbol."""
    m = re.match(r"(?:void )?hc::k_(\w+)<([^,>]+)((?:, *[^,>]+)*)>", demangled)
    if not m:
        return None
    base, dt = m.group(1), _DT.get(m.group(2).strip())
    args = [a.strip() for a in m.group(3).split(",") if a.strip()]
    if dt is None:
        return None
    if base == "inv_pass":
        kind = "inv_adj_pass" if args[3] == "true" else "inv_pass"
        return f"{kind}<{dt},{args[0]}+{args[1]}>"
    if base == "fused_inner":
        return f"{base}<{dt},K={args[0]}>"
    if base == "fused_inner_adj":
        return f"{base}<{dt},K={args[0]},t={args[2]}>"
    if base in ("fwd_pass", "fwd_adj_pass"):
        return f"{base}<{dt},M={args[0]}>"
    return None


def write_traffic(args) -> None:
    """Turns rocprofv3 counter passes into the traffic table.  `args` lists
    triples WORKLOAD FETCH_CSV WRITE_CSV, each pair of passes taken over one
    `--workload WORKLOAD --copy-calibration` run: KiB per dispatch averaged
    per kernel and workload, and the factors that map each counter onto the
    calibration copy's known bytes (averaged over the runs)."""
    import csv

    if len(args) % 3:
        raise SystemExit("--write-traffic takes WORKLOAD FETCH_CSV WRITE_CSV triples")

    def per_kernel(path, counter):
        # dispatches of one kernel whose grid is under half the largest grid
        # of that kernel in the run (the shared-weight backward's single-item
        # passes) are different launches from the timed ones and are left out
        rows, cal = {}, []
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name, val = row["Kernel_Name"], float(row["Counter_Value"])
                if "neg" in name and "hc::" not in name:
                    cal.append(val)
                    continue
                pn = profiler_name(name)
                if pn is not None:
                    rows.setdefault(pn, []).append((int(row["Grid_Size"]), val))
        if len(cal) != 1:
            raise SystemExit(f"{path}: expected one calibration copy dispatch, found {len(cal)}")
        acc = {}
        for pn, lst in rows.items():
            top = max(g for g, _ in lst)
            acc[pn] = [v for g, v in lst if 2 * g >= top]
        return acc, cal[0]

    workloads, fcals, wcals = {}, [], []
    for i in range(0, len(args), 3):
        wl, fpath, wpath = args[i:i + 3]
        f, fc = per_kernel(fpath, "FETCH_SIZE")
        w, wc = per_kernel(wpath, "WRITE_SIZE")
        fcals.append(fc)
        wcals.append(wc)
        workloads[wl] = {k: {"fetch_kib": sum(f[k]) / len(f[k]), "write_kib": sum(w[k]) / len(w[k])}
                         for k in sorted(f) if k in w}
    fcal = sum(fcals) / len(fcals)
    wcal = sum(wcals) / len(wcals)
    out = {"kernel_source_sha": kernel_source_hash(), "unit": "KiB per dispatch",
           "copy_calibration_bytes": COPY_CAL_BYTES, "copy_fetch_kib": fcal, "copy_write_kib": wcal,
           "fetch_scale": COPY_CAL_BYTES / (fcal * 1024.0), "write_scale": COPY_CAL_BYTES / (wcal * 1024.0),
           "workloads": workloads}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


def time_steps(fn, steps: int, warmup: int, torch):
    """Runs fn warmup times, then times exactly `steps` calls bracketed by
    device synchronisation; the library profiler records every launch."""
    from paper_1608_00206_amd import _abi
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    _abi.hc_profile_collect()  # drop anything recorded so far
    _abi.hc_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _abi.hc_profile_enable(False)
    stats = _abi.hc_profile_collect()
    return ev0.elapsed_time(ev1) / steps, wall, stats


def roofline(stats, steps: int, workload: str):
    dom = max(stats, key=lambda s: s[2])
    name, launches, total_ms, alg_bytes = dom
    avg_s = total_ms / launches / 1e3
    per_launch = alg_bytes / launches
    achieved = per_launch / avg_s / 1e9
    traffic = measured_traffic(name, workload)
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "alg_bytes_per_launch": round(per_launch), "avg_launch_ms": round(avg_s * 1e3, 4)}


def kernel_table(stats, steps):
    out = []
    for name, launches, total_ms, alg_bytes in sorted(stats, key=lambda s: -s[2]):
        avg_ms = total_ms / launches
        out.append({"kernel": name, "launches_per_step": launches / steps, "avg_ms": round(avg_ms, 4),
                    "alg_GBps": round(alg_bytes / launches / (avg_ms / 1e3) / 1e9, 1)})
    return out


def cpu_baseline(x, y, z_gpu, D):
    """The oracle (the three-subproblem recursion) timed on the workload
    itself, on up to 16 host threads; the GPU output is then compared with
    it bit for bit, chunk by chunk."""
    import numpy as np

    import oracle
    threads = host_threads()
    out = np.empty(3 ** D, dtype=x.dtype)
    log(f"cpu baseline: oracle recursion D={D} on {threads} threads")
    t0 = time.perf_counter()
    oracle.recursive(x, y, threads=threads, out=out)
    dt = time.perf_counter() - t0
    equal = True
    chunk = 1 << 26
    for s in range(0, out.size, chunk):
        e = min(s + chunk, out.size)
        g = z_gpu[s:e].cpu().numpy()
        iv = np.int32 if g.dtype.itemsize == 4 else np.int64
        if not np.array_equal(g.view(iv), out[s:e].view(iv)):
            equal = False
            break
    log(f"cpu baseline: {dt:.2f} s; GPU output bitwise equal: {equal}")
    del out
    # the same recursion on one thread, as the paper times its own method, on
    # a smaller pair of the same kind
    import hc_inputs
    Ds = min(D, 17)
    xs, ys = hc_inputs.pair_masses(Ds, hc_inputs.W_D20_F64)
    t0 = time.perf_counter()
    oracle.recursive(xs, ys, threads=1)
    dt1 = time.perf_counter() - t0
    log(f"cpu baseline, one thread, D={Ds}: {dt1:.2f} s")
    return {"value": round(3 ** D / dt, 1), "unit": "output elems/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole workload (one D={D} pair), three-subproblem recursion",
            "seconds": round(dt, 3), "gpu_output_bitwise_equal": equal, "cpu_model": cpu_model(),
            "host_nproc": os.cpu_count(), "host_cpus_allowed": len(os.sched_getaffinity(0)),
            "single_thread": {"value": round(3 ** Ds / dt1, 1), "unit": "output elems/s", "cores": 1,
                              "sample": f"one D={Ds} float64 pair of the same distribution",
                              "seconds": round(dt1, 3)}}


# Host CPUs the job may use: every CPU the process is allowed to run on, at
# most 16 (the host CPU share that comes with one GPU of the machine).
HOST_CPU_SHARE = 16


def host_threads() -> int:
    return max(1, min(HOST_CPU_SHARE, len(os.sched_getaffinity(0))))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_single(args, torch, hc, D, dtype_name, steps=None, warmup=None, cpu=True, parity=False):
    import numpy as np

    import hc_inputs
    dev = torch.device("cuda:0")
    if dtype_name == "i64":
        x, y = hc_inputs.pair_ints(D, hc_inputs.W_D16)
        tdt = torch.int64
        desc = f"single pair D={D} int64, iid integers in [0,15] (seeded)"
    elif dtype_name == "f32":
        x, y = hc_inputs.pair_masses(D, hc_inputs.W_D20_F64)
        x, y = x.astype(np.float32), y.astype(np.float32)
        tdt = torch.float32
        desc = f"single pair D={D} float32, iid U[0,1) normalised to sum 1 in float64, then rounded (seeded)"
    else:
        wl = {20: hc_inputs.W_D20_F64, 16: hc_inputs.W_D16, 10: hc_inputs.W_D10_F64}[D]
        x, y = hc_inputs.pair_masses(D, wl)
        tdt = torch.float64
        desc = f"single pair D={D} float64, iid U[0,1) normalised to sum 1 (seeded)"
    tx = torch.from_numpy(x).to(dev)
    ty = torch.from_numpy(y).to(dev)
    z = torch.empty(3 ** D, dtype=tdt, device=dev)
    hc.convolve(tx, ty, out=z)  # first call outside the timed region: module load
    nb = hc.workspace_bytes(D, tdt)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    log(f"workload {desc}: z {z.numel() * z.element_size() / 1e9:.2f} GB, workspace {nb / 1e9:.2f} GB")

    def step():
        hc.convolve(tx, ty, out=z, workspace=ws)

    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    ms, wall, stats = time_steps(step, steps, warmup, torch)
    log(f"timed {steps} steps: {ms:.3f} ms/step (wall {wall:.3f} s)")
    n_out = 3 ** D
    wl_name = {("f64", 20): "d20", ("f32", 20): "d20-f32", ("f64", 16): "d16-f64", ("i64", 16): "d16-i64",
               ("f64", 10): "d10"}.get((dtype_name, D), f"d{D}-{dtype_name}")
    res = {
        "metric": METRIC, "value": round(n_out / (ms / 1e3), 1), "unit": "output elems/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_name, "data": "synthetic",
        "config": {"workload": desc, "D": D, "outputs_per_step": n_out, "global_batch": 1,
                   "parallelism": "single GPU"},
        "roofline": roofline(stats, steps, wl_name),
        "compulsory_hbm_frac": round((n_out + 2 * (1 << D)) * z.element_size() / (ms / 1e3) / 1e9
                                     / HBM_PEAK_GBS, 4),
        "kernels": kernel_table(stats, steps),
    }
    if parity:
        # every output bitwise against the oracle's recursion (which the CPU
        # tests pin to Algorithm 1 and to the per-axis method)
        import oracle
        ref = oracle.recursive(x, y, threads=host_threads())
        iv = np.int32 if ref.dtype.itemsize == 4 else np.int64
        res["oracle_bitwise_equal"] = bool(np.array_equal(z.cpu().numpy().view(iv), ref.view(iv)))
        log(f"{wl_name}: every output bitwise equal to the oracle: {res['oracle_bitwise_equal']}")
    if cpu and not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(x, y, z, D)
    del z, ws
    return res


def run_apps(args, torch, hc, steps=None, warmup=None):
    """The applications built on the forward path (Discussion): carry-free
    convolution of two length-10^6 float64 vectors (D = 20 after padding) and
    the distribution of X - Y for two D = 20 float64 distributions."""
    import numpy as np

    import hc_inputs
    dev = torch.device("cuda:0")
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    out = {}
    n = 1_000_000
    g = hc_inputs.rng(hc_inputs.W_D20_F64, 0, 9)
    x = torch.from_numpy(g.random(n)).to(dev)
    y = torch.from_numpy(g.random(n)).to(dev)
    D = hc.carryfree_dim(n)
    z = torch.empty(3 ** D, dtype=torch.float64, device=dev)
    ws = torch.empty(hc._abi.hc_carryfree_workspace_bytes(n, hc._abi.HC_F64), dtype=torch.uint8, device=dev)
    ms, _, st = time_steps(lambda: hc.carryfree_convolve(x, y, out=z, workspace=ws), steps, warmup, torch)
    log(f"carry-free n={n}: {ms:.3f} ms/step")
    out["carryfree_n1e6_f64"] = {"n": n, "D": D, "ms_per_step": round(ms, 4),
                                 "output_elems_per_s": round(3 ** D / (ms / 1e3), 1),
                                 "kernels": kernel_table(st, steps)}
    del x, y, ws
    D = 20
    xa, ya = hc_inputs.pair_masses(D, hc_inputs.W_D20_F64)
    x = torch.from_numpy(xa).to(dev)
    y = torch.from_numpy(ya).to(dev)
    ws = torch.empty(hc._abi.hc_difference_workspace_bytes(D, hc._abi.HC_F64, 1), dtype=torch.uint8, device=dev)
    ms, _, st = time_steps(lambda: hc.difference(x, y, out=z, workspace=ws), steps, warmup, torch)
    log(f"difference D={D}: {ms:.3f} ms/step")
    out["difference_D20_f64"] = {"D": D, "ms_per_step": round(ms, 4),
                                 "output_elems_per_s": round(3 ** D / (ms / 1e3), 1),
                                 "kernels": kernel_table(st, steps)}
    del ws
    ws = torch.empty(hc._abi.hc_maxconv_workspace_bytes(D, hc._abi.HC_F64, 1), dtype=torch.uint8, device=dev)
    ms, _, st = time_steps(lambda: hc.maxconv_pnorm(x, y, 32.0, out=z, workspace=ws), steps, warmup, torch)
    log(f"p-norm max-convolution D={D} p=32: {ms:.3f} ms/step")
    out["maxconv_p32_D20_f64"] = {"D": D, "p": 32.0, "ms_per_step": round(ms, 4),
                                  "output_elems_per_s": round(3 ** D / (ms / 1e3), 1),
                                  "kernels": kernel_table(st, steps)}
    del x, y, z, ws
    torch.cuda.empty_cache()
    # distribution of X1 + X2 + X3 (three Bernoulli-axis vectors), D = 14
    D = 14
    xs = [torch.from_numpy(hc_inputs.masses(D, hc_inputs.W_D16, 0, role)).to(dev) for role in range(3)]
    z = torch.empty(4 ** D, dtype=torch.float64, device=dev)
    ws = torch.empty(max(hc._abi.hc_sum3_workspace_bytes(D, hc._abi.HC_F64, 1), 1), dtype=torch.uint8, device=dev)
    ms, _, st = time_steps(lambda: hc.sum3(*xs, out=z, workspace=ws), steps, warmup, torch)
    log(f"sum of three D={D}: {ms:.3f} ms/step")
    out["sum3_D14_f64"] = {"D": D, "ms_per_step": round(ms, 4), "output_elems_per_s": round(4 ** D / (ms / 1e3), 1),
                           "kernels": kernel_table(st, steps)}
    del xs, z, ws
    torch.cuda.empty_cache()
    # distribution of X1 + X2 + X3 + X4, D = 12: the two pair sums, then
    # their ternary convolution
    D = 12
    xs = [torch.from_numpy(hc_inputs.masses(D, hc_inputs.W_D16, 1, role)).to(dev) for role in range(4)]
    p12 = torch.empty(3 ** D, dtype=torch.float64, device=dev)
    p34 = torch.empty(3 ** D, dtype=torch.float64, device=dev)
    z = torch.empty(5 ** D, dtype=torch.float64, device=dev)
    ws = torch.empty(max(hc._abi.hc_ternary_workspace_bytes(D, hc._abi.HC_F64, 1), hc.workspace_bytes(D, torch.float64),
                         1), dtype=torch.uint8, device=dev)

    def sum4_step():
        hc.convolve(xs[0], xs[1], out=p12, workspace=ws)
        hc.convolve(xs[2], xs[3], out=p34, workspace=ws)
        hc.ternary_convolve(p12, p34, out=z, workspace=ws)
    ms, _, st = time_steps(sum4_step, steps, warmup, torch)
    log(f"sum of four D={D}: {ms:.3f} ms/step")
    out["sum4_D12_f64"] = {"D": D, "ms_per_step": round(ms, 4), "output_elems_per_s": round(5 ** D / (ms / 1e3), 1),
                           "kernels": kernel_table(st, steps)}
    del xs, p12, p34, z, ws
    torch.cuda.empty_cache()
    return out


def run_batched(args, torch, hc, steps=None, warmup=None):
    """4096 pairs with D drawn uniformly from {6, ..., 14}: one graph launch of
    the batched plan per step, in float64 and float32; compared with a loop
    of single-pair calls, and (float32) against the float64 oracle on a
    sample of pairs.  The same batch is also timed as one persistent kernel
    launch (a workgroup per pair) and compared with the graph bit for bit."""
    import numpy as np

    import hc_inputs
    import oracle
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    dev = torch.device("cuda:0")
    Ds = hc_inputs.batched_dims(4096)
    xs = [hc_inputs.pair_masses(int(D), hc_inputs.W_BATCHED, i) for i, D in enumerate(Ds)]
    out = {"pairs": int(len(Ds)), "outputs": int(sum(3 ** int(D) for D in Ds))}
    for tdt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        npdt = np.float64 if name == "f64" else np.float32
        plan = hc.BatchedPlan(Ds, tdt, tune=True)
        X = torch.from_numpy(np.concatenate([a.astype(npdt) for a, _ in xs])).to(dev)
        Y = torch.from_numpy(np.concatenate([b.astype(npdt) for _, b in xs])).to(dev)
        Z = torch.empty(plan.n_outputs, dtype=tdt, device=dev)
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        log(f"batched {name}: {len(Ds)} pairs, z {Z.numel() * Z.element_size() / 1e9:.1f} GB; schedule "
            f"{[(g['D'], g['items'], g['K'], g['inverse_groups']) for g in plan.schedule['groups']]}")
        ms, _, stats = time_steps(lambda: plan.run(X, Y, out=Z, workspace=ws), steps, warmup, torch)
        plan.check()
        # the same pairs as a loop of single-pair calls (one call per pair)
        xo, zo = plan.x_offsets, plan.z_offsets
        Zl = torch.empty_like(Z)
        wsl = torch.empty(max(hc.workspace_bytes(14, tdt), 1), dtype=torch.uint8, device=dev)

        def loop():
            for i, D in enumerate(Ds):
                hc.convolve(X[xo[i]:xo[i + 1]], Y[xo[i]:xo[i + 1]], out=Zl[zo[i]:zo[i + 1]], workspace=wsl)

        ms_loop, _, _ = time_steps(loop, 2, 1, torch)
        same = bool(torch.equal(Z.view(torch.int64 if name == "f64" else torch.int32),
                                Zl.view(torch.int64 if name == "f64" else torch.int32)))
        res = {"ms_per_step": round(ms, 3), "pairs_per_s": round(len(Ds) / (ms / 1e3), 1),
               "outputs_per_s": round(out["outputs"] / (ms / 1e3), 1),
               "loop_of_single_calls_ms": round(ms_loop, 3), "speedup_vs_loop": round(ms_loop / ms, 2),
               "bitwise_equal_to_loop": same, "kernels": kernel_table(stats, steps)}
        # parity on a sample of pairs: bitwise against the per-axis oracle in the
        # same precision; float32 error against the float64 oracle reported
        rng = np.random.default_rng(7)
        sample = rng.choice(len(Ds), 16, replace=False)
        worst32 = 0.0
        ok = True
        for i in sample:
            zi = Z[zo[i]:zo[i + 1]].cpu().numpy()
            xi, yi = xs[i][0].astype(npdt), xs[i][1].astype(npdt)
            ok &= bool(np.array_equal(zi.view(np.int64 if name == "f64" else np.int32),
                                      oracle.canonical(xi, yi).view(np.int64 if name == "f64" else np.int32)))
            if name == "f32":
                r64 = oracle.canonical(xs[i][0], xs[i][1])
                worst32 = max(worst32, float(np.abs(zi.astype(np.float64) - r64).max() / np.abs(r64).max()))
        res["sample_pairs_bitwise_equal_oracle"] = ok
        if name == "f32":
            res["f32_vs_f64_oracle_max_rel_err"] = worst32
        del Zl, wsl
        # the same batch as one persistent kernel launch, a workgroup per pair
        pplan = hc.BatchedPlan(Ds, tdt, tune=True, persistent_pairs=True)
        Zp = torch.empty_like(Z)
        wsp = torch.empty(max(pplan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        ms_p, _, stats_p = time_steps(lambda: pplan.run(X, Y, out=Zp, workspace=wsp), steps, warmup, torch)
        pplan.check()
        iv = torch.int64 if name == "f64" else torch.int32
        res["persistent_pairs"] = {
            "ms_per_step": round(ms_p, 3), "pairs_per_s": round(len(Ds) / (ms_p / 1e3), 1),
            "outputs_per_s": round(out["outputs"] / (ms_p / 1e3), 1), "grid": pplan.schedule["grid"],
            "workgroups_per_cu": pplan.schedule["workgroups_per_cu"],
            "schedule": [[g["D"], g["forward_groups"], g["inverse_groups"]] for g in pplan.schedule["groups"]],
            "bitwise_equal_to_graph": bool(torch.equal(Zp.view(iv), Z.view(iv))), "kernels": kernel_table(stats_p, steps)}
        out[name] = res
        log(f"batched {name}: {ms:.3f} ms/step, loop of single calls {ms_loop:.3f} ms, sample parity {ok}; "
            f"one persistent launch {ms_p:.3f} ms/step")
        del X, Y, Z, ws, Zp, wsp
        pplan.close()
        plan.close()
        torch.cuda.empty_cache()
    return out


def run_backward(args, torch, hc, steps=None, warmup=None):
    """64 pairs at D=16 float64, forward then backward of L = sum(w * z)."""
    import numpy as np

    import hc_inputs
    dev = torch.device("cuda:0")
    D, B = 16, 64
    X = torch.from_numpy(np.stack([hc_inputs.pair_masses(D, hc_inputs.W_BACKWARD, b)[0] for b in range(B)])).to(dev)
    Y = torch.from_numpy(np.stack([hc_inputs.pair_masses(D, hc_inputs.W_BACKWARD, b)[1] for b in range(B)])).to(dev)
    W = torch.empty((B, 3 ** D), dtype=torch.float64, device=dev)
    for b in range(B):
        W[b].copy_(torch.from_numpy(hc_inputs.loss_weights(D, pair=b)))
    Z = torch.empty((B, 3 ** D), dtype=torch.float64, device=dev)
    wsf = torch.empty(max(hc.workspace_bytes(D, torch.float64, B), 1), dtype=torch.uint8, device=dev)
    wsb = torch.empty(max(hc.backward_workspace_bytes(D, torch.float64, B), 1), dtype=torch.uint8, device=dev)
    log(f"workload backward: {B} pairs D={D}; z and w {2 * Z.numel() * 8 / 1e9:.1f} GB")

    def fwd():
        hc.convolve_batch(X, Y, out=Z, workspace=wsf)

    def bwd():
        hc.convolve_backward(X, Y, W, workspace=wsb)

    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    fwd_ms, _, fstats = time_steps(fwd, steps, warmup, torch)
    bwd_ms, _, bstats = time_steps(bwd, steps, warmup, torch)
    log(f"backward: fwd {fwd_ms:.3f} ms, bwd {bwd_ms:.3f} ms")
    # the same backward with one weight vector shared by all pairs (grad_z
    # with batch stride 0): the library computes its adjoint transform once
    Wb = W[0].expand(B, 3 ** D)

    def bwd_shared():
        hc.convolve_backward(X, Y, Wb, workspace=wsb)

    bwd_shared_ms, _, _ = time_steps(bwd_shared, steps, warmup, torch)
    log(f"backward with one shared w: {bwd_shared_ms:.3f} ms")
    n_out = B * 3 ** D
    del Z, wsf, wsb, W, Wb
    torch.cuda.empty_cache()
    return {
        "metric": METRIC, "value": round(n_out / ((fwd_ms + bwd_ms) / 1e3), 1), "unit": "output elems/s (fwd+bwd)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fwd_ms + bwd_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{B} pairs D={D} float64 masses, loss sum(w*z), w iid N(0,1) per pair",
                   "D": D, "global_batch": B, "parallelism": "single GPU"},
        "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4), "fwd_bwd_ms": round(fwd_ms + bwd_ms, 4),
        "bwd_shared_w_ms": round(bwd_shared_ms, 4),
        "roofline": roofline(bstats, steps, "backward"),
        "kernels": kernel_table(fstats, steps) + kernel_table(bstats, steps),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all",
                    choices=["all", "d20", "d20-f32", "d16-f64", "d16-i64", "d10", "batched", "backward", "apps"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain copy kernel of known size before the workload (for counter passes)")
    ap.add_argument("--write-traffic", nargs="+", metavar="ARG",
                    help="write profiles/traffic.json from rocprofv3 counter CSVs given as WORKLOAD FETCH_CSV "
                         "WRITE_CSV triples, and exit")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1608_00206_amd as hc
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
    if args.workload == "backward":
        res = run_backward(args, torch, hc)
    elif args.workload == "apps":
        res = {"metric": METRIC, "applications": run_apps(args, torch, hc)}
    elif args.workload == "batched":
        b = run_batched(args, torch, hc)
        res = {"metric": METRIC, "value": b["f64"]["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["f64"]["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic", "config": {"workload": "4096 pairs, D uniform in {6..14}, masses",
                                               "global_batch": 4096, "parallelism": "single GPU"},
               "batched": b}
    else:
        D = {"all": 20, "d20": 20, "d20-f32": 20, "d16-f64": 16, "d16-i64": 16, "d10": 10}[args.workload]
        dt = {"d16-i64": "i64", "d20-f32": "f32"}.get(args.workload, "f64")
        res = run_single(args, torch, hc, D, dt)
        if args.workload == "all":
            # the other parts of the metric, measured after the headline and
            # outside its timed region
            torch.cuda.empty_cache()
            sec_steps = max(2, min(args.steps, 5))
            single = {}
            for name, Dq, dq, n_steps in (("d10_f64", 10, "f64", 200), ("d16_f64", 16, "f64", 20),
                                          ("d16_i64", 16, "i64", 20)):
                r = run_single(args, torch, hc, Dq, dq, n_steps, 5, cpu=False, parity=True)
                single[name] = {k: r[k] for k in ("value", "unit", "ms_per_step", "steps", "dtype", "config",
                                                  "roofline", "kernels", "oracle_bitwise_equal")}
            torch.cuda.empty_cache()
            res["secondary"] = {**single,
                                "batched_4096_pairs": run_batched(args, torch, hc, sec_steps, 1),
                                "backward_64xD16_f64": run_backward(args, torch, hc, sec_steps, 1),
                                "applications": run_apps(args, torch, hc, sec_steps, 1)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
