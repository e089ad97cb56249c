"""GPU parity of batched plans (ragged pairs grouped by D, one graph launch)
against the per-pair oracle and against single-pair calls."""
import numpy as np
import pytest
import torch

import hc_inputs
import oracle
import paper_1608_00206_amd as hc
from tests import pins

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
NP2T = {np.dtype(np.float64): torch.float64, np.dtype(np.float32): torch.float32, np.dtype(np.int64): torch.int64}


def packed_inputs(Ds, dtype, seed):
    xs, ys = [], []
    for i, D in enumerate(Ds):
        kind = "int" if dtype == np.int64 else "mass"
        x, y = hc_inputs.random_pair(D, dtype, seed * 1000 + i, kind)
        xs.append(x)
        ys.append(y)
    return xs, ys


def run_plan(plan, xs, ys):
    X = torch.from_numpy(np.concatenate(xs)).to(DEV)
    Y = torch.from_numpy(np.concatenate(ys)).to(DEV)
    Z = plan.run(X, Y)
    plan.check()
    return Z.cpu().numpy()


def check_pairs(plan, Ds, xs, ys, Z):
    zo = plan.z_offsets
    for i in range(len(Ds)):
        pins.assert_bitwise(Z[zo[i]:zo[i + 1]], oracle.canonical(xs[i], ys[i]), f"pair {i} D={Ds[i]}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int64])
def test_batched_matches_oracle(dtype):
    Ds = [0, 1, 5, 8, 9, 12, 3, 10, 13, 6, 11, 2, 14, 7, 9]
    plan = hc.BatchedPlan(Ds, NP2T[np.dtype(dtype)])
    xs, ys = packed_inputs(Ds, dtype, seed=1)
    check_pairs(plan, Ds, xs, ys, run_plan(plan, xs, ys))
    plan.close()


def test_batched_many_pairs_config_mix():
    """A slice of the batched workload: D drawn from {6, ..., 14}."""
    Ds = hc_inputs.batched_dims(96)
    plan = hc.BatchedPlan(Ds, torch.float64)
    xs = [hc_inputs.pair_masses(int(D), hc_inputs.W_BATCHED, i)[0] for i, D in enumerate(Ds)]
    ys = [hc_inputs.pair_masses(int(D), hc_inputs.W_BATCHED, i)[1] for i, D in enumerate(Ds)]
    Z = run_plan(plan, xs, ys)
    check_pairs(plan, Ds, xs, ys, Z)


def test_batched_equals_single_pair_calls():
    Ds = [7, 12, 9, 13]
    plan = hc.BatchedPlan(Ds, torch.float64)
    xs, ys = packed_inputs(Ds, np.float64, seed=2)
    Z = run_plan(plan, xs, ys)
    for i, D in enumerate(Ds):
        z1 = hc.convolve(torch.from_numpy(xs[i]).to(DEV), torch.from_numpy(ys[i]).to(DEV)).cpu().numpy()
        pins.assert_bitwise(Z[plan.z_offsets[i]:plan.z_offsets[i + 1]], z1, f"pair {i}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_tuned_plan_and_cache(dtype, tmp_path, monkeypatch):
    monkeypatch.setenv("HC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    Ds = [6, 9, 11, 12, 8, 10, 12]
    plan = hc.BatchedPlan(Ds, NP2T[np.dtype(dtype)], tune=True)
    assert (tmp_path / "tune.txt").exists()
    again = hc.BatchedPlan(Ds, NP2T[np.dtype(dtype)], tune=True)   # served from the cache
    assert again.schedule == plan.schedule
    xs, ys = packed_inputs(Ds, dtype, seed=3)
    check_pairs(plan, Ds, xs, ys, run_plan(plan, xs, ys))


def test_replay_and_new_buffers():
    """The graph is replayed, and recaptured when the buffers change."""
    Ds = [10, 5, 12]
    plan = hc.BatchedPlan(Ds, torch.float64)
    xs, ys = packed_inputs(Ds, np.float64, seed=4)
    X = torch.from_numpy(np.concatenate(xs)).to(DEV)
    Y = torch.from_numpy(np.concatenate(ys)).to(DEV)
    Z1 = plan.run(X, Y)
    Z2 = plan.run(X, Y, out=torch.empty_like(Z1))
    Z3 = plan.run(X.clone(), Y.clone())
    plan.check()
    for Z in (Z1, Z2, Z3):
        check_pairs(plan, Ds, xs, ys, Z.cpu().numpy())
    for _ in range(3):
        plan.run(X, Y, out=Z1)
    plan.check()
    check_pairs(plan, Ds, xs, ys, Z1.cpu().numpy())


def test_plan_errors():
    with pytest.raises(hc.HCError):
        hc.BatchedPlan([4, 17], torch.float64)
    plan = hc.BatchedPlan([4, 9], torch.float64)
    X = torch.zeros(plan.n_inputs, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        plan.run(X[:-1], X[:-1])
    with pytest.raises(hc.HCError) as e:
        hc._abi.check(hc._abi.hc_plan_execute(plan._h, X.data_ptr(), X.data_ptr(), X.data_ptr() + 8, 0, 0, 0))
    assert e.value.status in ("HC_ERR_ALIAS", "HC_ERR_MISALIGNED", "HC_ERR_WORKSPACE")


@pytest.mark.skip(reason="the single persistent batched kernel (workgroups taking tasks by ticket and "
                         "spinning on per-phase counters) did not complete on MI355X twice; it is disabled "
                         "and the flag raises HC_ERR_UNSUPPORTED")
def test_persistent_batched_kernel():
    Ds = [0, 1, 5, 8, 9, 12, 3, 10, 13, 6, 11, 2, 14, 7, 9]
    plan = hc.BatchedPlan(Ds, torch.float64, persistent=True)
    xs, ys = packed_inputs(Ds, np.float64, seed=1)
    check_pairs(plan, Ds, xs, ys, run_plan(plan, xs, ys))


def test_persistent_request_is_rejected():
    with pytest.raises(hc.HCError) as e:
        hc.BatchedPlan([9, 12], torch.float64, persistent=True)
    assert e.value.status == "HC_ERR_UNSUPPORTED"


# ------------------------------------------- one persistent launch (HC_PLAN_PERSISTENT_PAIRS)

@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int64])
def test_persistent_pairs_match_oracle(dtype):
    """Every schedule shape of the persistent kernel: single tiles (D up to
    the largest fused depth), one to six outer axes (one inverse pass of 1+0,
    2+0, 3+0, 2+2, 3+2 or 4+2), against the oracle pair by pair."""
    Ds = [0, 1, 5, 8, 9, 12, 3, 10, 13, 6, 11, 2, 14, 7, 9, 4]
    print(f"persistent pairs {np.dtype(dtype).name} Ds={Ds}", flush=True)
    plan = hc.BatchedPlan(Ds, NP2T[np.dtype(dtype)], persistent_pairs=True)
    assert plan.schedule["mode"] == "persistent_pairs"
    assert 1 <= plan.schedule["grid"] <= len(Ds)
    xs, ys = packed_inputs(Ds, dtype, seed=11)
    check_pairs(plan, Ds, xs, ys, run_plan(plan, xs, ys))
    plan.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int64])
def test_persistent_pairs_largest_d_equal_single_calls(dtype):
    """D = 15 and 16: three outer forward groups and two inverse passes;
    bitwise equal to single-pair calls."""
    Ds = [16, 3, 15, 9]
    print(f"persistent pairs {np.dtype(dtype).name} Ds={Ds}", flush=True)
    plan = hc.BatchedPlan(Ds, NP2T[np.dtype(dtype)], persistent_pairs=True)
    xs, ys = packed_inputs(Ds, dtype, seed=12)
    Z = run_plan(plan, xs, ys)
    for i, D in enumerate(Ds):
        z1 = hc.convolve(torch.from_numpy(xs[i]).to(DEV), torch.from_numpy(ys[i]).to(DEV)).cpu().numpy()
        pins.assert_bitwise(Z[plan.z_offsets[i]:plan.z_offsets[i + 1]], z1, f"pair {i} D={D}")
    plan.close()


def test_persistent_pairs_many_tickets_per_workgroup():
    """Far more pairs than workgroups: every workgroup takes many tickets.
    Replays of the captured launch (the counters reset themselves) and a new
    set of buffers all give the graph mode's bits."""
    rng = np.random.default_rng(5)
    Ds = [int(d) for d in rng.integers(0, 11, 1500)]
    print(f"persistent pairs f64 {len(Ds)} pairs", flush=True)
    plan = hc.BatchedPlan(Ds, torch.float64, persistent_pairs=True)
    assert plan.schedule["grid"] < len(Ds)
    ref = hc.BatchedPlan(Ds, torch.float64)
    xs, ys = packed_inputs(Ds, np.float64, seed=13)
    X = torch.from_numpy(np.concatenate(xs)).to(DEV)
    Y = torch.from_numpy(np.concatenate(ys)).to(DEV)
    Zr = ref.run(X, Y).cpu().numpy()
    Z1 = plan.run(X, Y)
    for _ in range(3):
        plan.run(X, Y, out=Z1)
    Z2 = plan.run(X.clone(), Y.clone())
    plan.check()
    pins.assert_bitwise(Z1.cpu().numpy(), Zr, "replayed")
    pins.assert_bitwise(Z2.cpu().numpy(), Zr, "new buffers")
    zo = plan.z_offsets
    for i in (0, 1, 777, len(Ds) - 1):
        pins.assert_bitwise(Zr[zo[i]:zo[i + 1]], oracle.canonical(xs[i], ys[i]), f"pair {i}")
    plan.close()
    ref.close()


def test_persistent_pairs_config_mix():
    """A slice of the batched workload (D drawn from {6, ..., 14}), bitwise
    equal to the graph mode and, pair by pair, to the oracle."""
    Ds = hc_inputs.batched_dims(96)
    print(f"persistent pairs f64 config mix {len(Ds)} pairs", flush=True)
    plan = hc.BatchedPlan(Ds, torch.float64, persistent_pairs=True)
    xs = [hc_inputs.pair_masses(int(D), hc_inputs.W_BATCHED, i)[0] for i, D in enumerate(Ds)]
    ys = [hc_inputs.pair_masses(int(D), hc_inputs.W_BATCHED, i)[1] for i, D in enumerate(Ds)]
    Z = run_plan(plan, xs, ys)
    check_pairs(plan, Ds, xs, ys, Z)
    groups = {g["D"]: g for g in plan.schedule["groups"]}
    assert groups[14]["inverse_groups"] == ["4+2"] and groups[14]["forward_groups"] == [3, 3]
    assert groups[8]["inverse_groups"] == [] and groups[8]["K"] == 8


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_persistent_pairs_tuned_and_cached(dtype, tmp_path, monkeypatch):
    """The autotuner of persistent plans: every candidate schedule agrees
    bitwise (else plan creation fails), the choice is cached, and the tuned
    plan gives the default plan's bits."""
    monkeypatch.setenv("HC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    Ds = [14, 9, 12, 13, 7, 10, 11, 14, 13]
    tdt = NP2T[np.dtype(dtype)]
    print(f"persistent pairs tuned {np.dtype(dtype).name} Ds={Ds}", flush=True)
    plan = hc.BatchedPlan(Ds, tdt, tune=True, persistent_pairs=True)
    assert plan.schedule["tuned"] and plan.schedule["mode"] == "persistent_pairs"
    lines = (tmp_path / "tune.txt").read_text().split()
    with_outer = {D for D in Ds if D > (9 if dtype == np.float32 else 8)}
    assert sum(1 for w in lines if w.startswith("p1:")) == len(with_outer)
    again = hc.BatchedPlan(Ds, tdt, tune=True, persistent_pairs=True)
    assert again.schedule == plan.schedule
    default = hc.BatchedPlan(Ds, tdt, persistent_pairs=True)
    xs, ys = packed_inputs(Ds, dtype, seed=14)
    Zt = run_plan(plan, xs, ys)
    pins.assert_bitwise(Zt, run_plan(default, xs, ys), "tuned vs default")
    check_pairs(plan, Ds, xs, ys, Zt)


@pytest.mark.parametrize("Ds", [[16], [0], [0, 0, 0], [8, 8], [9]])
def test_persistent_pairs_edge_batches(Ds):
    """One pair (a grid of one workgroup), pairs that need no workspace, the
    largest D alone: bitwise equal to single-pair calls."""
    print(f"persistent pairs f64 edge Ds={Ds}", flush=True)
    plan = hc.BatchedPlan(Ds, torch.float64, persistent_pairs=True)
    assert 1 <= plan.schedule["grid"] <= len(Ds)
    assert (plan.workspace_bytes == 0) == all(D <= 8 for D in Ds)
    xs, ys = packed_inputs(Ds, np.float64, seed=15)
    Z = run_plan(plan, xs, ys)
    for i, D in enumerate(Ds):
        z1 = hc.convolve(torch.from_numpy(xs[i]).to(DEV), torch.from_numpy(ys[i]).to(DEV)).cpu().numpy()
        pins.assert_bitwise(Z[plan.z_offsets[i]:plan.z_offsets[i + 1]], z1, f"pair {i} D={D}")
    plan.close()


def test_plan_log_on_stderr():
    """HC_LOG=1 prints the plan (and the tuner's candidates) on stderr; the
    library reads the variable once, so this runs in a child process."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import torch, paper_1608_00206_amd as hc; "
            "hc.BatchedPlan([3, 9, 9], torch.float64, tune=True, persistent_pairs=True).close(); "
            "hc.BatchedPlan([3, 10], torch.float64).close()")
    env = dict(os.environ, HC_LOG="1", PYTHONPATH=root)
    env.pop("HC_TUNE_CACHE", None)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("[hc] ")]
    assert sum(1 for l in lines if l.startswith('[hc] plan: {"mode": "persistent_pairs"')) == 1
    assert sum(1 for l in lines if l.startswith('[hc] plan: {"mode": "graph"')) == 1


def test_more_pairs_than_one_launch_holds():
    """70000 small pairs: the grouped graph splits a D group above 65535
    items (the grid's y extent) into two launches; the persistent launch
    takes them all by ticket.  Both against a vectorised definition."""
    rng = np.random.default_rng(17)
    Ds = [1] * 66000 + [2] * 4000
    print(f"batched {len(Ds)} small pairs", flush=True)
    xs = rng.integers(0, 16, size=sum(2 ** d for d in Ds)).astype(np.int64)
    ys = rng.integers(0, 16, size=xs.size).astype(np.int64)
    # the definition, vectorised per D: z[tern(i) + tern(j)] += x[i] y[j]
    want = []
    off = 0
    for D, n in ((1, 66000), (2, 4000)):
        x = xs[off:off + n * 2 ** D].reshape(n, 2 ** D)
        y = ys[off:off + n * 2 ** D].reshape(n, 2 ** D)
        off += n * 2 ** D
        tern = np.array([int(np.base_repr(i, 2), 3) for i in range(2 ** D)])
        z = np.zeros((n, 3 ** D), dtype=np.int64)
        for i in range(2 ** D):
            for j in range(2 ** D):
                z[:, tern[i] + tern[j]] += x[:, i] * y[:, j]
        want.append(z.ravel())
    want = np.concatenate(want)
    X = torch.from_numpy(xs).to(DEV)
    Y = torch.from_numpy(ys).to(DEV)
    for kw in ({}, {"persistent_pairs": True}):
        plan = hc.BatchedPlan(Ds, torch.int64, **kw)
        if not kw:
            assert [(g["D"], g["items"]) for g in plan.schedule["groups"]] == [(2, 4000), (1, 65535), (1, 465)]
        Z = plan.run(X, Y)
        plan.check()
        pins.assert_bitwise(Z.cpu().numpy(), want, f"70000 pairs {kw}")
        plan.close()


@pytest.mark.parametrize("seed", [21, 22, 23])
@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int64])
def test_persistent_pairs_random_batches_equal_graph(dtype, seed):
    """Random ragged batches (D from 0 to 13 in random order, repeats
    included): the persistent launch and the grouped graph give the same
    bits, and a sample of pairs equals the oracle."""
    rng = np.random.default_rng(seed)
    Ds = [int(d) for d in rng.integers(0, 14, int(rng.integers(1, 300)))]
    print(f"random batch {np.dtype(dtype).name} seed={seed}: {len(Ds)} pairs", flush=True)
    xs, ys = packed_inputs(Ds, dtype, seed=seed)
    X = torch.from_numpy(np.concatenate(xs)).to(DEV)
    Y = torch.from_numpy(np.concatenate(ys)).to(DEV)
    tdt = NP2T[np.dtype(dtype)]
    with hc.BatchedPlan(Ds, tdt) as g, hc.BatchedPlan(Ds, tdt, persistent_pairs=True) as p:
        Zg = g.run(X, Y)
        Zp = p.run(X, Y)
        p.check()
        Zg, Zp = Zg.cpu().numpy(), Zp.cpu().numpy()
        pins.assert_bitwise(Zp, Zg, "persistent vs graph")
        zo = p.z_offsets
        for i in rng.choice(len(Ds), min(len(Ds), 4), replace=False):
            pins.assert_bitwise(Zp[zo[i]:zo[i + 1]], oracle.canonical(xs[i], ys[i]), f"pair {i} D={Ds[i]}")
