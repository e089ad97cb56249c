"""Host logic of batched plans (CPU only): how pairs are grouped."""
import pytest

import hc_inputs
from paper_1608_00206_amd import _abi


def test_every_pair_in_one_group_largest_first():
    Ds = list(hc_inputs.batched_dims(500)) + [0, 3, 16]
    groups = _abi.hc_plan_inspect(Ds, _abi.HC_F64)
    assert sum(g["pairs"] for g in groups) == len(Ds)
    assert [g["D"] for g in groups] == sorted({int(d) for d in Ds}, reverse=True)
    for g in groups:
        assert Ds[g["first_pair"]] == g["D"]
        assert g["pairs"] == sum(1 for d in Ds if d == g["D"])


# float32 default fused depth for D = 9..16: 9 where it saves an outer pass
# (D = 9, 15) or where depth 8 would leave a 5-axis last pass (D = 13), else 8
F32_DEPTH = {9: 9, 10: 8, 11: 8, 12: 8, 13: 9, 14: 8, 15: 9, 16: 8}


@pytest.mark.parametrize("dtype", [_abi.HC_F64, _abi.HC_F32, _abi.HC_I64])
def test_group_schedules(dtype):
    groups = _abi.hc_plan_inspect(list(range(0, 17)), dtype)
    for g in groups:
        D = g["D"]
        if dtype == _abi.HC_F32:
            assert g["K"] == F32_DEPTH.get(D, D)
        else:
            assert g["K"] == min(D, 8)
        p = D - g["K"]
        assert (g["fwd_passes"] == 0) == (p == 0)
        assert g["fwd_passes"] == -(-p // 4)          # outer forward groups of at most 4 axes
        assert g["inv_passes"] == -(-p // 6)          # outer inverse groups of at most 6 axes


def test_inspect_and_plan_validation():
    with pytest.raises(_abi.HCError):
        _abi.hc_plan_inspect([4, 17], _abi.HC_F64)
    with pytest.raises(_abi.HCError):
        _abi.hc_plan_inspect([4], 9)
    with pytest.raises(_abi.HCError) as e:
        _abi.hc_plan_inspect([9, 12], _abi.HC_F64, _abi.HC_PLAN_PERSISTENT)
    assert e.value.status == "HC_ERR_UNSUPPORTED"


@pytest.mark.parametrize("dtype", [_abi.HC_F64, _abi.HC_F32, _abi.HC_I64])
def test_persistent_pair_schedules(dtype):
    """One persistent launch, a workgroup per pair: the largest fused tile
    (9 axes for 4-byte elements, else 8), outer forward groups of at most
    three axes, outer inverse groups of at most six."""
    groups = _abi.hc_plan_inspect(list(range(0, 17)), dtype, _abi.HC_PLAN_PERSISTENT_PAIRS)
    kmax = 9 if dtype == _abi.HC_F32 else 8
    assert [g["D"] for g in groups] == list(range(16, -1, -1))
    for g in groups:
        D = g["D"]
        assert g["K"] == min(D, kmax)
        p = D - g["K"]
        assert g["fwd_passes"] == -(-p // 3)
        assert g["inv_passes"] == -(-p // 6)
