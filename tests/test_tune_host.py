"""The autotuner's built-in candidate lists (host only, no GPU): every
schedule the precision has times the segment lengths of the bin kind."""
import ctypes

import pytest

from paper_2308_07487_amd import sdc


def _candidates(kind, prec, **spec):
    bs = sdc.bin_spec(kind, spec.get("cells", (0, 0, 0)), spec.get("n_shells", 0), spec.get("r_max", 0.0))
    cs = sdc.corr_spec(16, 24, prec, 1)
    n = ctypes.c_int32()
    assert sdc.lib().sdc_autotune_candidates(ctypes.byref(bs), ctypes.byref(cs), None, 0, ctypes.byref(n)) == 0
    arr = (sdc.Tuning * n.value)()
    got = ctypes.c_int32()
    assert sdc.lib().sdc_autotune_candidates(ctypes.byref(bs), ctypes.byref(cs), ctypes.cast(arr, ctypes.c_void_p),
                                             n.value, ctypes.byref(got)) == 0
    inv = {v: k for k, v in sdc.SCHEDULES.items()}
    return {(inv[t.schedule], t.segment_pairs) for t in arr}


@pytest.mark.parametrize("prec,schedules", [
    ("split_bf16", {"one_pass", "two_pass", "lag_split", "fold"}),
    ("split_fp16", {"one_pass", "two_pass", "lag_split", "fold"}),
    ("bf16x3", {"one_pass", "lag_split", "fold"}),
    ("fp32", {"one_pass", "lag_split"}),
])
def test_builtin_candidates(prec, schedules):
    periodic = _candidates(sdc.BINS_SC, prec, cells=(8, 8, 8))
    assert periodic == {(s, g) for s in schedules for g in (16, 32, 48, 96, 192)}
    radial = _candidates(sdc.BINS_RADIAL, prec, n_shells=64, r_max=4.0)
    assert radial == {(s, g) for s in schedules for g in (64, 256, 1 << 20)}
