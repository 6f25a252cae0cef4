"""The matrix-core behaviour the fused product's design rests on, read off
single MFMA instructions (sdc_mfma_probe) and the sustained-rate loop
(sdc_mfma_peak).

BF16 32x32x16: each result is the exact sum rounded to nearest as long as
every addend's bits lie within a window of about 7 places below the last
place of the largest addend; bits further down are dropped, always
downwards (a tiny negative addend still lowers a tie, a tiny positive one
vanishes), and inside one instruction the products are aligned to the
largest product with bits below about 2^-24 of it dropped.  This is why the
small split products are never added to a sum that already holds the large
ones.  The FP32 form adds its products one at a time, rounding each."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2308_07487_amd import sdc
    return sdc


def _probe(S, form, c, prods):
    a = np.array([p[0] for p in prods], dtype=np.float32)
    b = np.array([p[1] for p in prods], dtype=np.float32)
    return S.mfma_probe(form, c, a, b)


def test_bf16_rounds_to_nearest_within_the_window(S):
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -23)
    # exact sums that need rounding: 1 + 3/4 ulp -> 1 + ulp, 1 - 3/4 ulp(below 1) -> 1 - 2^-24
    assert _probe(S, "bf16", 1.0, [(1.5, 2.0 ** -24)]) == one + ulp
    assert _probe(S, "bf16", 1.0, [(-1.5, 2.0 ** -24)]) == np.float32(1.0 - 2.0 ** -23)
    # two half-ulp addends: the exact 1 + 2^-23 ... a tie for each alone, exact together
    assert _probe(S, "bf16", 1.0, [(-(2.0 ** -12), 2.0 ** -13), (-(2.0 ** -12), 2.0 ** -13)]) == \
        np.float32(1.0 - 2.0 ** -24)
    for e in (26, 28, 30):
        # 1 + 2^-24 + 2^-e: above the tie, rounds up
        assert _probe(S, "bf16", 1.0, [(2.0 ** -12, 2.0 ** -12), (2.0 ** -e, 1.0)]) == one + ulp


def test_bf16_drops_addend_bits_below_the_window_downwards(S):
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -23)
    for e in (32, 36, 40, 44):
        # 1 + 2^-24 + 2^-e: the tiny positive addend is dropped -> a tie -> even (1.0)
        assert _probe(S, "bf16", 1.0, [(2.0 ** -12, 2.0 ** -12), (2.0 ** -e, 1.0)]) == one
        # (1 + ulp) + 2^-24 - 2^-e: the tiny negative addend is not dropped but
        # floored to the window's last place, so the tie is missed -> 1 + ulp
        assert _probe(S, "bf16", 1.0 + 2.0 ** -23, [(2.0 ** -12, 2.0 ** -12), (-(2.0 ** -e), 1.0)]) == one + ulp
    # products aligned to the largest product: 1 + 2^-24 + 2^-26 from zero -> 1.0 (the exact sum rounds up)
    assert _probe(S, "bf16", 0.0, [(1.0, 1.0), (2.0 ** -12, 2.0 ** -12), (2.0 ** -13, 2.0 ** -13)]) == one


def test_f32_form_adds_products_one_at_a_time(S):
    # 1 - 2^-25 - 2^-25: each step rounds back to 1.0 (the exact 1 - 2^-24 is representable)
    assert _probe(S, "f32", 1.0, [(-(2.0 ** -12), 2.0 ** -13), (-(2.0 ** -12), 2.0 ** -13)]) == np.float32(1.0)


def test_probe_rejects_inexact_operands(S):
    with pytest.raises(S.SdcError):
        S.mfma_probe("bf16", 0.0, np.array([1.0 + 2.0 ** -10], dtype=np.float32), np.array([1.0], dtype=np.float32))


@pytest.mark.parametrize("form", ["bf16", "f32"])
def test_mfma_rate_loop(S, form):
    """The sustained-rate loop runs and reports a rate below the vendor peak
    (2.5 PFLOP/s BF16, 157.3 TFLOP/s FP32) and above a tenth of it."""
    peak = {"bf16": 2500.0, "f32": 157.3}[form]
    ms, tf = S.mfma_peak(form, random_operands=True, iterations=200)
    print(f"  {form}: {tf:.1f} TFLOP/s in {ms:.2f} ms", flush=True)
    assert 0.1 * peak < tf < 1.05 * peak
