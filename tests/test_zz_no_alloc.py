"""The structure-factor entry point that allocates nothing
(sdc_plan_structure_factor_static, fixed device scratch) against the one
that allocates per call (sdc_plan_structure_factor): two calls in a row,
the second with a smaller input than the first, each equal to the existing
entry point's result bit for bit (same kernels, same reduction order); and
the scratch limit refused before any GPU work."""
import numpy as np
import pytest

from paper_2308_07487_amd import inputs

pytestmark = pytest.mark.gpu


def _plan_case(torch, sdc, kind, L, n_o, n_L, seed):
    pos = inputs.sc_positions(L) if kind == "sc" else inputs.bcc_positions(L)
    fr = inputs.random_unit_frames(n_o + n_L - 1, pos.shape[0], seed=seed)
    p = sdc.Plan(pos, sdc.BINS_SC if kind == "sc" else sdc.BINS_BCC, n_o, n_L, "split_bf16", cells=L)
    p.accumulate(torch.from_numpy(fr).cuda())
    return p


def test_static_structure_factor_matches_allocating_one():
    import torch

    from paper_2308_07487_amd import sdc
    assert torch.cuda.is_available(), "GPU tests need a device"
    rng = np.random.default_rng(0x5DC0A110)
    # first call: 24 wave vectors x 40 lags; second: 3 x 6 (smaller)
    cases = [("sc", (6, 5, 4), 7, 40, 24), ("bcc", (3, 2, 3), 4, 6, 3)]
    for k, (kind, L, n_o, n_L, n_q) in enumerate(cases):
        print(f"[case] static structure factor, call {k + 1}: {kind} {L}, {n_o} origins x {n_L} lags, "
              f"{n_q} wave vectors", flush=True)
        m = rng.integers(-7, 8, size=(n_q, 3)).astype(np.int32)
        m[0] = 0
        p = _plan_case(torch, sdc, kind, L, n_o, n_L, seed=40 + k)
        try:
            want_t, want_w = p.structure_factor(m)
            got_t, got_w = p.structure_factor_static(m)
        finally:
            p.close()
        assert got_t.shape == (n_q, n_L)
        np.testing.assert_array_equal(got_t, want_t)
        np.testing.assert_array_equal(got_w, want_w)


def test_static_structure_factor_limit():
    import torch

    from paper_2308_07487_amd import sdc
    assert torch.cuda.is_available(), "GPU tests need a device"
    pos = inputs.sc_positions((2, 2, 2))
    with sdc.Plan(pos, sdc.BINS_SC, 1, 1024, "fp32", cells=(2, 2, 2)) as p:
        m = np.zeros((600, 3), dtype=np.int32)  # 32 * 600 * 1024 bytes > 16 MiB
        with pytest.raises(sdc.SdcError) as ex:
            p.structure_factor_static(m)
        assert ex.value.status == sdc.ERR_UNSUPPORTED
        # a request that fits still works on the same plan (nothing accumulated: zeros)
        t, w = p.structure_factor_static(m[:10])
        assert not np.any(t) and not np.any(w)
