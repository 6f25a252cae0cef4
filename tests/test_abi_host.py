"""Host-side checks of the C-ABI library (no GPU needed).

- the library loads and exports every function declared in include/sdc.h;
- the tile layout maps every ordered pair to the same bin as the oracle's
  key rule, bit for bit (periodic sc/bcc including ragged boxes, radial);
- argument validation returns the documented status codes before any
  device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2308_07487_amd import inputs, sdc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "sdc.h")).read()
    declared = set(re.findall(r"^(?:sdc_status|const char\*)\s+(sdc_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    L = sdc.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(sdc.EXPORTS)


@pytest.mark.parametrize("L", [(1, 1, 1), (2, 3, 4), (5, 6, 7), (8, 8, 8), (9, 4, 10), (11, 13, 3)])
def test_layout_keys_sc_match_oracle(orc, L):
    pos = inputs.sc_positions(L)
    pos, _, _ = inputs.permute_sites(pos, np.zeros((1, pos.shape[0], 3), np.float32), seed=1)
    n = pos.shape[0]
    keys = sdc.layout_keys(pos, sdc.BINS_SC, cells=L)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ref = orc.pair_keys(pos, orc.SC, ii.ravel(), jj.ravel(), cells=L).reshape(n, n)
    np.testing.assert_array_equal(keys, ref)


@pytest.mark.parametrize("L", [(1, 1, 1), (2, 2, 3), (3, 5, 4), (6, 6, 6)])
def test_layout_keys_bcc_match_oracle(orc, L):
    pos = inputs.bcc_positions(L)
    pos, _, _ = inputs.permute_sites(pos, np.zeros((1, pos.shape[0], 3), np.float32), seed=2)
    n = pos.shape[0]
    keys = sdc.layout_keys(pos, sdc.BINS_BCC, cells=L)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ref = orc.pair_keys(pos, orc.BCC, ii.ravel(), jj.ravel(), cells=L).reshape(n, n)
    np.testing.assert_array_equal(keys, ref)


@pytest.mark.parametrize("n,ns,rm", [(1, 1, 1.0), (100, 64, 10.0), (777, 1024, 50.0), (300, 7, 2.0)])
def test_layout_keys_radial_match_oracle(orc, n, ns, rm):
    pos = inputs.ball_positions(n, rm / 2, seed=n)
    keys = sdc.layout_keys(pos, sdc.BINS_RADIAL, n_shells=ns, r_max=rm)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ref = orc.pair_keys(pos, orc.RADIAL, ii.ravel(), jj.ravel(), n_shells=ns, r_max=rm).reshape(n, n)
    np.testing.assert_array_equal(keys, ref)


def test_layout_keys_radial_edge_ties(orc):
    """Points placed exactly on shell edges (squared distances equal to an edge)."""
    w = 0.25
    xs = np.array([0.0, 0.25, 0.5, 1.0, 1.75, 3.0], dtype=np.float32)
    pos = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], axis=1)
    keys = sdc.layout_keys(pos, sdc.BINS_RADIAL, n_shells=12, r_max=12 * w)
    n = pos.shape[0]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ref = orc.pair_keys(pos, orc.RADIAL, ii.ravel(), jj.ravel(), n_shells=12, r_max=3.0).reshape(n, n)
    np.testing.assert_array_equal(keys, ref)


def _create(pos, bins, corr):
    h = ctypes.c_void_p()
    p = np.ascontiguousarray(pos, dtype=np.float32)
    st = sdc.lib().sdc_plan_create(p.ctypes.data_as(ctypes.c_void_p), p.shape[0], ctypes.byref(bins),
                                   ctypes.byref(corr), 0, ctypes.byref(h))
    return st, h


def test_validation_codes():
    pos = inputs.sc_positions((4, 4, 4))
    good_b = sdc.bin_spec(sdc.BINS_SC, (4, 4, 4))
    good_c = sdc.corr_spec(8, 16)
    cases = [
        (sdc.corr_spec(0, 16), good_b),
        (sdc.corr_spec(8, 0), good_b),
        (sdc.corr_spec(8, 16, origin_stride=0), good_b),
        (sdc.corr_spec(8, 16, precision=7), good_b),
        (sdc.corr_spec(8, 16, flags=16), good_b),
        (good_c, sdc.bin_spec(9, (4, 4, 4))),
        (good_c, sdc.bin_spec(sdc.BINS_SC, (4, 4, 5))),       # wrong site count
        (good_c, sdc.bin_spec(sdc.BINS_RADIAL, n_shells=0, r_max=1.0)),
        (good_c, sdc.bin_spec(sdc.BINS_RADIAL, n_shells=8, r_max=0.0)),
    ]
    for corr, bins in cases:
        st, h = _create(pos, bins, corr)
        assert st == sdc.ERR_INVALID_ARG, (st, sdc.last_error())
        assert not h.value
    st, _ = _create(pos + 0.25, good_b, good_c)
    assert st == sdc.ERR_INVALID_ARG and "lattice" in sdc.last_error()
    st, _ = _create(pos, sdc.bin_spec(sdc.BINS_RADIAL, n_shells=5000, r_max=1.0), good_c)
    assert st == sdc.ERR_UNSUPPORTED
    # null pointers
    h = ctypes.c_void_p()
    assert sdc.lib().sdc_plan_create(None, 64, ctypes.byref(good_b), ctypes.byref(good_c), 0,
                                     ctypes.byref(h)) == sdc.ERR_INVALID_ARG
    assert sdc.lib().sdc_accumulate(None, None, 0, None, 0, None) == sdc.ERR_INVALID_ARG
    assert sdc.lib().sdc_finalize(None, None, None, None, None, None, None, None) == sdc.ERR_INVALID_ARG
    assert sdc.lib().sdc_plan_destroy(None) == sdc.OK
    nb = ctypes.c_int64()
    assert sdc.lib().sdc_plan_n_bins(None, ctypes.byref(nb)) == sdc.ERR_INVALID_ARG
    for s in range(7):
        assert sdc.status_string(s)
    # batch calls
    L = sdc.lib()
    hb = ctypes.c_void_p()
    one = (ctypes.c_void_p * 1)(None)
    one_p = ctypes.cast(one, ctypes.c_void_p)
    assert L.sdc_batch_create(None, 1, 0, ctypes.byref(hb)) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_create(one_p, 1, 0, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_create(one_p, 0, 0, ctypes.byref(hb)) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_create(one_p, 1, 0, ctypes.byref(hb)) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_create(one_p, 1, 4, ctypes.byref(hb)) == sdc.ERR_INVALID_ARG
    assert not hb.value
    assert L.sdc_batch_accumulate(None, None, None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_info(None, None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_timings(None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_batch_destroy(None) == sdc.OK


def test_no_device_reported_on_host():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _create(inputs.sc_positions((4, 4, 4)), sdc.bin_spec(sdc.BINS_SC, (4, 4, 4)),
                    sdc.corr_spec(8, 16))
    assert st == sdc.ERR_NO_DEVICE
    assert not h.value


def _sq_create(pos, q, spec):
    h = ctypes.c_void_p()
    p = np.ascontiguousarray(pos, dtype=np.float32)
    qv = np.ascontiguousarray(q, dtype=np.float64)
    st = sdc.lib().sdc_sq_create(p.ctypes.data_as(ctypes.c_void_p), p.shape[0], qv.ctypes.data_as(ctypes.c_void_p),
                                 qv.shape[0], ctypes.byref(spec), 0, ctypes.byref(h))
    return st, h


def test_sq_validation_codes():
    pos = inputs.ball_positions(50, 2.0, seed=3)
    q = np.array([[0.1, 0.2, 0.3], [1.0, 0.0, 0.0]])
    bad_specs = [sdc.SqSpec(0, 8, 1, 0), sdc.SqSpec(4, 0, 1, 0), sdc.SqSpec(4, 2000, 1, 0),
                 sdc.SqSpec(4, 8, 0, 0), sdc.SqSpec(4, 8, 65, 0), sdc.SqSpec(4, 8, 1, 4),
                 sdc.SqSpec(4, 8, 1, 8), sdc.SqSpec(5000, 8, 1, 0)]
    for spec in bad_specs:
        st, h = _sq_create(pos, q, spec)
        assert st == sdc.ERR_INVALID_ARG, (spec.n_origins, spec.n_lags, spec.flags, sdc.last_error())
        assert not h.value
    good = sdc.SqSpec(4, 8, 1, 0)
    p_nan = pos.copy()
    p_nan[7, 1] = np.nan
    q_inf = q.copy()
    q_inf[1, 2] = np.inf
    for pp, qq in [(p_nan, q), (pos, q_inf)]:
        st, h = _sq_create(pp, qq, good)
        assert st == sdc.ERR_INVALID_ARG and "non-finite" in sdc.last_error()
    st, _ = _sq_create(pos, np.zeros((0, 3)), good)
    assert st == sdc.ERR_INVALID_ARG
    st, _ = _sq_create(pos * np.float32(1e5), np.array([[3.0, 2.0, 1.0]]), good)  # |q.r| up to ~1e6 rad
    assert st == sdc.ERR_UNSUPPORTED and "2^20" in sdc.last_error()
    L = sdc.lib()
    h = ctypes.c_void_p()
    assert L.sdc_sq_create(None, 50, None, 1, ctypes.byref(good), 0, ctypes.byref(h)) == sdc.ERR_INVALID_ARG
    assert L.sdc_sq_accumulate(None, None, 0, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_sq_finalize(None, None, None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_sq_timings(None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_sq_reset(None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_sq_destroy(None) == sdc.OK


def test_sq_no_device_reported_on_host():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _sq_create(inputs.ball_positions(50, 2.0, seed=3), np.zeros((1, 3)), sdc.SqSpec(4, 8, 1, 0))
    assert st == sdc.ERR_NO_DEVICE
    assert not h.value


def test_mc_validation_codes():
    L = sdc.lib()
    good = sdc.mc_spec(sdc.BINS_SC, cells=(4, 4, 4), T_start=1.0, T_end=0.5, sweeps_final=2)
    n = ctypes.c_int64()
    assert L.sdc_mc_n_sweeps(ctypes.byref(good), ctypes.byref(n)) == sdc.OK and n.value == 7 + 2  # 1.0 .. 0.9^6
    for field, value in [("cool", 1.0), ("cool", 0.0), ("T_end", 0.0), ("T_start", float("nan")), ("cone0", 4.0),
                         ("acc_target", 0.7), ("sweeps_per_T", 0), ("sweeps_final", -1), ("Hz", float("inf"))]:
        bad = sdc.mc_spec(sdc.BINS_SC, cells=(4, 4, 4), T_start=1.0, T_end=0.5, sweeps_final=2)
        setattr(bad, field, value)
        assert L.sdc_mc_n_sweeps(ctypes.byref(bad), ctypes.byref(n)) == sdc.ERR_INVALID_ARG, field
    huge = sdc.mc_spec(sdc.BINS_SC, cells=(4, 4, 4), T_start=1.0, T_end=1e-300, cool=0.999999,
                       sweeps_per_T=10 ** 9)
    assert L.sdc_mc_n_sweeps(ctypes.byref(huge), ctypes.byref(n)) == sdc.ERR_UNSUPPORTED
    h = ctypes.c_void_p()
    assert L.sdc_mc_create(None, 64, ctypes.byref(good), 0, ctypes.byref(h)) == sdc.ERR_INVALID_ARG
    assert L.sdc_mc_run(None, ctypes.byref(good), None, None, None, None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_mc_timings(None, None) == sdc.ERR_INVALID_ARG
    assert L.sdc_mc_destroy(None) == sdc.OK
    assert L.sdc_mc_anneal(None, 64, ctypes.byref(good), None, None, None, None, 0, None) == sdc.ERR_INVALID_ARG


def test_mc_no_device_reported_on_host():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    pos = np.ascontiguousarray(inputs.sc_positions((4, 4, 4)))
    good = sdc.mc_spec(sdc.BINS_SC, cells=(4, 4, 4), T_start=1.0, T_end=0.5, sweeps_final=2)
    h = ctypes.c_void_p()
    st = sdc.lib().sdc_mc_create(pos.ctypes.data_as(ctypes.c_void_p), 64, ctypes.byref(good), 0, ctypes.byref(h))
    assert st == sdc.ERR_NO_DEVICE and not h.value
