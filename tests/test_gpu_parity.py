"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars (see the tolerance derivation in the design notes):
- pair counts: bit-exact;
- dyadic inputs: raw bins H bit-exact for every precision;
- FP32 and split-FP16: normwise error <= 1e-6 on C(r,t);
- split-BF16: normwise error <= 5e-5 (deterministic bound 3*2^-16 plus FP32
  accumulation); on random unit spins the off-diagonal rounding is unbiased
  noise, bounded by six standard deviations for the sparsest bin and by 1e-6
  once bins hold enough pairs x origins (the diagonal lo*lo term is added
  exactly; the small split products never enter a sum holding the large
  ones, so the matrix cores' downward truncation of low addend bits leaves
  only a residual of ~1e-10 of the pair mass, which the full-size summed-bin
  checks bound).
Normwise error e = max |C_gpu - C_ref| / max |C_ref| over all bins and lags.
"""
import numpy as np
import pytest

from paper_2308_07487_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-6, "split_fp16": 1e-6, "split_bf16": 5e-5, "bf16x3": 1e-6}
TOL_RANDOM = {"fp32": 1e-6, "split_fp16": 1e-6, "split_bf16": 1e-6, "bf16x3": 1e-6}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch


@pytest.fixture(scope="module")
def S():
    from paper_2308_07487_amd import sdc
    return sdc


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _run_gpu(torch, S, pos, frames, kind, n_o, n_L, prec, lags=None, stride=1, **kw):
    with S.Plan(pos, kind, n_o, n_L, prec, origin_stride=stride, **kw) as p:
        d = torch.from_numpy(frames).cuda()
        p.accumulate(d, lags=lags)
        out = p.finalize()
        H, no, sf, ms = p.raw()
        torch.cuda.synchronize()
    return out, H, no, sf


def _oracle(orc, pos, frames, kind, n_o, lags, stride=1, **kw):
    H, c = orc.binned_corr(pos, frames, kind, n_o, lags, stride=stride, **kw)
    sf = orc.self_corr(frames, n_o, lags, stride=stride)
    return H, c, sf


def _tol_random(prec, counts, n_o):
    """Random unit spins: split-BF16 rounding is unbiased noise of RMS about
    2^-17 per product, so a bin's C error shrinks like 2^-17 / sqrt(count n_o);
    the bar is six such standard deviations for the sparsest bin, and never
    looser than needed above 1e-6."""
    if prec != "split_bf16":
        return TOL_RANDOM[prec]
    m = float(np.min(counts[counts > 0])) * n_o
    return max(TOL_RANDOM[prec], 6 * 2.0 ** -17 / np.sqrt(m))


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


SC_CASES = [
    # (name, L, n_o, n_L, stride)
    ("c1-geometry 8^3", (8, 8, 8), 32, 64, 1),
    ("ragged 5x6x7, n_o=20, n_L=21", (5, 6, 7), 20, 21, 1),
    ("stride 3", (4, 4, 8), 10, 20, 3),
    ("tiny 2x2x2", (2, 2, 2), 3, 5, 1),
]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
@pytest.mark.parametrize("case", SC_CASES, ids=[c[0] for c in SC_CASES])
def test_sc_random(torch_dev, S, orc, case, prec):
    name, L, n_o, n_L, s = case
    _say(f"sc {name} {prec}")
    pos = inputs.sc_positions(L)
    pos, _, _ = inputs.permute_sites(pos, np.zeros((1, pos.shape[0], 3), np.float32), seed=3)
    T = (n_o - 1) * s + n_L
    fr = inputs.random_unit_frames(T, pos.shape[0], seed=11)
    out, H, no, sf = _run_gpu(torch_dev, S, pos, fr, S.BINS_SC, n_o, n_L, prec, stride=s, cells=L)
    lags = np.arange(n_L)
    Hr, cr, sfr = _oracle(orc, pos, fr, orc.SC, n_o, lags, stride=s, cells=L)
    np.testing.assert_array_equal(out["counts"], cr)
    C, Cs, Cf, Ss, Sf = orc.finalize(Hr, cr, pos.shape[0], float(n_o), sfr)
    e = _normwise(out["C"], C)
    print(f"  normwise error {e:.3e}", flush=True)
    assert e <= _tol_random(prec, cr, n_o)
    np.testing.assert_allclose(no, n_o)
    np.testing.assert_allclose(sf, sfr, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(out["Cself"], Cf, rtol=1e-12, atol=1e-12)
    assert _normwise(out["Csum"], Cs) <= TOL[prec] * 4
    assert np.max(np.abs(out["Ssum"] - Ss)) <= TOL[prec] * 4 * n_L
    np.testing.assert_allclose(out["Sself"], Sf, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
def test_dyadic_bit_exact(torch_dev, S, orc, prec):
    """Components in (1/16)Z: every product and partial sum is exact, so the
    raw bins must agree bit for bit whatever the summation order."""
    for kind, pos, kw in [
        (S.BINS_SC, inputs.sc_positions((6, 5, 4)), dict(cells=(6, 5, 4))),
        (S.BINS_BCC, inputs.bcc_positions((3, 3, 2)), dict(cells=(3, 3, 2))),
        (S.BINS_RADIAL, inputs.ball_positions(150, 3.0, 5), dict(n_shells=40, r_max=6.0)),
    ]:
        _say(f"dyadic kind={kind} {prec}")
        n_o, n_L = 8, 18
        fr = inputs.dyadic_frames(n_o + n_L - 1, pos.shape[0], seed=kind + 1)
        out, H, _, _ = _run_gpu(torch_dev, S, pos, fr, kind, n_o, n_L, prec, **kw)
        Hr, cr, _ = _oracle(orc, pos, fr, kind, n_o, np.arange(n_L), **kw)
        np.testing.assert_array_equal(out["counts"], cr)
        np.testing.assert_array_equal(H, Hr)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "bf16x3"])
def test_bcc_and_radial_random(torch_dev, S, orc, prec):
    for kind, pos, kw in [
        (S.BINS_BCC, inputs.bcc_positions((4, 3, 5)), dict(cells=(4, 3, 5))),
        (S.BINS_RADIAL, inputs.ball_positions(700, 5.0, 8), dict(n_shells=1024, r_max=10.0)),
        (S.BINS_RADIAL, inputs.ball_positions(130, 2.0, 9), dict(n_shells=33, r_max=3.0)),
    ]:
        _say(f"random kind={kind} n={pos.shape[0]} {prec}")
        n_o, n_L = 17, 19
        fr = inputs.random_unit_frames(n_o + n_L - 1, pos.shape[0], seed=21)
        out, H, _, _ = _run_gpu(torch_dev, S, pos, fr, kind, n_o, n_L, prec, **kw)
        Hr, cr, sfr = _oracle(orc, pos, fr, kind, n_o, np.arange(n_L), **kw)
        np.testing.assert_array_equal(out["counts"], cr)
        C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), sfr)
        e = _normwise(out["C"], C)
        print(f"  normwise error {e:.3e}", flush=True)
        assert e <= _tol_random(prec, cr, n_o)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
def test_static_ferromagnet_z_exact(torch_dev, S, prec):
    """Every spin along z in every frame: C = 1 exactly in every occupied bin."""
    _say(f"static z ferromagnet {prec}")
    L = (4, 4, 6)
    pos = inputs.sc_positions(L)
    fr = inputs.static_frames(40, pos.shape[0], (0, 0, 1))
    out, H, _, _ = _run_gpu(torch_dev, S, pos, fr, S.BINS_SC, 20, 21, prec, cells=L)
    np.testing.assert_array_equal(out["C"], 1.0)
    np.testing.assert_array_equal(out["Cself"], 1.0)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
def test_static_ferromagnet_generic_axis(torch_dev, S, prec):
    """Every spin along one generic axis: C = |s|^2 in every bin (the fp32
    axis is not exactly unit), with the rounding of every product coherent.
    This is the worst case of the reduced forms: split-BF16 only meets its
    deterministic bound, split-FP16 and the three-piece BF16 form meet 1e-6."""
    _say(f"static generic-axis ferromagnet {prec}")
    L = (4, 6, 5)
    pos = inputs.sc_positions(L)
    fr = inputs.static_frames(30, pos.shape[0], (0.3, -0.55, 0.7))
    out, *_ = _run_gpu(torch_dev, S, pos, fr, S.BINS_SC, 16, 15, prec, cells=L)
    a = fr[0, 0].astype(np.float64)
    ref = float(a @ a)
    e = float(np.max(np.abs(out["C"] - ref)) / ref)
    print(f"  normwise error {e:.3e}", flush=True)
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
def test_planted_spiral(torch_dev, S, prec):
    _say(f"planted spiral {prec}")
    L = (8, 4, 6)
    pos = inputs.sc_positions(L)
    q = 2 * np.pi * np.array([1, 1, 2]) / np.array(L)
    theta, omega, dt = np.pi / 2, 0.9, 0.1
    n_o, n_L = 16, 24
    fr = inputs.spiral_frames(pos, q, theta, omega, n_o + n_L - 1, dt)
    out, *_ = _run_gpu(torch_dev, S, pos, fr, S.BINS_SC, n_o, n_L, prec, cells=L)
    b = np.arange(pos.shape[0])
    d = np.stack([b // (L[1] * L[2]), (b // L[2]) % L[1], b % L[2]], axis=1)
    t = np.arange(n_L)[:, None]
    ref = np.cos(d @ q - omega * t * dt)
    tol = {"fp32": 2e-6, "split_fp16": 2e-6, "split_bf16": 5e-5, "bf16x3": 2e-6}[prec]
    assert np.max(np.abs(out["C"] - ref)) <= tol


def test_lag_subset_and_accumulation(torch_dev, S, orc):
    _say("lag subset, two accumulates, reset, raw round trip")
    L = (4, 5, 4)
    pos = inputs.sc_positions(L)
    n_o, n_L = 9, 40
    fr1 = inputs.random_unit_frames(n_o + n_L, pos.shape[0], seed=1)
    fr2 = inputs.random_unit_frames(n_o + n_L, pos.shape[0], seed=2)
    lags = np.array([0, 5, 17, 39])
    with S.Plan(pos, S.BINS_SC, n_o, n_L, "fp32", cells=L) as p:
        p.accumulate(torch_dev.from_numpy(fr1).cuda(), lags=lags)
        p.accumulate(torch_dev.from_numpy(fr2).cuda(), lags=lags[:2])
        H, no, sf, ms = p.raw()
        H1, c1 = orc.binned_corr(pos, fr1, orc.SC, n_o, lags, cells=L)
        H2, _ = orc.binned_corr(pos, fr2, orc.SC, n_o, lags[:2], cells=L)
        ref = np.zeros((n_L, pos.shape[0]))
        ref[lags] += H1
        ref[lags[:2]] += H2
        assert _normwise(H, ref) < 1e-6
        # site sums: the magnetisation products equal the oracle's sum over bins
        np.testing.assert_allclose(ms, ref.sum(axis=1), rtol=1e-10, atol=1e-10 * np.abs(ref).sum())
        expect_no = np.zeros(n_L)
        expect_no[lags] += n_o
        expect_no[lags[:2]] += n_o
        np.testing.assert_array_equal(no, expect_no)
        out = p.finalize()
        untouched = np.setdiff1d(np.arange(n_L), lags)
        np.testing.assert_array_equal(out["C"][untouched], 0.0)
        # raw round trip and reset
        p.reset()
        H0, no0, _, ms0 = p.raw()
        assert not H0.any() and not no0.any() and not ms0.any()
        p.load_raw(H, no, sf, ms)
        H3, no3, sf3, ms3 = p.raw()
        np.testing.assert_array_equal(H3, H)
        np.testing.assert_array_equal(no3, no)
        np.testing.assert_array_equal(ms3, ms)


def test_nan_propagates(torch_dev, S):
    _say("nan propagation")
    L = (4, 4, 4)
    pos = inputs.sc_positions(L)
    fr = inputs.random_unit_frames(40, 64, seed=4)
    fr[3, 10, 1] = np.nan
    out, H, _, _ = _run_gpu(torch_dev, S, pos, fr, S.BINS_SC, 8, 16, "split_bf16", cells=L)
    assert np.isnan(H).any()


def test_invalid_calls(torch_dev, S):
    _say("invalid calls")
    L = (4, 4, 4)
    pos = inputs.sc_positions(L)
    with S.Plan(pos, S.BINS_SC, 8, 16, "fp32", cells=L) as p:
        d = torch_dev.zeros((10, 64, 3), device="cuda")
        with pytest.raises(S.SdcError) as ei:
            p.accumulate(d)  # needs 8 - 1 + 16 frames
        assert ei.value.status == S.ERR_INVALID_ARG
        with pytest.raises(S.SdcError):
            p.accumulate(torch_dev.zeros((40, 64, 3), device="cuda"), lags=[16])
        with pytest.raises(S.SdcError):
            p.accumulate(torch_dev.zeros((40, 64, 3), device="cuda"), lags=[3, 3])
        # the plan stays usable after rejected calls
        p.accumulate(torch_dev.zeros((40, 64, 3), device="cuda"))
        p.finalize()


CONNECTED_CASES = [
    ("sc 5x4x6", "sc", (5, 4, 6), {}),
    ("bcc 3x4x3", "bcc", (3, 4, 3), {}),
    ("radial 400 points, 64 shells", "radial", None, dict(n_shells=64, r_max=8.0)),
]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
@pytest.mark.parametrize("case", CONNECTED_CASES, ids=[c[0] for c in CONNECTED_CASES])
def test_connected_matches_oracle(torch_dev, S, orc, case, prec):
    """Connected form (Eq. (4) with its second term): the GPU centres the
    origin side (Eq. (5)); the oracle subtracts the product of the averages."""
    name, lat, L, spec = case
    _say(f"connected {name} {prec}")
    if lat == "sc":
        pos, kind, okind, kw = inputs.sc_positions(L), S.BINS_SC, orc.SC, dict(cells=L)
    elif lat == "bcc":
        pos, kind, okind, kw = inputs.bcc_positions(L), S.BINS_BCC, orc.BCC, dict(cells=L)
    else:
        pos, kind, okind, kw = inputs.ball_positions(400, 4.0, 3), S.BINS_RADIAL, orc.RADIAL, spec
    n = pos.shape[0]
    n_o, n_L, s = 21, 19, 2
    fr = inputs.random_unit_frames((n_o - 1) * s + n_L, n, seed=31).astype(np.float64)
    fr[:, :, 2] += 0.4  # a non-zero average that the connected form removes
    fr = fr.astype(np.float32)
    with S.Plan(pos, kind, n_o, n_L, prec, origin_stride=s, connected=True, **kw) as p:
        p.accumulate(torch_dev.from_numpy(fr).cuda())
        out = p.finalize()
    lags = np.arange(n_L)
    Hr, cr = orc.binned_corr(pos, fr, okind, n_o, lags, stride=s, connected=True, **kw)
    sfr = orc.self_corr(fr, n_o, lags, stride=s, connected=True)
    np.testing.assert_array_equal(out["counts"], cr)
    C, Cs, Cf, Ss, Sf = orc.finalize(Hr, cr, n, float(n_o), sfr)
    e = _normwise(out["C"], C)
    print(f"  normwise error {e:.3e}", flush=True)
    assert e <= max(_tol_random(prec, cr, n_o), TOL[prec] if prec == "split_bf16" else 0.0)
    # the origin side is centred in fp32, as the packed operand is
    np.testing.assert_allclose(out["Cself"], Cf, rtol=1e-7, atol=1e-7)
    assert _normwise(out["Csum"], Cs) <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "bf16x3"])
def test_connected_static_is_zero(torch_dev, S, prec):
    """Spins constant in time: the origin side equals its average, so the
    connected correlation vanishes identically."""
    _say(f"connected static {prec}")
    L = (4, 4, 5)
    pos = inputs.sc_positions(L)
    fr = inputs.static_frames(30, pos.shape[0], (0.3, -0.55, 0.7))
    with S.Plan(pos, S.BINS_SC, 16, 15, prec, cells=L, connected=True) as p:
        p.accumulate(torch_dev.from_numpy(fr).cuda())
        out = p.finalize()
    assert np.max(np.abs(out["C"])) == 0.0
    assert np.max(np.abs(out["Cself"])) == 0.0
    assert np.max(np.abs(out["Csum"])) < 1e-12


def test_radial_key_table_and_on_the_fly_agree(torch_dev, S, orc):
    """The stored per-pair shells and the epilogue's own distance computation
    give the same bins (and both match the oracle)."""
    _say("radial key table vs on-the-fly shells")
    pos = inputs.ball_positions(900, 6.0, 17)
    n_o, n_L = 12, 10
    fr = inputs.random_unit_frames(n_o + n_L - 1, pos.shape[0], seed=5)
    outs = []
    for table in (True, False):
        with S.Plan(pos, S.BINS_RADIAL, n_o, n_L, "split_bf16", n_shells=300, r_max=13.0,
                    key_table=table) as p:
            p.accumulate(torch_dev.from_numpy(fr).cuda())
            outs.append((p.finalize(), p.raw()[0]))
    np.testing.assert_array_equal(outs[0][0]["counts"], outs[1][0]["counts"])
    np.testing.assert_allclose(outs[0][1], outs[1][1], rtol=1e-12, atol=1e-12 * np.max(np.abs(outs[1][1])))
    Hr, cr = orc.binned_corr(pos, fr, orc.RADIAL, n_o, np.arange(n_L), n_shells=300, r_max=13.0)
    np.testing.assert_array_equal(outs[0][0]["counts"], cr)
    C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), orc.self_corr(fr, n_o, np.arange(n_L)))
    assert _normwise(outs[0][0]["C"], C) <= _tol_random("split_bf16", cr, n_o)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("lat", ["sc", "bcc"])
def test_structure_factor_matches_oracle(torch_dev, S, orc, prec, lat):
    """S(q, t) of Eq. (3) from the GPU bins against the oracle's direct double
    sum over site pairs, and its windowed transform against the oracle DFT."""
    _say(f"structure factor {lat} {prec}")
    L = (5, 4, 6) if lat == "sc" else (3, 4, 3)
    pos = inputs.sc_positions(L) if lat == "sc" else inputs.bcc_positions(L)
    kind = S.BINS_SC if lat == "sc" else S.BINS_BCC
    pos, _, _ = inputs.permute_sites(pos, np.zeros((1, pos.shape[0], 3), np.float32), seed=9)
    n_o, n_L = 10, 12
    fr = inputs.random_unit_frames(n_o + n_L - 1, pos.shape[0], seed=19)
    ms = np.array([[0, 0, 0], [1, 0, 0], [2, 1, 3], [-1, 2, 1], [5, 4, 6]], dtype=np.int32)
    with S.Plan(pos, kind, n_o, n_L, prec, cells=L) as p:
        p.accumulate(torch_dev.from_numpy(fr).cuda())
        sqt, sqw = p.structure_factor(ms)
    ref = orc.structure_factor(pos, fr, n_o, list(range(n_L)), ms, L)
    scale = max(1.0, float(np.max(np.abs(ref))))
    e = float(np.max(np.abs(sqt - ref))) / scale
    # S sums every pair once: split-BF16's per-product noise (2^-17, unbiased
    # up to the ~1e-10 residual of the matrix cores' truncation) averages
    # only over the origins, so its bar is statistical
    bar = 1e-6 if prec != "split_bf16" else max(1e-6, 6 * 2.0 ** -17 / np.sqrt(n_o))
    print(f"  S(q,t) error {e:.3e} (bar {bar:.2e})", flush=True)
    assert e <= bar
    for qi in range(ms.shape[0]):
        w_ref = orc.dft(ref[qi].real) + 1j * orc.dft(ref[qi].imag)
        assert np.max(np.abs(sqw[qi] - w_ref)) <= bar * scale * n_L
    with pytest.raises(S.SdcError):
        with S.Plan(inputs.ball_positions(64, 2.0, 1), S.BINS_RADIAL, 4, 4, prec, n_shells=8, r_max=4.0) as pr:
            pr.structure_factor(ms)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_deterministic_mode_bit_identical(torch_dev, S, orc, prec):
    """SDC_FLAG_DETERMINISTIC: fixed-point sums make two runs (and a batch
    run) bit-identical, and the result stays within the bar of the oracle."""
    _say(f"deterministic mode {prec}")
    cases = [
        (S.BINS_SC, orc.SC, inputs.sc_positions((9, 10, 8)), dict(cells=(9, 10, 8))),
        (S.BINS_BCC, orc.BCC, inputs.bcc_positions((5, 4, 6)), dict(cells=(5, 4, 6))),
        (S.BINS_RADIAL, orc.RADIAL, inputs.ball_positions(600, 5.0, 4), dict(n_shells=128, r_max=10.0)),
    ]
    n_o, n_L = 24, 20
    for kind, okind, pos, kw in cases:
        fr = inputs.random_unit_frames(n_o + n_L - 1, pos.shape[0], seed=44)
        d = torch_dev.from_numpy(fr).cuda()
        runs = []
        for _ in range(2):
            with S.Plan(pos, kind, n_o, n_L, prec, deterministic=True, **kw) as p:
                p.accumulate(d)
                out = p.finalize()
                runs.append((p.raw(), out))
        (H0, no0, sf0, ms0), out0 = runs[0]
        (H1, no1, sf1, ms1), out1 = runs[1]
        np.testing.assert_array_equal(H0, H1)
        np.testing.assert_array_equal(sf0, sf1)
        np.testing.assert_array_equal(out0["C"], out1["C"])
        np.testing.assert_array_equal(out0["Sself"], out1["Sself"])
        Hr, cr = orc.binned_corr(pos, fr, okind, n_o, np.arange(n_L), **kw)
        C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), orc.self_corr(fr, n_o, np.arange(n_L)))
        e = _normwise(out0["C"], C)
        print(f"  kind {kind}: normwise error {e:.3e}", flush=True)
        assert e <= _tol_random(prec, cr, n_o)
        # one partial per site is rounded to 2^-20: at most N * 2^-21 in all
        np.testing.assert_allclose(sf0, orc.self_corr(fr, n_o, np.arange(n_L)), rtol=1e-12,
                                   atol=pos.shape[0] * 2.0 ** -21)
    # a batch in deterministic mode gives the same bits as the single plan
    pos, kw = cases[0][2], cases[0][3]
    fr = inputs.random_unit_frames(n_o + n_L - 1, pos.shape[0], seed=44)
    d = torch_dev.from_numpy(fr).cuda()
    with S.Plan(pos, S.BINS_SC, n_o, n_L, prec, deterministic=True, **kw) as a, \
            S.Plan(pos, S.BINS_SC, n_o, n_L, prec, deterministic=True, **kw) as b:
        a.accumulate(d)
        with S.Batch([b]) as bt:
            bt.accumulate([d])
        np.testing.assert_array_equal(a.raw()[0], b.raw()[0])


def test_edge_cases(torch_dev, S, orc):
    """Single site, single origin, single lag, and the options combined."""
    _say("edge cases")
    # one site, one origin, one lag: C(0, 0) = |S|^2 = 1 for an axis spin
    for kind, pos, kw in [(S.BINS_SC, inputs.sc_positions((1, 1, 1)), dict(cells=(1, 1, 1))),
                          (S.BINS_RADIAL, np.zeros((1, 3), np.float32), dict(n_shells=4, r_max=1.0))]:
        fr = inputs.axis_frames(1, 1, seed=3)
        with S.Plan(pos, kind, 1, 1, "split_bf16", **kw) as p:
            p.accumulate(torch_dev.from_numpy(fr).cuda())
            out = p.finalize()
        assert out["counts"][0] == 1 and out["C"][0, 0] == 1.0 and out["Cself"][0] == 1.0
    # one origin, several lags, ragged box
    L = (3, 1, 5)
    pos = inputs.sc_positions(L)
    fr = inputs.random_unit_frames(4, pos.shape[0], seed=6)
    with S.Plan(pos, S.BINS_SC, 1, 4, "fp32", cells=L) as p:
        p.accumulate(torch_dev.from_numpy(fr).cuda())
        out = p.finalize()
    Hr, cr = orc.binned_corr(pos, fr, orc.SC, 1, np.arange(4), cells=L)
    C, *_ = orc.finalize(Hr, cr, pos.shape[0], 1.0, orc.self_corr(fr, 1, np.arange(4)))
    assert _normwise(out["C"], C) <= 1e-6
    # connected + deterministic + BF16x3 + origin stride 2, single plan and batch
    L = (4, 3, 5)
    pos = inputs.bcc_positions(L)
    n_o, n_L, s = 9, 7, 2
    fr = inputs.random_unit_frames((n_o - 1) * s + n_L, pos.shape[0], seed=8).astype(np.float64)
    fr[:, :, 0] += 0.5
    fr = fr.astype(np.float32)
    d = torch_dev.from_numpy(fr).cuda()
    Hr, cr = orc.binned_corr(pos, fr, orc.BCC, n_o, np.arange(n_L), stride=s, cells=L, connected=True)
    sfr = orc.self_corr(fr, n_o, np.arange(n_L), stride=s, connected=True)
    C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), sfr)
    kw = dict(cells=L, origin_stride=s, connected=True, deterministic=True)
    with S.Plan(pos, S.BINS_BCC, n_o, n_L, "bf16x3", **kw) as a, \
            S.Plan(pos, S.BINS_BCC, n_o, n_L, "bf16x3", **kw) as b:
        a.accumulate(d)
        with S.Batch([b]) as bt:
            bt.accumulate([d])
        oa, ob = a.finalize(), b.finalize()
        np.testing.assert_array_equal(oa["C"], ob["C"])
        assert _normwise(oa["C"], C) <= 1e-6


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_square_lattice_2d(torch_dev, S, orc, prec):
    """The paper's geometry, a 2D square lattice, is the sc kind with one cell
    along z; an RK4 trajectory of it (the +-z bonds close on the site itself
    and drop out of the precession) against the oracle."""
    _say(f"2D square lattice {prec}")
    L = (24, 18, 1)
    pos = inputs.sc_positions(L)
    n_o, n_L = 20, 16
    fr = torch_dev.empty((n_o + n_L - 1, pos.shape[0], 3), dtype=torch_dev.float32, device="cuda")
    S.traj_generate(pos, S.BINS_SC, fr, cells=L, J=-1.0, dt=0.02, init=S.INIT_PERTURBED_Z, sigma=0.4, seed=7)
    with S.Plan(pos, S.BINS_SC, n_o, n_L, prec, cells=L) as p:
        p.accumulate(fr)
        out = p.finalize()
    frh = fr.cpu().numpy()
    Hr, cr = orc.binned_corr(pos, frh, orc.SC, n_o, np.arange(n_L), cells=L)
    np.testing.assert_array_equal(out["counts"], cr)
    C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), orc.self_corr(frh, n_o, np.arange(n_L)))
    e = _normwise(out["C"], C)
    print(f"  normwise error {e:.3e}", flush=True)
    assert e <= TOL[prec]
