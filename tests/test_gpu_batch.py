"""GPU tests of the batched entry points and of graph capture.

- a batch of mixed sc / bcc samples (ragged boxes, different origin and lag
  counts) accumulated with one persistent launch agrees with the FP64 oracle
  per sample (counts bit-exact, C within the random-spin bar) and, on dyadic
  inputs, bit for bit;
- the batch gives the same bins as accumulating each plan on its own;
- a captured accumulate (single plan and batch) replayed several times, with
  eager work and synchronisations between the replays, gives after every
  replay the eager result (origin totals are counted on the device);
- argument checks of the batch calls.
"""
import numpy as np
import pytest

from paper_2308_07487_amd import inputs

pytestmark = pytest.mark.gpu

TOL_RANDOM = {"fp32": 1e-6, "split_bf16": 1e-6, "split_fp16": 1e-6, "bf16x3": 1e-6}


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


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _tol_random(prec, counts, n_o):
    if prec != "split_bf16":
        return TOL_RANDOM[prec]
    m = float(np.min(counts[counts > 0])) * n_o
    return max(TOL_RANDOM[prec], 6 * 2.0 ** -17 / np.sqrt(m))


# (lattice, cells, n_origins, n_lags)
SAMPLES = [
    ("sc", (6, 6, 6), 20, 33),
    ("bcc", (4, 4, 4), 17, 40),
    ("sc", (5, 7, 4), 32, 17),
    ("bcc", (3, 3, 5), 9, 24),
    ("sc", (10, 10, 10), 16, 20),
    ("bcc", (2, 2, 2), 3, 5),
]


def _sample(S, lattice, cells, seed, dyadic=False, n_frames=0):
    pos = inputs.sc_positions(cells) if lattice == "sc" else inputs.bcc_positions(cells)
    pos, _, _ = inputs.permute_sites(pos, np.zeros((1, pos.shape[0], 3), np.float32), seed=seed)
    kind = S.BINS_SC if lattice == "sc" else S.BINS_BCC
    gen = inputs.dyadic_frames if dyadic else inputs.random_unit_frames
    return pos, kind, gen(n_frames, pos.shape[0], seed=seed + 100)


def _plans_and_frames(torch, S, prec, samples, dyadic=False):
    plans, frames, host = [], [], []
    for k, (lat, cells, n_o, n_L) in enumerate(samples):
        pos, kind, fr = _sample(S, lat, cells, seed=7 + k, dyadic=dyadic, n_frames=n_o + n_L - 1 + k % 3)
        plans.append(S.Plan(pos, kind, n_o, n_L, prec, cells=cells))
        frames.append(torch.from_numpy(fr).cuda())
        host.append((pos, kind, fr, cells, n_o, n_L))
    return plans, frames, host


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "bf16x3"])
def test_batch_matches_oracle(torch_dev, S, orc, prec):
    _say(f"batch of {len(SAMPLES)} mixed samples, {prec}")
    plans, frames, host = _plans_and_frames(torch_dev, S, prec, SAMPLES)
    with S.Batch(plans) as b:
        n_tasks, grid = b.info()
        print(f"  tasks {n_tasks}, grid {grid}", flush=True)
        assert grid % 8 == 0 and grid >= 8
        b.accumulate(frames)
        torch_dev.cuda.synchronize()
    for p, (pos, kind, fr, cells, n_o, n_L) in zip(plans, host):
        okind = orc.SC if kind == S.BINS_SC else orc.BCC
        out = p.finalize()
        H, no, sf, ms = p.raw()
        lags = np.arange(n_L)
        Hr, cr = orc.binned_corr(pos, fr, okind, n_o, lags, cells=cells)
        sfr = orc.self_corr(fr, n_o, lags)
        np.testing.assert_array_equal(out["counts"], cr)
        np.testing.assert_array_equal(no, float(n_o))
        C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), sfr)
        e = _normwise(out["C"], C)
        print(f"  N={pos.shape[0]} n_o={n_o} n_L={n_L}: normwise error {e:.3e}", flush=True)
        assert e <= _tol_random(prec, cr, n_o)
        np.testing.assert_allclose(sf, sfr, rtol=1e-12, atol=1e-9)
        p.close()


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_batch_dyadic_bit_exact(torch_dev, S, orc, prec):
    """Dyadic components: exact arithmetic, so a task that is lost, run twice
    or merged into the wrong plan changes the raw bins."""
    _say(f"batch dyadic {prec}")
    samples = [(lat, cells, min(n_o, 8), n_L) for lat, cells, n_o, n_L in SAMPLES]
    plans, frames, host = _plans_and_frames(torch_dev, S, prec, samples, dyadic=True)
    with S.Batch(plans) as b:
        b.accumulate(frames)
    for p, (pos, kind, fr, cells, n_o, n_L) in zip(plans, host):
        okind = orc.SC if kind == S.BINS_SC else orc.BCC
        H, no, _, _ = p.raw()
        Hr, _ = orc.binned_corr(pos, fr, okind, n_o, np.arange(n_L), cells=cells)
        np.testing.assert_array_equal(H, Hr)
        p.close()


def test_batch_radial(torch_dev, S, orc):
    _say("batch of radial samples")
    specs = [(300, 3.0, 64, 6.0, 12, 15), (700, 5.0, 1024, 10.0, 9, 20), (64, 1.5, 7, 3.0, 5, 6)]
    plans, frames, host = [], [], []
    for k, (n, R, ns, rm, n_o, n_L) in enumerate(specs):
        pos = inputs.ball_positions(n, R, seed=30 + k)
        fr = inputs.random_unit_frames(n_o + n_L - 1, n, seed=40 + k)
        plans.append(S.Plan(pos, S.BINS_RADIAL, n_o, n_L, "split_bf16", n_shells=ns, r_max=rm))
        frames.append(torch_dev.from_numpy(fr).cuda())
        host.append((pos, fr, ns, rm, n_o, n_L))
    with S.Batch(plans) as b:
        b.accumulate(frames)
    for p, (pos, fr, ns, rm, n_o, n_L) in zip(plans, host):
        out = p.finalize()
        lags = np.arange(n_L)
        Hr, cr = orc.binned_corr(pos, fr, orc.RADIAL, n_o, lags, n_shells=ns, r_max=rm)
        np.testing.assert_array_equal(out["counts"], cr)
        C, *_ = orc.finalize(Hr, cr, pos.shape[0], float(n_o), orc.self_corr(fr, n_o, lags))
        e = _normwise(out["C"], C)
        print(f"  N={pos.shape[0]} shells={ns}: normwise error {e:.3e}", flush=True)
        assert e <= _tol_random("split_bf16", cr, n_o)
        p.close()


def test_batch_equals_single_plans(torch_dev, S):
    _say("batch vs one accumulate per plan")
    samples = SAMPLES[:4]
    plans_b, frames, host = _plans_and_frames(torch_dev, S, "split_bf16", samples)
    plans_s, _, _ = _plans_and_frames(torch_dev, S, "split_bf16", samples)
    with S.Batch(plans_b) as b:
        b.accumulate(frames)
    for p, fr in zip(plans_s, frames):
        p.accumulate(fr)
    for pb, ps in zip(plans_b, plans_s):
        Hb, nob, sfb, msb = pb.raw()
        Hs, nos, sfs, mss = ps.raw()
        np.testing.assert_array_equal(nob, nos)
        np.testing.assert_allclose(sfb, sfs, rtol=1e-12)  # FP64 atomics: order varies
        np.testing.assert_array_equal(msb, mss)
        # same tasks, same FP32 sums; only the order of the FP64 merges differs
        np.testing.assert_allclose(Hb, Hs, rtol=1e-12, atol=1e-12 * np.max(np.abs(Hs)))
        pb.close()
        ps.close()


def test_graph_capture_replays(torch_dev, S):
    """Captured accumulates (one plan, and a batch) replayed three times with
    eager work and synchronisations in between: after every replay the
    normalised result equals the eager one and the origin totals count the
    replays."""
    torch = torch_dev
    _say("graph capture of sdc_accumulate and sdc_batch_accumulate")
    samples = SAMPLES[:3]
    ref_plans, frames, host = _plans_and_frames(torch, S, "split_bf16", samples)
    for p, fr in zip(ref_plans, frames):
        p.accumulate(fr)
    ref = [p.finalize() for p in ref_plans]

    cap_plans, _, _ = _plans_and_frames(torch, S, "split_bf16", samples)
    single, _, _ = _plans_and_frames(torch, S, "split_bf16", samples[:1])
    single = single[0]
    # the single plan's lag selection is uploaded by an uncaptured call first
    single.accumulate(frames[0])
    single.reset()
    torch.cuda.synchronize()
    batch = S.Batch(cap_plans)
    g_batch = torch.cuda.CUDAGraph()
    g_single = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_batch):
        batch.accumulate(frames)
    with torch.cuda.graph(g_single):
        single.accumulate(frames[0])
    torch.cuda.synchronize()
    # capture executes nothing
    for p in cap_plans + [single]:
        _, no, _, _ = p.raw()
        assert not no.any()
    x = torch.randn(512, 512, device="cuda")
    for rep in range(1, 4):
        g_batch.replay()
        y = x @ x  # eager work of the program between replays
        g_single.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        for k, p in enumerate(cap_plans + [single]):
            r = ref[k if k < len(cap_plans) else 0]
            out = p.finalize()
            _, no, _, _ = p.raw()
            n_o = samples[k if k < len(cap_plans) else 0][2]
            np.testing.assert_array_equal(no, float(rep * n_o))
            np.testing.assert_array_equal(out["counts"], r["counts"])
            e = _normwise(out["C"], r["C"])
            assert e <= 1e-12, (rep, k, e)
            np.testing.assert_allclose(out["Cself"], r["Cself"], rtol=1e-12)
    batch.close()
    for p in ref_plans + cap_plans + [single]:
        p.close()


def test_batch_invalid(torch_dev, S):
    _say("batch argument checks")
    a = S.Plan(inputs.sc_positions((4, 4, 4)), S.BINS_SC, 8, 16, "split_bf16", cells=(4, 4, 4))
    b = S.Plan(inputs.sc_positions((4, 4, 4)), S.BINS_SC, 8, 16, "fp32", cells=(4, 4, 4))
    r = S.Plan(inputs.ball_positions(100, 2.0, 1), S.BINS_RADIAL, 8, 16, "split_bf16", n_shells=8, r_max=4.0)
    for bad in ([a, b], [a, a], [a, r]):
        with pytest.raises(S.SdcError) as ei:
            S.Batch(bad)
        assert ei.value.status == S.ERR_INVALID_ARG
    batch = S.Batch([a])
    # a plan held by a batch cannot be destroyed
    with pytest.raises(S.SdcError) as ei:
        a.close()
    assert ei.value.status == S.ERR_STATE
    with pytest.raises(S.SdcError) as ei:
        batch.accumulate([torch_dev.zeros((10, 64, 3), device="cuda")])  # too few frames
    assert ei.value.status == S.ERR_INVALID_ARG
    with pytest.raises(ValueError):
        batch.accumulate([])
    batch.accumulate([torch_dev.zeros((23, 64, 3), device="cuda")])
    batch.close()
    a.close()
    b.close()
    r.close()
