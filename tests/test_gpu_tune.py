"""The autotuner on the device (sdc_autotune through the C ABI): it times
every candidate, keeps the longest segment among the candidates within 0.5%
of the fastest, writes its size class into the JSON tuning file without
touching other entries, and plan creation picks the entry up through
SDC_TUNING_FILE unless the caller gives the tuning explicitly."""
import json

import pytest

from paper_2308_07487_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2308_07487_amd import sdc
    return sdc


def test_autotune_cache_and_plan_creation(S, tmp_path, monkeypatch):
    L = (8, 8, 8)
    pos = inputs.sc_positions(L)
    cache = tmp_path / "tuning.json"
    cands = [("two_pass", 16), ("one_pass", 48), ("lag_split", 1 << 20), ("fold", 32)]
    print("[case] autotune sc 8^3, 16 origins x 24 lags, split_bf16", flush=True)
    best, ms, times = S.autotune(pos, S.BINS_SC, 16, 24, "split_bf16", cells=L, candidates=cands,
                                 cache_path=str(cache))
    print(f"  best {best} {ms:.3f} ms; {times}", flush=True)
    assert [(c["schedule"], c["segment_pairs"]) for c, _ in times] == cands
    assert all(t > 0 for _, t in times)
    fastest = min(t for _, t in times)
    ties = [c for c, t in times if t <= fastest * 1.005]
    assert best["segment_pairs"] == max(c["segment_pairs"] for c in ties)
    assert best in ties and ms == dict((tuple(c.values()), t) for c, t in times)[tuple(best.values())]

    entries = json.loads(cache.read_text())["entries"]
    assert len(entries) == 1 and entries[0]["segment_pairs"] == best["segment_pairs"]
    assert len(entries[0]["candidates"].split()) == len(cands)
    assert S.tuning_lookup(str(cache), pos.shape[0], S.BINS_SC, 16, 24, "split_bf16", cells=L) == best
    # another size class (more K-steps) is not in the file yet
    assert S.tuning_lookup(str(cache), pos.shape[0], S.BINS_SC, 64, 24, "split_bf16", cells=L) is None

    monkeypatch.setenv("SDC_TUNING_FILE", str(cache))
    with S.Plan(pos, S.BINS_SC, 16, 24, "split_bf16", cells=L) as p:
        assert p.tuning == best
    with S.Plan(pos, S.BINS_SC, 16, 24, "split_bf16", cells=L, schedule="one_pass", segment_pairs=24) as p:
        assert p.tuning == {"schedule": "one_pass", "segment_pairs": 24}
    with S.Plan(pos, S.BINS_SC, 64, 24, "split_bf16", cells=L) as p:  # not in the file: the defaults
        assert p.tuning == {"schedule": "two_pass", "segment_pairs": 96}

    # a second class is added beside the first
    S.autotune(pos, S.BINS_SC, 64, 24, "split_bf16", cells=L, candidates=[("one_pass", 32)], cache_path=str(cache))
    entries = json.loads(cache.read_text())["entries"]
    assert len(entries) == 2
    assert S.tuning_lookup(str(cache), pos.shape[0], S.BINS_SC, 16, 24, "split_bf16", cells=L) == best
    assert S.tuning_lookup(str(cache), pos.shape[0], S.BINS_SC, 64, 24, "split_bf16",
                           cells=L) == {"schedule": "one_pass", "segment_pairs": 32}


def test_autotune_rejects_bad_candidates(S, tmp_path):
    pos = inputs.sc_positions((4, 4, 4))
    with pytest.raises(S.SdcError):  # two-pass exists only for the hi/lo splits
        S.autotune(pos, S.BINS_SC, 8, 8, "fp32", cells=(4, 4, 4), candidates=[("two_pass", 16)])
