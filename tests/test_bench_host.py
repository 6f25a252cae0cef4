"""Host-side checks of the benchmark script's contract (no GPU)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_lookup_checks_the_sources(tmp_path, monkeypatch):
    """A committed traffic figure is reported only while the kernel sources it
    was taken on are unchanged; workloads without one report none."""
    assert bench.measured_traffic("sc8_afm", "split_bf16") is None
    prof, srcs = bench.TRAFFIC_PROFILES["sc36_afm"]
    text = open(prof).read()
    copy = tmp_path / "profile.md"
    copy.write_text(text)
    monkeypatch.setitem(bench.TRAFFIC_PROFILES, "sc36_afm", (str(copy), srcs))
    current = bench.measured_traffic("sc36_afm", "split_bf16")
    edited = "\n".join(("kernel_source_sha256: " + "0" * 64) if ln.startswith("kernel_source_sha256:") else ln
                       for ln in text.splitlines())
    copy.write_text(edited)
    assert bench.measured_traffic("sc36_afm", "split_bf16") is None
    assert bench.measured_traffic("sc36_afm", "fp32") is None
    if current is not None:
        assert current > 0


def test_workloads_are_defined():
    for name in ("sc36_afm", "sc32_fm", "ball65k", "batch48", "sq420", "ball65k_sq", "mc_sc128"):
        assert name in bench.WORKLOADS


def test_unknown_compare_precision_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--compare", "''"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "--compare" in r.stderr


def test_contraction_sum_against_brute_force():
    """The summed-bin reference of each form (the exact sum of the piece
    products the contraction keeps, plus the diagonal dropped ones) against a
    plain loop over all ordered pairs; the pieces rebuild each value to the
    form's precision (BF16x3 and FP32 exactly), and the splits' sum differs
    from sum_o M.M by their dropped products."""
    import numpy as np
    import torch
    rng = np.random.default_rng(11)
    f = torch.from_numpy(rng.standard_normal((7, 23, 3)).astype(np.float32))
    n_o, n_L = 4, 4
    M = f.double().sum(dim=1)
    mm = np.array([float((M[:n_o] * M[t:t + n_o]).sum()) for t in range(n_L)])
    for prec, rec_bar in (("fp32", 0.0), ("split_bf16", 2.0 ** -16), ("split_fp16", 2.0 ** -22), ("bf16x3", 0.0)):
        ps = bench._pieces(torch, f, prec)
        rec = sum(p.double() for p in ps)
        assert float((rec - f.double()).abs().max()) <= rec_bar * float(f.abs().max())
        kept, diag = bench._PIECE_PRODUCTS[prec]
        P = [p.double().numpy() for p in ps]
        brute = np.zeros(n_L)
        for t in range(n_L):
            for o in range(n_o):
                for i in range(f.shape[1]):
                    for j in range(f.shape[1]):
                        for a, b in kept + (diag if i == j else []):
                            brute[t] += P[a][o, i] @ P[b][o + t, j]
        got = bench.contraction_sum(torch, f, prec, n_o, n_L)
        np.testing.assert_allclose(got, brute, rtol=1e-13, atol=1e-12)
        if prec == "fp32":
            np.testing.assert_allclose(got, mm, rtol=1e-13)
        else:
            assert np.max(np.abs(got - mm)) > 0.0
