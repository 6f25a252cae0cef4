"""Tunes the fused product for the benchmarked sample shapes on this GPU and
writes the tuning file plan creation reads (SDC_TUNING_FILE).

    python -m paper_2308_07487_amd.tune [--out FILE] [--only all|full|batch] [--batch-lags 0]

Every distinct size class (bin kind, size, K-steps, precision) of the
workloads gets one sdc_autotune run on its first sample shape, with seeded
unit spins; classes already in the file are kept.  The single-sample
workloads (sc 36^3 in split-BF16 and split-FP16, sc 32^3, sc 8^3, the 420^2
square lattice, the 65536-point ball) run over all their lags with every
schedule of the precision and the segment lengths 16, 32, 48 and 96 (the
ball: the built-in radial candidates); the 48 batch samples with the
two-pass schedule (the batch's work-weighted vote) and segments of 16, 32
and 48 pairs, over all their lags by default (--batch-lags N: the first N;
the segment choice depends on the number of lag groups that run together).
Each class's winner and every candidate's median time go to the file, and
the library prints every candidate's time as it is measured.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2308_07487_amd import inputs, sdc  # noqa: E402


def shapes():
    """(label, positions, kind, spec, n_origins, n_lags, precision, full) of every shape tuned."""
    out = []
    sc36 = inputs.sc_positions((36, 36, 36))
    out.append(("sc36", sc36, sdc.BINS_SC, dict(cells=(36, 36, 36)), 128, 256, "split_bf16", True))
    out.append(("sc36", sc36, sdc.BINS_SC, dict(cells=(36, 36, 36)), 128, 256, "split_fp16", True))
    out.append(("sc32", inputs.sc_positions((32, 32, 32)), sdc.BINS_SC, dict(cells=(32, 32, 32)), 64, 256,
                "split_bf16", True))
    out.append(("sc8", inputs.sc_positions((8, 8, 8)), sdc.BINS_SC, dict(cells=(8, 8, 8)), 32, 64, "split_bf16", True))
    out.append(("sq420", inputs.sc_positions((420, 420, 1)), sdc.BINS_SC, dict(cells=(420, 420, 1)), 50, 64,
                "split_bf16", True))
    out.append(("ball65k", inputs.ball_positions(65536, 25.0, seed=0x5DC00013), sdc.BINS_RADIAL,
                dict(n_shells=1024, r_max=50.0), 64, 128, "split_bf16", True))
    for s in inputs.batch_samples(48, 0x5DC00500):
        sc = s["lattice"] == "sc"
        pos = inputs.sc_positions(s["cells"]) if sc else inputs.bcc_positions(s["cells"])
        out.append((f"batch {s['lattice']} {s['cells'][0]}", pos, sdc.BINS_SC if sc else sdc.BINS_BCC,
                    dict(cells=s["cells"]), s["n_origins"], s["n_lags"], "split_bf16", False))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "gfx950.json"))
    ap.add_argument("--batch-lags", type=int, default=0, help="lags timed per batch sample (0: all)")
    ap.add_argument("--only", default="all", choices=["all", "full", "batch"])
    args = ap.parse_args()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    os.environ["SDC_TUNE_VERBOSE"] = "1"  # the library prints each candidate's time as it is measured
    t_all = time.perf_counter()
    for label, pos, kind, spec, n_o, n_L, prec, full in shapes():
        if (args.only == "full" and not full) or (args.only == "batch" and full):
            continue
        if sdc.tuning_lookup(args.out, pos.shape[0], kind, n_o, n_L, prec, **spec) is not None:
            continue  # its size class is tuned already
        t0 = time.perf_counter()
        if full and kind == sdc.BINS_RADIAL:
            best, ms, cands = sdc.autotune(pos, kind, n_o, n_L, prec, max_lags=0, cache_path=args.out, **spec)
        elif full:
            cands = [(sch, seg) for sch in ("one_pass", "two_pass", "lag_split", "fold") for seg in (16, 32, 48, 96)]
            best, ms, cands = sdc.autotune(pos, kind, n_o, n_L, prec, max_lags=0, candidates=cands,
                                           cache_path=args.out, **spec)
        else:
            cands = [("two_pass", seg) for seg in (16, 32, 48)]
            best, ms, cands = sdc.autotune(pos, kind, n_o, n_L, prec, max_lags=args.batch_lags, candidates=cands,
                                           cache_path=args.out, **spec)
        times = " ".join(f"{c['schedule'][:4]}/{c['segment_pairs']}:{t:.2f}" for c, t in cands)
        print(f"{label:18s} N={pos.shape[0]:7d} {n_o:4d}x{n_L:<4d} {prec:10s} -> {best['schedule']}/"
              f"{best['segment_pairs']} {ms:.2f} ms  [{times}]  ({time.perf_counter() - t0:.1f} s)", flush=True)
    print(f"tuning file {args.out} written in {time.perf_counter() - t_all:.1f} s", flush=True)


if __name__ == "__main__":
    main()
