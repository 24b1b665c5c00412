"""Records l_eff(t) of seeded capillary runs on the GPU (the training and
held-out data of the surrogate, or the sweep itself).

    python -m paper_0911_0459_amd.data.generate --kind train --part 0 --parts 8 --out runs_train_0.npz

kind: train (master seeds 1000..5095), heldout (9000..9511) or sweep (the 256
capillaries of master seed 4).  Each run lasts 100000 steps, sampled every 625.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from paper_0911_0459_amd import inputs as I
from paper_0911_0459_amd import surrogate as S


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kind", choices=["train", "heldout", "sweep"], required=True)
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    works = I.sweep_batch(4, 256, a.steps) if a.kind == "sweep" else I.surrogate_runs(a.kind, a.steps)
    n = len(works)
    lo, hi = a.part * n // a.parts, (a.part + 1) * n // a.parts
    works = works[lo:hi]
    every = a.steps // S.N_SAMPLES
    print(f"{a.kind} runs {lo}..{hi - 1}: {len(works)} capillaries, {a.steps} steps", flush=True)
    t0 = time.perf_counter()
    hist, health, wall = S.simulate(works, a.steps, every, log=lambda m: print(m, flush=True))
    p = S.RunParams.of(works)
    np.savez_compressed(a.out, hist=hist.astype(np.float32), health=health, wall=wall, index=np.arange(lo, hi),
                        seeds=np.array([w.seed for w in works]), steps=a.steps, **p.arrays())
    bad = int(np.sum(health != 0))
    print(f"done: {wall:.1f} s stepping, {time.perf_counter() - t0:.1f} s total, unstable {bad}", flush=True)
    return 0 if bad == 0 else 3


if __name__ == "__main__":
    sys.exit(main())
