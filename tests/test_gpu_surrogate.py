"""The trained surrogate ensemble on the held-out runs, and the early-stopping
sweep driver on the GPU.

The held-out runs (master seeds 9000..9511, 100000 steps each, recorded by
the library) are the reference: an accepted run's predicted tail must be within
1 % of the recorded l_eff everywhere, and the network must accept more runs
than the Washburn extrapolation without it, with fewer wrong acceptances.
"""
import os

import numpy as np
import pytest

from paper_0911_0459_amd import inputs as I
from paper_0911_0459_amd import surrogate as S

pytestmark = pytest.mark.gpu

T = 100_000
NET = os.path.join(S.DATA_DIR, "surrogate_net.npz")
HELDOUT = os.path.join(S.DATA_DIR, "runs_heldout.npz")


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_0459_amd import lbcap
    return lbcap


@pytest.fixture(scope="module")
def heldout():
    p, h, health = S.load_runs(HELDOUT)
    keep = (health == 0) & ~S.drained(h)
    return p.subset(keep), h[keep], np.nonzero(keep)[0]


def test_accepted_tails_are_within_one_percent(L, heldout):
    p, h, _ = heldout
    sur = S.Surrogate.load(NET, L)
    assert len(sur.nets) == S.N_NETS
    mean, spread = sur.predict(p, h[:, :S.N_EARLY])
    ev = S.evaluate(p, mean, h, T, spread, sur.gate_tol, sur.spread_tol)
    assert ev["false_accepts"] == 0
    assert ev["accepted_true_err_max"] <= S.ACCEPT_ERR
    assert ev["accept_rate"] >= 0.5


def test_network_beats_the_washburn_extrapolation(L, heldout):
    p, h, _ = heldout
    sur = S.Surrogate.load(NET, L)
    mean, spread = sur.predict(p, h[:, :S.N_EARLY])
    ev = S.evaluate(p, mean, h, T, spread, sur.gate_tol, sur.spread_tol)
    wb = S.evaluate(p, S.washburn_predict(p, h[:, :S.N_EARLY], T), h, T)
    assert ev["accept_rate"] > 2 * wb["accept_rate"]
    assert wb["false_accepts"] > ev["false_accepts"]
    assert ev["true_err_median"] < 0.2 * wb["true_err_median"]


def test_recorded_runs_are_reproduced(L, heldout):
    """The stored held-out histories are what the library computes."""
    p, h, idx = heldout
    works = I.surrogate_runs("heldout", T)
    pick = [int(idx[0]), int(idx[1])]
    hist, health, _ = S.simulate([works[k] for k in pick], 20_000, T // S.N_SAMPLES, autotune=False)
    assert not health.any()
    d = np.load(HELDOUT)
    ref = d["hist"][pick, :hist.shape[1]].astype(float)
    assert np.abs(hist - ref).max() <= 1e-3 * np.abs(ref).max()


def test_early_stopping_sweep_driver(L, heldout):
    """A small sweep with the gate: accepted runs stop at 20 % and their
    predicted tails match the recorded runs; the others run to the end and
    reproduce the recorded histories."""
    p, h, idx = heldout
    works = I.surrogate_runs("heldout", T)
    pick = [int(k) for k in idx[:6]]
    sur = S.Surrogate.load(NET, L)
    out = S.run_sweep([works[k] for k in pick], T, sur, autotune=False)
    d = np.load(HELDOUT)
    truth_hist = d["hist"][pick].astype(float)
    truth = S.interp_history(truth_hist, T, S.out_times(T))
    for k, acc in enumerate(out["accept"]):
        if acc:
            assert len(out["hist"][k]) == int(S.GATE_OVERLAP_END * S.N_SAMPLES)
            assert (np.abs(out["pred"][k] - truth[k]) / truth[k]).max() <= S.ACCEPT_ERR
        else:
            assert len(out["hist"][k]) == S.N_SAMPLES
            assert np.abs(out["hist"][k] - truth_hist[k]).max() <= 1e-3 * truth_hist[k].max()
