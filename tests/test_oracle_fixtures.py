"""The recorded surrogate data tied to the oracle.

The training and held-out l_eff(t) histories under paper_0911_0459_amd/data/
were recorded by the GPU library (they are the LB-generated runs the learned
surrogate is trained on).  Here the oracle re-runs a held-out capillary from
the same seeded input and must reproduce its early history: the first 16
samples (t = 625 .. 10^4, the surrogate's input window) within 0.5 lattice
units, the filled-length bar of the GPU parity gates."""
import numpy as np
import pytest

from paper_0911_0459_amd import inputs as I
from paper_0911_0459_amd import surrogate as S
from tests.helpers import run_oracle

pytestmark = pytest.mark.slow


def test_heldout_fixture_early_history_matches_the_oracle():
    d = np.load(f"{S.DATA_DIR}/runs_heldout.npz", allow_pickle=False)
    nodes = (256 + d["L"]) * (d["H"] + 40)
    i = int(np.argmin(nodes))                       # the smallest held-out lattice (813 x 51)
    T = int(d["steps"])
    every = T // S.N_SAMPLES
    w = I.surrogate_runs("heldout", T)[int(d["index"][i])]
    assert (w.geom.tube_h, w.geom.tube_len, w.seed) == (int(d["H"][i]), int(d["L"][i]), int(d["seeds"][i]))
    _, lo = run_oracle(w, 16 * every, sample_every=every)
    rec = d["hist"][i, :16].astype(np.float64)
    print(f"held-out run {i}: oracle {lo[-1]:.3f}, recorded {rec[-1]:.3f}, max |dl| {np.abs(lo - rec).max():.3e}")
    assert np.abs(lo - rec).max() <= 0.5
    assert lo[-1] > lo[0] + 2.0                     # the meniscus moves in the window
