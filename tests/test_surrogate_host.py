"""Host-side logic of the surrogate sweep (no GPU): sampling grids, the
physics anchor, the Washburn extrapolation, the gate and the run filters."""
import math

import numpy as np

from paper_0911_0459_amd import surrogate as S

T = 100_000


def _params(n=3, H=40.0, L=2000.0, ratio=10.0, theta=60.0):
    nu0 = 1 / 6
    nl, ng = nu0 * math.sqrt(ratio), nu0 / math.sqrt(ratio)
    f = lambda v: np.full(n, float(v))
    return S.RunParams(H=f(H), L=f(L), ratio=f(ratio), theta=f(theta), nu_l=f(nl), nu_g=f(ng),
                       V_liq=f(0.5 * 256 * (H + 40)))


def test_grids():
    t = S.out_times(T)
    assert t.size == 64 and t[0] == 10_000 + 1406.25 and t[-1] == T
    ts = S.sample_times(T)
    assert ts.size == 160 and ts[15] == 10_000 and ts[-1] == T
    assert S.overlap_count(T) == 7          # t_7 = 19843.75 <= 0.2 T < t_8


def test_interpolation_is_exact_on_linear_histories():
    hist = np.stack([3.0 + 1e-3 * S.sample_times(T), 7.0 - 2e-5 * S.sample_times(T)])
    t = S.out_times(T)
    assert np.allclose(S.interp_history(hist, T, t), np.stack([3.0 + 1e-3 * t, 7.0 - 2e-5 * t]), rtol=0, atol=1e-12)


def test_anchor_passes_through_the_last_early_sample():
    p = _params()
    early = np.tile(np.linspace(20, 30, 16), (3, 1))
    a = S.anchor(p, early, T, t=np.array([S.sample_times(T)[15]]))
    assert np.allclose(a[:, 0], 30.0, rtol=0, atol=1e-9)


def test_anchor_is_washburn_without_gas_drag():
    """nu_g -> 0: l^2 - l16^2 = H gamma cos(theta) (t - t16) / (3 eta_l), Eq. 3."""
    p = _params(n=1)
    p.nu_g[:] = 0.0
    early = np.full((1, 16), 25.0)
    t = S.out_times(T)
    a = S.anchor(p, early, T)[0]
    c = p.H[0] * S.GAMMA_LG * math.cos(math.radians(60.0)) / 6.0
    ref = np.sqrt(25.0 ** 2 + 2 * c * (t - 10_000) / p.nu_l[0])
    assert np.allclose(a, ref, rtol=1e-12)


def test_anchor_at_ninety_degrees_stays_put():
    p = _params(n=1, theta=90.0)
    a = S.anchor(p, np.full((1, 16), 21.0), T)
    assert np.allclose(a, 21.0, atol=1e-9)


def test_washburn_fit_recovers_its_own_law():
    """Histories that follow the balance exactly are extrapolated exactly."""
    p = _params(n=2, ratio=30.0)
    a = 0.5 * (p.nu_l - p.nu_g)
    b = p.nu_g * (p.L + 0.5 * p.H)
    c, d = np.array([0.05, 0.11]), np.array([500.0, 900.0])
    ts = S.sample_times(T)
    rhs = c[:, None] * ts[None, :] + d[:, None]
    hist = (-b[:, None] + np.sqrt(b[:, None] ** 2 + 4 * a[:, None] * rhs)) / (2 * a[:, None])
    pred = S.washburn_predict(p, hist[:, :16], T)
    truth = S.interp_history(hist, T, S.out_times(T))
    assert np.abs(pred - truth).max() / truth.max() < 1e-3    # interpolation of the truth dominates


def test_gate_and_decision():
    p = _params(n=4)
    sim = np.full((4, 7), 50.0)
    pred = np.full((4, 64), 50.0)
    pred[1, 3] = 50.0 * 1.006          # gate error 0.6 % > 0.5 %
    pred[2, 40] = 300.0                # liquid column beyond the reservoir's liquid
    spread = np.array([0.001, 0.001, 0.001, 0.02])   # run 3: networks disagree
    early = np.full((4, 16), 0.5 * 40 + 3.0)
    acc, err = S.decide(p, pred, sim, early, spread)
    assert acc.tolist() == [True, False, False, False]
    assert abs(err[1] - 0.006) < 1e-12
    early[0, -1] = 0.5 * 40 + 0.5                     # meniscus not yet a node into the tube
    assert not S.decide(p, pred, sim, early, spread)[0][0]


def test_drained_and_eligible():
    h = np.tile(np.linspace(20, 80, 160), (2, 1))
    h[1, 150:] = 20.0
    assert S.drained(h).tolist() == [False, True]
    p = _params(n=2, H=60.0)
    V = p.V_liq[0]
    l_ok = 0.5 * 60 + 0.7 * V / 60
    l_bad = 0.5 * 60 + 0.9 * V / 60
    early = np.full((2, 16), 0.5 * 60 + 2.0)
    assert S.eligible(p, np.array([[l_ok] * 64, [l_bad] * 64]), early).tolist() == [True, False]


def test_features_and_targets_round_trip():
    p = _params(n=2)
    rng = np.random.default_rng(0)
    early = 20 + np.cumsum(rng.uniform(0, 1, (2, 16)), axis=1)
    late = 40 + np.cumsum(rng.uniform(0, 1, (2, 64)), axis=1)
    x = S.raw_features(p, early)
    assert x.shape == (2, 19) and np.allclose(np.exp(x[:, 18]) * p.H, early[:, -1])
    y = S.raw_targets(p, early, late, T)
    assert np.allclose(S.targets_to_l(p, early, y, T), late)
