"""Learned early stopping of capillary-filling sweeps.

A run of T steps records the filled length l_eff = l + H/2 every T/160 steps.
The surrogate reads the capillary's parameters and the first 16 samples (the
first 10 % of the run) and predicts l_eff at 64 times evenly spaced over the
remaining 90 %.

Prediction = physics anchor x learned correction.  The anchor is the
capillary-filling balance of Sec. 1 (Eq. 1 for the mean velocity, Eq. 3) with
the viscous drag of both the liquid column and the gas still to be displaced:
    (eta_l - eta_g) l^2 / 2 + eta_g Ltot l = (H gamma cos(theta) / 6) t + d,
eta = rho nu with rho = 1, Ltot = tube length + H/2, gamma the binary
interface tension (Sec. 3.1), theta the equilibrium angle, and d chosen so
that the curve passes through the last early sample.  The network (the
library's MLP 19 -> 256 -> 256 -> 256 -> 64, trained on the GPU) outputs
ln(l_eff / anchor) at the 64 times: the dynamic angle, the entrance losses
and the wall slip the anchor leaves out.  Several networks trained from
different seeds form an ensemble; its mean is the prediction and its spread
a measure of doubt.

The gate: run to 10 %, predict, continue to 20 %, compare with the simulation
where prediction and simulation overlap (predicted times up to 0.2 T).  A run
stops early only if that error is at most GATE_TOL, the ensemble spread over
the whole tail is at most SPREAD_TOL, the meniscus had entered the tube by
the end of the early window, and the predicted liquid column stays well
inside the reservoir's liquid; otherwise it continues to T.  Both limits
are tighter than the 1 % accuracy asked of the accepted tails (ACCEPT_ERR).
The lattice Boltzmann run always has the final
word.

The comparison method without the network fits the same balance with both c
and d free (least squares on the second half of the early window) and
extrapolates it.

Feature encoding (host-side input preparation; the network's arithmetic runs
in the library's kernels):
    x = [H / 80, ln(ratio) / ln(100), cos(theta),
         ln(l_k / l_16) for k = 1..15, ln(l_16 / H)]
    y = [ln(l_eff(t_j) / anchor(t_j)) for j = 1..64]
both standardised with the training set's mean and standard deviation.
"""
from __future__ import annotations

import math
import os
import time
from dataclasses import dataclass

import numpy as np

N_SAMPLES = 160            # samples per run (every T/160 steps)
N_EARLY = 16               # the first 10 %
N_OUT = 64                 # predicted times over the remaining 90 %
GATE_OVERLAP_END = 0.2     # the gate runs to 20 % of T
ACCEPT_ERR = 0.01          # accuracy asked of an accepted tail (relative, on l_eff)
GATE_TOL = 0.005           # largest error allowed on the gate window
SPREAD_TOL = 0.005         # largest ensemble spread allowed over the tail
L_ENTERED = 1.0            # filled length (nodes) needed at the end of the early window
N_NETS = 4                 # networks in the ensemble

# binary free-energy constants of the sweep (Sec. 3.1) and its interface tension
KAPPA, A_BULK = 0.04, 0.04
GAMMA_LG = 2.0 * math.sqrt(2.0) / 3.0 * math.sqrt(KAPPA * A_BULK)

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def out_times(T: int) -> np.ndarray:
    """t_j = 0.1 T + j 0.9 T / 64, j = 1..64."""
    return 0.1 * T + np.arange(1, N_OUT + 1) * (0.9 * T / N_OUT)


def sample_times(T: int) -> np.ndarray:
    """Steps of the recorded samples: k T / 160, k = 1..160."""
    return np.arange(1, N_SAMPLES + 1) * (T / N_SAMPLES)


def overlap_count(T: int) -> int:
    """Number of predicted times inside the gate window (t <= 0.2 T)."""
    return int(np.sum(out_times(T) <= GATE_OVERLAP_END * T + 1e-9))


def interp_history(hist: np.ndarray, T: int, t: np.ndarray) -> np.ndarray:
    """l_eff at times t by linear interpolation of the recorded samples
    (rows of hist are runs; sample k at step k T/160)."""
    ts = sample_times(T)
    return np.stack([np.interp(t, ts, h) for h in np.atleast_2d(hist)])


@dataclass
class RunParams:
    H: np.ndarray          # tube height (fluid rows)
    L: np.ndarray          # tube length
    ratio: np.ndarray      # viscosity ratio nu_l / nu_g
    theta: np.ndarray      # contact angle (degrees)
    nu_l: np.ndarray
    nu_g: np.ndarray
    V_liq: np.ndarray      # liquid area of the reservoir at t = 0

    @staticmethod
    def of(works) -> "RunParams":
        return RunParams(H=np.array([w.geom.tube_h for w in works], float),
                         L=np.array([w.geom.tube_len for w in works], float),
                         ratio=np.array([w.nu_l / w.nu_g for w in works], float),
                         theta=np.array([w.theta_deg for w in works], float),
                         nu_l=np.array([w.nu_l for w in works], float),
                         nu_g=np.array([w.nu_g for w in works], float),
                         V_liq=np.array([(1.0 - w.gas_frac) * (w.geom.nx - w.geom.tube_len) * w.geom.ny
                                         for w in works], float))

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in ("H", "L", "ratio", "theta", "nu_l", "nu_g", "V_liq")}

    def subset(self, idx) -> "RunParams":
        return RunParams(**{k: v[idx] for k, v in self.arrays().items()})


def load_runs(paths):
    """Recorded runs (data/generate.py output): parameters, l_eff histories,
    health flags.  Files without V_liq hold runs of the sweep distribution
    (reservoir 256 x (H + 40), liquid in half of it)."""
    ds = [np.load(p) for p in ([paths] if isinstance(paths, str) else paths)]
    cat = lambda k: np.concatenate([np.asarray(d[k]) for d in ds])
    H = cat("H").astype(float)
    V = cat("V_liq") if all("V_liq" in d.files for d in ds) else 0.5 * 256.0 * (H + 40.0)
    p = RunParams(H=H, L=cat("L").astype(float), ratio=cat("ratio").astype(float),
                  theta=cat("theta").astype(float), nu_l=cat("nu_l").astype(float),
                  nu_g=cat("nu_g").astype(float), V_liq=V.astype(float))
    return p, cat("hist").astype(float), cat("health")


def drained(hist: np.ndarray, drop: float = 1.0) -> np.ndarray:
    """Runs whose reservoir ran out of liquid: the liquid column leaves the
    inlet and the filled length (measured from the inlet) falls back."""
    return np.diff(np.atleast_2d(hist), axis=1).min(axis=1) < -drop


def eligible(p: RunParams, pred: np.ndarray, early: np.ndarray, frac: float = 0.8,
             l_min: float = L_ENTERED) -> np.ndarray:
    """A run may end early only if (1) the meniscus has advanced at least
    l_min nodes into the tube by the end of the early window (before that the
    early samples hold no filling to extrapolate from), and (2) the liquid the
    prediction puts in the tube stays below frac of the reservoir's liquid
    (otherwise the reservoir may drain before the end)."""
    l = np.atleast_2d(pred) - 0.5 * p.H[:, None]
    entered = np.atleast_2d(early)[:, -1] - 0.5 * p.H >= l_min
    return entered & (l.max(axis=1) * p.H < frac * p.V_liq)


def raw_features(p: RunParams, early: np.ndarray) -> np.ndarray:
    early = np.atleast_2d(early)
    ref = early[:, -1:]
    x = np.empty((early.shape[0], 19))
    x[:, 0] = p.H / 80.0
    x[:, 1] = np.log(p.ratio) / math.log(100.0)
    x[:, 2] = np.cos(np.radians(p.theta))
    x[:, 3:18] = np.log(early[:, :15] / ref)
    x[:, 18] = np.log(ref[:, 0] / p.H)
    return x


def anchor(p: RunParams, early: np.ndarray, T: int, t: np.ndarray | None = None) -> np.ndarray:
    """The capillary-filling balance with liquid and gas drag, surface tension
    GAMMA_LG and the equilibrium angle, through the last early sample."""
    early = np.atleast_2d(early)
    t = out_times(T) if t is None else t
    l16 = early[:, -1]
    t16 = sample_times(T)[N_EARLY - 1]
    a = 0.5 * (p.nu_l - p.nu_g)
    b = p.nu_g * (p.L + 0.5 * p.H)
    c = p.H * GAMMA_LG * np.cos(np.radians(p.theta)) / 6.0
    rhs = (a * l16 * l16 + b * l16)[:, None] + c[:, None] * (t - t16)[None, :]
    disc = np.maximum(b[:, None] ** 2 + 4.0 * a[:, None] * rhs, 0.0)
    lin = rhs / np.where(b > 0, b, 1.0)[:, None]
    quad = (-b[:, None] + np.sqrt(disc)) / (2.0 * np.where(np.abs(a) > 1e-12, a, 1.0)[:, None])
    return np.maximum(np.where(np.abs(a)[:, None] > 1e-12, quad, lin), 1e-3)


def raw_targets(p: RunParams, early: np.ndarray, late: np.ndarray, T: int) -> np.ndarray:
    return np.log(np.atleast_2d(late) / anchor(p, early, T))


def targets_to_l(p: RunParams, early: np.ndarray, y: np.ndarray, T: int) -> np.ndarray:
    return np.exp(y) * anchor(p, early, T)


@dataclass
class Scaler:
    xm: np.ndarray
    xs: np.ndarray
    ym: np.ndarray
    ys: np.ndarray

    @staticmethod
    def fit(X: np.ndarray, Y: np.ndarray) -> "Scaler":
        return Scaler(X.mean(0), X.std(0) + 1e-6, Y.mean(0), Y.std(0) + 1e-6)

    def x(self, X):
        return ((X - self.xm) / self.xs).astype(np.float32)

    def y(self, Y):
        return ((Y - self.ym) / self.ys).astype(np.float32)

    def y_inv(self, Yn):
        return np.asarray(Yn, float) * self.ys + self.ym


def washburn_predict(p: RunParams, early: np.ndarray, T: int, t: np.ndarray | None = None) -> np.ndarray:
    """Extrapolation of the capillary-filling law fitted to the early samples
    (second half of the early window, after the entrance transient)."""
    early = np.atleast_2d(early)
    t = out_times(T) if t is None else t
    ts = sample_times(T)[N_EARLY // 2:N_EARLY]
    out = np.empty((early.shape[0], t.size))
    for r in range(early.shape[0]):
        eta_l, eta_g = p.nu_l[r], p.nu_g[r]
        a = 0.5 * (eta_l - eta_g)
        b = eta_g * (p.L[r] + 0.5 * p.H[r])
        le = early[r, N_EARLY // 2:N_EARLY]
        q = a * le * le + b * le
        A = np.stack([ts, np.ones_like(ts)], axis=1)
        c, d = np.linalg.lstsq(A, q, rcond=None)[0]
        rhs = c * t + d
        if abs(a) < 1e-12:
            l = rhs / b
        else:
            disc = np.maximum(b * b + 4.0 * a * rhs, 0.0)
            l = (-b + np.sqrt(disc)) / (2.0 * a)
        out[r] = np.maximum(l, 1e-3)
    return out


class Surrogate:
    """An ensemble of trained networks and the feature scaling."""

    def __init__(self, nets, scaler: Scaler, T: int = 100_000, gate_tol: float = GATE_TOL,
                 spread_tol: float = SPREAD_TOL):
        self.nets = list(nets)
        self.scaler = scaler
        self.T = T
        self.gate_tol = gate_tol        # limits of the early-stopping decision,
        self.spread_tol = spread_tol    # chosen on validation runs (select_limits)

    def predict_all(self, p: RunParams, early: np.ndarray) -> np.ndarray:
        X = self.scaler.x(raw_features(p, early))
        return np.stack([targets_to_l(p, early, self.scaler.y_inv(n.predict(X)), self.T) for n in self.nets])

    def predict(self, p: RunParams, early: np.ndarray):
        """Ensemble mean of l_eff at out_times(T), and the largest relative
        spread of the members over the tail, per run."""
        P = self.predict_all(p, early)
        mean = P.mean(axis=0)
        spread = ((P.max(axis=0) - P.min(axis=0)) / mean).max(axis=1)
        return mean, spread

    def save(self, path: str):
        np.savez(path, T=self.T, xm=self.scaler.xm, xs=self.scaler.xs, ym=self.scaler.ym, ys=self.scaler.ys,
                 gate_tol=self.gate_tol, spread_tol=self.spread_tol,
                 **{f"params_{k}": n.get_params() for k, n in enumerate(self.nets)})

    def select_limits(self, p: RunParams, hist: np.ndarray,
                      grid=(0.002, 0.003, 0.004, 0.005)) -> dict:
        """Choose (gate_tol, spread_tol) on validation runs: the pair that
        accepts the most runs with no accepted tail off by more than
        ACCEPT_ERR (ties go to the tighter pair)."""
        mean, spread = self.predict(p, hist[:, :N_EARLY])
        best = None
        for g in grid:
            for s_ in grid:
                ev = evaluate(p, mean, hist, self.T, spread, g, s_)
                key = (ev["false_accepts"] == 0, ev["accept_rate"], -g - s_)
                if best is None or key > best[0]:
                    best = (key, g, s_, ev)
        _, self.gate_tol, self.spread_tol, ev = best
        return {"gate_tol": self.gate_tol, "spread_tol": self.spread_tol, "val_accept_rate": ev["accept_rate"],
                "val_false_accepts": ev["false_accepts"], "val_runs": len(hist)}

    @staticmethod
    def load(path: str, L=None) -> "Surrogate":
        if L is None:
            from . import lbcap as L
        d = np.load(path)
        nets = []
        k = 0
        while f"params_{k}" in d.files:
            n = L.MLP(seed=0)
            n.set_params(d[f"params_{k}"])
            nets.append(n)
            k += 1
        lim = {k: float(d[k]) for k in ("gate_tol", "spread_tol") if k in d.files}
        return Surrogate(nets, Scaler(d["xm"], d["xs"], d["ym"], d["ys"]), int(d["T"]), **lim)

    @staticmethod
    def train(p: RunParams, hist: np.ndarray, T: int, n_nets: int = N_NETS, epochs: int = 3000,
              batch: int = 512, lr: float = 1e-3, seed: int = 0, L=None, log=None) -> "Surrogate":
        """Train the ensemble on recorded runs with the library's kernels:
        Adam at lr for two thirds of the epochs, then at lr / 10."""
        if L is None:
            from . import lbcap as L
        early = hist[:, :N_EARLY]
        X = raw_features(p, early)
        Y = raw_targets(p, early, interp_history(hist, T, out_times(T)), T)
        sc = Scaler.fit(X, Y)
        Xn, Yn = sc.x(X), sc.y(Y)
        nets = []
        e1 = 2 * epochs // 3
        for k in range(n_nets):
            net = L.MLP(seed=seed + 101 * k)
            l1 = net.train(Xn, Yn, epochs=e1, batch=batch, lr=lr, seed=seed + 7 * k)
            l2 = net.train(Xn, Yn, epochs=epochs - e1, batch=batch, lr=lr / 10, seed=seed + 7 * k + 1)
            if log:
                log(f"  network {k}: loss {l1:.5f} -> {l2:.5f}")
            nets.append(net)
        return Surrogate(nets, sc, T)


def gate(pred: np.ndarray, sim_overlap: np.ndarray, tol: float = GATE_TOL):
    """Accept where the largest relative error on the overlap is <= tol."""
    err = np.abs(pred[:, :sim_overlap.shape[1]] - sim_overlap) / sim_overlap
    e = err.max(axis=1)
    return e <= tol, e


def decide(p: RunParams, pred: np.ndarray, sim_overlap: np.ndarray, early: np.ndarray,
           spread: np.ndarray | None = None, tol: float = GATE_TOL, spread_tol: float = SPREAD_TOL):
    """The early-stopping decision per run (see the module docstring)."""
    acc, gate_err = gate(pred, sim_overlap, tol)
    acc &= eligible(p, pred, early)
    if spread is not None:
        acc &= spread <= spread_tol
    return acc, gate_err


def evaluate(p: RunParams, pred: np.ndarray, hist: np.ndarray, T: int, spread: np.ndarray | None = None,
             tol: float = GATE_TOL, spread_tol: float = SPREAD_TOL) -> dict:
    """Gate decisions from the first 20 % of recorded runs and the true error
    of every prediction against the whole run."""
    truth = interp_history(hist, T, out_times(T))
    acc, gate_err = decide(p, pred, truth[:, :overlap_count(T)], np.atleast_2d(hist)[:, :N_EARLY], spread, tol,
                           spread_tol)
    true_err = (np.abs(pred - truth) / truth).max(axis=1)
    return {"accept": acc, "gate_err": gate_err, "true_err": true_err,
            "accept_rate": float(acc.mean()),
            "false_accepts": int(np.sum(acc & (true_err > ACCEPT_ERR))),
            "accepted_true_err_max": float(true_err[acc].max()) if acc.any() else 0.0,
            "accepted_true_err_median": float(np.median(true_err[acc])) if acc.any() else 0.0,
            "true_err_median": float(np.median(true_err))}


# ---- running the lattice ---------------------------------------------------------

def simulate(works, steps: int, sample_every: int, log=None, chunk: int = 10_000, autotune: bool = True):
    """Advance a batch of capillaries for `steps` steps recording l_eff every
    sample_every steps.  Returns (histories n x steps/sample_every, health
    flags, wall seconds)."""
    import torch
    from . import lbcap as L
    params = [L.params_from_workload(w) for w in works]
    geoms = [L.geometry_from_workload(w) for w in works]
    fields = [w.initial_field() for w in works]
    lat = L.Lattice(params, geoms, fields)
    del fields
    if log:
        log(f"  {len(works)} lattices on the device, {lat.fluid_nodes} fluid nodes")
    if autotune:
        cfg, us = lat.autotune(trial_steps=10)
        if log:
            log(f"  launch shape {cfg.asdict()}: {us:.0f} us per step")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        lat.step(n, sample_every=sample_every)
        done += n
        if log:
            torch.cuda.synchronize()
            log(f"  {done}/{steps} steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    health = lat.health()
    hist = np.stack([lat.l_history(k)[1] for k in range(len(works))])
    lat.close()
    return hist, health, wall


def run_sweep(works, T: int, sur: "Surrogate | None" = None, log=None, chunk: int = 10_000,
              autotune: bool = True) -> dict:
    """A batched sweep of T steps per capillary, with or without learned early
    stopping (the gate described at the top of this module).  Returns the wall
    time of the stepping and gating, the recorded histories, and with a
    surrogate the accepted runs and their predicted tails."""
    import torch
    from . import lbcap as L
    every = T // N_SAMPLES
    lat = L.Lattice([L.params_from_workload(w) for w in works], [L.geometry_from_workload(w) for w in works],
                    [w.initial_field() for w in works])
    if autotune:
        lat.autotune(trial_steps=10)
    n = len(works)
    p = RunParams.of(works)
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def advance(steps):
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            lat.step(k, sample_every=every)
            done += k
            if log:
                torch.cuda.synchronize()
                log(f"  t = {lat.t}, {time.perf_counter() - t0:.1f} s")

    out = {"n": n, "T": T}
    if sur is None:
        advance(T)
    else:
        t_early, t_gate = T // 10, int(GATE_OVERLAP_END * T)
        advance(t_early)
        early = np.stack([lat.l_history(k)[1][:N_EARLY] for k in range(n)])
        pred, spread = sur.predict(p, early)
        advance(t_gate - t_early)
        k_ov = overlap_count(T)
        ts = sample_times(T)[:t_gate // every]
        sim = np.stack([np.interp(out_times(T)[:k_ov], ts, lat.l_history(k)[1][:ts.size]) for k in range(n)])
        acc, gate_err = decide(p, pred, sim, early, spread, sur.gate_tol, sur.spread_tol)
        for k in np.nonzero(acc)[0]:
            lat.retire(int(k))
        if log:
            log(f"  gate at t = {lat.t}: {int(acc.sum())} of {n} runs accepted")
        if not acc.all():
            advance(T - t_gate)
        out.update(accept=acc, gate_err=gate_err, pred=pred, spread=spread)
    torch.cuda.synchronize()
    out["wall_s"] = time.perf_counter() - t0
    out["health"] = lat.health()
    out["hist"] = [lat.l_history(k)[1] for k in range(n)]
    lat.close()
    return out


def plain_sequential(works, T: int, log=None) -> dict:
    """Measured time of running the capillaries one after another, each alone
    for all T steps (tuned launch shape, graph replays, l sampled as in the
    sweep): the stepping time of every run, setup and tuning excluded as in
    run_sweep."""
    import torch
    from . import lbcap as L
    per_run = []
    for i, w in enumerate(works):
        lat = L.Lattice(L.params_from_workload(w), L.geometry_from_workload(w), w.initial_field())
        lat.autotune(trial_steps=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(T, sample_every=T // N_SAMPLES)
        torch.cuda.synchronize()
        per_run.append(time.perf_counter() - t0)
        lat.check()
        lat.close()
        if log and (i % 16 == 15 or i + 1 == len(works)):
            log(f"  plain (full runs): {i + 1} of {len(works)} runs, {sum(per_run):.1f} s")
    return {"measured_s": float(sum(per_run)), "per_run_s": per_run, "steps": T}


def plain_sequential_estimate(works, T: int, sample_steps: int = 1000, log=None) -> dict:
    """Time of running the capillaries one after another (each alone, tuned
    launch shape, graph replays), from sample_steps timed steps of each run,
    scaled to T steps."""
    import torch
    from . import lbcap as L
    total, sampled, per_run = 0.0, 0.0, []
    for i, w in enumerate(works):
        lat = L.Lattice(L.params_from_workload(w), L.geometry_from_workload(w), w.initial_field())
        lat.autotune(trial_steps=10)
        lat.step(64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(sample_steps, sample_every=T // N_SAMPLES)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sampled += dt
        total += dt * T / sample_steps
        per_run.append(dt * T / sample_steps)
        lat.close()
        if log and i % 64 == 63:
            log(f"  plain: {i + 1} runs sampled")
    return {"estimated_s": total, "sampled_s": sampled, "sample_steps": sample_steps, "per_run_s": per_run}
