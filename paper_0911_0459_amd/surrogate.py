"""Learned early stopping of capillary-filling sweeps.

A run of T steps records the filled length l_eff = l + H/2 every T/160 steps.
The network (the library's MLP, 19 -> 256 -> 256 -> 256 -> 64) reads the
capillary's parameters and the first 16 samples (the first 10 % of the run)
and predicts l_eff at 64 times evenly spaced over the remaining 90 %.

The gate: run to 10 %, predict, continue to 20 %, compare the prediction with
the simulation where they overlap (the predicted times up to 0.2 T).  If the
largest relative error there is at most 1 % the run stops and its tail is the
prediction; otherwise it continues to T.  The lattice Boltzmann run is always
the judge.

The comparison method without the network extrapolates the capillary-filling
law fitted to the same early samples: the Washburn balance of capillary
pressure against viscous drag in the liquid column and in the gas still to be
displaced (Eq. 3 with the gas term), integrated in time:
    (eta_l - eta_g) l_eff^2 / 2 + eta_g Ltot l_eff = c t + d,
with eta = rho nu (rho = 1), Ltot the tube length plus H/2, and c, d fitted
by least squares; l_eff(t) is the positive root.

Feature encoding (host-side input preparation; all arithmetic of the network
runs in the library's kernels):
    x = [H / 80, ln(ratio) / ln(100), cos(theta),
         ln(l_k / l_16) for k = 1..15, ln(l_16 / H)]
    y = [ln(l(t_j) / l_16) for j = 1..64]
then standardised with the training set's mean and standard deviation.
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
TOL = 0.01                 # accepted relative error

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

    @staticmethod
    def of(works) -> "RunParams":
        return RunParams(H=np.array([w.geom.tube_h for w in works], float),
                         L=np.array([w.geom.tube_len for w in works], float),
                         ratio=np.array([w.nu_l / w.nu_g for w in works], float),
                         theta=np.array([w.theta_deg for w in works], float),
                         nu_l=np.array([w.nu_l for w in works], float),
                         nu_g=np.array([w.nu_g for w in works], float))

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in ("H", "L", "ratio", "theta", "nu_l", "nu_g")}


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


def raw_targets(early: np.ndarray, late: np.ndarray) -> np.ndarray:
    return np.log(np.atleast_2d(late) / np.atleast_2d(early)[:, -1:])


def targets_to_l(early: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.exp(y) * np.atleast_2d(early)[:, -1:]


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
    """The trained network and its feature scaling."""

    def __init__(self, net, scaler: Scaler):
        self.net = net
        self.scaler = scaler

    def predict(self, p: RunParams, early: np.ndarray) -> np.ndarray:
        X = self.scaler.x(raw_features(p, early))
        return targets_to_l(early, self.scaler.y_inv(self.net.predict(X)))

    def save(self, path: str):
        np.savez(path, params=self.net.get_params(), xm=self.scaler.xm, xs=self.scaler.xs, ym=self.scaler.ym,
                 ys=self.scaler.ys)

    @staticmethod
    def load(path: str, L=None) -> "Surrogate":
        if L is None:
            from . import lbcap as L
        d = np.load(path)
        net = L.MLP(seed=0)
        net.set_params(d["params"])
        return Surrogate(net, Scaler(d["xm"], d["xs"], d["ym"], d["ys"]))


def gate(pred: np.ndarray, sim_overlap: np.ndarray, tol: float = TOL):
    """Accept where the largest relative error on the overlap is <= tol."""
    err = np.abs(pred[:, :sim_overlap.shape[1]] - sim_overlap) / sim_overlap
    e = err.max(axis=1)
    return e <= tol, e


def evaluate(pred: np.ndarray, hist: np.ndarray, T: int, tol: float = TOL) -> dict:
    """Gate decisions from the first 20 % and the true error of every
    prediction against the full recorded run."""
    t = out_times(T)
    truth = interp_history(hist, T, t)
    k = overlap_count(T)
    acc, gate_err = gate(pred, truth[:, :k], tol)
    true_err = (np.abs(pred - truth) / truth).max(axis=1)
    return {"accept": acc, "gate_err": gate_err, "true_err": true_err,
            "accept_rate": float(acc.mean()),
            "accepted_true_err_max": float(true_err[acc].max()) if acc.any() else 0.0,
            "accepted_true_err_median": float(np.median(true_err[acc])) if acc.any() else 0.0,
            "false_accepts": int(np.sum(acc & (true_err > tol))),
            "all_true_err_median": float(np.median(true_err))}


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
    if autotune:
        lat.autotune(trial_steps=10)
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
