"""Shared helpers of the test suite: run the same seeded workload through the
oracle and through the GPU library, compare fields."""
from __future__ import annotations

import os

import numpy as np

from oracle import Oracle, OracleGeom, OracleParams
from oracle import physics as P
from paper_0911_0459_amd import inputs as I


def oracle_wall_grad(w: I.Workload) -> float:
    """Wall gradient of a workload on the oracle side: given directly, else the
    oracle's own Cahn construction for its contact angle."""
    if w.wall_grad is not None:
        return w.wall_grad
    if w.model == "binary":
        return P.binary_wall_gradient(w.theta_deg, w.kappa, w.A, w.B)
    return P.vdw_wall_gradient(w.theta_deg, w.kappa, w.a, w.b, w.T)


def oracle_params(w: I.Workload, **over) -> OracleParams:
    d = dict(model=w.model, kappa=w.kappa, a=w.a, b=w.b, T=w.T, A=w.A, B=w.B, Gamma=w.Gamma,
             nu_l=w.nu_l, nu_g=w.nu_g, wall_grad=oracle_wall_grad(w))
    d.update(over)
    return OracleParams(**d)


def q_mid(w: I.Workload) -> float:
    if w.model == "binary":
        return 0.0
    rl, rg = P.vdw_maxwell(w.a, w.b, w.T)
    return 0.5 * (rl + rg)


def run_oracle(w: I.Workload, steps: int, sample_every: int = 0, init=None, **over):
    """Fields after `steps` and the l_eff samples every `sample_every` steps."""
    o = Oracle(oracle_params(w, **over), OracleGeom(**w.geom.asdict()),
               w.initial_field() if init is None else init)
    ls = []
    if sample_every:
        for _ in range(steps // sample_every):
            o.step(sample_every)
            ls.append(o.interface_length(q_mid(w))[1])
        o.step(steps - o.t)
    else:
        o.step(steps)
    return o.moments(), np.array(ls)


def field_errors(w: I.Workload, gpu, orc):
    """max relative rho deviation, max |dphi|, max |du| over fluid nodes."""
    fluid = ~w.geom.solid()
    rho, ux, uy, phi = gpu
    r_o, ux_o, uy_o, phi_o = orc
    drho = float((np.abs(rho - r_o)[fluid] / np.abs(r_o)[fluid]).max())
    dphi = float(np.abs(phi - phi_o)[fluid].max())
    du = float(max(np.abs(ux - ux_o)[fluid].max(), np.abs(uy - uy_o)[fluid].max()))
    return drho, dphi, du


def printed_values():
    """Values printed in the paper, with their tolerances, from
    tests/golden/paper_values.txt (name -> (value, tolerance or None))."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, value, tol = line.split()[:3]
            out[name] = (float(value), None if tol == "-" else float(tol))
    return out
