"""Continuum results the oracle is pinned against (test infrastructure only).

Each function states the physics it encodes.  None of them is used by the
lattice code; they are the independent side of the pins:
  - the Maxwell equal-area coexistence of the van der Waals bulk pressure (Sec. 2);
  - the Cahn construction of the equilibrium contact angle for a wall that
    fixes the normal gradient of the order field (Sec. 2.2 and 3.2 wetting),
    by numerical quadrature for both free energies;
  - the flat-interface tension integral (Laplace law, Sec. 1);
  - least-squares fits used to read lattice results: circle through an
    interface contour (Sec. 3.2), straight lines for Washburn's law (Eq. 3),
    a parabola for Poiseuille flow (Eq. 1).
The binary interface tension here is the continuum (phi^4) value; the value
the paper prints for it (Sec. 3.1) is not reproduced by it or by the lattice:
parity with that printed number is unpinned.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

# ---------------------------------------------------------------------------
# van der Waals free energy, W(rho) = rho T ln(rho/(1-b rho)) - a rho^2, whose
# Legendre transform rho W' - W is the bulk pressure p0 of Sec. 2.
# ---------------------------------------------------------------------------


def vdw_p0(rho, a, b, T):
    return rho * T / (1.0 - b * rho) - a * rho * rho


def vdw_mu(rho, a, b, T):
    return T * np.log(rho / (1.0 - b * rho)) + T / (1.0 - b * rho) - 2.0 * a * rho


def vdw_W(rho, a, b, T):
    return rho * T * np.log(rho / (1.0 - b * rho)) - a * rho * rho


def vdw_maxwell(a=9.0 / 49.0, b=2.0 / 21.0, T=0.56, guess=(4.5, 2.5)):
    """Coexisting densities: equal pressure and equal chemical potential."""
    def eqs(v):
        rl, rg = v
        return [vdw_p0(rl, a, b, T) - vdw_p0(rg, a, b, T), vdw_mu(rl, a, b, T) - vdw_mu(rg, a, b, T)]
    rl, rg = optimize.fsolve(eqs, guess, xtol=1e-14)
    return float(rl), float(rg)


def _excess(W, mu_b, p_b):
    """Grand-potential excess over the coexisting bulk, Delta W(q) >= 0."""
    return lambda q: W(q) - mu_b * q + p_b


def _sqrt_pos(v):
    return math.sqrt(max(v, 0.0))


def interface_tension(dW, kappa, q_lo, q_hi):
    """gamma = integral of sqrt(2 kappa DeltaW) over the profile."""
    val, _ = integrate.quad(lambda q: _sqrt_pos(2.0 * kappa * dW(q)), q_lo, q_hi, limit=200,
                            epsabs=1e-13, epsrel=1e-12)
    return val


def _cahn_angle(dW, kappa, q_lo, q_hi, G):
    """Cahn construction with a surface energy -h q_s, h = -kappa G.

    The minimising wall value q_s solves sqrt(2 kappa DeltaW(q_s)) = |h| on the
    branch that leaves each bulk phase towards the favoured phase.  Returns the
    angle in degrees measured through the liquid (q_hi) phase."""
    h = -kappa * G
    gamma_lg = interface_tension(dW, kappa, q_lo, q_hi)
    if h == 0.0:
        return 90.0
    s = 1.0 if h > 0 else -1.0
    target = abs(h)
    F = lambda q: _sqrt_pos(2.0 * kappa * dW(q)) - target
    # wall next to the liquid: q_s beyond q_hi in the direction of s (h > 0: q_s > q_hi)
    # wall next to the gas: q_s moves from q_lo towards q_hi for h > 0
    if s > 0:
        q_hump = optimize.minimize_scalar(lambda q: -dW(q), bounds=(q_lo, q_hi), method="bounded").x
        if F(q_hump) < 0:
            raise ValueError("wall field too strong: complete wetting")
        qs_g = optimize.brentq(F, q_lo, q_hump, xtol=1e-15)
        hi = q_hi + 1e-6
        step = 0.01 * (q_hi - q_lo)
        while F(hi) < 0:
            hi += step
        qs_l = q_hi if F(q_hi) >= 0 else optimize.brentq(F, q_hi, hi, xtol=1e-15)
    else:
        q_hump = optimize.minimize_scalar(lambda q: -dW(q), bounds=(q_lo, q_hi), method="bounded").x
        if F(q_hump) < 0:
            raise ValueError("wall field too strong: complete drying")
        qs_l = optimize.brentq(F, q_hump, q_hi, xtol=1e-15)
        lo = q_lo - 1e-6
        step = 0.01 * (q_hi - q_lo)
        while F(lo) < 0:
            lo -= step
        qs_g = q_lo if F(q_lo) >= 0 else optimize.brentq(F, lo, q_lo, xtol=1e-15)

    def gamma_wall(qs, qb):
        a, b = (qs, qb) if qs < qb else (qb, qs)
        return -h * qs + interface_tension(dW, kappa, a, b)

    cos_t = (gamma_wall(qs_g, q_lo) - gamma_wall(qs_l, q_hi)) / gamma_lg
    return math.degrees(math.acos(max(-1.0, min(1.0, cos_t))))


def vdw_contact_angle(G, kappa=0.02, a=9.0 / 49.0, b=2.0 / 21.0, T=0.56):
    rl, rg = vdw_maxwell(a, b, T)
    W = lambda r: vdw_W(r, a, b, T)
    mu_b = float(vdw_mu(rl, a, b, T))
    p_b = float(vdw_p0(rl, a, b, T))
    return _cahn_angle(_excess(W, mu_b, p_b), kappa, rg, rl, G)


def vdw_tension(kappa=0.02, a=9.0 / 49.0, b=2.0 / 21.0, T=0.56):
    rl, rg = vdw_maxwell(a, b, T)
    W = lambda r: vdw_W(r, a, b, T)
    dW = _excess(W, float(vdw_mu(rl, a, b, T)), float(vdw_p0(rl, a, b, T)))
    return interface_tension(dW, kappa, rg, rl)


def binary_bulk(A=0.04, B=0.04):
    return math.sqrt(A / B)


def binary_excess(A=0.04, B=0.04):
    """phi^4 free energy -A phi^2/2 + B phi^4/4 relative to its minima."""
    pb = binary_bulk(A, B)
    return lambda p: 0.25 * B * (p * p - pb * pb) ** 2


def binary_contact_angle(G, kappa=0.04, A=0.04, B=0.04):
    pb = binary_bulk(A, B)
    return _cahn_angle(binary_excess(A, B), kappa, -pb, pb, G)


def binary_tension(kappa=0.04, A=0.04, B=0.04):
    pb = binary_bulk(A, B)
    return interface_tension(binary_excess(A, B), kappa, -pb, pb)


def binary_wall_gradient(theta_deg, kappa=0.04, A=0.04, B=0.04):
    """Inverse of binary_contact_angle by root finding (numeric quadrature)."""
    if abs(theta_deg - 90.0) < 1e-12:
        return 0.0
    sgn = -1.0 if theta_deg < 90.0 else 1.0
    # complete wetting bound: sqrt(2 kappa DeltaW(0)) = kappa |G|
    gmax = math.sqrt(2.0 * kappa * binary_excess(A, B)(0.0)) / kappa
    f = lambda g: binary_contact_angle(sgn * g, kappa, A, B) - theta_deg
    return sgn * optimize.brentq(f, 1e-4, gmax * (1 - 1e-9), xtol=1e-14)


def vdw_wall_gradient(theta_deg, kappa=0.02, a=9.0 / 49.0, b=2.0 / 21.0, T=0.56):
    if abs(theta_deg - 90.0) < 1e-12:
        return 0.0
    sgn = -1.0 if theta_deg < 90.0 else 1.0
    f = lambda g: vdw_contact_angle(sgn * g, kappa, a, b, T) - theta_deg
    lo, hi = 1e-4, 0.01
    while f(hi) * f(lo) > 0:
        hi *= 1.5
    return sgn * optimize.brentq(f, lo, hi, xtol=1e-14)


# ---------------------------------------------------------------------------
# fits
# ---------------------------------------------------------------------------


def fit_circle(xs, ys):
    """Algebraic least-squares circle (Kasa fit): x^2 + y^2 + D x + E y + F = 0."""
    xs, ys = np.asarray(xs, float), np.asarray(ys, float)
    Amat = np.column_stack([xs, ys, np.ones_like(xs)])
    rhs = -(xs * xs + ys * ys)
    (D, E, F), *_ = np.linalg.lstsq(Amat, rhs, rcond=None)
    xc, yc = -D / 2.0, -E / 2.0
    R = math.sqrt(xc * xc + yc * yc - F)
    return xc, yc, R


def contour_points(field, level, mask=None):
    """Linear-interpolated crossings of `level` along rows and columns."""
    pts = []
    ny, nx = field.shape
    ok = np.ones_like(field, dtype=bool) if mask is None else ~mask
    for y in range(ny):
        for x in range(nx - 1):
            a, b = field[y, x], field[y, x + 1]
            if ok[y, x] and ok[y, x + 1] and (a - level) * (b - level) < 0:
                pts.append((x + (a - level) / (a - b), y))
    for x in range(nx):
        for y in range(ny - 1):
            a, b = field[y, x], field[y + 1, x]
            if ok[y, x] and ok[y + 1, x] and (a - level) * (b - level) < 0:
                pts.append((x, y + (a - level) / (a - b)))
    return np.array(pts)


def drop_contact_angle(field, level, y_wall, mask=None, y_min_fit=None):
    """Angle (degrees, through the drop) of a circular cap on the wall y = y_wall."""
    pts = contour_points(field, level, mask)
    if y_min_fit is not None:
        pts = pts[pts[:, 1] >= y_min_fit]
    xc, yc, R = fit_circle(pts[:, 0], pts[:, 1])
    # cap above the wall: cos(theta) = (y_wall - yc)/R ... angle through the liquid
    c = (y_wall - yc) / R
    return math.degrees(math.acos(max(-1.0, min(1.0, c)))), (xc, yc, R)


def meniscus_angle(q, x_in, tube_len, y0, tube_h, q_mid, edge_rows=2):
    """Contact angle (degrees, through the liquid, liquid on the inlet side) of
    the meniscus in a channel of width tube_h (walls half a node outside the
    boundary rows), as analysed for the dynamic angles of Sec. 3.2: interface
    crossings of q_mid scanned from the inlet in the rows away from the walls,
    an unconstrained algebraic circle fit, and cos(theta) = (tube_h / 2) / R with
    the sign of the side (gas: +, liquid: -) on which the centre lies."""
    xs, ys = [], []
    for y in range(y0 + edge_rows, y0 + tube_h - edge_rows):
        row = q[y]
        if row[x_in] < q_mid:
            continue
        for k in range(1, tube_len):
            a, b = row[x_in + k - 1], row[x_in + k]
            if b < q_mid:
                xs.append(x_in + k - 1 + (a - q_mid) / (a - b))
                ys.append(float(y))
                break
    xs, ys = np.array(xs), np.array(ys)
    xc, yc, R = fit_circle(xs, ys)
    apex = xs[np.argmin(np.abs(ys - (y0 + 0.5 * (tube_h - 1))))]
    sign = 1.0 if xc > apex else -1.0
    c = sign * min(1.0, 0.5 * tube_h / R)
    return math.degrees(math.acos(c)), R


def linear_fit(x, y):
    """Least-squares line and its coefficient of determination."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    A = np.column_stack([x, np.ones_like(x)])
    (m, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    pred = m * x + c
    ss_res = float(((y - pred) ** 2).sum())
    ss_tot = float(((y - y.mean()) ** 2).sum())
    return float(m), float(c), 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
