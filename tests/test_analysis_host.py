"""Host-side analysis entry points of the library (no GPU): the capillary
balance with gas drag behind Fig. "10" and the tube-flow statistics of Fig. 3.

These run in the library's host code; the expected values come from the
closed forms the balance reduces to, an independent numerical integration of
its differential form, and fields built here with known answers."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_0911_0459_amd import lbcap as L

H, LT, GAMMA, COS = 40.0, 350.0, 0.0112, 0.5


@pytest.mark.parametrize("t", [0.0, 1e3, 5e4, 2e5])
def test_washburn_without_gas_drag_is_eq3(t):
    """eta_g = 0: l^2 = l0^2 + gamma H cos(theta) t / (3 eta_l) (Eq. 3)."""
    eta = 4.513 / 6
    got = L.lb_washburn_length(t, 10.0, H, LT, GAMMA, COS, eta, 0.0)
    assert abs(got - math.sqrt(100.0 + GAMMA * H * COS * t / (3 * eta))) < 1e-10 * got


def test_washburn_with_equal_viscosities_is_linear():
    """eta_l = eta_g: the drag no longer depends on l, so l grows linearly,
    l = l0 + gamma H cos(theta) t / (6 eta L)."""
    eta = 1 / 6
    for t in (1e3, 1e4, 1e5):
        got = L.lb_washburn_length(t, 10.0, H, LT, GAMMA, COS, eta, eta)
        assert abs(got - (10.0 + GAMMA * H * COS * t / (6 * eta * LT))) < 1e-10 * got


@pytest.mark.parametrize("eta_g", [0.05, 2.543 / 6, 0.9])
def test_washburn_with_gas_drag_integrates_the_force_balance(eta_g):
    """The closed form against the force balance it integrates,
    2 gamma cos(theta)/H = 12 (dl/dt)(eta_l l + eta_g (L - l))/H^2, solved
    numerically from l(0) = 10; more gas drag fills more slowly."""
    eta_l = 4.513 / 6
    rhs = lambda t, l: [GAMMA * H * COS / (6.0 * (eta_l * l[0] + eta_g * (LT - l[0])))]
    ts = np.array([1e3, 1e4, 5e4])
    sol = solve_ivp(rhs, (0.0, ts[-1]), [10.0], t_eval=ts, rtol=1e-11, atol=1e-12, method="DOP853")
    for t, l_ode in zip(ts, sol.y[0]):
        got = L.lb_washburn_length(t, 10.0, H, LT, GAMMA, COS, eta_l, eta_g)
        assert abs(got - l_ode) < 1e-7 * l_ode
        assert got < L.lb_washburn_length(t, 10.0, H, LT, GAMMA, COS, eta_l, 0.0)


def test_washburn_rejects_bad_arguments():
    for args in [(-1, 10, H, LT, GAMMA, COS, 1.0, 0.0), (1, 400, H, LT, GAMMA, COS, 1.0, 0.0),
                 (1, 10, 0.0, LT, GAMMA, COS, 1.0, 0.0), (1, 10, H, LT, GAMMA, COS, 0.0, 0.0),
                 (1, 10, H, LT, GAMMA, COS, 1.0, -0.1)]:
        with pytest.raises(L.LbError):
            L.lb_washburn_length(*args)


def test_tube_flow_statistics_of_a_built_field():
    """A tube 30 x 8 (rows 2..9 of a 50 x 12 lattice, inlet at 10) with liquid
    (rho 4.5, u 0.02) up to x_in + 12 and gas (rho 2.5, u -0.01) beyond, the
    centre rows with a known profile: the filled length, the centreline
    velocity, the region means and the two condensation rates."""
    g = L.make_geometry(50, 12, 10, 30, 8, 2)
    q = np.full((12, 50), 2.5)
    q[:, :22] = 4.5
    q[:, 22] = 3.0                       # crossing of q_mid = 3.5 between x = 21 and 22
    rho = q.copy()
    ux = np.where(q > 3.5, 0.02, -0.01)
    ux[5, 10:40] = np.linspace(-0.05, 0.05, 30)   # centre rows 5 and 6 (even H: their mean)
    ux[6, 10:40] = np.linspace(0.05, 0.15, 30)
    rows = slice(2, 10)
    out, line = L.lb_tube_flow_field(q, rho, ux, g, 3.5, margin=2, v_meniscus=0.03)
    # l = (k - 1) + (q(k-1) - q_mid)/(q(k-1) - q(k)) with k = 12 (x = 22)
    assert abs(out.l - (11 + (4.5 - 3.5) / (4.5 - 3.0))) < 1e-12
    assert np.abs(line - 0.5 * (ux[5, 10:40] + ux[6, 10:40])).max() < 1e-15
    # the meniscus lies in column x_in + floor(l) = 21: liquid x 12 .. 18
    # (x_in + 2 up to 21 - 2, exclusive), gas x 24 .. 37 (21 + 1 + 2 up to the
    # tube's end 40 - 2, exclusive)
    m = rho[rows, 12:19]
    u_l = (m * ux[rows, 12:19]).sum() / m.sum()
    assert out.liquid_cols == 7 and abs(out.u_liquid - u_l) < 1e-15 and abs(out.rho_liquid - 4.5) < 1e-15
    mg = rho[rows, 24:38]
    u_g = (mg * ux[rows, 24:38]).sum() / mg.sum()
    assert out.gas_cols == 14 and abs(out.u_gas - u_g) < 1e-15
    assert abs(out.condensation_liquid_side - out.rho_liquid * (0.03 - u_l)) < 1e-15
    assert abs(out.condensation_gas_side - out.rho_gas * (0.03 - u_g)) < 1e-15
    with pytest.raises(L.LbError):
        L.lb_tube_flow_field(q, rho, ux, L.make_geometry(50, 12), 3.5)
