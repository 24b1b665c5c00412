"""The meniscus contact angle (library host function and oracle), pinned on
fields whose interface is an exact circular arc of known angle, and compared
with each other on oracle runs; the GPU-side entry point is exercised in
test_gpu_parity.py."""
import math

import numpy as np
import pytest

from oracle import Oracle, OracleGeom, OracleParams
from oracle import physics as P
from paper_0911_0459_amd import inputs as I
from tests.helpers import oracle_wall_grad

NX, NY, X_IN, LEN, H, Y0 = 220, 50, 50, 170, 30, 10


@pytest.fixture(scope="module")
def L():
    from paper_0911_0459_amd.build import build_library
    build_library(force=False)
    from paper_0911_0459_amd import lbcap
    return lbcap


def arc_field(theta, apex=120.0, w=2.0):
    """Liquid (+1) on the inlet side of a circular arc through (apex, centreline)
    that meets walls H apart at theta (flat at 90 degrees); tanh profile in x."""
    y, x = np.mgrid[0:NY, 0:NX].astype(float)
    yc = Y0 + 0.5 * (H - 1)
    c = math.cos(math.radians(theta))
    if abs(c) < 1e-12:
        x_arc = np.full_like(y, apex)
    else:
        R = 0.5 * H / abs(c)
        s = np.sqrt(np.maximum(R * R - (y - yc) ** 2, 0.0))
        # wetting: centre on the gas side, the arc bulges back into the liquid
        x_arc = (apex + R) - s if c > 0 else (apex - R) + s
    return np.tanh((x_arc - x) / w)


@pytest.mark.parametrize("theta", [30.0, 45.0, 60.0, 75.0, 90.0, 105.0, 120.0])
def test_library_recovers_arc_angle(L, theta):
    g = L.make_geometry(NX, NY, X_IN, LEN, H, Y0)
    th, R, apex = L.lb_meniscus_angle_field(arc_field(theta), g, 0.0)
    assert abs(th - theta) < 0.5
    assert abs(apex - 120.0) < 0.1
    if theta != 90.0:
        assert abs(R - 0.5 * H / abs(math.cos(math.radians(theta)))) < 0.02 * R


@pytest.mark.parametrize("theta", [30.0, 45.0, 60.0, 75.0, 105.0, 120.0])
def test_oracle_recovers_arc_angle(theta):
    th, R = P.meniscus_angle(arc_field(theta), X_IN, LEN, Y0, H, 0.0)
    assert abs(th - theta) < 0.5


def test_errors(L):
    g = L.make_geometry(NX, NY, X_IN, LEN, H, Y0)
    with pytest.raises(L.LbError) as e:
        L.lb_meniscus_angle_field(-np.ones((NY, NX)), g, 0.0)      # gas everywhere: no meniscus
    assert e.value.code == L.LB_ESTATE
    with pytest.raises(L.LbError) as e:
        L.lb_meniscus_angle_field(arc_field(60.0), L.make_geometry(NX, NY), 0.0)   # no tube
    assert e.value.code == L.LB_EINVAL
    with pytest.raises(L.LbError):
        L.lb_meniscus_angle_field(arc_field(60.0), g, 0.0, edge_rows=14)


def test_library_and_oracle_agree_on_a_filling_capillary(L):
    """Binary capillary, ratio 10, 45 degrees, after the meniscus has formed."""
    g = I.Geometry(nx=240, ny=44, x_in=60, tube_len=180, tube_h=24, y0=10)
    nl, ng = I.viscosity_pair(10.0)
    w = I.Workload("m", "binary", g, 0, 0, 3, nu_l=nl, nu_g=ng, theta_deg=45.0, liquid=1.0, gas=-1.0,
                   **I.BIN_CONSTS)
    o = Oracle(OracleParams(model="binary", kappa=0.04, A=0.04, B=0.04, Gamma=1.0, nu_l=nl, nu_g=ng,
                            wall_grad=oracle_wall_grad(w)), OracleGeom(**g.asdict()), w.initial_field())
    o.step(3000)
    phi = o.moments()[3]
    th_o, R_o = P.meniscus_angle(phi, g.x_in, g.tube_len, g.y0, g.tube_h, 0.0)
    th_l, R_l, _ = L.lb_meniscus_angle_field(phi, L.make_geometry(**g.asdict()), 0.0)
    assert 20.0 < th_l < 80.0
    assert abs(th_l - th_o) < 1.0
