"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP32 populations against FP64):
  - after 10^4 steps: max relative rho deviation <= 1e-4, max |dphi| <= 1e-4,
    filled length within 0.5 lattice units (the acceptance gates);
  - short runs (<= 500 steps) must agree much more tightly: 2e-5 relative on
    rho, 2e-5 on phi, 1e-6 on u, which catches any wrong term long before the
    accumulated FP32 rounding matters.
"""
import numpy as np
import pytest

from paper_0911_0459_amd import inputs as I
from tests.helpers import field_errors, oracle_wall_grad, q_mid, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_0459_amd import lbcap
    return lbcap


def gpu_run(L, w, steps, sample_every=0, cfg=None, init=None, **over):
    p = L.params_from_workload(w)           # the library maps the contact angle itself
    for k, v in over.items():
        setattr(p, k, v)
    lat = L.Lattice(p, L.geometry_from_workload(w), w.initial_field() if init is None else init)
    if cfg is not None:
        lat.set_launch_config(**cfg)
    ls = []
    if sample_every:
        for _ in range(steps // sample_every):
            lat.step(sample_every)
            ls.append(lat.interface_length()[1])
        lat.step(steps - lat.t)
    else:
        lat.step(steps)
    out = lat.moments()
    lat.close()
    return out, np.array(ls)


def small_binary(nx=256, ny=64, H=20, ratio=10.0, seed=5, theta=60.0):
    g = I.Geometry(nx=nx, ny=ny, x_in=nx // 2, tube_len=nx - nx // 2, tube_h=H, y0=(ny - H) // 2)
    nl, ng = I.viscosity_pair(ratio)
    return I.Workload(f"binary_{nx}x{ny}", "binary", g, steps=0, sample_every=0, seed=seed, nu_l=nl, nu_g=ng,
                      theta_deg=theta, liquid=1.0, gas=-1.0, **I.BIN_CONSTS)


# ---- the 10^4-step gates ---------------------------------------------------------
def test_vdw_capillary_256x64_1e4_steps(L):
    """Liquid-gas capillary 256x64 (H=20, length 128, tau 0.8, gradient -0.144)."""
    w = I.vdw_capillary_256x64()
    gpu, lg = gpu_run(L, w, 10_000, sample_every=500)
    orc, lo = run_oracle(w, 10_000, sample_every=500)
    drho, _, du = field_errors(w, gpu, orc)
    print(f"vdw 1e4: max rel drho {drho:.3e}, max du {du:.3e}, max dl {np.abs(lg - lo).max():.3e}")
    assert drho <= 1e-4
    assert np.abs(lg - lo).max() <= 0.5
    assert lo[-1] > lo[0]          # the tube is filling


def test_binary_capillary_1e4_steps(L):
    """Binary capillary (ratio 10, 60 degrees) on a 256x64 lattice."""
    w = small_binary()
    orc, lo = run_oracle(w, 10_000, sample_every=500)
    # population storage; two steps per sweep; the default, moment storage
    for cfg in (dict(schedule=4, chunk_rows=8), dict(schedule=5, chunk_rows=16), None):
        gpu, lg = gpu_run(L, w, 10_000, sample_every=500, cfg=cfg)
        drho, dphi, du = field_errors(w, gpu, orc)
        print(f"binary 1e4 {cfg}: max rel drho {drho:.3e}, max dphi {dphi:.3e}, du {du:.3e}, "
              f"max dl {np.abs(lg - lo).max():.3e}")
        assert drho <= 1e-4 and dphi <= 1e-4
        assert np.abs(lg - lo).max() <= 0.5


def test_binary_capillary_1024x128_1e4_steps(L):
    """The binary capillary at its real size: 1024x128, tube H=40 and length
    768, ratio 10, 60 degrees, seed 2, 10^4 steps against the oracle in the
    population storage (schedule 4) and in the default launch shape (the
    moment storage, schedule 6), the filled length compared every 500 steps."""
    w = I.binary_capillary_1024x128()
    print(f"binary 1024x128 1e4: oracle run", flush=True)
    orc, lo = run_oracle(w, 10_000, sample_every=500)
    assert lo[-1] > lo[0] + 5.0          # the liquid is filling the tube
    # population storage; two steps per sweep; the default, moment storage
    for cfg in (dict(schedule=4, chunk_rows=8), dict(schedule=5, chunk_rows=16), None):
        print(f"binary 1024x128 1e4: GPU run {cfg}", flush=True)
        gpu, lg = gpu_run(L, w, 10_000, sample_every=500, cfg=cfg)
        drho, dphi, du = field_errors(w, gpu, orc)
        print(f"binary 1024x128 1e4 {cfg}: max rel drho {drho:.3e}, max dphi {dphi:.3e}, du {du:.3e}, "
              f"max dl {np.abs(lg - lo).max():.3e}, l_oracle {lo[0]:.2f} -> {lo[-1]:.2f}")
        assert drho <= 1e-4 and dphi <= 1e-4
        assert np.abs(lg - lo).max() <= 0.5


# ---- tight short-run parity across tiles, tails and launch shapes --------------
SHAPES = [
    dict(tile_rows=1, schedule=0, persist_blocks_per_cu=4, graph_steps=0, fp64_arith=0),
    dict(tile_rows=2, schedule=1, persist_blocks_per_cu=4, graph_steps=2, fp64_arith=1),
    dict(tile_rows=4, schedule=2, persist_blocks_per_cu=4, graph_steps=64, fp64_arith=0),
    dict(tile_rows=8, schedule=1, persist_blocks_per_cu=4, graph_steps=16, fp64_arith=0),
    dict(schedule=3, chunk_rows=0, graph_steps=64, fp64_arith=1),
    dict(schedule=3, chunk_rows=8, graph_steps=0, fp64_arith=0),
    dict(schedule=4, chunk_rows=0, graph_steps=64, fp64_arith=1),
    dict(schedule=4, chunk_rows=8, graph_steps=0, fp64_arith=0),
    dict(schedule=4, chunk_rows=5, graph_steps=2, fp64_arith=1),
    dict(schedule=4, chunk_rows=16, graph_steps=64, fp64_arith=1),   # long chunks end in short tails
]


@pytest.mark.parametrize("cfg", SHAPES, ids=lambda c: "-".join(f"{k[:2]}{v}" for k, v in c.items()))
@pytest.mark.parametrize("model", ["vdw", "binary"])
def test_ragged_lattice_short_run(L, model, cfg):
    """150x37 lattice (ragged in x and y), odd tube height, several tiles."""
    g = I.Geometry(nx=150, ny=37, x_in=53, tube_len=97, tube_h=13, y0=11)
    if model == "vdw":
        w = I.Workload("vdw_ragged", "vdw", g, 0, 0, seed=21, nu_l=0.13, nu_g=0.13, wall_grad=-0.1,
                       liquid=4.5, gas=2.6, **I.VDW_CONSTS)
    else:
        nl, ng = I.viscosity_pair(30.0)
        w = I.Workload("bin_ragged", "binary", g, 0, 0, seed=22, nu_l=nl, nu_g=ng, theta_deg=45.0,
                       liquid=1.0, gas=-1.0, **I.BIN_CONSTS)
    gpu, _ = gpu_run(L, w, 300, cfg=cfg)
    orc, _ = run_oracle(w, 300)
    drho, dphi, du = field_errors(w, gpu, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (drho, dphi, du)


@pytest.mark.parametrize("model", ["vdw", "binary"])
def test_wide_strips_across_strip_boundaries(L, model):
    """700x45 lattice: four 192-column strips (the inlet inside the second,
    two tube-only strips, the last one ragged and ending with the tube),
    against the oracle and against the one-wavefront strips (to rounding)."""
    g = I.Geometry(nx=700, ny=45, x_in=250, tube_len=450, tube_h=17, y0=14)
    if model == "vdw":
        w = I.Workload("vdw_wide", "vdw", g, 0, 0, seed=31, nu_l=0.13, nu_g=0.13, wall_grad=-0.1,
                       liquid=4.5, gas=2.6, **I.VDW_CONSTS)
    else:
        nl, ng = I.viscosity_pair(20.0)
        w = I.Workload("bin_wide", "binary", g, 0, 0, seed=32, nu_l=nl, nu_g=ng, theta_deg=50.0,
                       liquid=1.0, gas=-1.0, **I.BIN_CONSTS)
    wide, _ = gpu_run(L, w, 200, cfg=dict(schedule=4, chunk_rows=8, fp64_arith=1))
    narrow, _ = gpu_run(L, w, 200, cfg=dict(schedule=3, chunk_rows=8, fp64_arith=1))
    gap = max(float(np.abs(x - y).max()) for x, y in zip(wide, narrow))
    print(f"{model}: wide vs one-wavefront strips, max |difference| {gap:.3e}")
    assert gap <= 1e-6
    orc, _ = run_oracle(w, 200)
    drho, dphi, du = field_errors(w, wide, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (drho, dphi, du)


@pytest.mark.parametrize("model", ["vdw", "binary"])
def test_strips_that_the_tube_enters_or_leaves(L, model):
    """520x41 lattice, reservoirs on both sides of the tube (inlet at 150,
    outlet at 430, neither on a 32-column boundary), odd tube height and wall
    thickness. The strips that the tube enters or leaves sweep their channel
    rows, and their wall rows in strips of their own over the reservoir
    columns. Against the oracle (as are the tiles), the one-wavefront strips
    (to rounding), and across chunkings (bitwise)."""
    g = I.Geometry(nx=520, ny=41, x_in=150, tube_len=280, tube_h=15, y0=13)
    if model == "vdw":
        w = I.Workload("vdw_ends", "vdw", g, 0, 0, seed=33, nu_l=0.13, nu_g=0.13, wall_grad=-0.1,
                       liquid=4.5, gas=2.6, **I.VDW_CONSTS)
    else:
        nl, ng = I.viscosity_pair(20.0)
        w = I.Workload("bin_ends", "binary", g, 0, 0, seed=34, nu_l=nl, nu_g=ng, theta_deg=50.0,
                       liquid=1.0, gas=-1.0, **I.BIN_CONSTS)
    wide, _ = gpu_run(L, w, 200, cfg=dict(schedule=4, chunk_rows=0, fp64_arith=1))
    orc, _ = run_oracle(w, 200)
    drho, dphi, du = field_errors(w, wide, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (drho, dphi, du)
    for cfg in (dict(schedule=4, chunk_rows=5), dict(schedule=4, chunk_rows=12)):
        got, _ = gpu_run(L, w, 200, cfg=dict(cfg, fp64_arith=1))
        for x, y in zip(wide, got):
            assert np.array_equal(x, y), cfg
    narrow, _ = gpu_run(L, w, 200, cfg=dict(schedule=3, chunk_rows=6, fp64_arith=1))
    gap = max(float(np.abs(x - y).max()) for x, y in zip(wide, narrow))
    print(f"{model}: wide vs one-wavefront strips, max |difference| {gap:.3e}")
    assert gap <= 1e-6
    tile, _ = gpu_run(L, w, 200, cfg=dict(tile_rows=4, schedule=1, fp64_arith=1))
    drho, dphi, du = field_errors(w, tile, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, ("tiles", drho, dphi, du)


@pytest.mark.parametrize("cfg", [dict(schedule=4, chunk_rows=0), dict(schedule=4, chunk_rows=4),
                                 dict(schedule=3, chunk_rows=0), dict(tile_rows=2, schedule=1)],
                         ids=["wide", "wide-ch4", "strip", "tile"])
@pytest.mark.parametrize("model", ["vdw", "binary"])
def test_smallest_lattice(L, model, cfg):
    """5x3, fully periodic (the smallest lattice the library accepts is 3x3):
    every row and column index of the sweeps wraps, and one strip covers the
    lattice many times over."""
    g = I.Geometry(nx=5, ny=3)
    if model == "vdw":
        w = I.Workload("vdw_5x3", "vdw", g, 0, 0, seed=41, nu_l=0.13, nu_g=0.13, wall_grad=0.0,
                       liquid=4.5, gas=2.6, **I.VDW_CONSTS)
        init = np.array([[4.5, 4.4, 3.0, 2.6, 2.7], [4.5, 4.2, 3.1, 2.6, 2.8], [4.3, 4.5, 2.9, 2.7, 2.6]])
    else:
        nl, ng = I.viscosity_pair(10.0)
        w = I.Workload("bin_5x3", "binary", g, 0, 0, seed=42, nu_l=nl, nu_g=ng, wall_grad=0.0,
                       liquid=1.0, gas=-1.0, **I.BIN_CONSTS)
        init = np.array([[1.0, 0.8, -0.2, -1.0, -0.9], [0.9, 0.7, 0.1, -0.8, -1.0], [1.0, 0.6, -0.3, -0.9, -0.7]])
    gpu, _ = gpu_run(L, w, 100, cfg=cfg, init=init)
    orc, _ = run_oracle(w, 100, init=init)
    drho, dphi, du = field_errors(w, gpu, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (drho, dphi, du)


def test_lambda_off_and_full_periodic_box(L):
    """No walls at all (tube_len 0) and the Galilean term switched off."""
    g = I.Geometry(nx=96, ny=40)
    w = I.Workload("vdw_box", "vdw", g, 0, 0, seed=23, nu_l=0.2, nu_g=0.2, wall_grad=0.0, liquid=4.5,
                   gas=2.6, **I.VDW_CONSTS)
    y, x = np.mgrid[0:40, 0:96]
    init = np.where(np.hypot(x - 48, y - 20) < 12, 4.5, 2.6) + I.node_noise(23, 96, 40)
    for lam in (0, 1):
        gpu, _ = gpu_run(L, w, 400, init=init, lambda_mode=lam)
        orc, _ = run_oracle(w, 400, init=init, lambda_mode=lam)
        drho, _, du = field_errors(w, gpu, orc)
        assert drho < 2e-5 and du < 1e-6


@pytest.mark.parametrize("cfg", [None, dict(schedule=4, chunk_rows=8), dict(schedule=5, chunk_rows=8)],
                         ids=["default", "populations", "two_steps_per_sweep"])
def test_poiseuille_body_force_narrow_lattice(L, cfg):
    """nx = 3 (narrower than one tile, and than the halo of the two-step sweep)
    with the Guo body force, in each binary row sweep."""
    H = 20
    g = I.Geometry(nx=3, ny=H + 2, x_in=0, tube_len=3, tube_h=H, y0=1)
    w = I.Workload("pois", "binary", g, 0, 0, seed=24, nu_l=1 / 6, nu_g=1 / 6, wall_grad=0.0, liquid=1.0,
                   gas=1.0, noise=0.0, **I.BIN_CONSTS)
    init = np.ones((H + 2, 3))
    gpu, _ = gpu_run(L, w, 3000, cfg=cfg, init=init, force_x=1e-5)
    orc, _ = run_oracle(w, 3000, init=init, force_x=1e-5)
    rho, ux, _, _ = gpu
    assert np.abs(ux - orc[1]).max() / np.abs(orc[1]).max() < 1e-4
    assert np.abs(rho - orc[0])[1:-1].max() < 1e-5


def test_binary_1024x128_full_size_short(L):
    """The 1024x128 binary workload at its real size, 300 steps, every node."""
    w = I.binary_capillary_1024x128()
    gw = oracle_wall_grad(w)
    gpu, _ = gpu_run(L, w, 300)
    orc, _ = run_oracle(w, 300)
    drho, dphi, du = field_errors(w, gpu, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6
    assert abs(gw - (-0.236834)) < 1e-5


def test_binary_4096x256_properties(L):
    """The 4096x256 throughput lattice at its real size: conservation of mass
    and order parameter, bounded phi, liquid entering the tube (no oracle run
    at this size)."""
    w = I.binary_capillary_4096x256()
    p = L.params_from_workload(w)
    lat = L.Lattice(p, L.geometry_from_workload(w), w.initial_field())
    rho0, _, _, phi0 = lat.moments()
    g = w.geom
    tube = np.zeros_like(phi0, dtype=bool)
    tube[g.y0:g.y0 + g.tube_h, g.x_in:g.x_in + g.tube_len] = True
    liquid0 = phi0[tube].sum()
    lat.step(10000)
    lat.check()
    rho, ux, uy, phi = lat.moments()
    fluid = ~g.solid()
    assert abs(rho[fluid].sum() - rho0[fluid].sum()) / rho0[fluid].sum() < 1e-5
    assert abs(phi[fluid].sum() - phi0[fluid].sum()) / np.abs(phi0[fluid]).sum() < 1e-5
    # the wetting walls hold phi above 1 on the wall rows: phi_s^2 = 1 + Omega (Cahn), 1.155 at 60 degrees
    assert np.abs(phi[fluid]).max() < 1.2
    # liquid (phi > 0) has entered the hydrophilic tube
    assert phi[tube].sum() - liquid0 > 100.0
    lat.close()


# ---- determinism, checkpoints, batches -------------------------------------------
def test_bitwise_determinism_and_launch_shape_independence(L):
    w = small_binary(nx=200, ny=48, H=16)
    a, _ = gpu_run(L, w, 200, cfg=SHAPES[0])
    b, _ = gpu_run(L, w, 200, cfg=SHAPES[0])
    c, _ = gpu_run(L, w, 200, cfg=SHAPES[2])
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    # row-sweep strips: the chunking of the rows does not change any node's arithmetic
    d, _ = gpu_run(L, w, 200, cfg=SHAPES[4])
    e, _ = gpu_run(L, w, 200, cfg=dict(schedule=3, chunk_rows=16, fp64_arith=1))
    for x, y in zip(d, e):
        assert np.array_equal(x, y)
    # workgroup-wide strips: bitwise independent of their chunking, and the
    # one-wavefront strips' values up to the rounding of differently compiled
    # (contracted) arithmetic
    f, _ = gpu_run(L, w, 200, cfg=dict(schedule=4, chunk_rows=0, fp64_arith=1))
    h, _ = gpu_run(L, w, 200, cfg=dict(schedule=4, chunk_rows=12, fp64_arith=1))
    for x, y, z in zip(d, f, h):
        assert np.array_equal(y, z)
        assert float(np.abs(x - y).max()) <= 1e-6


@pytest.mark.parametrize("schedule", [3, 4])
@pytest.mark.parametrize("model", ["vdw", "binary"])
def test_row_sweeps_do_not_depend_on_the_chunking(L, model, schedule):
    """Chunks of 0 (whole columns), 5, 7, 12 and 20 rows give bitwise the same
    fields: every chunk starts in step with the kernels' unrolled row loops."""
    g = I.Geometry(nx=300, ny=61, x_in=120, tube_len=180, tube_h=23, y0=19)
    if model == "vdw":
        w = I.Workload("vdw_chunks", "vdw", g, 0, 0, seed=51, nu_l=0.13, nu_g=0.13, wall_grad=-0.1,
                       liquid=4.5, gas=2.6, **I.VDW_CONSTS)
    else:
        nl, ng = I.viscosity_pair(10.0)
        w = I.Workload("bin_chunks", "binary", g, 0, 0, seed=52, nu_l=nl, nu_g=ng, theta_deg=50.0,
                       liquid=1.0, gas=-1.0, **I.BIN_CONSTS)
    ref, _ = gpu_run(L, w, 60, cfg=dict(schedule=schedule, chunk_rows=0, fp64_arith=1))
    for ch in (5, 7, 12, 20):
        got, _ = gpu_run(L, w, 60, cfg=dict(schedule=schedule, chunk_rows=ch, fp64_arith=1))
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), (model, schedule, ch)


@pytest.mark.parametrize("cfg", [None, dict(schedule=5, chunk_rows=16)], ids=["default", "two_steps_per_sweep"])
def test_checkpoint_resume_is_bitwise(L, cfg):
    """A checkpoint taken after 120 steps, resumed elsewhere, ends bitwise
    where the run without it ends (the same stepping calls: with two steps per
    sweep each call of the binary model ends with a single step)."""
    w = small_binary(nx=200, ny=48, H=16)
    p = L.params_from_workload(w, wall_grad=oracle_wall_grad(w))
    g = L.geometry_from_workload(w)
    ref = L.Lattice(p, g, w.initial_field())
    if cfg:
        ref.set_launch_config(**cfg)
    ref.step(120)
    ref.step(180)
    full = ref.moments()
    lat = L.Lattice(p, g, w.initial_field())
    if cfg:
        lat.set_launch_config(**cfg)
    lat.step(120)
    blob = lat.save()
    lat.step(77)                     # wander off, then come back
    lat.load(blob)
    assert lat.t == 120
    lat.step(180)
    for x, y in zip(full, lat.moments()):
        assert np.array_equal(x, y)
    other = L.Lattice(p, L.make_geometry(210, 48, 100, 110, 16, 16), I.initial_field(
        I.Geometry(210, 48, 100, 110, 16, 16), 1.0, -1.0, 0.5, 3))
    with pytest.raises(L.LbError):
        other.load(blob)


@pytest.mark.parametrize("cfg", [dict(schedule=4, chunk_rows=8), None], ids=["populations", "default"])
def test_batch_equals_single_runs_and_oracle(L, cfg):
    """Uneven capillaries advanced together give bitwise the single-run result."""
    ws = [I.sweep_capillary(77, k, steps=0) for k in range(3)]
    # shrink the draws so the oracle stays fast
    ws = [I.Workload(w.name, w.model, I.Geometry(nx=96 + w.geom.tube_h * 2, ny=w.geom.tube_h + 12, x_in=96,
                                                  tube_len=w.geom.tube_h * 2, tube_h=w.geom.tube_h, y0=6),
                     0, 0, w.seed, nu_l=w.nu_l, nu_g=w.nu_g, theta_deg=w.theta_deg, liquid=1.0, gas=-1.0,
                     **I.BIN_CONSTS) for w in ws]
    P = [L.params_from_workload(w, wall_grad=oracle_wall_grad(w)) for w in ws]
    G = [L.geometry_from_workload(w) for w in ws]
    Q = [w.initial_field() for w in ws]
    batch = L.Lattice(P, G, Q)
    if cfg is not None:
        batch.set_launch_config(**cfg)
    batch.step(250, sample_every=50)
    for k, w in enumerate(ws):
        single = L.Lattice(P[k], G[k], Q[k])
        if cfg is not None:
            single.set_launch_config(**cfg)
        single.step(250)
        for x, y in zip(batch.moments(k), single.moments()):
            assert np.array_equal(x, y)
        orc, lo = run_oracle(w, 250, sample_every=50)
        drho, dphi, du = field_errors(w, batch.moments(k), orc)
        assert drho < 2e-5 and dphi < 2e-5
        steps, hist = batch.l_history(k)
        assert list(steps) == [50, 100, 150, 200, 250]
        assert np.abs(hist - lo).max() < 0.05
    batch.close()


def test_retire_freezes_and_revive_resumes(L):
    """Population storage (the moment storage's own test is in
    test_gpu_moment_storage.py)."""
    S4 = dict(schedule=4, chunk_rows=8)
    ws = [small_binary(nx=160, ny=40, H=12, seed=s) for s in (31, 32)]
    P = [L.params_from_workload(w, wall_grad=oracle_wall_grad(w)) for w in ws]
    G = [L.geometry_from_workload(w) for w in ws]
    Q = [w.initial_field() for w in ws]
    b = L.Lattice(P, G, Q)
    b.set_launch_config(**S4)
    b.step(101)
    frozen = b.moments(1)
    b.retire(1)
    b.step(51)
    for x, y in zip(frozen, b.moments(1)):
        assert np.array_equal(x, y)
    b.revive(1)
    b.step(99)
    ref = L.Lattice(P[1], G[1], Q[1])
    ref.set_launch_config(**S4)
    ref.step(200)
    for x, y in zip(ref.moments(), b.moments(1)):
        assert np.array_equal(x, y)
    ref0 = L.Lattice(P[0], G[0], Q[0])
    ref0.set_launch_config(**S4)
    ref0.step(251)
    for x, y in zip(ref0.moments(), b.moments(0)):
        assert np.array_equal(x, y)


def test_instability_is_reported(L):
    """Density driven through the van der Waals pole: lb_check reports
    LB_EUNSTABLE, as the oracle reports ORC_EUNSTABLE on the same input."""
    g = I.Geometry(nx=16, ny=8)
    q = np.full((8, 16), 3.0)
    q[:, :8] = 10.4
    p = L.make_params("vdw", kappa=0.02, nu_l=0.01)
    lat = L.Lattice(p, L.make_geometry(16, 8), q)
    lat.step(200)
    with pytest.raises(L.LbError) as e:
        lat.check()
    assert e.value.code == L.LB_EUNSTABLE


def test_autotune_keeps_state(L):
    w = small_binary(nx=300, ny=64, H=24)
    p = L.params_from_workload(w, wall_grad=oracle_wall_grad(w))
    g = L.geometry_from_workload(w)
    a = L.Lattice(p, g, w.initial_field())
    cfg0 = a.launch_config()
    a.step(40)
    cfg, us = a.autotune(trial_steps=6)
    assert cfg.schedule in (0, 1, 2, 3, 4, 6) and us > 0
    assert a.t == 40
    a.step(60)
    # a new lattice starts from the default shape, and takes the tuned one only
    # when asked: replay a's history
    b = L.Lattice(p, g, w.initial_field())
    assert b.launch_config().asdict() == cfg0.asdict()
    b.step(40)
    assert b.use_tuned_launch_config()
    assert b.launch_config().asdict() == cfg.asdict()
    b.step(60)
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)


def test_results_do_not_depend_on_earlier_tuning(L):
    """Two identical runs give the same bits whatever was tuned in between:
    a tuning run in the other arithmetic on a lattice of the same size class
    leaves the next context at the default shape and arithmetic, and applying
    the tuned shape keeps the context's own arithmetic."""
    w = small_binary(nx=260, ny=56, H=20, seed=61)
    p = L.params_from_workload(w, wall_grad=oracle_wall_grad(w))
    g = L.geometry_from_workload(w)
    first = L.Lattice(p, g, w.initial_field())
    default = first.launch_config().asdict()
    first.step(120)
    ref = first.moments()
    first.close()
    other = L.Lattice(p, g, w.initial_field())
    other.set_launch_config(**dict(default, fp64_arith=1 - default["fp64_arith"]))
    other.autotune(trial_steps=4)
    other.close()
    again = L.Lattice(p, g, w.initial_field())
    assert again.launch_config().asdict() == default
    again.step(120)
    for x, y in zip(ref, again.moments()):
        assert np.array_equal(x, y)
    assert again.use_tuned_launch_config()
    assert again.launch_config().fp64_arith == default["fp64_arith"]
    again.close()


def test_every_strip_chunking_fits_one_capillary(L):
    """Sweep capillary 144 alone (an 11-row tube): with tail chunks a column
    can need one strip more than at the finest chunking. Every row-sweep
    chunking is accepted, and all give bitwise the same fields."""
    w = I.sweep_capillary(4, 144)
    assert w.geom.tube_h == 11
    lat = L.Lattice(L.params_from_workload(w), L.geometry_from_workload(w), w.initial_field())
    for schedule in (3, 4):
        for ch in (0, 4, 6, 8, 12, 16, 32):
            lat.set_launch_config(schedule=schedule, chunk_rows=ch, fp64_arith=1)
        lat.set_launch_config(schedule=4, chunk_rows=12, fp64_arith=1)
    lat.step(20)
    ref = lat.moments()
    lat.close()
    for ch in (16, 32):
        got, _ = gpu_run(L, w, 20, cfg=dict(schedule=4, chunk_rows=ch, fp64_arith=1))
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), ch
    tuned = L.Lattice(L.params_from_workload(w), L.geometry_from_workload(w), w.initial_field())
    cfg, us = tuned.autotune(trial_steps=4)
    assert us > 0
    tuned.close()


def test_moments_device_matches_host(L):
    import torch
    w = small_binary(nx=130, ny=40, H=12)
    lat = L.Lattice(L.params_from_workload(w, wall_grad=oracle_wall_grad(w)), L.geometry_from_workload(w),
                    w.initial_field())
    lat.step(37)
    n = w.geom.nx * w.geom.ny
    bufs = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4)]
    lat.moments_device(*bufs)
    torch.cuda.synchronize()
    host = lat.moments()
    for d, h in zip(bufs, host):
        assert np.array_equal(d.cpu().numpy().reshape(h.shape).astype(np.float64), h)


@pytest.mark.parametrize("cfg", [dict(schedule=4, chunk_rows=12), None], ids=["populations", "moment-storage"])
def test_throughput_runs_follow_the_filling_balance(L, cfg):
    """The six 4096x256 throughput runs (ratios 1, 10, 100 x 30 and 60 degrees)
    at their real size and length (200000 steps), batched: over the second half
    of each run the filling obeys the capillary balance of Eq. 1 and Eq. 3 with
    the drag of the liquid column and of the gas still in the tube,
        (eta_l - eta_g) l^2 / 2 + eta_g Ltot l = c t + d   (eta = nu, rho = 1),
    linear in t (R^2 >= 0.999); at equal viscosities this says l is linear in
    t (Sec. 3.2).  Smaller contact angles fill faster; mass and phi are kept."""
    works = I.throughput_runs()
    P = [L.params_from_workload(w) for w in works]
    lat = L.Lattice(P, [L.geometry_from_workload(w) for w in works], [w.initial_field() for w in works])
    if cfg is not None:
        lat.set_launch_config(**cfg)
    m0 = [lat.moments(k) for k in range(len(works))]
    every, steps = 2000, works[0].steps
    lat.step(steps, sample_every=every)
    lat.check()
    fluid = ~works[0].geom.solid()
    ends = {}
    for k, w in enumerate(works):
        t, le = lat.l_history(k)
        assert len(t) == steps // every
        rho, _, _, phi = lat.moments(k)
        assert abs(rho[fluid].sum() - m0[k][0][fluid].sum()) / m0[k][0][fluid].sum() < 1e-5
        # phi is stored in fixed point on a 2^-29 grid and each step adds its
        # update as a whole number of grid steps.  Stored in FP32 (half an ulp,
        # 6e-8 at |phi| ~ 1) the small updates in the tails of an interface were
        # rounded away, and these runs lost up to 2.7e-4 of their phi; the
        # budget is now 1e-5 for the whole run (the FP64 oracle conserves to
        # 1e-12).
        drift = abs(phi[fluid].sum() - m0[k][3][fluid].sum()) / np.abs(m0[k][3][fluid]).sum()
        print(f"{'moment storage' if cfg is None else 'populations'} run {k}: relative phi drift {drift:.3e}")
        assert drift < 1e-5
        half = t >= steps // 2
        Ltot = w.geom.tube_len + 0.5 * w.geom.tube_h
        q = 0.5 * (w.nu_l - w.nu_g) * le[half] ** 2 + w.nu_g * Ltot * le[half]
        A = np.stack([t[half], np.ones(half.sum())], axis=1)
        coef, res, *_ = np.linalg.lstsq(A, q, rcond=None)
        r2 = 1.0 - res[0] / np.sum((q - q.mean()) ** 2)
        assert coef[0] > 0 and r2 >= 0.999, (w.ratio, w.theta_deg, r2)
        ends[(round(w.ratio), w.theta_deg)] = le[-1]
    for r in (1, 10, 100):
        assert ends[(r, 30.0)] > ends[(r, 60.0)]
    lat.close()


def test_graph_replays_equal_direct_launches(L):
    """The step run from HIP graphs (64 steps per replay, several replays with
    host reads and direct launches in between) is bitwise the step launched
    directly, for the row-sweep and the tile kernels."""
    w = small_binary(nx=300, ny=64, H=24)
    p = L.params_from_workload(w, wall_grad=oracle_wall_grad(w))
    g = L.geometry_from_workload(w)
    for shape in (dict(schedule=3, chunk_rows=8), dict(schedule=4, chunk_rows=8), dict(tile_rows=4, schedule=1)):
        direct = L.Lattice(p, g, w.initial_field())
        direct.set_launch_config(**shape, graph_steps=0)
        direct.step(300)
        ref = direct.moments()
        direct.close()
        rep = L.Lattice(p, g, w.initial_field())
        rep.set_launch_config(**shape, graph_steps=64)
        for n in (64, 70, 64, 1, 101):        # replays, replays plus direct steps, direct steps
            rep.step(n)
            rep.interface_length()
            rep.moments()
        assert rep.t == 300
        for x, y in zip(rep.moments(), ref):
            assert np.array_equal(x, y)
        rep.close()


# ---- two time steps per sweep (schedule 5), van der Waals model -----------------
FUSED_GEOMS = {
    "ragged150x37": I.Geometry(nx=150, ny=37, x_in=53, tube_len=97, tube_h=13, y0=11),
    "wide700x45": I.Geometry(nx=700, ny=45, x_in=250, tube_len=450, tube_h=17, y0=14),
    "ends520x41": I.Geometry(nx=520, ny=41, x_in=150, tube_len=280, tube_h=15, y0=13),
    "periodic5x3": I.Geometry(nx=5, ny=3),
    # one-row walls: the tube's wall rows are neighbours through the periodic y boundary
    "thinwall300x22": I.Geometry(nx=300, ny=22, x_in=100, tube_len=200, tube_h=20, y0=1),
}


@pytest.mark.parametrize("name", list(FUSED_GEOMS))
def test_fused_vdw_equals_single_steps_and_oracle(L, name):
    """Schedule 5 (two steps per sweep, the intermediate step in LDS) against
    single-step wide strips: bitwise equal, whatever the chunking (0, 5, 12, 24
    rows), graphs or direct launches, with an odd step count (the last step a
    single-step launch); and against the oracle."""
    g = FUSED_GEOMS[name]
    w = I.Workload(f"vdw_fused_{name}", "vdw", g, 0, 0, seed=71, nu_l=0.13, nu_g=0.13, wall_grad=-0.1,
                   liquid=4.5, gas=2.6, **I.VDW_CONSTS)
    init = None
    if name == "periodic5x3":
        init = np.array([[4.5, 4.4, 3.0, 2.6, 2.7], [4.5, 4.2, 3.1, 2.6, 2.8], [4.3, 4.5, 2.9, 2.7, 2.6]])
    steps = 201
    print(f"fused vdw {name}: single-step reference", flush=True)
    ref, _ = gpu_run(L, w, steps, cfg=dict(schedule=4, chunk_rows=8, graph_steps=0, fp64_arith=1), init=init)
    for cfg in (dict(schedule=5, chunk_rows=0, graph_steps=64), dict(schedule=5, chunk_rows=5, graph_steps=0),
                dict(schedule=5, chunk_rows=12, graph_steps=2), dict(schedule=5, chunk_rows=24, graph_steps=64)):
        print(f"fused vdw {name}: {cfg}", flush=True)
        got, _ = gpu_run(L, w, steps, cfg=dict(cfg, fp64_arith=1), init=init)
        gap = max(float(np.abs(x - y).max()) for x, y in zip(ref, got))
        assert gap == 0.0, (cfg, gap)
    orc, _ = run_oracle(w, steps, init=init)
    drho, _, du = field_errors(w, ref, orc)
    assert drho < 2e-5 and du < 1e-6, (drho, du)
    got32, _ = gpu_run(L, w, steps, cfg=dict(schedule=5, chunk_rows=12, graph_steps=64, fp64_arith=0), init=init)
    drho, _, du = field_errors(w, got32, orc)
    assert drho < 2e-5 and du < 1e-6, ("fp32", drho, du)


def test_fused_vdw_graph_replays_and_sampling(L):
    """Schedule 5 run from graphs (64 steps = 32 fused launches per replay)
    interleaved with direct launches, odd step counts and host reads, and a
    batch sampled every 25 steps (odd): bitwise the single-step run, and the
    same filled-length history."""
    w = I.vdw_capillary_256x64()
    p = L.params_from_workload(w)
    g = L.geometry_from_workload(w)
    direct = L.Lattice(p, g, w.initial_field())
    direct.set_launch_config(schedule=4, chunk_rows=8, graph_steps=0)
    direct.step(300)
    ref = direct.moments()
    direct.close()
    rep = L.Lattice(p, g, w.initial_field())
    rep.set_launch_config(schedule=5, chunk_rows=12, graph_steps=64)
    for n in (64, 70, 64, 1, 101):
        rep.step(n)
        rep.interface_length()
        rep.moments()
    assert rep.t == 300
    for x, y in zip(rep.moments(), ref):
        assert np.array_equal(x, y)
    rep.close()
    hists = []
    for shape in (dict(schedule=4, chunk_rows=8), dict(schedule=5, chunk_rows=16)):
        b = L.Lattice([p, p], [g, g], [w.initial_field(), w.initial_field()])
        b.set_launch_config(**shape, graph_steps=64)
        b.step(275, sample_every=25)
        hists.append([b.l_history(k) for k in range(2)])
        b.close()
    for (t0, h0), (t1, h1) in zip(*hists):
        assert list(t0) == list(t1) == list(range(25, 276, 25))
        assert np.array_equal(h0, h1)


def test_vdw_capillary_256x64_1e4_steps_fused(L):
    """The liquid-gas 10^4-step gate (256x64, H=20, tau 0.8) with two steps per sweep."""
    w = I.vdw_capillary_256x64()
    gpu, lg = gpu_run(L, w, 10_000, sample_every=500, cfg=dict(schedule=5, chunk_rows=12))
    orc, lo = run_oracle(w, 10_000, sample_every=500)
    drho, _, du = field_errors(w, gpu, orc)
    print(f"vdw fused 1e4: max rel drho {drho:.3e}, max du {du:.3e}, max dl {np.abs(lg - lo).max():.3e}")
    assert drho <= 1e-4
    assert np.abs(lg - lo).max() <= 0.5


# ---- two time steps per sweep, binary model ----------------------------------
@pytest.mark.parametrize("name", list(FUSED_GEOMS))
def test_fused_binary_equals_single_steps_and_oracle(L, name):
    """Schedule 5 for the binary model (two steps per sweep; f*(t) and
    phi(t+1) in LDS, with a halo of four nodes): bitwise the same whatever the
    chunking (0, 5, 12, 24 rows), with graphs or direct launches, in either
    arithmetic; against single-step wide strips to rounding (the same
    arithmetic per step, compiled apart: single nodes differ in the last bit
    after a few steps); against the oracle at the short-run tolerances."""
    g = FUSED_GEOMS[name]
    nl, ng = I.viscosity_pair(30.0)
    wet = dict(theta_deg=45.0) if g.tube_h else dict(wall_grad=0.0)
    w = I.Workload(f"bin_fused_{name}", "binary", g, 0, 0, seed=73, nu_l=nl, nu_g=ng, liquid=1.0, gas=-1.0,
                   **wet, **I.BIN_CONSTS)
    init = None
    if name == "periodic5x3":
        init = np.array([[1.0, 0.8, -0.2, -1.0, -0.9], [0.9, 0.7, 0.1, -0.8, -1.0], [1.0, 0.6, -0.3, -0.9, -0.7]])
    steps = 201
    for arith in (1, 0):
        print(f"fused binary {name}: single-step reference, fp64_arith {arith}", flush=True)
        ref, _ = gpu_run(L, w, steps, cfg=dict(schedule=4, chunk_rows=8, graph_steps=0, fp64_arith=arith), init=init)
        first = None
        for cfg in (dict(schedule=5, chunk_rows=0, graph_steps=64), dict(schedule=5, chunk_rows=5, graph_steps=0),
                    dict(schedule=5, chunk_rows=12, graph_steps=2), dict(schedule=5, chunk_rows=24, graph_steps=64)):
            got, _ = gpu_run(L, w, steps, cfg=dict(cfg, fp64_arith=arith), init=init)
            if first is None:
                first = got
                gap = max(float(np.abs(x - y).max()) for x, y in zip(ref, got))
                print(f"fused binary {name}: fp64_arith {arith}: max |difference| to single steps {gap:.3e}",
                      flush=True)
                assert gap <= 2e-6, (arith, gap)
            else:
                for x, y in zip(first, got):
                    assert np.array_equal(x, y), (cfg, arith)
        orc, _ = run_oracle(w, steps, init=init)
        drho, dphi, du = field_errors(w, first, orc)
        assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (arith, drho, dphi, du)


def test_fused_binary_graph_replays_batch_and_sampling(L):
    """Binary schedule 5 run from graphs interleaved with direct launches, odd
    step counts and host reads: bitwise the same calls made with direct
    launches (every call ends with a single step, so that the read-outs see phi
    of the state's time), and the single-step run to rounding.  A batch of two
    capillaries with one retired for a while: each equals its single run
    bitwise, and the filled lengths sampled every 25 steps agree with those of
    the single-step strips."""
    w = small_binary(nx=200, ny=48, H=16, seed=87)
    p = L.params_from_workload(w)
    g = L.geometry_from_workload(w)
    calls = (64, 70, 64, 1, 101)
    direct = L.Lattice(p, g, w.initial_field())
    direct.set_launch_config(schedule=5, chunk_rows=12, graph_steps=0)
    for n in calls:
        direct.step(n)
    ref = direct.moments()
    direct.close()
    single = L.Lattice(p, g, w.initial_field())
    single.set_launch_config(schedule=4, chunk_rows=8, graph_steps=0)
    single.step(300)
    gap = max(float(np.abs(x - y).max()) for x, y in zip(single.moments(), ref))
    single.close()
    print(f"fused binary 300 steps: max |difference| to single steps {gap:.3e}")
    assert gap <= 2e-6
    rep = L.Lattice(p, g, w.initial_field())
    rep.set_launch_config(schedule=5, chunk_rows=12, graph_steps=64)
    for n in calls:
        rep.step(n)
        rep.interface_length()
        rep.moments()
    assert rep.t == 300
    rep.check()
    for x, y in zip(rep.moments(), ref):
        assert np.array_equal(x, y)
    rep.close()

    ws = [small_binary(nx=160, ny=40, H=12, seed=s) for s in (88, 89)]
    P = [L.params_from_workload(v) for v in ws]
    G = [L.geometry_from_workload(v) for v in ws]
    Q = [v.initial_field() for v in ws]
    F5 = dict(schedule=5, chunk_rows=16, graph_steps=64)
    b = L.Lattice(P, G, Q)
    b.set_launch_config(**F5)
    b.step(101)
    frozen = b.moments(1)
    b.retire(1)
    b.step(51)
    for x, y in zip(frozen, b.moments(1)):
        assert np.array_equal(x, y)
    b.revive(1)
    b.step(99)
    for k, ns in ((0, (101, 51, 99)), (1, (101, 99))):   # the same calls (capillary 1 retired for one)
        single = L.Lattice(P[k], G[k], Q[k])
        single.set_launch_config(**F5)
        for n in ns:
            single.step(n)
        for x, y in zip(single.moments(), b.moments(k)):
            assert np.array_equal(x, y), k
        single.close()
    b.close()
    hists = []
    for shape in (dict(schedule=4, chunk_rows=8), dict(schedule=5, chunk_rows=16)):
        bb = L.Lattice(P, G, Q)
        bb.set_launch_config(**shape, graph_steps=64)
        bb.step(275, sample_every=25)
        hists.append([bb.l_history(k) for k in range(2)])
        bb.close()
    for (t0, h0), (t1, h1) in zip(*hists):
        assert list(t0) == list(t1) == list(range(25, 276, 25))
        assert np.abs(h0 - h1).max() <= 1e-4


def test_fused_binary_storage_switches(L):
    """Switching between the two-step sweep (population storage) and the
    moment storage mid-run converts the state; the result agrees with the
    single-step population storage to rounding."""
    w = small_binary(nx=200, ny=48, H=16, seed=91)
    p = L.params_from_workload(w)
    g = L.geometry_from_workload(w)
    ref = L.Lattice(p, g, w.initial_field())
    ref.set_launch_config(schedule=4, chunk_rows=8, graph_steps=64)
    ref.step(181)
    want = ref.moments()
    ref.close()
    lat = L.Lattice(p, g, w.initial_field())
    for cfg, n in ((dict(schedule=5, chunk_rows=16), 60), (dict(schedule=6, chunk_rows=20), 61),
                   (dict(schedule=5, chunk_rows=12), 60)):
        lat.set_launch_config(**cfg, graph_steps=64)
        lat.step(n)
    assert lat.t == 181
    got = lat.moments()
    lat.check()
    lat.close()
    gap = max(float(np.abs(x - y).max()) for x, y in zip(want, got))
    print(f"fused/moment storage switches: max |difference| {gap:.3e}")
    assert gap <= 2e-6
