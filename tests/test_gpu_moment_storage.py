"""Schedule 6 (binary model): the row sweep over the stored post-collision state
(seven moment planes instead of nine populations).

The state of a node after the collision of Appendix A is fixed by seven numbers,
so storing them instead of the populations changes only where the populations
are rounded to FP32 (after the rebuild instead of before the store).  Against
the oracle at the tolerances of the population storage; against the population
storage to rounding; bitwise across chunkings, graphs and checkpoints of its own
storage; storage switches and checkpoints of the other storage converted.
"""
import numpy as np
import pytest

from paper_0911_0459_amd import inputs as I
from tests.helpers import field_errors, oracle_wall_grad, run_oracle
from tests.test_gpu_parity import FUSED_GEOMS, gpu_run, small_binary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_0459_amd import lbcap
    return lbcap


INIT_5X3 = np.array([[1.0, 0.8, -0.2, -1.0, -0.9], [0.9, 0.7, 0.1, -0.8, -1.0], [1.0, 0.6, -0.3, -0.9, -0.7]])


def _binary(name, g, seed):
    nl, ng = I.viscosity_pair(30.0)
    wet = dict(theta_deg=45.0) if g.tube_h else dict(wall_grad=0.0)
    return I.Workload(f"bin_mstore_{name}", "binary", g, 0, 0, seed=seed, nu_l=nl, nu_g=ng, liquid=1.0, gas=-1.0,
                      **wet, **I.BIN_CONSTS)


def _gap(a, b):
    return max(float(np.abs(x - y).max()) for x, y in zip(a, b))


@pytest.mark.parametrize("name", list(FUSED_GEOMS))
def test_moment_storage_equals_population_storage_and_oracle(L, name):
    """Ragged 150x37, four strips of 700x45, a tube that ends inside the
    lattice (520x41) and the fully periodic 5x3: bitwise the same whatever the
    chunking (0, 5, 12, 16 rows) and with graphs or direct launches; within
    the short-run tolerances of the oracle; the population storage to
    rounding.  FP32 arithmetic against the oracle too."""
    g = FUSED_GEOMS[name]
    w = _binary(name, g, seed=81)
    init = INIT_5X3 if name == "periodic5x3" else None
    steps = 201
    print(f"moment storage {name}: population storage", flush=True)
    ref, _ = gpu_run(L, w, steps, cfg=dict(schedule=4, chunk_rows=8, graph_steps=0, fp64_arith=1), init=init)
    first = None
    for cfg in (dict(schedule=6, chunk_rows=0, graph_steps=64), dict(schedule=6, chunk_rows=5, graph_steps=0),
                dict(schedule=6, chunk_rows=12, graph_steps=2), dict(schedule=6, chunk_rows=16, graph_steps=64)):
        print(f"moment storage {name}: {cfg}", flush=True)
        got, _ = gpu_run(L, w, steps, cfg=dict(cfg, fp64_arith=1), init=init)
        if first is None:
            first = got
        else:
            assert _gap(first, got) == 0.0, cfg
    gap = _gap(ref, first)
    print(f"moment storage {name}: max |difference| to the population storage {gap:.3e}")
    assert gap <= 2e-6
    orc, _ = run_oracle(w, steps, init=init)
    drho, dphi, du = field_errors(w, first, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (drho, dphi, du)
    got32, _ = gpu_run(L, w, steps, cfg=dict(schedule=6, chunk_rows=12, graph_steps=64, fp64_arith=0), init=init)
    drho, dphi, du = field_errors(w, got32, orc)
    assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, ("fp32", drho, dphi, du)


def test_storage_switches_and_checkpoints(L):
    """Switching the storage mid-run (populations -> state -> populations)
    converts it in place; a checkpoint of either storage resumes in either:
    bitwise in its own, to rounding in the other."""
    w = small_binary(nx=200, ny=48, H=16, seed=83)
    p = L.params_from_workload(w, wall_grad=oracle_wall_grad(w))
    g = L.geometry_from_workload(w)
    S4 = dict(schedule=4, chunk_rows=8, graph_steps=64, fp64_arith=1)
    S6 = dict(schedule=6, chunk_rows=12, graph_steps=64, fp64_arith=1)

    def lattice(cfg):
        lat = L.Lattice(p, g, w.initial_field())
        lat.set_launch_config(**cfg)
        return lat

    pop = lattice(S4)
    pop.step(120)
    blob4 = pop.save()
    pop.step(61)
    ref4 = pop.moments()
    pop.close()
    mom = lattice(S6)
    mom.step(120)
    blob6 = mom.save()
    mom.step(61)
    ref6 = mom.moments()
    mom.check()
    mom.close()
    gap = _gap(ref4, ref6)
    print(f"storages after 181 steps: max |difference| {gap:.3e}")
    assert gap <= 2e-6

    mixed = lattice(S4)
    mixed.step(60)
    mixed.set_launch_config(**S6)
    mixed.step(60)
    mixed.set_launch_config(**S4)
    mixed.step(61)
    assert _gap(mixed.moments(), ref4) <= 2e-6
    mixed.close()

    for cfg, blob, ref, exact in ((S6, blob6, ref6, True), (S4, blob6, ref4, False),
                                  (S6, blob4, ref6, False), (S4, blob4, ref4, True)):
        lat = lattice(cfg)
        lat.step(33)                     # elsewhere, then back
        lat.load(blob)
        assert lat.t == 120
        lat.step(61)
        got = lat.moments()
        lat.close()
        if exact:
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), (cfg["schedule"], "own storage")
        else:
            assert _gap(got, ref) <= 2e-6, (cfg["schedule"], "other storage")


def test_moment_storage_batch_retire_revive_and_sampling(L):
    """A batch in schedule 6: a retired capillary stays frozen, revived it
    resumes, and each capillary equals its single run bitwise; the filled
    length sampled every 25 steps matches the population storage's."""
    ws = [small_binary(nx=160, ny=40, H=12, seed=s) for s in (85, 86)]
    P = [L.params_from_workload(w, wall_grad=oracle_wall_grad(w)) for w in ws]
    G = [L.geometry_from_workload(w) for w in ws]
    Q = [w.initial_field() for w in ws]
    S6 = dict(schedule=6, chunk_rows=8, graph_steps=64, fp64_arith=1)
    b = L.Lattice(P, G, Q)
    b.set_launch_config(**S6)
    b.step(101)
    frozen = b.moments(1)
    b.retire(1)
    b.step(51)
    for x, y in zip(frozen, b.moments(1)):
        assert np.array_equal(x, y)
    b.revive(1)
    b.step(99)
    for k, n in ((0, 251), (1, 200)):
        single = L.Lattice(P[k], G[k], Q[k])
        single.set_launch_config(**S6)
        single.step(n)
        for x, y in zip(single.moments(), b.moments(k)):
            assert np.array_equal(x, y), k
        single.close()
    b.close()
    hists = []
    for shape in (dict(schedule=4, chunk_rows=8), dict(schedule=6, chunk_rows=12)):
        bb = L.Lattice(P, G, Q)
        bb.set_launch_config(**shape, graph_steps=64)
        bb.step(275, sample_every=25)
        hists.append([bb.l_history(k) for k in range(2)])
        bb.close()
    for (t0, h0), (t1, h1) in zip(*hists):
        assert list(t0) == list(t1) == list(range(25, 276, 25))
        assert np.abs(h0 - h1).max() <= 1e-4


def test_every_moment_storage_chunking_fits_one_capillary(L):
    """Sweep capillary 144 alone (an 11-row tube): every chunking of schedule 6
    is accepted and gives bitwise the same fields."""
    w = I.sweep_capillary(4, 144)
    ref, _ = gpu_run(L, w, 20, cfg=dict(schedule=6, chunk_rows=0, fp64_arith=1))
    for ch in (4, 6, 8, 12, 16, 32):
        got, _ = gpu_run(L, w, 20, cfg=dict(schedule=6, chunk_rows=ch, fp64_arith=1))
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), ch


def test_moment_storage_is_refused_for_the_vdw_model(L):
    w = I.vdw_capillary_256x64()
    lat = L.Lattice(L.params_from_workload(w), L.geometry_from_workload(w), w.initial_field())
    with pytest.raises(L.LbError) as e:
        lat.set_launch_config(schedule=6, chunk_rows=8)
    assert e.value.code == L.LB_EINVAL
    assert lat.launch_config().schedule == 4
    lat.close()


@pytest.mark.parametrize("shape", [dict(schedule=6, chunk_rows=16), dict(schedule=5, chunk_rows=48)],
                         ids=["moment_storage", "two_steps_per_sweep"])
def test_full_sweep_in_the_bench_shape_matches_oracle_on_sampled_capillaries(L, shape):
    """The benchmark's workload at its full size (the 256 uneven capillaries of
    the sweep, 32.95 M fluid nodes) in the launch shape the bench times
    (moment storage, chunks of 16 rows as tuned there, 64-step graphs; other
    chunkings give bitwise the same fields) and in the two-step sweep the
    autotuner also tries there, sampled: after 400 steps the two
    smallest capillaries, a middle one and the largest agree with the oracle
    run on each alone, at the short-run tolerances, and their filled lengths,
    sampled every 100 steps, within 0.05."""
    ws = I.sweep_batch(4, 256)
    lat = L.Lattice([L.params_from_workload(w) for w in ws], [L.geometry_from_workload(w) for w in ws],
                    [w.initial_field() for w in ws])
    lat.set_launch_config(**shape, graph_steps=64)
    lat.step(400, sample_every=100)
    lat.check()
    fluid = [int((~w.geom.solid()).sum()) for w in ws]
    order = np.argsort(fluid)
    picks = [int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1])]
    for k in picks:
        w = ws[k]
        print(f"sweep capillary {k}: {w.geom.nx}x{w.geom.ny}, H {w.geom.tube_h}, {fluid[k]} fluid nodes", flush=True)
        orc, lo = run_oracle(w, 400, sample_every=100)
        drho, dphi, du = field_errors(w, lat.moments(k), orc)
        steps, lg = lat.l_history(k)
        assert list(steps) == [100, 200, 300, 400]
        assert drho < 2e-5 and dphi < 2e-5 and du < 1e-6, (k, drho, dphi, du)
        assert np.abs(lg - lo).max() < 0.05, (k, lg, lo)
    lat.close()
