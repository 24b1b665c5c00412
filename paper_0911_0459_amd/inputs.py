"""Seeded synthetic inputs shared by the GPU path, its tests and the benchmark.

This module holds no lattice Boltzmann arithmetic.  It draws random numbers
with SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used counter-style so that node (x, y) of a lattice
with seed s always receives the same number, and it lays out the workloads:
lattice sizes, tube placement, model constants and the sharp liquid/gas
initial field with +-1e-3 noise.

Geometry convention (shared with the C-ABI ``lb_geometry``): x is the tube
axis and is periodic; the tube occupies columns [x_in, x_in + tube_len) with
fluid rows [y0, y0 + tube_h) and solid rows above and below; every other node
is reservoir, periodic in y.  The initial field puts liquid in the reservoir
half next to the tube inlet and gas in the half that touches the tube outlet
through the periodic x wrap, and gas in the tube (filled length 0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def splitmix64(seed: int, idx) -> np.ndarray:
    """Output number idx+1 of a SplitMix64 stream started at state ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK) + (idx + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, idx) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    return (splitmix64(seed, idx) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def node_noise(seed: int, nx: int, ny: int, amp: float = 1e-3) -> np.ndarray:
    """U(-amp, amp) per node, counter y*nx + x."""
    idx = np.arange(nx * ny, dtype=np.uint64)
    return (amp * (2.0 * uniform01(seed, idx) - 1.0)).reshape(ny, nx)


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    x_in: int = 0
    tube_len: int = 0
    tube_h: int = 0
    y0: int = 0

    def solid(self) -> np.ndarray:
        """Boolean (ny, nx) solid mask of this geometry (layout only)."""
        s = np.zeros((self.ny, self.nx), dtype=bool)
        if self.tube_len > 0:
            xs = slice(self.x_in, self.x_in + self.tube_len)
            s[: self.y0, xs] = True
            s[self.y0 + self.tube_h:, xs] = True
        return s

    def fluid_count(self) -> int:
        return int(self.nx * self.ny - self.solid().sum())

    def asdict(self):
        return asdict(self)


@dataclass(frozen=True)
class Workload:
    """One capillary run: model constants, geometry, initial field recipe."""
    name: str
    model: str                 # "vdw" or "binary"
    geom: Geometry
    steps: int
    sample_every: int
    seed: int
    # model constants (paper Sec. 2 and Sec. 3.1 values)
    kappa: float
    a: float = 9.0 / 49.0
    b: float = 2.0 / 21.0
    T: float = 0.56
    A: float = 0.04
    B: float = 0.04
    Gamma: float = 1.0
    nu_l: float = 0.1
    nu_g: float = 0.1
    theta_deg: float = 60.0
    wall_grad: float | None = None   # given directly (vdW at 60 deg) or None = map theta
    liquid: float = 1.0
    gas: float = -1.0
    gas_frac: float = 0.5
    noise: float = 1e-3

    @property
    def ratio(self) -> float:
        return self.nu_l / self.nu_g

    def initial_field(self) -> np.ndarray:
        return initial_field(self.geom, self.liquid, self.gas, self.gas_frac, self.seed, self.noise)


def initial_field(geom: Geometry, liquid: float, gas: float, gas_frac: float, seed: int,
                  amp: float = 1e-3, l0: int = 0) -> np.ndarray:
    """Sharp liquid/gas step plus node noise, shape (ny, nx), y major; with
    l0 > 0 the liquid column already reaches l0 nodes into the tube (the
    paper's capillary starts at l = 10)."""
    q = np.full((geom.ny, geom.nx), gas, dtype=np.float64)
    if geom.tube_len > 0:
        x_gas_end = int(round(gas_frac * geom.x_in))
        q[:, x_gas_end: geom.x_in] = liquid
        if l0 > 0:
            q[geom.y0: geom.y0 + geom.tube_h, geom.x_in: geom.x_in + min(l0, geom.tube_len)] = liquid
    q += node_noise(seed, geom.nx, geom.ny, amp)
    return q


def viscosity_pair(ratio: float, nu0: float = 1.0 / 6.0):
    """(nu_l, nu_g) with nu_l / nu_g = ratio and geometric mean nu0."""
    s = math.sqrt(ratio)
    return nu0 * s, nu0 / s


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
VDW_CONSTS = dict(kappa=0.02, a=9.0 / 49.0, b=2.0 / 21.0, T=0.56)
BIN_CONSTS = dict(kappa=0.04, A=0.04, B=0.04, Gamma=1.0)


def vdw_capillary_256x64(seed: int = 1) -> Workload:
    """Liquid-gas vdW, 256x64, tube H=20 and length 128, tau=0.8 (nu=0.1),
    wall gradient -0.144 (60 degrees), 2000 steps, l sampled every 50."""
    g = Geometry(nx=256, ny=64, x_in=128, tube_len=128, tube_h=20, y0=22)
    return Workload("vdw_256x64", "vdw", g, steps=2000, sample_every=50, seed=seed,
                    nu_l=0.1, nu_g=0.1, theta_deg=60.0, wall_grad=-0.144,
                    liquid=4.54, gas=2.59, **VDW_CONSTS)


def vdw_capillary_4096x256(seed: int = 9) -> Workload:
    """The liquid-gas model at the size of the binary throughput runs: 4096x256,
    tube H=100 and length 3072, the C1 constants (nu = 0.1, -0.144)."""
    g = Geometry(nx=4096, ny=256, x_in=1024, tube_len=3072, tube_h=100, y0=78)
    return Workload("vdw_4096x256", "vdw", g, steps=200_000, sample_every=2000, seed=seed,
                    nu_l=0.1, nu_g=0.1, theta_deg=60.0, wall_grad=-0.144,
                    liquid=4.54, gas=2.59, **VDW_CONSTS)


def vdw_capillary_16384x1024(seed: int = 10) -> Workload:
    """The liquid-gas model on a lattice far larger than the last-level cache:
    16384x1024 (9.1 M fluid nodes), tube H=400 and length 12288, the C1
    constants (nu = 0.1, -0.144)."""
    g = Geometry(nx=16384, ny=1024, x_in=4096, tube_len=12288, tube_h=400, y0=312)
    return Workload("vdw_16384x1024", "vdw", g, steps=200_000, sample_every=2000, seed=seed,
                    nu_l=0.1, nu_g=0.1, theta_deg=60.0, wall_grad=-0.144,
                    liquid=4.54, gas=2.59, **VDW_CONSTS)


def binary_capillary_16384x1024(seed: int = 11, ratio: float = 10.0) -> Workload:
    """One binary capillary far larger than the last-level cache: 16384x1024
    (9.1 M fluid nodes), tube H=400 and length 12288, ratio 10, 60 degrees."""
    g = Geometry(nx=16384, ny=1024, x_in=4096, tube_len=12288, tube_h=400, y0=312)
    nl, ng = viscosity_pair(ratio)
    return Workload("binary_16384x1024", "binary", g, steps=200_000, sample_every=2000, seed=seed,
                    nu_l=nl, nu_g=ng, theta_deg=60.0, liquid=1.0, gas=-1.0, **BIN_CONSTS)


def binary_capillary_1024x128(seed: int = 2, ratio: float = 10.0) -> Workload:
    """Binary, 1024x128, tube H=40 and length 768, reservoir 256 wide,
    viscosity ratio 10, 60 degrees, 50k steps."""
    g = Geometry(nx=1024, ny=128, x_in=256, tube_len=768, tube_h=40, y0=44)
    nl, ng = viscosity_pair(ratio)
    return Workload("binary_1024x128", "binary", g, steps=50_000, sample_every=500, seed=seed,
                    nu_l=nl, nu_g=ng, theta_deg=60.0, liquid=1.0, gas=-1.0, **BIN_CONSTS)


def binary_capillary_4096x256(seed: int = 3, ratio: float = 10.0, theta_deg: float = 60.0) -> Workload:
    """Binary throughput run, 4096x256, tube H=100 and length 3072, 200k steps."""
    g = Geometry(nx=4096, ny=256, x_in=1024, tube_len=3072, tube_h=100, y0=78)
    nl, ng = viscosity_pair(ratio)
    return Workload("binary_4096x256", "binary", g, steps=200_000, sample_every=2000, seed=seed,
                    nu_l=nl, nu_g=ng, theta_deg=theta_deg, liquid=1.0, gas=-1.0, **BIN_CONSTS)


def throughput_runs():
    """Viscosity ratios 1, 10, 100 x contact angles 30, 60: seeds 3..8."""
    out, seed = [], 3
    for r in (1.0, 10.0, 100.0):
        for th in (30.0, 60.0):
            out.append(binary_capillary_4096x256(seed=seed, ratio=r, theta_deg=th))
            seed += 1
    return out


def sweep_capillary(master_seed: int, cap: int, steps: int = 100_000,
                    sample_every: int | None = None) -> Workload:
    """One capillary of the uneven batched sweep: H ~ U{10..80}, tube length
    ~ U[500, 4000], reservoir 256 x (H+40), ratio log-uniform in [1, 100],
    contact angle ~ U[30, 90] degrees; draws from SplitMix64(master, 16 cap + k)."""
    u = uniform01(master_seed, np.arange(16 * cap, 16 * cap + 5, dtype=np.uint64))
    H = 10 + int(u[0] * 71)                      # 10..80
    L = int(round(500.0 + u[1] * 3500.0))        # 500..4000
    ratio = math.exp(u[2] * math.log(100.0))     # 1..100
    theta = 30.0 + 60.0 * float(u[3])            # 30..90
    nseed = int(splitmix64(master_seed, 16 * cap + 15)) & 0x7FFFFFFF
    g = Geometry(nx=256 + L, ny=H + 40, x_in=256, tube_len=L, tube_h=H, y0=20)
    nl, ng = viscosity_pair(ratio)
    if sample_every is None:
        sample_every = max(1, steps // 160)
    return Workload(f"sweep{master_seed}_{cap}", "binary", g, steps=steps, sample_every=sample_every,
                    seed=nseed, nu_l=nl, nu_g=ng, theta_deg=theta, liquid=1.0, gas=-1.0, **BIN_CONSTS)


def sweep_batch(master_seed: int = 4, n: int = 256, steps: int = 100_000):
    return [sweep_capillary(master_seed, c, steps) for c in range(n)]


def surrogate_runs(kind: str = "train", steps: int = 100_000):
    """Training runs use master seeds 1000..5095, held-out runs 9000..9511; each
    run is capillary 0 of its own master seed (the sweep distribution)."""
    seeds = range(1000, 5096) if kind == "train" else range(9000, 9512)
    return [sweep_capillary(s, 0, steps) for s in seeds]
