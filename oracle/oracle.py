"""ctypes binding of the FP64 oracle (``lb_oracle.c``).

TEST INFRASTRUCTURE ONLY: see the package docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB = os.path.join(_HERE, "liblb_oracle.so")


def lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP rows)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("model", C.c_int), ("kappa", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("T", C.c_double), ("A", C.c_double),
                ("B", C.c_double), ("Gamma", C.c_double), ("nu_l", C.c_double),
                ("nu_g", C.c_double), ("wall_grad", C.c_double), ("force_x", C.c_double),
                ("lambda_mode", C.c_int)]


class _Geom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x_in", C.c_int), ("tube_len", C.c_int),
                ("tube_h", C.c_int), ("y0", C.c_int)]


@dataclass
class OracleParams:
    model: str = "vdw"          # "vdw" or "binary"
    kappa: float = 0.02
    a: float = 9.0 / 49.0
    b: float = 2.0 / 21.0
    T: float = 0.56
    A: float = 0.04
    B: float = 0.04
    Gamma: float = 1.0
    nu_l: float = 0.1
    nu_g: float = 0.1
    wall_grad: float = 0.0
    force_x: float = 0.0
    lambda_mode: int = 0

    def c(self) -> _Params:
        return _Params(0 if self.model == "vdw" else 1, self.kappa, self.a, self.b, self.T,
                       self.A, self.B, self.Gamma, self.nu_l, self.nu_g, self.wall_grad,
                       self.force_x, self.lambda_mode)


@dataclass
class OracleGeom:
    nx: int
    ny: int
    x_in: int = 0
    tube_len: int = 0
    tube_h: int = 0
    y0: int = 0

    def c(self) -> _Geom:
        return _Geom(self.nx, self.ny, self.x_in, self.tube_len, self.tube_h, self.y0)


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle(force=False)
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    lib.orc_error.restype = C.c_char_p
    lib.orc_threads.restype = C.c_int
    lib.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(_Geom), dp, C.POINTER(C.c_void_p)]
    lib.orc_create.restype = C.c_int
    lib.orc_create_flow.argtypes = [C.POINTER(_Params), C.POINTER(_Geom), dp, dp, dp, C.POINTER(C.c_void_p)]
    lib.orc_create_flow.restype = C.c_int
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_step.argtypes = [C.c_void_p, C.c_long]
    lib.orc_step.restype = C.c_int
    lib.orc_time.argtypes = [C.c_void_p]
    lib.orc_time.restype = C.c_long
    lib.orc_set_wall_gradient.argtypes = [C.c_void_p, C.c_double]
    lib.orc_set_wall_gradient.restype = C.c_int
    lib.orc_moments.argtypes = [C.c_void_p, dp, dp, dp, dp]
    lib.orc_get_pop.argtypes = [C.c_void_p, C.c_int, dp]
    lib.orc_interface_length.argtypes = [C.c_void_p, C.c_double, dp, dp]
    lib.orc_interface_length.restype = C.c_int
    lib.orc_matrix_M.argtypes = [dp]
    lib.orc_matrix_Minv.argtypes = [dp]
    lib.orc_solid_mask.argtypes = [C.POINTER(_Geom), C.POINTER(C.c_ubyte)]
    lib.orc_gradients.argtypes = [C.POINTER(_Geom), C.c_double, dp, dp, dp, dp]
    lib.orc_gradients.restype = C.c_int
    lib.orc_feq.argtypes = [C.POINTER(_Params)] + [C.c_double] * 7 + [dp]
    lib.orc_geq.argtypes = [C.POINTER(_Params)] + [C.c_double] * 4 + [dp]
    lib.orc_collide.argtypes = [C.POINTER(_Params), dp, dp] + [C.c_double] * 5 + [dp]
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc: int):
    if rc != 0:
        raise OracleError(rc, _load().orc_error().decode())


def threads() -> int:
    """OpenMP threads used by the oracle's row loops."""
    return int(_load().orc_threads())


def matrix_M() -> np.ndarray:
    out = np.zeros(81)
    _load().orc_matrix_M(_dp(out))
    return out.reshape(9, 9)


def matrix_Minv() -> np.ndarray:
    out = np.zeros(81)
    _load().orc_matrix_Minv(_dp(out))
    return out.reshape(9, 9)


def solid_mask(geom: OracleGeom) -> np.ndarray:
    out = np.zeros(geom.ny * geom.nx, dtype=np.uint8)
    g = geom.c()
    _load().orc_solid_mask(C.byref(g), out.ctypes.data_as(C.POINTER(C.c_ubyte)))
    return out.reshape(geom.ny, geom.nx).astype(bool)


def gradients(geom: OracleGeom, wall_grad: float, q: np.ndarray):
    q = np.ascontiguousarray(q, dtype=np.float64)
    dx, dy, lap = (np.zeros_like(q) for _ in range(3))
    g = geom.c()
    _check(_load().orc_gradients(C.byref(g), wall_grad, _dp(q), _dp(dx), _dp(dy), _dp(lap)))
    return dx, dy, lap


def feq(p: OracleParams, rho, ux, uy, omega, X, dxq, dyq) -> np.ndarray:
    out = np.zeros(9)
    pc = p.c()
    _load().orc_feq(C.byref(pc), rho, ux, uy, omega, X, dxq, dyq, _dp(out))
    return out


def geq(p: OracleParams, phi, ux, uy, mu) -> np.ndarray:
    out = np.zeros(9)
    pc = p.c()
    _load().orc_geq(C.byref(pc), phi, ux, uy, mu, _dp(out))
    return out


def collide(p: OracleParams, f, fe, omega, ux, uy, Fx=0.0, Fy=0.0) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    fe = np.ascontiguousarray(fe, dtype=np.float64)
    out = np.zeros(9)
    pc = p.c()
    _load().orc_collide(C.byref(pc), _dp(f), _dp(fe), omega, ux, uy, Fx, Fy, _dp(out))
    return out


class Oracle:
    """One lattice advanced by the FP64 oracle."""

    def __init__(self, params: OracleParams, geom: OracleGeom, init_q: np.ndarray, init_u=None):
        """init_q: rho (vdW) or phi (binary), (ny, nx); init_u: optional (ux, uy)
        initial velocity, each (ny, nx) or a scalar (uniform); default at rest."""
        self.params, self.geom = params, geom
        n = geom.ny * geom.nx
        q = np.ascontiguousarray(init_q, dtype=np.float64).reshape(n)
        self._p, self._g = params.c(), geom.c()
        h = C.c_void_p()
        if init_u is None:
            _check(_load().orc_create(C.byref(self._p), C.byref(self._g), _dp(q), C.byref(h)))
        else:
            ux, uy = (np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (geom.ny, geom.nx)))
                      .reshape(n) for v in init_u)
            _check(_load().orc_create_flow(C.byref(self._p), C.byref(self._g), _dp(q), _dp(ux), _dp(uy),
                                           C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _load().orc_free(h)
            self._h = None

    @property
    def t(self) -> int:
        return int(_load().orc_time(self._h))

    def step(self, n: int):
        _check(_load().orc_step(self._h, int(n)))

    def set_wall_gradient(self, wall_grad: float):
        """Wall gradient for the following steps (the scan of Sec. 2.2, Fig. 2)."""
        _check(_load().orc_set_wall_gradient(self._h, float(wall_grad)))
        self.params.wall_grad = float(wall_grad)

    def moments(self):
        n = self.geom.nx * self.geom.ny
        rho, ux, uy, phi = (np.zeros(n) for _ in range(4))
        _load().orc_moments(self._h, _dp(rho), _dp(ux), _dp(uy), _dp(phi))
        shp = (self.geom.ny, self.geom.nx)
        return rho.reshape(shp), ux.reshape(shp), uy.reshape(shp), phi.reshape(shp)

    def populations(self, which: str = "f") -> np.ndarray:
        out = np.zeros(9 * self.geom.nx * self.geom.ny)
        _load().orc_get_pop(self._h, 0 if which == "f" else 1, _dp(out))
        return out.reshape(9, self.geom.ny, self.geom.nx)

    def interface_length(self, q_mid: float):
        l, le = C.c_double(), C.c_double()
        _check(_load().orc_interface_length(self._h, q_mid, C.byref(l), C.byref(le)))
        return l.value, le.value
