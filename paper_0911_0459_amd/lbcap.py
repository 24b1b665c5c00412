"""Python binding of liblbcap.so (C ABI in include/lbcap.h).

Argument marshalling only: every step of the lattice Boltzmann path and of the
surrogate runs in the library's HIP kernels.  PyTorch supplies device memory
and the stream.  If the library has not been built this module raises at
import time; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
# PyTorch first: the library then binds to the HIP runtime PyTorch already
# loaded (same soname), so both share one runtime and one device context.
import torch  # noqa: F401

from .build import LIB

if not os.path.exists(LIB):
    raise ImportError(f"liblbcap.so not found at {LIB}: build it first: python -m paper_0911_0459_amd.build (hipcc, gfx950)")

_lib = C.CDLL(LIB)

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_ESTATE = 0, -1, -2, -3, -4, -5
LB_VDW, LB_BINARY = 0, 1
LB_HISTORY_CAP = 4096
MLP_NOALLOC_MAX_ROWS = 1024


class LbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbcap error {code}: {msg}")
        self.code = code


class lb_params(C.Structure):
    _fields_ = [("model", C.c_int), ("kappa", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("T", C.c_double), ("A", C.c_double), ("B", C.c_double), ("Gamma", C.c_double),
                ("nu_l", C.c_double), ("nu_g", C.c_double), ("wall_grad", C.c_double),
                ("theta_deg", C.c_double), ("force_x", C.c_double), ("lambda_mode", C.c_int),
                ("q_mid", C.c_double)]


class lb_geometry(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x_in", C.c_int), ("tube_len", C.c_int),
                ("tube_h", C.c_int), ("y0", C.c_int)]


class lb_launch_config(C.Structure):
    _fields_ = [("tile_rows", C.c_int), ("schedule", C.c_int), ("persist_blocks_per_cu", C.c_int),
                ("graph_steps", C.c_int), ("fp64_arith", C.c_int), ("chunk_rows", C.c_int)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _dp, _fp, _ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)

_SIGS = {
    "lb_last_error": (C.c_char_p, []),
    "lb_state_bytes": (C.c_size_t, [C.POINTER(lb_params), C.POINTER(lb_geometry)]),
    "lb_init": (C.c_int, [C.POINTER(_vp), C.POINTER(lb_params), C.POINTER(lb_geometry), _dp, _vp, C.c_size_t, _vp]),
    "lb_step": (C.c_int, [_vp, C.c_long]),
    "lb_time": (C.c_long, [_vp]),
    "lb_check": (C.c_int, [_vp]),
    "lb_moments": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "lb_moments_device": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lb_interface_length": (C.c_int, [_vp, _dp, _dp]),
    "lb_wall_gradient_for_angle": (C.c_int, [C.POINTER(lb_params), C.c_double, _dp]),
    "lb_vdw_coexistence": (C.c_int, [C.POINTER(lb_params), _dp, _dp]),
    "lb_checkpoint_bytes": (C.c_size_t, [_vp]),
    "lb_save": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lb_load": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lb_free": (None, [_vp]),
    "lb_batch_init": (C.c_int, [C.POINTER(_vp), C.c_int, C.POINTER(lb_params), C.POINTER(lb_geometry),
                                C.POINTER(_dp), _vp]),
    "lb_batch_step": (C.c_int, [_vp, C.c_long, C.c_int]),
    "lb_batch_l_history": (C.c_int, [_vp, C.c_int, _dp, _lp, C.c_int, _ip]),
    "lb_batch_retire": (C.c_int, [_vp, C.c_int]),
    "lb_batch_revive": (C.c_int, [_vp, C.c_int]),
    "lb_batch_moments": (C.c_int, [_vp, C.c_int, _dp, _dp, _dp, _dp]),
    "lb_batch_health": (C.c_int, [_vp, _ip]),
    "lb_batch_size": (C.c_int, [_vp]),
    "lb_fluid_nodes": (C.c_longlong, [_vp]),
    "lb_get_launch_config": (C.c_int, [_vp, C.POINTER(lb_launch_config)]),
    "lb_set_launch_config": (C.c_int, [_vp, C.POINTER(lb_launch_config)]),
    "lb_autotune": (C.c_int, [_vp, C.c_int, C.POINTER(lb_launch_config), _dp]),
    "lb_use_tuned_launch_config": (C.c_int, [_vp, _ip]),
    "lb_last_step_kernel_us": (C.c_int, [_vp, _dp]),
    "lb_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "lb_meniscus_angle_field": (C.c_int, [_dp, C.POINTER(lb_geometry), C.c_double, C.c_int, _dp, _dp, _dp]),
    "lb_meniscus_angle": (C.c_int, [_vp, C.c_int, C.c_int, _dp, _dp, _dp]),
    "lb_tube_flow_field": (C.c_int, [_dp, _dp, _dp, C.POINTER(lb_geometry), C.c_double, C.c_int, C.c_double, _dp,
                                     _vp]),
    "lb_tube_flow": (C.c_int, [_vp, C.c_int, C.c_int, C.c_double, _dp, _vp]),
    "lb_washburn_length": (C.c_int, [C.c_double] * 8 + [_dp]),
    "lb_set_wall_gradient": (C.c_int, [_vp, C.c_int, C.c_double]),
    "mlp_init": (C.c_int, [C.POINTER(_vp), C.c_int, _vp]),
    "mlp_free": (None, [_vp]),
    "mlp_param_count": (C.c_long, [_vp]),
    "mlp_get_params": (C.c_int, [_vp, _fp, C.c_long]),
    "mlp_set_params": (C.c_int, [_vp, _fp, C.c_long]),
    "mlp_predict": (C.c_int, [_vp, _fp, C.c_int, _fp]),
    "mlp_predict_device_noalloc": (C.c_int, [_vp, _vp, C.c_int, _vp]),
    "mlp_loss_grad": (C.c_int, [_vp, _fp, _fp, C.c_int, _fp, _fp]),
    "mlp_train": (C.c_int, [_vp, _fp, _fp, C.c_int, C.c_int, C.c_int, C.c_float, C.c_int, _fp]),
}

EXPORTED = tuple(_SIGS)

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc: int):
    if rc != LB_OK:
        raise LbError(rc, _lib.lb_last_error().decode())


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f32(a: np.ndarray):
    return a.ctypes.data_as(_fp)


def _torch_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(model: str, *, kappa: float, a: float = 9 / 49, b: float = 2 / 21, T: float = 0.56,
                A: float = 0.04, B: float = 0.04, Gamma: float = 1.0, nu_l: float = 0.1,
                nu_g: float | None = None, wall_grad: float = 0.0, theta_deg: float | None = None,
                force_x: float = 0.0, lambda_mode: int = 0, q_mid: float | None = None) -> lb_params:
    return lb_params(LB_VDW if model == "vdw" else LB_BINARY, kappa, a, b, T, A, B, Gamma, nu_l,
                     nu_l if nu_g is None else nu_g, wall_grad,
                     math.nan if theta_deg is None else theta_deg, force_x, lambda_mode,
                     math.nan if q_mid is None else q_mid)


def make_geometry(nx, ny, x_in=0, tube_len=0, tube_h=0, y0=0) -> lb_geometry:
    return lb_geometry(nx, ny, x_in, tube_len, tube_h, y0)


def params_from_workload(w, wall_grad: float | None = None) -> lb_params:
    """lb_params of an inputs.Workload; the contact angle goes through the
    library's own wall-gradient map unless a gradient is given."""
    g = w.wall_grad if wall_grad is None else wall_grad
    return make_params(w.model, kappa=w.kappa, a=w.a, b=w.b, T=w.T, A=w.A, B=w.B, Gamma=w.Gamma,
                       nu_l=w.nu_l, nu_g=w.nu_g, wall_grad=0.0 if g is None else g,
                       theta_deg=None if g is not None else w.theta_deg)


def geometry_from_workload(w) -> lb_geometry:
    g = w.geom
    return make_geometry(g.nx, g.ny, g.x_in, g.tube_len, g.tube_h, g.y0)


def lb_wall_gradient_for_angle(p: lb_params, theta_deg: float) -> float:
    out = C.c_double()
    _check(_lib.lb_wall_gradient_for_angle(C.byref(p), theta_deg, C.byref(out)))
    return out.value


def lb_vdw_coexistence(p: lb_params):
    l, g = C.c_double(), C.c_double()
    _check(_lib.lb_vdw_coexistence(C.byref(p), C.byref(l), C.byref(g)))
    return l.value, g.value


def lb_stream_copy(dst, src, stream=None):
    """Copy torch tensor src into dst (same byte size) with the library's copy kernel."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    _check(_lib.lb_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, C.c_void_p(s)))


def lb_meniscus_angle_field(q: np.ndarray, g: lb_geometry, q_mid: float, edge_rows: int = 2):
    """(theta_deg, radius, apex_x) of the meniscus in a host field q (ny x nx)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    if q.size != g.nx * g.ny:
        raise LbError(LB_EINVAL, "field size does not match the geometry")
    th, R, ax = C.c_double(), C.c_double(), C.c_double()
    _check(_lib.lb_meniscus_angle_field(_d(q), C.byref(g), float(q_mid), int(edge_rows), C.byref(th),
                                        C.byref(R), C.byref(ax)))
    return th.value, R.value, ax.value


class lb_tube_flow_stats(C.Structure):
    _fields_ = [("l", C.c_double), ("rho_liquid", C.c_double), ("u_liquid", C.c_double), ("rho_gas", C.c_double),
                ("u_gas", C.c_double), ("condensation_liquid_side", C.c_double),
                ("condensation_gas_side", C.c_double), ("liquid_cols", C.c_int), ("gas_cols", C.c_int)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lb_tube_flow_field(q: np.ndarray, rho: np.ndarray, ux: np.ndarray, g: lb_geometry, q_mid: float,
                       margin: int = 3, v_meniscus: float = 0.0):
    """(lb_tube_flow_stats, centreline u_x over the tube) of host fields (ny x nx)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (q, rho, ux)]
    if any(a.size != g.nx * g.ny for a in arrs):
        raise LbError(LB_EINVAL, "field size does not match the geometry")
    out, line = lb_tube_flow_stats(), np.zeros(max(g.tube_len, 0))
    _check(_lib.lb_tube_flow_field(*[_d(a) for a in arrs], C.byref(g), float(q_mid), int(margin),
                                   float(v_meniscus), _d(line), C.byref(out)))
    return out, line


def lb_washburn_length(t: float, l0: float, H: float, L: float, gamma: float, cos_theta: float, eta_l: float,
                       eta_g: float = 0.0) -> float:
    """Filled length of the capillary balance with liquid and gas drag
    (eta_g = 0: Washburn's law, Eq. 3)."""
    out = C.c_double()
    _check(_lib.lb_washburn_length(float(t), float(l0), float(H), float(L), float(gamma), float(cos_theta),
                                   float(eta_l), float(eta_g), C.byref(out)))
    return out.value


def lb_state_bytes(p: lb_params, g: lb_geometry) -> int:
    return int(_lib.lb_state_bytes(C.byref(p), C.byref(g)))


class Lattice:
    """One capillary or a batch of capillaries advanced on the GPU."""

    def __init__(self, params, geoms, init_q, *, torch_memory: bool = True, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise LbError(LB_EDEVICE, "no GPU visible to PyTorch")
        single = isinstance(params, lb_params)
        self.params = [params] if single else list(params)
        self.geoms = [geoms] if single else list(geoms)
        fields = [init_q] if single else list(init_q)
        self.n = len(self.params)
        self._fields = [np.ascontiguousarray(q, dtype=np.float64).reshape(-1) for q in fields]
        for q, g in zip(self._fields, self.geoms):
            if q.size != g.nx * g.ny:
                raise LbError(LB_EINVAL, "initial field size does not match the geometry")
        if stream is None:
            # a dedicated (default-priority) stream, so that step runs can be
            # captured into HIP graphs
            self._torch_stream = torch.cuda.Stream()
            self._stream = C.c_void_p(self._torch_stream.cuda_stream)
        else:
            self._stream = C.c_void_p(stream)
        h = C.c_void_p()
        self._mem = None
        if single:
            if torch_memory:
                nbytes = lb_state_bytes(self.params[0], self.geoms[0])
                if nbytes == 0:
                    raise LbError(LB_EINVAL, _lib.lb_last_error().decode())
                self._mem = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
                ptr, nb = C.c_void_p(self._mem.data_ptr()), nbytes
            else:
                ptr, nb = None, 0
            _check(_lib.lb_init(C.byref(h), C.byref(self.params[0]), C.byref(self.geoms[0]),
                                _d(self._fields[0]), ptr, nb, self._stream))
        else:
            P = (lb_params * self.n)(*self.params)
            G = (lb_geometry * self.n)(*self.geoms)
            Q = (_dp * self.n)(*[_d(q) for q in self._fields])
            _check(_lib.lb_batch_init(C.byref(h), self.n, P, G, Q, self._stream))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lb_free(self._h)
            self._h = None
        self._mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- time stepping -------------------------------------------------------
    def step(self, n: int, sample_every: int = 0):
        _check(_lib.lb_batch_step(self._h, int(n), int(sample_every)))

    @property
    def t(self) -> int:
        return int(_lib.lb_time(self._h))

    def check(self):
        _check(_lib.lb_check(self._h))

    def health(self) -> np.ndarray:
        flags = np.zeros(self.n, dtype=np.int32)
        rc = _lib.lb_batch_health(self._h, flags.ctypes.data_as(_ip))
        if rc not in (LB_OK, LB_EUNSTABLE):
            _check(rc)
        return flags

    def last_step_kernel_us(self) -> float:
        us = C.c_double()
        _check(_lib.lb_last_step_kernel_us(self._h, C.byref(us)))
        return us.value

    # -- observables -----------------------------------------------------------
    def moments(self, cap: int = 0):
        g = self.geoms[cap]
        out = [np.zeros(g.nx * g.ny) for _ in range(4)]
        _check(_lib.lb_batch_moments(self._h, cap, *[_d(o) for o in out]))
        return tuple(o.reshape(g.ny, g.nx) for o in out)

    def moments_device(self, rho, ux=None, uy=None, phi=None):
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        _check(_lib.lb_moments_device(self._h, ptr(rho), ptr(ux), ptr(uy), ptr(phi)))

    def interface_length(self):
        l, le = C.c_double(), C.c_double()
        _check(_lib.lb_interface_length(self._h, C.byref(l), C.byref(le)))
        return l.value, le.value

    def l_history(self, cap: int = 0):
        buf = np.zeros(LB_HISTORY_CAP)
        steps = np.zeros(LB_HISTORY_CAP, dtype=np.int64)
        n = C.c_int()
        _check(_lib.lb_batch_l_history(self._h, cap, _d(buf), steps.ctypes.data_as(_lp), LB_HISTORY_CAP,
                                       C.byref(n)))
        m = min(n.value, LB_HISTORY_CAP)
        return steps[:m].copy(), buf[:m].copy()

    def meniscus_angle(self, cap: int = 0, edge_rows: int = 2):
        """(theta_deg, radius, apex_x) of capillary cap's meniscus."""
        th, R, ax = C.c_double(), C.c_double(), C.c_double()
        _check(_lib.lb_meniscus_angle(self._h, cap, int(edge_rows), C.byref(th), C.byref(R), C.byref(ax)))
        return th.value, R.value, ax.value

    def tube_flow(self, cap: int = 0, margin: int = 3, v_meniscus: float = 0.0):
        """(lb_tube_flow_stats, centreline u_x over the tube) of capillary cap (Fig. 3)."""
        out = lb_tube_flow_stats()
        line = np.zeros(self.geoms[cap].tube_len)
        _check(_lib.lb_tube_flow(self._h, cap, int(margin), float(v_meniscus), _d(line), C.byref(out)))
        return out, line

    def set_wall_gradient(self, grad: float, cap: int = 0):
        """Wall gradient of capillary cap for the following steps (the
        quasistatic scan of Sec. 2.2, Fig. 2)."""
        _check(_lib.lb_set_wall_gradient(self._h, cap, float(grad)))

    def retire(self, cap: int):
        _check(_lib.lb_batch_retire(self._h, cap))

    def revive(self, cap: int):
        _check(_lib.lb_batch_revive(self._h, cap))

    @property
    def fluid_nodes(self) -> int:
        return int(_lib.lb_fluid_nodes(self._h))

    # -- launch configuration ----------------------------------------------------
    def launch_config(self) -> lb_launch_config:
        cfg = lb_launch_config()
        _check(_lib.lb_get_launch_config(self._h, C.byref(cfg)))
        return cfg

    def set_launch_config(self, tile_rows=4, schedule=4, persist_blocks_per_cu=4, graph_steps=64, fp64_arith=None,
                          chunk_rows=8):
        """fp64_arith None keeps the context's current arithmetic."""
        if fp64_arith is None:
            fp64_arith = self.launch_config().fp64_arith
        cfg = lb_launch_config(tile_rows, schedule, persist_blocks_per_cu, graph_steps, fp64_arith, chunk_rows)
        _check(_lib.lb_set_launch_config(self._h, C.byref(cfg)))

    def autotune(self, trial_steps: int = 20):
        cfg, us = lb_launch_config(), C.c_double()
        _check(_lib.lb_autotune(self._h, trial_steps, C.byref(cfg), C.byref(us)))
        return cfg, us.value

    def use_tuned_launch_config(self) -> bool:
        """Apply the shape last tuned in this process for this model and size
        class (the arithmetic stays); False if there is none."""
        found = C.c_int()
        _check(_lib.lb_use_tuned_launch_config(self._h, C.byref(found)))
        return bool(found.value)

    # -- checkpoints -----------------------------------------------------------------
    def save(self) -> bytes:
        n = int(_lib.lb_checkpoint_bytes(self._h))
        buf = C.create_string_buffer(n)
        _check(_lib.lb_save(self._h, C.cast(buf, C.c_void_p), n))
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(_lib.lb_load(self._h, C.cast(buf, C.c_void_p), len(blob)))


class MLP:
    """The l(t) surrogate network, resident on the GPU."""

    N_IN, N_OUT = 19, 64

    def __init__(self, seed: int = 0, stream=None):
        h = C.c_void_p()
        _check(_lib.mlp_init(C.byref(h), int(seed), _torch_stream() if stream is None else C.c_void_p(stream)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.mlp_free(self._h)
            self._h = None

    @property
    def param_count(self) -> int:
        return int(_lib.mlp_param_count(self._h))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.param_count, dtype=np.float32)
        _check(_lib.mlp_get_params(self._h, _f32(out), out.size))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.mlp_set_params(self._h, _f32(p), p.size))

    def predict(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros((X.shape[0], self.N_OUT), dtype=np.float32)
        _check(_lib.mlp_predict(self._h, _f32(X), X.shape[0], _f32(Y)))
        return Y

    def predict_device_noalloc(self, X, Y) -> None:
        """Forward pass from device tensor X (n x 19, float32, contiguous) into
        device tensor Y (n x 64), n <= MLP_NOALLOC_MAX_ROWS, without any device
        allocation; enqueued on the network's stream, not synchronised."""
        for t, cols in ((X, self.N_IN), (Y, self.N_OUT)):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4 and t.is_contiguous()
                    and t.dim() == 2 and t.shape[1] == cols):
                raise LbError(LB_EINVAL, "X and Y must be contiguous float32 device tensors (n x 19, n x 64)")
        if X.shape[0] != Y.shape[0]:
            raise LbError(LB_EINVAL, "X and Y row counts differ")
        _check(_lib.mlp_predict_device_noalloc(self._h, C.c_void_p(X.data_ptr()), int(X.shape[0]),
                                               C.c_void_p(Y.data_ptr())))

    def loss_grad(self, X: np.ndarray, Y: np.ndarray):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        g = np.zeros(self.param_count, dtype=np.float32)
        loss = C.c_float()
        _check(_lib.mlp_loss_grad(self._h, _f32(X), _f32(Y), X.shape[0], C.byref(loss), _f32(g)))
        return loss.value, g

    def train(self, X, Y, epochs: int, batch: int = 512, lr: float = 1e-3, seed: int = 0) -> float:
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        last = C.c_float()
        _check(_lib.mlp_train(self._h, _f32(X), _f32(Y), X.shape[0], epochs, batch, lr, seed, C.byref(last)))
        return last.value
