"""FP64 CPU oracle of the free-energy MRT lattice Boltzmann scheme
(Pooley, Kusumaatmaja & Yeomans, arXiv:0911.0459).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    OracleError,
    OracleParams,
    OracleGeom,
    Oracle,
    build_oracle,
    lib_path,
    threads,
    matrix_M,
    matrix_Minv,
    solid_mask,
    gradients,
    feq,
    geq,
    collide,
)
from . import mlp_oracle  # noqa: F401,E402
