"""MI355X-native free-energy MRT lattice Boltzmann for capillary filling
(Pooley, Kusumaatmaja & Yeomans, arXiv:0911.0459).

The compute path is liblbcap.so (HIP kernels for gfx950 behind the C ABI of
include/lbcap.h); ``paper_0911_0459_amd.lbcap`` is its ctypes binding and
``paper_0911_0459_amd.inputs`` builds the seeded synthetic workloads.
"""
