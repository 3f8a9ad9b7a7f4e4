"""MI355X (gfx950) alternating-direction isogeometric wave solver.

The compute path is the HIP library ``lib/libads.so`` (sources in ``csrc/``,
C-ABI in ``include/ads.h``).  This package only marshals arguments to it:
PyTorch provides device memory and streams.  Build with
``python -m paper_1911_08158_amd.build``.
"""
from .binding import AdsError, Params, Pool, PooledSim, Sim, lib_path, load_library, quad_points  # noqa: F401
