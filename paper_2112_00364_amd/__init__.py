"""SMC over PPL control-flow graphs on AMD Instinct MI355X (gfx950).

The data-parallel path of Lunden et al. (ESOP 2022): particles execute a
PCFG's basic blocks (Sec. 3.1) under Algorithm 1 (Sec. 3.2) with systematic
resampling and a log Z estimate (Sec. 3.3). The path runs in hand-written HIP
kernels behind the C interface include/pcfgsmc.h (libpcfgsmc.so); ``smc`` is
its Python binding and ``inputs`` builds seeded synthetic workloads.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "smc", "build"]
