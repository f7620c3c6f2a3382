"""MI355X-native cumulant lattice Boltzmann solver and Fourier neural
operator surrogate (gfx950 HIP kernels behind a C ABI, include/mi355lbm.h).

The HIP library must be built (``python -m paper_2606_16765_amd.build``);
there is no CPU fallback.
"""
from .lbm import Lbm, nu_from_re, bytes_per_cell_update, STORAGE  # noqa: F401

__all__ = ["Lbm", "nu_from_re", "bytes_per_cell_update", "STORAGE"]
from .fno import Fno, FnoError  # noqa: F401,E402

__all__ += ["Fno", "FnoError"]
from .unet import Unet, UnetError  # noqa: F401,E402

__all__ += ["Unet", "UnetError"]
