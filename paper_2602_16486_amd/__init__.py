"""MI355X (gfx950) implementation of the fused stream-and-collide step of the
fluctuating orthogonal-central-moment lattice Boltzmann method (De Rosis &
Zhou, arXiv 2602.16486) for D2Q9, D3Q19 and D3Q27.

The compute path is the HIP library ``libcmflb.so`` (C ABI in
``include/cmflb.h``); this package is its ctypes binding.  Importing the
package does not load the library; creating a :class:`Lattice` does, and fails
loudly when it has not been built.
"""
from ._lib import CmfError, STAT_COLUMNS, load, noise_sample, philox_words, version  # noqa: F401
from .ensemble import Ensemble  # noqa: F401
from .lattice import Lattice, external_bytes, rate_vector  # noqa: F401
