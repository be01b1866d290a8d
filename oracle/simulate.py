"""The simulator's map, end to end, in FP64 (test infrastructure only).

The 3-D Fourier method of Sec. II D 1 with the definitions of ``noise``, ``field`` and
``gather``: realisation b of a plan uses seed + b; its map is the interpolated inverse DFT
of the weighted half grid, sampled at c + r n for every pixel direction n.
"""
import numpy as np

from . import field as _field
from . import gather as _gather
from . import noise as _noise


def simulate(N, L, seed, r, dirs, k_tab, p_tab, interp, noise_dtype=np.float64, workers=None):
    """(map, field) for one realisation. ``noise_dtype`` is the precision the modes are
    rounded to (the GPU path's working precision); everything after is FP64."""
    h = _noise.halfgrid(N, L, seed, k_tab, p_tab, dtype=noise_dtype)
    fld = _field.field(h, workers=workers)
    return _gather.gather(fld, L, r, dirs, interp), fld
