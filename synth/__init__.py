"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds no arithmetic of the method itself: it only builds the
inputs that both sides consume (grid sizes, time step, transducer voxels,
region-of-interest masks, sound-speed phantoms, source pulses).  Everything is
drawn from numpy's PCG64 with an explicit seed so that both sides see
identical arrays.

Stand-ins for the paper's data (Sec. 4.1): the OA-Breast MRI phantom and the
PAMMOTH scanner geometry are not available, so seeded breast-like phantoms and
a golden-section hemispherical bowl with the paper's value ranges replace them.
"""

from .configs import (  # noqa: F401
    Problem,
    make_config,
    make_small,
    random_traces,
    CONFIG_NAMES,
)
