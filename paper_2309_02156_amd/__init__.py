"""MI355X-native subspace-accelerated solver for sequences of sparse linear systems.

HIP kernels for gfx950 behind a C-ABI (include/sacc.h, libsacc.so); this package is a
thin binding: ``Sequence`` (push / initial_guess / solve), ``DeviceCSR``, ``spmv`` and the
coefficient-predictor ``MLP``.
"""

from .native import SaccError  # noqa: F401
from .sequence import MLP, Batch, DeviceCSR, Sequence, spmv  # noqa: F401
