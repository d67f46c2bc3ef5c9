"""Plain FP64 CPU oracle for the time-spectral GLS Navier-Stokes hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code, tables or helpers with the HIP library in ``paper_2311_09465_amd``
and never imports it.

Independence by construction: the oracle works with complex modes -K..K,
forms the paper's Toeplitz convolution matrices explicitly, takes tau from a
LAPACK Hermitian eigendecomposition, and assembles with ``numpy.add.at``.  The
library works in a real orthonormal basis, uses sampled (dealiased) products
and its own Jacobi eigensolver, and sums element rows per node in a fixed order.

``oracle.mlp`` is the FP64 reference of the warm-start network (forward,
backward, Adam) and of the greedy reduced basis.
"""
from .tsref import (Params, geometry, slots_to_modes, modes_to_slots, toeplitz,
                    tau_from_velocity, residual, linearize, jv, picard_blocks,
                    picard_matvec, jacobian_diagonal, gmres, solve,
                    QP_BARY, FACE_QP_BARY)

__all__ = ["Params", "geometry", "slots_to_modes", "modes_to_slots", "toeplitz",
           "tau_from_velocity", "residual", "linearize", "jv", "picard_blocks",
           "picard_matvec", "jacobian_diagonal", "gmres", "solve", "QP_BARY",
           "FACE_QP_BARY"]
