"""CPU FP64 oracle for messenger-field mapmaking (Huffenberger & Naess).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and this package imports nothing from the library.

Every routine is written in float64 NumPy straight from the paper's equations,
with library primitives (``numpy.fft``, ``numpy.bincount``, ``numpy.linalg``)
as the only building blocks and no blocking, fusion or reordering beyond what
the equations state.

Modules
-------
noise      noise power spectrum, messenger covariance, spectral filters (Sections 2, 2.1, 2.3, 4.2)
pointing   pointing weights, projection P, back-projection P^T, weight blocks P^T T^-1 P (Sections 2, 2.1)
messenger  the messenger iteration in its three algebraic forms, chi^2, cooling schedule (Section 2.1)
cg         diagonal-preconditioned conjugate gradients on the same operators (Sections 1, 2, 3.1)
dense      explicit matrices on tiny problems: circulant N^-1, P, GLS solution, m(lambda), F(lambda)
grad       implicit gradients of the solved map (adjoint of the mapmaking equation)
"""

from .noise import noise_psd, chi2_weights, messenger_filter, NoiseModel
from .pointing import Pointing
from .messenger import (Setup, make_setup, residual, apply_filter, chi2, chi2_lambda,
                        messenger_step, messenger_step_two_equation, messenger_step_mapsized,
                        cooling_schedule, messenger_solve, binned_map)
from .cg import pcg_solve

__all__ = [
    "noise_psd", "chi2_weights", "messenger_filter", "NoiseModel", "Pointing", "Setup", "make_setup",
    "residual", "apply_filter", "chi2", "chi2_lambda", "messenger_step", "messenger_step_two_equation",
    "messenger_step_mapsized", "cooling_schedule", "messenger_solve", "binned_map", "pcg_solve",
]
