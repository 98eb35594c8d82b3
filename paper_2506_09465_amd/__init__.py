"""MI355X (gfx950) implementation of the implicit unified gas-kinetic particle
(IUGKP) steady-state solver for multiscale gray phonon transport.

The compute path is the HIP library libiugkp.so (C ABI in include/iugkp.h);
this package only marshals arguments to it.
"""
from ._lib import (EST_ANALOG, EST_EXPECTED, FACES_EVERY, FACES_FINAL, FACES_OFF, PRECOND_MG,
                   PRECOND_NONE, RNG_CRN, RNG_FRESH, SCHEME_EMITTERS, SCHEME_PERSISTENT,
                   IugkpError, lib as library)

__all__ = ["Solver", "BatchSolver", "steady_temperature", "d_eff", "diffusion_solve",
           "dev_philox", "dev_math",
           "dev_segments", "dev_atomics", "step_group", "solve",
           "FACES_EVERY",
           "FACES_FINAL", "FACES_OFF", "RNG_CRN", "RNG_FRESH", "SCHEME_EMITTERS", "EST_ANALOG",
           "EST_EXPECTED", "PRECOND_NONE", "PRECOND_MG",
           "SCHEME_PERSISTENT", "IugkpError", "library"]


def __getattr__(name):
    # torch is imported lazily so that the C-ABI declarations load without it
    if name in ("Solver", "d_eff", "diffusion_solve", "dev_philox", "dev_math", "dev_segments", "dev_atomics",
                "step_group", "solve"):
        from . import solver
        return getattr(solver, name)
    if name == "BatchSolver":
        from . import batch
        return batch.BatchSolver
    if name == "steady_temperature":
        from . import adjoint
        return adjoint.steady_temperature
    raise AttributeError(name)
