"""MI355X (gfx950) full-state simulator: HIP kernels behind a C ABI
(include/qsim.h, libqsim.so), with a thin ctypes binding.

Importing the package fails if libqsim.so is missing; nothing runs on the CPU
in its place.
"""
from . import native  # noqa: F401  (raises ImportError if the library is absent)
from .native import QS_C64, QS_C128  # noqa: F401


def __getattr__(name):
    # Qureg pulls in torch; load it on first use.
    if name == "Qureg":
        from .qureg import Qureg
        return Qureg
    if name == "Circuit":
        from .circuit import Circuit
        return Circuit
    if name == "Batch":
        from .batch import Batch
        return Batch
    if name in ("BatchEnergy", "energies"):
        from . import batch
        return getattr(batch, name)
    if name in ("CircuitEnergy", "circuit_energy"):
        from . import circuit
        return getattr(circuit, name)
    raise AttributeError(name)
