"""MI355X-native multigrid waveform relaxation for the time-fractional heat equation.

The solver is a C-ABI shared library (``libmgwr.so``, HIP for gfx950) declared
in ``include/mgwr.h``; :mod:`paper_1608_05400_amd.binding` is a thin ctypes
layer over it.  :mod:`paper_1608_05400_amd.workloads` synthesises seeded
inputs and imports nothing else from the package.
:mod:`paper_1608_05400_amd.sama` is the semi-algebraic mode analysis of the
two-grid cycle (a CPU analysis tool, not part of the solve path).
"""

__all__ = ["binding", "workloads", "sama", "build"]
