"""FP64 CPU oracle for the 3D Helmholtz hot path -- TEST INFRASTRUCTURE.

This package is a plain, slow, obviously-correct NumPy/SciPy implementation of
what the GPU library computes: the PML-stretched 7-point and compact 27-point
Helmholtz operators and their adjoints, restarted GMRES / flexible GMRES, the
recursive multilevel GMRES (ML-GMRES) preconditioner, and the adjoint-state
least-squares misfit gradient.  Everything runs in complex128 / float64.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run it.  The product library never does, and this
package shares no code with it (the two are independent implementations of
the same definitions, compared element by element by the tests).

Modules
-------
operators  grid, absorbing-layer profiles, 7-pt / 27-pt apply and adjoint,
           independent sparse-matrix assembly
krylov     GMRES(k) and FGMRES(k) with modified Gram-Schmidt and Givens
mlgmres    transfer operators, level hierarchy, V-cycle, ML-GMRES solve
fwi        sources, receivers, misfit, adjoint source, gradient, exact FD
"""
from . import operators, krylov, mlgmres, fwi  # noqa: F401
