"""CPU oracle for the entropy-stable DGSEM right-hand side (test infrastructure).

This package is a plain, slow, FP64 NumPy implementation of what the HIP
library computes.  It exists to check the library: only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The library never calls it, and it shares no code with the
library (no operators, tables, helpers or constants); both only receive the
same seeded inputs from ``paper_2511_17551_amd.workloads``.

Every function cites the passage of the paper it follows (section and
equation labels of arXiv 2511.17551).  Where the paper is silent, garbled
or self-contradictory, the reading taken is stated at the function.

Modules
  basis      LGL nodes/weights, derivative matrix, Legendre modes
  geometry   metric terms, Jacobian, face and subcell normals
  gas        perfect-gas closures and two-point / Riemann fluxes
  thermo     RRHO mixture energies and the temperature Newton solve
  kinetics   Arrhenius rates, equilibrium constants, species sources
  indicator  modal shock indicator and blending factor
  dgsem      semi-discrete operator du/dt = L(u)
  br1        BR1 viscous terms
  mortar     mortar interpolation / L2 projection
  ssprk      SSPRK3 time stepping
  mlp        temperature-guess MLP forward/backward, Adam
"""
