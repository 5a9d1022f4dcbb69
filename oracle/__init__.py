"""CPU float64 oracle of the registration prefix scan.  TEST INFRASTRUCTURE ONLY.

A plain, slow, directly checkable implementation of what the GPU library
computes, written from the paper's definitions.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use it; the library never imports
it and it imports nothing from the library (inputs come from ``synth``).

Modules
  registration  bilinear warp, energy and gradient, gradient descent, the
                multilevel solve, composition, operators A and B
  plans         prefix-scan plans (sequential, dissemination, Ladner-Fischer,
                Brent-Kung, hierarchical reduce-then-scan) and work formulas
  scan          the series registration executed as a scan
  autodiff      gradients of the warp + energy step w.r.t. both images and u
  mock          the scan on an artificial operator (microbenchmarks): operator
                times, expected outputs, simulation of the execution forms
  rigid         the rigid normalized-cross-correlation operator: energy,
                gradient, multilevel flow, composition, its series scan
"""
from . import autodiff, mock, plans, registration, rigid, scan

__all__ = ["autodiff", "mock", "plans", "registration", "rigid", "scan"]
