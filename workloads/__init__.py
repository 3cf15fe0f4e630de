"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This package holds only input generation: grid descriptions, random-phase
initial data, metric tables of the background spacetime and training samples.
None of the numerical method (reconstruction, Riemann flux, finite-difference
derivative, constrained transport, time stepping, conservative-to-primitive
inversion) lives here; each side computes those itself from these inputs.
"""
from .grid import GridSpec, BC_PERIODIC, BC_OUTFLOW, BC_AXIS, CART, LOGSPH  # noqa: F401
