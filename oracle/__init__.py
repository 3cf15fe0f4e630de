"""Plain FP64 CPU oracle of the GRMHD right-hand side and time update.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the HIP path; the only common inputs come from the seeded generators in
``workloads``.

The paper states the method in one sentence (Introduction: general-relativistic
MHD solved with 3-D finite differences and high-order reconstruction, based on
the ECHO scheme).  Every step below therefore follows the standard published
form of that scheme family, named in each module:
  fd       : sixth-order staggered finite-difference derivative D_d and
             midpoint interpolation I_d (ECHO's high-order flux correction)
  mp5      : monotonicity-preserving fifth-order reconstruction (Suresh &
             Huynh 1997) with the point-value interpolant
  physics  : 3+1 (Valencia/ECHO) conserved variables, fluxes, fast speeds
  hll      : HLL flux (Harten, Lax & van Leer 1983)
  ct       : upwind constrained transport edge field (Londrillo & Del Zanna 2004)
  sources  : metric source terms of the stationary 3+1 equations
  c2p      : 1-D safeguarded Newton conservative-to-primitive inversion
  boundary : ghost-zone fill (periodic, outflow, polar axis)
  scheme   : RHS assembly, SSP-RK3 (Shu & Osher 1988), CFL step, diagnostics
  mlp      : FP64 reference of the learned Newton initial guess
Precision: float64 throughout.
"""
