"""CPU oracle for the VOF droplet-evaporation time step (test infrastructure).

This package is a plain, slow, FP64 CPU statement of what one time step of
the method computes.  It exists only to check the GPU library: the tests,
the smoke check and the benchmark's CPU-baseline leg import it; the product
library never does, and it shares no code with the HIP path (only the seeded
input generators in ``workloads`` feed both sides).

Modules, in the order of the paper's segregated step (Section 3.1):
  thermo     -- Section 2.5 (phase equilibrium, eqs. 22-25) and eq. 24
  gas        -- eq. 24 per cell and eq. 7's compressibility term (variable gas)
  interface  -- Section 2.4 (evaporation flux, eqs. 12-21)
  vof        -- Section 2.1 (eqs. 3-4) with a flux-limited face interpolation
  geo        -- Section 2.1's geometric advection: a plane per surface cell, swept face areas
  operators  -- implicit diffusion / pressure operators and a Jacobi PCG
  momentum   -- Section 2.2 and 2.6 (eqs. 6, 7, 28-30): predictor, projection
  viscous    -- eqs. 5 and 30: the implicit viscous part of the predictor
  step       -- the whole step and its diagnostics

All floating point is torch.float64 on the CPU.
"""
