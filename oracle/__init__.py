"""FP64 CPU oracle of the immersed interface method (IIM) for the 2D
vorticity-velocity Navier-Stokes equations with multiple bodies
(Gabbard, Gillis, Chatelain & van Rees, arXiv:2109.13628).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of the discretisation, used to prove the HIP
library right.  Only the tests, the `smoke()` entry point and the benchmark's
CPU-baseline leg may import it; the product path (the C-ABI library and its
Python binding) never does, and shares no code, table or constant generator
with it.

Modules
  lgf        lattice Green's function of the 5-point Laplacian (free space)
  poisson    solution operators G = (-lap_h)^-1: Dirichlet box (sine transform),
             free space (zero-padded convolution with the lattice Green's
             function), free space with an even outflow mirror
  geometry   boundary point sets -> spline -> control points, affected points,
             extrapolation stencils (Sec. 2.1-2.2, App. A)
  reconstruct  IIM Poisson / Schur complement / circulation rows, velocity
             (Sec. 4.2)
  transport  vorticity boundary condition, extensions, conservative fluxes,
             Kelvin circulation ODE (Sec. 3, Sec. 5.1, 5.3)
  ns         low-storage RK3 step and the time-step rule (Sec. 5.5, App. B)
  network    FP64 reference of the warm-start 1D convolution network
"""
