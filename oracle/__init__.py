"""Plain FP64 CPU oracle for the polarized subsurface BRDF of a flat homogeneous layer.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the package's smoke check and the benchmark's CPU
baseline leg may import this package. The GPU library never calls it, and it shares no code,
tables or constants with the GPU library.

What it computes (Collin & Pattanaik, "GPU accelerated computation of Polarized Subsurface BRDF
for Flat Particulate Layers"): the discrete-ordinate solution of the vector radiative transfer
equation (Sec. 2.A, eq. 2-4) for one homogeneous layer over a black base, split into Fourier orders
(Sec. 2.B, eq. 6-15), solved per order through the full 8N eigensystem of the homogeneous
equation (Sec. 2.C, eq. 16-25) and the boundary conditions (Sec. 3.C, eq. 49-56), and synthesised
into the BRDF Mueller matrix (Sec. 2.D, eq. 1 and 39) on the Gauss-node zenith grid.

It is written for clarity, not speed: the full 8N eigenproblem (no half-size reduction), a full
8N boundary solve (no block-symmetric split) and direct Fourier summation.

Modules:
  quadrature  double-Gauss nodes and weights (eq. 15)
  legendre    Wigner d-functions and the Legendre matrices P_l^m (eq. 9-11)
  phase       scattering matrix from coefficients, geometric phase matrix, its Fourier projection
  dom         per-order operator, eigen solution, boundary solve, synthesis of F_r
  particular  off-node incidence through the particular solution (eq. 28-33)
  stack       layer stacks (interface continuity, Sec. 2.C) and reflecting bases (eq. 57-66)
  reconstruct radiance towards arbitrary outgoing directions by source-function integration
              (eq. 36-38)
  brute       matrix-exponential propagator solve at extended precision (tiny N), also for stacks
              and bases (product of the layers' propagators)
  analytic    single-scattering limit and Chandrasekhar's H-function (isotropic scattering)
"""
