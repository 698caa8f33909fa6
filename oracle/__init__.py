"""CPU FP64 oracle for the NUFFT derivative-Radon projector and its adjoint.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library and never calls it; the library never calls it either.

Modules
  nudft      exact non-uniform DFT and its adjoint (the plain definitions)
  kernels    Kaiser-Bessel kernel, its Fourier transform, deapodization
             factors and the min-max interpolation coefficients
  nufft      the straightforward oversampled NUFFT (Section 2.1.3, eq 2.10-2.11)
             and its transpose
  radial     the derivative factor and the radial 1D inverse DFT that turn
             Fourier-slice samples into derivative-Radon values (Section 2.2.1,
             eq 2.17-2.18) and its adjoint
  projector  the composition image -> radially sampled derivative-Radon space
  recon      direct reconstruction from derivative-Radon data: the 3D ramp
             and the NUFFT transpose with angular quadrature (Section 2.3)
  umbrella   resampling of the derivative-Radon space from the radial pattern
             onto the cone-beam umbrella planes, method 2 (eq 2.15)
  complexity the paper's multiplication-count model (Section 2.4, eq 2.16-2.27)

Conventions (where the paper is silent these are readings, not quotations):
  * volume x[n0, n1, n2], centred index m = n - N/2 (even N);
  * X(omega) = sum_n x[n] exp(-i omega . m), omega in radians per voxel;
  * oversampled grid K per axis, gamma = 2 pi / K, frequency kappa stored at
    index (kappa mod K) of numpy's FFT layout;
  * neighbour rule per axis: t = omega_d / gamma, k0 = floor(t - J/2), taps
    kappa_j = k0 + j for j = 1..J, offsets u_j = t - kappa_j in [-J/2, J/2);
  * FFTs are unnormalised in both directions; the adjoint is the exact
    conjugate transpose.

Parity status of each function is stated in its docstring; every function is
pinned by the tests in tests/test_oracle_*.py.
"""

from . import nudft, kernels, nufft, radial, projector, recon, umbrella, complexity  # noqa: F401
