"""FP64 CPU oracle for the flux reconstruction (FR) right-hand side.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path imports,
links or runs this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library:
it builds its own point sets, orthonormal modal bases, operators, geometry
and interface pairing from the definitions, in plain NumPy float64.

What it computes (paper: Section 2.1 and Section 3.4):

* per element type, constant operator matrices applied to state matrices
  (the "C <- c1 A B + c2 C" products of Section 2.1; the volume-to-surface
  interpolation operator M0 has the dimensions of Table 2);
* point-wise flux evaluations at solution and flux points (Section 2.1);
* a Rusanov Riemann solver at element interfaces and a DG-type correction,
  for the compressible Euler and Navier-Stokes equations with constant
  viscosity (Section 3.4);
* explicit Runge-Kutta stepping: classical RK4 and the five-stage
  two-register RK45[2R+] scheme of Kennedy, Carpenter and Lewis (Section 3.4,
  Table 1).

Where the paper is silent (point sets, bases, the viscous interface scheme,
initial conditions), each function's docstring states the reading it
takes; the readings are numbered R1..R8 consistently across modules.

Modules: ``basis`` (polynomials, point sets, quadrature), ``elements``
(reference elements and operators), ``mesh`` (geometry, face matching, flux
point pairing), ``physics`` (fluxes), ``fr`` (the right-hand side),
``rk`` (time stepping), ``reduce`` (global FP64 sums).
"""
