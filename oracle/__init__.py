"""CPU FP64 oracle for the macromodel + AIM matrix-vector product and its GMRES solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the device library or its Python binding
imports, links or runs this package; only the test suite, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the device path:
the only common input is the seeded data produced by the `synth` package, which
holds none of the method's arithmetic.

What it computes, each function citing the passage of the paper it follows:
  * RWG functions and the Galerkin EFIE entries of the exterior problem
    (section II-A, section IV eq. Gouter1) with singularity subtraction;
  * the AIM operator step by step (section V): stencils, projection P_psi,
    grid convolution H_psi by FFT and by direct sum, interpolation I_psi, the
    near-field matrix with its pre-correction;
  * the final-system product (D - G T A^-1 B) Y (section V eq. MV_product1),
    with T A^-1 B given as the per-type block M_t (section III);
  * GMRES(m) on the final system (section V, eq. finalsystem), optionally right
    preconditioned with the per-kind block-Jacobi inverse of the diagonal blocks;
  * the macromodel of one element (section II, section III): Buffa-Christiansen dual
    functions on the equivalent box, the L- and K-type Galerkin blocks between the
    scatterer and the box, D (section IV), and A, B, T, R = A^-1 B and M = T A^-1 B;
  * the plane-wave excitation vector (section IV eq. V1), the radiated far field and
    the field at finite points;
  * the Mie series of a perfectly conducting sphere, an analytic reference for the
    EFIE, excitation and far field together.

Floating point is IEEE double throughout; numpy / scipy supply matmul and FFT
steps.  Readings of points the paper leaves open are listed where they are used.
"""
