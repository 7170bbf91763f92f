"""FP64 CPU oracle for the SHT+MG lens-plane solve and multiple-plane ray
propagation of Becker (2013), "CALCLENS" (arXiv:1210.3069).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything in this package.  It is a
plain, slow, float64 numpy restatement of the paper's method, written to be
checked against the paper by eye; it shares no code with the HIP library.

Modules:
  healpix  HEALPix geometry, RING/NESTED numbering, degrade, interpolation
  sht      Legendre recurrence, ring transforms, analysis, synthesis,
           harmonic Poisson step, pure-SHT derivatives
  mg       patches, finite-volume Laplacian, red-black Gauss-Seidel FAS
           V-cycle, finite differences, evaluation at points
  rays     distances, direction/position update, Jacobian recurrence,
           parallel transport, radial interpolation for galaxies
"""
