"""Serial FP64 CPU oracle for the FFT phase-field-fracture toughness solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written
reference that the HIP path is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never calls it and shares no code with it.

Everything here is written from the paper (Aranda & Segurado, "Effective
toughness estimation by FFT based phase field fracture: application to
composites and polycrystals", arXiv 2508.07424) in float64 with numpy /
scipy primitives only (FFT, sparse direct solve).  Each function cites the
section or equation it follows.  Where the paper is silent or its printed
formula is inconsistent, the reading taken is stated in the docstring.

Modules
-------
mandel     tensors in Mandel notation, stiffness tensors, Eq. 13 rotation
spectral   frequency grid, Fourier-Galerkin projection (Eq. 26), DFT
           gradient / divergence with forward-difference symbols
model      constitutive law (Eq. 2, 12), AT2 functionals (Eq. 3, 4, 14),
           damage operator (Eq. 10b/17), crack-tip enrichment (Eq. 35-38)
solver     staggered dissipation-controlled step (Eq. 10/16 fixed point),
           effective toughness (Eq. 32-33)
"""
