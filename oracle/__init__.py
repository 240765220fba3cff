"""CPU FP64 oracle for the HDG-IMEX pressure-velocity update (test infrastructure).

This package is a plain, slow, deliberately unoptimised NumPy/SciPy
implementation of what the GPU path computes.  It exists only to check the
GPU library: only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the HIP library; the only
common module is ``hdg_inputs`` (meshes and analytic point values).

Module map (each function cites the passage of the paper it follows):

* ``quadrature`` - Gauss rules on [0,1] and on the reference triangle.
* ``basis``      - the documented orthonormal Dubiner / Legendre bases.
* ``mesh``       - facet numbering, cell/facet adjacency, affine geometry.
* ``forms``      - the weak forms: mass, f_im, g, Gamma, the weak divergence,
                   the BDM projection (Section 2, "Original fully-implicit DG
                   method", "Hybridisation", "Splitting method").
* ``hdg``        - the hybridised mixed solve: static condensation onto the
                   trace, direct trace solve, back-substitution
                   (Section "Solvers and preconditioners").
* ``tet``        - tetrahedral meshes, quadrature and bases (d = 3).
* ``forms3d``    - the same weak forms on tetrahedra, with the 3D BDM
                   interpolant (first-kind Nedelec interior moments).
* ``imex``       - Butcher tableaux (Appendix A), the preconditioned Richardson
                   iteration (Algorithm 2), the IMEX-HDG step (Algorithm 1) and
                   the pressure reconstruction (Section "Pressure reconstruction").
"""
