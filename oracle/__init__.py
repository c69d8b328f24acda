"""FP64 CPU oracle for the energy-based DG / Galerkin-difference wave solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference against which the HIP path is checked.  Only the test-suite, the
smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py``
may import it.  The product path (``paper_2105_01722_amd``) never imports,
links or executes anything from here, and nothing here imports the product.

Modules (each function cites the passage of Zhang, Appelo & Hagstrom,
"Energy-based discontinuous Galerkin difference methods for second-order wave
equations", arXiv:2105.01722, that it follows):

* ``gd1d``    -- 1D Galerkin-difference basis with the extrapolation closure
                 (Sec. 2.1, eq. GD_basis_lagrange, Sec. 2.1.1) and its mass,
                 stiffness and face-derivative data (Sec. 3.1, Sec. 3.2).
* ``dg2d``    -- the energy-DG semi-discretisation DG1, DG2 + the extra mean
                 equation with the (alpha, beta, tau) fluxes (Sec. 2.2,
                 Sec. 2.2.1) on periodic Cartesian element grids, dense direct
                 local solves, classical RK4, discrete energy.
* ``dg3d``    -- the same semi-discretisation on box elements in three dimensions
                 (Sec. 2.2 and the d = 3 Kronecker forms of Sec. 3.1, Sec. 3.2).
* ``analysis`` -- Bloch (dispersion) analysis of the scheme (Sec. 4).
* ``general`` -- the same weak form on mapped elements with a variable c^2
                 (Sec. 7.1 and the mapped case the paper names there),
                 assembled by Gauss-Legendre quadrature, dense direct solves.
* ``pcg``     -- preconditioned conjugate gradients for the element systems
                 (Sec. 7.1) with a tensor-product preconditioner.
* ``ic0``     -- the zero-fill incomplete Cholesky factor of the element
                 matrices (Sec. 7.1's preconditioner) and CG with it.
* ``mlp``     -- FP64 reference of the small network that corrects that
                 preconditioner (not in the paper).
"""
