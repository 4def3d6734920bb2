"""CPU reference ("oracle") for the immersed FD/DLM Jacobian hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call or link anything in this
package; the product (the HIP library and its Python binding) never does, and
this package never imports the product.  The two share no code: the only
module both read is ``fsi_workloads`` (seeded input synthesis, none of the
method's arithmetic).

Contents (each function cites the passage of the paper it follows):

* ``vms``      - dense element matrices of the VMS-stabilised Oseen operator
                 (section 2.1) and y = sum_e P_e^T K_e P_e x (C core, FP64).
* ``dlm``      - point location, the FSI constraint matrix C^lambda = B^T
                 (section 2.3, eqs. nodal_solid_velo / fsi_constraint_matrix)
                 and its transpose, by brute force and point by point.
* ``jacobian`` - the reduced 2x2 block system of section 2.4 with the
                 per-point solid stand-in, plus nodal 4x4 block-Jacobi blocks.
* ``krylov``   - textbook flexible GMRES (right preconditioned, restarted).
* ``schur``    - a block preconditioner from the 2x2 sub-matrices of section
                 2.4's reduced system: nodal velocity blocks and a pressure
                 Schur-complement Laplacian with one multigrid V-cycle.
* ``newton``   - the nonlinear residual of one implicit step and Newton.
* ``genalpha`` - generalized-alpha time stepping (section 2.4) in stage
                 variables on top of ``newton``.
* ``solid``    - the hyperelastic solid block of section 2.4's reduced system
                 (neo-Hookean energy of eq. inc_neoHk on trilinear hexahedra whose
                 nodes are the solid points), replacing the per-point stand-in.
* ``conv3d``   - 3x3x3 convolution layers for the learned warm start.
"""
