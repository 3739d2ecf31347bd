"""FP64 CPU oracle for the matrix-free CHNS hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does,
and this package never imports the product library.

Modules:
* mesh   - octree refinement, 2:1 balance, node enumeration, hanging constraints
* fem    - Q1 element matrices and assembled sparse operators (pressure Poisson,
           mass, rho-weighted mass)
* krylov - Jacobi-PCG and restarted GMRES in FP64
* chns   - Cahn-Hilliard residual/Jacobian, VMS momentum, velocity update and
           the two-block projection step
* unet   - direct-loop conv3d forward/backward for gradient checks
"""
