"""FP64 CPU oracle for the sigma-transformed pressure Poisson problem and its p-multigrid solver.

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check of the entry module and
the CPU-baseline leg of the benchmark may import it. The GPU library never does, and it shares no
code, tables or helpers with it.

It is written from the paper (Melander, Bitsch, Chen, Engsig-Karup, "A High-Order Hybrid-Spectral
Incompressible Navier-Stokes Model For Nonlinear Water Waves"):

- ``spectral``  Fourier and Chebyshev-Gauss-Lobatto grids and derivatives (Sec. 3.4, 3.5).
- ``operator``  sigma-metrics (eq. 1_Scoef), the mixed-stage operator (eq. poissonp with the
                boundary conditions eq. bcpd and eq. bcpdneu), dense assembly and direct solves.
- ``pmg``       the p-multigrid V-cycle (Alg. 1) with the coarsening of Sec. 4.1, the modal
                transfers of Sec. 4.2 and a block smoother in the role of Sec. 4.3.
- ``krylov``    GMRES / flexible GMRES with a V-cycle or a flat-mode preconditioner (Sec. 4.4).
- ``lserk``     the 2N low-storage Runge-Kutta scheme (eq. LSERK) and the stage of Sec. 3.2.
- ``adjoint``   the discrete adjoint of that stage with respect to the bathymetry.

Every function is plain NumPy/SciPy in float64; no blocking, fusion or reordering beyond what the
definitions state.
"""
