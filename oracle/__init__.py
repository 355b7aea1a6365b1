"""CPU oracle for the ORAS-preconditioned GMRES Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow complex128
implementation of what the solver computes, written from the paper
(Dolean, Jolivet, Tournier, Operto, "Iterative frequency-domain seismic wave
solvers based on multi-level domain-decomposition preconditioners"):

* ``fem``     -- the Helmholtz boundary-value problem (eq. eqh) and its P1/P2
                 Lagrange discretisation A u = b (eq. eq1);
* ``dd``      -- the overlapping decomposition, Boolean restrictions R_i,
                 partition of unity D_i and impedance local matrices A_i
                 (eq. oras);
* ``coarse``  -- the coarse interpolation Z and Galerkin matrix E = Z^T A Z
                 (eq. 2lvl);
* ``precond`` -- one- and two-level ORAS applications (eqs. oras, 2lvl);
* ``gmres``   -- right-preconditioned restarted GMRES with the relative
                 residual stop of the experiments section.

Only the tests, the smoke check of ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import it.  It shares no code with the HIP library:
the only common module is the seeded input generator
(``paper_2004_06309_amd.workloads``), which holds none of the method's
arithmetic.
"""
