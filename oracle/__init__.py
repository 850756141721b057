"""Independent CPU FP64 oracle for the piecewise-isoviscous Stokes hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, explicitly assembled
reference implementation written from the paper (Huber, Ruede, Waluga,
Wohlmuth, "Highly sparse surface couplings for subdomain-wise isoviscous
Stokes finite element discretizations", arXiv:1604.07994).  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
imports it; the HIP library never imports it either.

Modules
-------
mesh       Kuhn (Freudenthal) lattices, element lists, Bey refinement check.
fem        P1 element matrices written from the bilinear forms
           (eq. standard, eq. newbil, weak divergence of eq. weaks).
problem    element viscosity by centroid rule, interface classification,
           right-hand sides, pressure weights.
assemble   global COO->CSR assembly, Dirichlet masking, the row-wise
           decoupled+interface operator of eq. equivalence-stencil.
multigrid  Uzawa smoother (eq. Uzawa_smooth), transfers, coarse solve,
           V(3,3)-cycle, solve, FP64 iterative refinement.
net        FP64 direct-loop 3D convolution network on the interface band
           (forward, manual backward, MSE loss).

Every function cites the passage of the paper it follows by section,
equation or table.  Where the paper leaves a choice open, the reading taken
is stated in the docstring of the function that makes it.
"""
