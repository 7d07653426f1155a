"""Plain, slow FP64 CPU oracle for the variational MFG hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or call anything here; the GPU
library never does, and this package shares no code with it.

Every function follows a passage of the paper (Ljosheim, Kalise, Pearson,
Silva, "Parallel-in-Time Preconditioning for Time-Dependent Variational Mean
Field Games", arXiv 2507.01958), cited by section / equation / algorithm:

* grid.py       Section 2 grids (periodic torus, Neumann interior nodes)
* operators.py  Section 2 difference operators, Section 3 matrices A, B, C
                (eq. ABC), the reduced system (eq. largeA), Section 4.3
                divergence factors D^1, D^2 and the negative Laplacian K
* prox.py       Section 3 proximal step of the cost b-hat + F (per cell), with
                the couplings and terminal cost of Section 2.1 / Section 5
* cg.py         Section 3/4 conjugate gradients on the reduced system
* precond.py    Section 4 preconditioner (eq. prec, eqs. eigs/precrec,
                Algorithms 1 and 2, eq. pstrec)
* cp.py         Section 3 Chambolle-Pock iteration (eq. pasosChamPock) with
                the Section 5 step-size schedule
* adjoint.py    reverse-mode derivative of a fixed number of CP iterations
* value.py      value function from the CP multiplier and the residual of the
                discrete HJB equation of the scheme (MFG_T^2_h), Section 2
"""
