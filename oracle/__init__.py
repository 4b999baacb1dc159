"""Reference (oracle) implementation of one IPCS + BCE-IB time step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation written directly from the paper (Bourantas et al.,
"Immersed boundary finite element method for blood flow simulation",
Section 2: governing equations, the IPCS of Section 2.2, the BCE-IB method
of Section 2.3 with Eqs. 17-24 and the combined procedure of Section 2.4),
discretised with trilinear (Q1) hexahedra on a masked Cartesian grid.  It
exists to check the GPU library; only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
path and imports nothing from it.

Modules
-------
grid    derived node/cell sets, boundary tags and canonical ordering
fem     Q1 element matrices by 2x2x2 Gauss quadrature and global assembly
ib      the four-point delta kernel (Eq. 18), interpolation matrix (Eq. 17),
        the BCE force system (Eqs. 20-24) and the velocity correction
krylov  CG and BiCGStab iterated to stagnation, dense Cholesky
ipcs    one time step in the order of Section 2.4

Parity status: every function is pinned by the tests under tests/ (closed
forms, invariants, dense direct solves on tiny grids, the Poiseuille
closed form).  The inlet Womersley-type shapes are inputs, not computed here.
"""
