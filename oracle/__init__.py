"""CPU FP64 oracle for the block alpha-circulant preconditioned all-at-once solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
product library and its Python binding never do, and this package never
imports them.  Everything here is plain, slow and written to be checked by eye
against the paper (Tabeart, Guerol, Pearson, Weaver: "Block alpha-circulant
preconditioners for all-at-once diffusion-based covariance operators"):
numpy / scipy in float64 / complex128, no blocking, fusion or reordering.

Modules
-------
operators : the diffusion matrix A (Section 5, eq. (IminusLap), variable
            coefficient reading), the all-at-once matrix (eq. (1)), the
            sequential solve, spectral intervals (Appendix A).
precond   : shift and scaling tables (Section 2.2, eq. (3)), the explicit
            P_alpha (eq. (2)), exact P_alpha^{-1} by direct solves (eq. (4)),
            nested Chebyshev P_NC^{-1} (Section 3), the closed-form
            constant-coefficient multipliers (Appendix A + Proposition 1).
alloc     : Algorithm 1 (NC2 budget allocation) and the uniform NC1 split.
bounds    : Theorem 3, Proposition 1, Lemma 3 / Theorem 4 scalar bounds.
krylov    : right-preconditioned GMRES / FGMRES(m) with CGS2, and the paper's
            outer Chebyshev semi-iteration on P^{-1} A.
cnn       : the three-layer 3x3 convolutional warm start (forward, loss,
            hand-written backward); parity unpinned by the paper, pinned by
            finite differences and by reduction to a single linear filter.

Parity status of every function is stated in its module docstring.
"""
