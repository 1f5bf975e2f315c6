"""Plain FP64 CPU oracle for the block-preconditioned MINRES hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything under ``oracle/``.  Only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

Everything here is written from the paper (Pazner, Kolev, Vassilevski,
"Matrix-free GPU-accelerated saddle-point solvers for high-order problems in
H(div)"), in the paper's notation, with no blocking, fusion or reordering
beyond what the definitions state.  Where the paper is silent or ambiguous the
reading taken is stated in the docstring of the function that depends on it.

Modules
-------
basis     1D Gauss-Lobatto / Gauss-Legendre points, Lagrange and
          histopolation polynomials (Section 2.1).
element   reference RT_p / Q_{p-1} bases, trilinear geometry, Piola maps,
          element matrices M_e, W_e, B_e by quadrature (Section 2, eq. matrices).
assemble  structured global numbering, assembled sparse M, W, B, the
          divergence D by Algorithm 1, the transformed block operator
          (eq. transformed-system, eq. transformed-system-darcy).
precond   diagonals, the approximate Schur complement (eq. approx-schur,
          eq. approx-schur-entries), the aggregation AMG V-cycle and the
          block-diagonal preconditioner (Section 2.3, Prop. 5, remark on tau).
minres    preconditioned MINRES (the short-recurrence Krylov method the
          paper uses for the symmetric indefinite system, Section 3).
"""
