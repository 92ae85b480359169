"""Plain CPU FP64 reference implementation (the oracle) of recursive reduction
quadrature (RRQ) for the Laplace layer potentials S, D, S' and D'.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

Every function follows the paper (Jiang & Zhu, "Recursive reduction quadrature
for the evaluation of Laplace layer potentials in three dimensions") step by
step, in its notation, with numpy primitives (matmul, QR, linear solves) as the
only library steps.  Citations name the section, equation label, theorem or
algorithm step that each function restates.

Parity status: every function is pinned by the CPU tests (closed forms,
identities, brute-force adaptive quadrature); none is "parity unpinned".
"""
