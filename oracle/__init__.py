"""CPU oracle for the population evaluator -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct float64 implementation of what the GPU path
computes, written from the paper (arXiv 2603.12292, section 2.1) and the
conventions this library fixes where the paper is silent.  It shares no code
with the GPU path: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it.  The product path never calls it.

Modules
-------
interp      postfix (reverse-Polish) stack interpreter, modes "o64" (every
            operation in IEEE binary64) and "o32e" (each token's result
            rounded to binary32), plus program validation
tree        an independent recursive tree evaluator (scalar Python math),
            used to pin the stack interpreter by brute force
fitness     MSE and correlation fitness 1 - r^2 (Eq. 1), float64 sums
population  whole-population evaluation -> fitness[N]
bound       bound on the fitness change of a binary32 evaluation (running
            error bound per case, combined through the MSE and Eq. 1's r)
grad        reverse-mode gradient of MSE w.r.t. program constants, and
            central finite differences
philox      Philox4x32-10 counter-based generator (Salmon et al., SC'11)
gp          ramped half-and-half initialisation, tournament selection,
            subtree crossover and point mutation on postfix programs

Parity status: every function here is pinned by tests under tests/ against
hand-evaluated expressions, closed forms, invariants, library routines or
brute force, except the fitness of arbitrary random programs, whose values
have no closed form ("parity unpinned" beyond the interpreter pins).
"""
