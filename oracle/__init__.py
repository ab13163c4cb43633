"""CPU oracle for the GTQA Trotter step — TEST INFRASTRUCTURE ONLY.

A plain, slow, complex128 NumPy implementation of what the graph
tensor-network quantum annealer computes, written from the paper's
definitions (App. A-F, Alg. 1-3, Sec. II-III).  It exists to check the GPU
library: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  The product path never calls into this package and
shares no code with it; the only shared module is `synthetic`, which draws
the seeded problem instances and the random numbers a run uses, and holds
the product formulas' angle sequences, which both sides take as inputs.

Modules
-------
colouring   Misra-Gries edge colouring (a build addition; the paper applies
            the interaction layer edge by edge, Sec. III.A).
gtqa        Vidal-gauge state, simple update (App. E), truncation (Alg. 3),
            BP (Alg. 1), Vidal gauge from messages (Alg. 2), re-gauging with
            warm-started messages (Sec. II.C), single-qubit gates (Sec. II.D),
            readout and rounding (Eq. rounding_rule), objective E(x).
exact       Exact state-vector dynamics of the same Trotter circuit (App. F),
            contraction of a small tensor network to a state vector,
            brute-force maximisation of E(x).

Parity status of each function is listed in its docstring; every function
here is pinned by a `-m "not gpu"` test except where a docstring says
"parity unpinned".
"""
