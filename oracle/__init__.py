"""CPU oracle for the two-site DMRG sigma step -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 NumPy code written from the definitions, used to check the
GPU library.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the library never does, and the oracle never
imports the library.  The two share no code: only the seeded input
generators in ``synthetic`` feed both.

Modules
-------
fock        determinant (Fock) space, spin-orbital operators, the
            Hamiltonian of the Method section, FCI (plain definitions).
projection  the MPS of eq. (1) contracted into Fock vectors, the
            effective Hamiltonian P^T H P and its action (plain definition).
blocksparse renormalised block operators and the normal/complementary
            sigma (the standard ab initio DMRG algorithm, written out).
dmrg        two-site sweeps, truncation, Davidson (standard algorithm).
rdm         one- and two-particle reduced density matrices.

Parity status of every function is listed in its docstring; all functions
here are pinned by tests under tests/ (no function is "parity unpinned").
"""
