"""CPU oracle for the two-site DMRG sigma step -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 NumPy code written from the definitions, used to check the
GPU library.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the library never does, and the oracle never
imports the library.  The two share no code: only the seeded input
generators in ``synthetic`` feed both.

Modules
-------
fock        determinant (Fock) space, spin-orbital operators, the
            Hamiltonian of the Method section, FCI, transition 1-/2-RDMs and
            the total spin <S^2> (plain definitions).
projection  the MPS of eq. (1) contracted into Fock vectors, the
            effective Hamiltonian P^T H P and its action (plain definition).
blocksparse renormalised block operators, the normal/complementary sigma and
            diag(H_eff) (the standard ab initio DMRG algorithm, written out).
truncation  the two-site truncation (per-sector SVD, global selection of the
            D largest weights, truncation error) and the window move.
orbital     generalised Fock matrix and orbital gradient from the RDMs.
su2         spin adaptation: Clebsch-Gordan, 6j and 9j coefficients,
            multiplet bases of blocks, the spin-adapted window H_eff (plain
            definition), the scalar-product recoupling rule of a
            spin-adapted sigma and its block-by-block contraction, and the
            coupled block x site operator product of the renormalisation.

Every function is pinned by tests under tests/ (test_oracle_*.py) against
closed forms, brute force or the plain definitions; the pins are listed in
each module's docstring.
"""
