"""Pins of the spin-adaptation oracle (CPU).

Clebsch-Gordan and 6j coefficients against orthonormality, closed forms and
explicit spin matrices; multiplet bases against S^2 and S_+; the spin-adapted
effective Hamiltonian against full CI of the same spin; the scalar-product
rule of a spin-adapted sigma against the operator built on the Fock space.
"""
import itertools
from math import sqrt

import numpy as np
import pytest

from oracle import su2
from oracle.fock import DetSpace, s_squared
from synthetic import make_integrals

SPINS = range(0, 7)  # doubled: 0 .. 3


def spin_matrices(tj):
    """J_z, J_+ of spin j = tj/2 in the basis m = j, j-1, ..., -j."""
    j = tj / 2
    ms = [j - i for i in range(tj + 1)]
    jz = np.diag(ms)
    jp = np.zeros((tj + 1, tj + 1))
    for i in range(1, tj + 1):
        m = ms[i]
        jp[i - 1, i] = sqrt(j * (j + 1) - m * (m + 1))
    return jz, jp


def test_clebsch_gordan_orthonormal():
    for tj1, tj2 in itertools.product(SPINS, SPINS):
        for tM in range(-(tj1 + tj2), tj1 + tj2 + 1, 2):
            Js = [tJ for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2) if abs(tM) <= tJ]
            m1s = [tm1 for tm1 in range(-tj1, tj1 + 1, 2) if abs(tM - tm1) <= tj2]
            C = np.array([[su2.clebsch_gordan(tj1, tm1, tj2, tM - tm1, tJ, tM) for tJ in Js] for tm1 in m1s])
            assert C.shape[0] == C.shape[1]
            assert np.allclose(C.T @ C, np.eye(len(Js)), atol=1e-12)


def test_clebsch_gordan_spin_half_closed_form():
    # <j1 m-1/2; 1/2 1/2 | j1+1/2 m> = sqrt((j1 + m + 1/2) / (2 j1 + 1))
    for tj1 in SPINS:
        for tm in range(-(tj1 + 1), tj1 + 2, 2):
            if abs(tm - 1) > tj1:
                continue
            ref = sqrt((tj1 / 2 + tm / 2 + 0.5) / (tj1 + 1))
            assert abs(su2.clebsch_gordan(tj1, tm - 1, 1, 1, tj1 + 1, tm) - ref) < 1e-13


def test_clebsch_gordan_are_eigenvectors_of_total_spin():
    """Columns of CG are the J^2 eigenvectors of the product space built from
    spin matrices, with the Condon-Shortley phase fixed by the highest weight."""
    for tj1, tj2 in [(1, 1), (2, 1), (2, 2), (3, 2), (4, 3)]:
        z1, p1 = spin_matrices(tj1)
        z2, p2 = spin_matrices(tj2)
        I1, I2 = np.eye(tj1 + 1), np.eye(tj2 + 1)
        Jz = np.kron(z1, I2) + np.kron(I1, z2)
        Jp = np.kron(p1, I2) + np.kron(I1, p2)
        J2 = Jp.T @ Jp + Jz @ Jz + Jz
        for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for tM in range(-tJ, tJ + 1, 2):
                v = np.zeros((tj1 + 1) * (tj2 + 1))
                for a in range(tj1 + 1):
                    for b in range(tj2 + 1):
                        v[a * (tj2 + 1) + b] = su2.clebsch_gordan(tj1, tj1 - 2 * a, tj2, tj2 - 2 * b, tJ, tM)
                J = tJ / 2
                assert np.allclose(J2 @ v, J * (J + 1) * v, atol=1e-12)
                assert np.allclose(Jz @ v, tM / 2 * v, atol=1e-12)
            # highest weight: <j1 j1; j2 J-j1 | J J> > 0, and lowering
            # reproduces the M < J columns with positive normalisation
            top = np.array([su2.clebsch_gordan(tj1, tj1 - 2 * a, tj2, tj2 - 2 * b, tJ, tJ)
                            for a in range(tj1 + 1) for b in range(tj2 + 1)])
            assert su2.clebsch_gordan(tj1, tj1, tj2, tJ - tj1, tJ, tJ) > 0
            cur, tM = top, tJ
            while tM > -tJ:
                J, M = tJ / 2, tM / 2
                cur = Jp.T @ cur / sqrt(J * (J + 1) - M * (M - 1))
                tM -= 2
                ref = np.array([su2.clebsch_gordan(tj1, tj1 - 2 * a, tj2, tj2 - 2 * b, tJ, tM)
                                for a in range(tj1 + 1) for b in range(tj2 + 1)])
                assert np.allclose(cur, ref, atol=1e-12)


def test_6j_orthogonality_and_special_value():
    for ta, tb, tc, td in itertools.product(range(0, 5), repeat=4):
        es = [te for te in range(0, 9) if su2._triangle(ta, td, te) and su2._triangle(tc, tb, te)]
        xs = [tx for tx in range(0, 9) if su2._triangle(ta, tb, tx) and su2._triangle(tc, td, tx)]
        for te, te2 in itertools.product(es, es):
            s = sum((tx + 1) * (te + 1) * su2.wigner_6j(ta, tb, tx, tc, td, te)
                    * su2.wigner_6j(ta, tb, tx, tc, td, te2) for tx in xs)
            assert abs(s - (1.0 if te == te2 else 0.0)) < 1e-12
    # {a b c; 0 c b} = (-1)^(a+b+c) / sqrt((2b+1)(2c+1))
    for ta, tb, tc in itertools.product(range(0, 7), repeat=3):
        if not su2._triangle(ta, tb, tc):
            continue
        ref = (-1) ** ((ta + tb + tc) // 2) / sqrt((tb + 1) * (tc + 1))
        assert abs(su2.wigner_6j(ta, tb, tc, 0, tc, tb) - ref) < 1e-13


def test_scalar_coupling_equals_its_clebsch_gordan_sum():
    """The closed form against the defining sum over components:
    sum_q <k q; k -q|0 0> <a' b' S M|(<a M_a; k q|a' M_a'> <b M_b; k -q|b' M_b'>)|a b S M>."""
    n = 0
    for tSa, tSb, tSa2, tSb2, tk in itertools.product(range(0, 5), range(0, 5), range(0, 5), range(0, 5),
                                                      (0, 1, 2)):
        for tS in range(0, 9):
            if not (su2._triangle(tSa, tSb, tS) and su2._triangle(tSa2, tSb2, tS)
                    and su2._triangle(tSa, tk, tSa2) and su2._triangle(tSb, tk, tSb2)):
                continue
            tM = tS
            ref = 0.0
            for tq in range(-tk, tk + 1, 2):
                for tMa in range(-tSa, tSa + 1, 2):
                    tMb = tM - tMa
                    if abs(tMb) > tSb:
                        continue
                    tMa2, tMb2 = tMa + tq, tMb - tq
                    if abs(tMa2) > tSa2 or abs(tMb2) > tSb2:
                        continue
                    ref += (su2.clebsch_gordan(tk, tq, tk, -tq, 0, 0)
                            * su2.clebsch_gordan(tSa2, tMa2, tSb2, tMb2, tS, tM)
                            * su2.clebsch_gordan(tSa, tMa, tSb, tMb, tS, tM)
                            * su2.clebsch_gordan(tSa, tMa, tk, tq, tSa2, tMa2)
                            * su2.clebsch_gordan(tSb, tMb, tk, -tq, tSb2, tMb2))
            assert abs(su2.scalar_coupling(tSa2, tSb2, tSa, tSb, tS, tk) - ref) < 1e-12
            n += 1
    assert n > 200


@pytest.mark.parametrize("n_orb", [1, 2, 3])
def test_multiplets_are_spin_eigenstates_and_complete(n_orb):
    mults = su2.multiplets(n_orb)
    count = {}
    for M in mults:
        for tM, v in M.vec.items():
            space = M.space[tM]
            assert np.allclose(v.T @ v, np.eye(M.dim), atol=1e-12)
            for c in range(M.dim):
                S = M.tS / 2
                assert abs(s_squared(space, v[:, c]) - S * (S + 1)) < 1e-11
            count[(M.n, tM)] = count.get((M.n, tM), 0) + M.dim
    for (n, tM), c in count.items():
        assert c == DetSpace.sector(n_orb, n, tM).dim
    assert sum(M.dim * (M.tS + 1) for M in mults) == 4 ** n_orb


def fci_spin_levels(K, n, tS, h, eri):
    space = DetSpace.sector(K, n, tS)
    H = space.hamiltonian(h, eri).toarray()
    w, v = np.linalg.eigh(H)
    S = tS / 2
    keep = [w[i] for i in range(len(w)) if abs(s_squared(space, v[:, i]) - S * (S + 1)) < 1e-8]
    return np.array(keep)


@pytest.mark.parametrize("K,nl,n,tS", [(4, 2, 4, 0), (4, 2, 4, 2), (4, 1, 3, 1), (4, 3, 5, 3), (5, 2, 5, 1)])
def test_heff_su2_spectrum_is_fci_of_that_spin(K, nl, n, tS):
    h, eri = make_integrals(K, K)
    left, right = su2.multiplets(nl), su2.multiplets(K - nl)
    m, basis = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS)
    assert np.allclose(m, m.T, atol=1e-12)
    w = np.linalg.eigvalsh(m)
    ref = fci_spin_levels(K, n, tS, h, eri)
    assert len(w) == len(ref)
    assert np.allclose(np.sort(w), np.sort(ref), atol=1e-10)


def test_heff_su2_does_not_depend_on_m_and_its_states_are_orthonormal():
    K, nl, n, tS = 5, 2, 5, 3
    h, eri = make_integrals(K, K)
    rng = np.random.default_rng(11)
    left, right = su2.multiplets(nl, rng, keep=2), su2.multiplets(K - nl, rng, keep=2)
    basis = su2.coupled_basis(left, right, n, tS)
    P, _ = su2.coupled_vectors(left, right, nl, K - nl, n, tS, tS, basis)
    assert np.allclose(P.T @ P, np.eye(len(basis)), atol=1e-12)
    a, _ = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS, tS)
    b, _ = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS, tS - 2)
    c, _ = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS, -tS)
    assert np.allclose(a, b, atol=1e-12) and np.allclose(a, c, atol=1e-12)


def test_heff_su2_energy_equals_the_u1_rayleigh_quotient():
    """A spin-adapted window vector is a U(1) vector of S_z = S: its Rayleigh
    quotient under H_eff equals that of the Fock vector under H."""
    K, nl, n, tS = 5, 2, 5, 1
    h, eri = make_integrals(K, K)
    rng = np.random.default_rng(12)
    left, right = su2.multiplets(nl, rng, keep=2), su2.multiplets(K - nl, rng, keep=3)
    m, basis = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS)
    psi = rng.normal(size=len(basis))
    P, space = su2.coupled_vectors(left, right, nl, K - nl, n, tS, tS, basis)
    v = P @ psi
    H = space.hamiltonian(h, eri)
    assert abs(psi @ m @ psi / (psi @ psi) - v @ (H @ v) / (v @ v)) < 1e-10
    assert abs(s_squared(space, v) - (tS / 2) * (tS / 2 + 1)) < 1e-10


def block_tensor(mults, n_orb, dn, tk, rng):
    """A random rank-k tensor operator on a block (particle change dn): random
    reduced blocks for every allowed (a', a), expanded into components
    T_q = sum CG <S M; k q|S' M'> t |a' M'><a M| on the block's full Fock
    space.  Returns (reduced dict, {tq: dense matrix})."""
    full = DetSpace.full(n_orb)
    red = {}
    for i2, A2 in enumerate(mults):
        for i, A in enumerate(mults):
            if A2.n == A.n + dn and su2._triangle(A.tS, tk, A2.tS):
                red[(i2, i)] = rng.normal(size=(A2.dim, A.dim))
    comp = {}
    for tq in range(-tk, tk + 1, 2):
        T = np.zeros((full.dim, full.dim))
        for (i2, i), t in red.items():
            A2, A = mults[i2], mults[i]
            for tM in range(-A.tS, A.tS + 1, 2):
                tM2 = tM + tq
                if abs(tM2) > A2.tS:
                    continue
                cg = su2.clebsch_gordan(A.tS, tM, tk, tq, A2.tS, tM2)
                if cg == 0.0:
                    continue
                rows = full.index(A2.space[tM2].dets)
                cols = full.index(A.space[tM].dets)
                T[np.ix_(rows, cols)] += cg * (A2.vec[tM2] @ t @ A.vec[tM].T)
        comp[tq] = T
    return red, comp


@pytest.mark.parametrize("dn,tk", [(0, 0), (0, 2), (1, 1), (-1, 1), (2, 0), (2, 2)])
def test_scalar_product_rule_against_the_fock_space_operator(dn, tk):
    """[A^k x B^k]^0 with A on the left block (particle change dn) and B on the
    right (-dn), built component by component on the Fock space with the
    Jordan-Wigner sign of B passing the left electrons, against the reduced
    rule: (-1)^(p(B) N_a) scalar_coupling t_A t_B."""
    nl, nr, n, tS = 2, 2, 4, 2
    rng = np.random.default_rng(20 + 3 * dn + tk)
    left, right = su2.multiplets(nl), su2.multiplets(nr)
    ta, A = block_tensor(left, nl, dn, tk, rng)
    tb, B = block_tensor(right, nr, -dn, tk, rng)
    full_l, full_r = DetSpace.full(nl), DetSpace.full(nr)
    nL = np.bitwise_count(full_l.dets.astype(np.uint64)).astype(int)
    pb = abs(dn) % 2
    sign = np.diag((-1.0) ** (pb * nL))
    O = sum(su2.clebsch_gordan(tk, tq, tk, -tq, 0, 0) * np.kron(B[-tq], A[tq] @ sign)
            for tq in range(-tk, tk + 1, 2))
    # full index = left det + (right det << 2 nl): kron(B, A) orders (right, left)
    basis = su2.coupled_basis(left, right, n, tS)
    P, space = su2.coupled_vectors(left, right, nl, nr, n, tS, tS, basis)
    idx = np.asarray(space.dets)  # full determinant integers = positions in kron order
    brute = P.T @ O[np.ix_(idx, idx)] @ P
    rule = np.zeros_like(brute)
    for c2, (ia2, al2, ib2, be2) in enumerate(basis):
        for c, (ia, al, ib, be) in enumerate(basis):
            if (ia2, ia) not in ta or (ib2, ib) not in tb:
                continue
            coef = su2.scalar_coupling(left[ia2].tS, right[ib2].tS, left[ia].tS, right[ib].tS, tS, tk)
            rule[c2, c] = ((-1) ** (pb * left[ia].n)) * coef * ta[(ia2, ia)][al2, al] * tb[(ib2, ib)][be2, be]
    assert np.abs(brute).max() > 1e-3
    assert np.allclose(rule, brute, atol=1e-11)


def test_contract_scalar_products_against_the_fock_space_operators():
    """The block-by-block spin-adapted contraction (the rule a spin-adapted
    sigma runs as block GEMMs) against the sum of the operators built on the
    Fock space, for several pairs of ranks 0, 1/2, 1 and particle changes."""
    nl, nr, n, tS = 2, 2, 4, 2
    rng = np.random.default_rng(31)
    left, right = su2.multiplets(nl), su2.multiplets(nr)
    lsec = [(M.n, M.tS, M.dim) for M in left]
    rsec = [(M.n, M.tS, M.dim) for M in right]
    full_l = DetSpace.full(nl)
    nL = np.bitwise_count(full_l.dets.astype(np.uint64)).astype(int)
    pairs, O = [], 0
    for (dn, tk), c in zip([(0, 0), (1, 1), (-1, 1), (0, 2), (2, 2)], [0.7, -1.3, 0.4, 2.0, -0.5]):
        ta, A = block_tensor(left, nl, dn, tk, rng)
        tb, B = block_tensor(right, nr, -dn, tk, rng)
        pb = abs(dn) % 2
        sign = np.diag((-1.0) ** (pb * nL))
        O = O + c * sum(su2.clebsch_gordan(tk, tq, tk, -tq, 0, 0) * np.kron(B[-tq], A[tq] @ sign)
                        for tq in range(-tk, tk + 1, 2))
        pairs.append((c, tk, pb, ta, tb))
    basis = su2.coupled_basis(left, right, n, tS)
    P, space = su2.coupled_vectors(left, right, nl, nr, n, tS, tS, basis)
    idx = np.asarray(space.dets)
    psi_flat = rng.normal(size=len(basis))
    ref = P.T @ (O[np.ix_(idx, idx)] @ (P @ psi_flat))
    blocks = su2.coupled_blocks(lsec, rsec, n, tS)
    psi = {k: np.zeros((lsec[k[0]][2], rsec[k[1]][2])) for k in blocks}
    for c, (ia, al, ib, be) in enumerate(basis):
        psi[(ia, ib)][al, be] = psi_flat[c]
    got = su2.contract_scalar_products(lsec, rsec, n, tS, psi, pairs)
    got_flat = np.array([got[(ia, ib)][al, be] for (ia, al, ib, be) in basis])
    assert np.abs(ref).max() > 1e-2
    assert np.allclose(got_flat, ref, atol=1e-11)
