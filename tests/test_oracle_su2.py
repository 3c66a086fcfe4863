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


@pytest.mark.parametrize("spins", [(1, 1, 2, 1, 1, 2), (2, 1, 1, 1, 2, 3), (3, 2, 1, 1, 2, 2), (2, 2, 2, 2, 2, 4)])
def test_9j_with_a_zero_entry_is_a_6j(spins):
    """{a b e; c d e; f f 0} = (-1)^(b + c + e + f) {a b e; d c f} / sqrt((2e + 1)(2f + 1))."""
    a, b, e, c, d, f = spins
    got = su2.wigner_9j(a, b, e, c, d, e, f, f, 0)
    want = (-1) ** ((b + c + e + f) // 2) * su2.wigner_6j(a, b, e, d, c, f) / sqrt((e + 1) * (f + 1))
    assert abs(got - want) < 1e-13


@pytest.mark.parametrize("j1,j2,j3,j4,J", [(1, 1, 1, 1, 2), (2, 1, 1, 2, 2), (1, 2, 3, 1, 3), (2, 2, 2, 2, 4)])
def test_9j_recoupling_matrix_is_orthogonal(j1, j2, j3, j4, J):
    """The transformation between the couplings ((j1 j2) j12, (j3 j4) j34) J
    and ((j1 j3) j13, (j2 j4) j24) J, sqrt((2j12+1)(2j34+1)(2j13+1)(2j24+1))
    times the 9j symbol, is an orthogonal matrix (and square)."""
    def pairs(ja, jb, jc, jd):
        return [(x, y) for x in range(abs(ja - jb), ja + jb + 1, 2) for y in range(abs(jc - jd), jc + jd + 1, 2)
                if su2._triangle(x, y, J)]
    rows, cols = pairs(j1, j2, j3, j4), pairs(j1, j3, j2, j4)
    M = np.array([[sqrt((x + 1) * (y + 1) * (u + 1) * (v + 1)) * su2.wigner_9j(j1, j2, x, j3, j4, y, u, v, J)
                   for (u, v) in cols] for (x, y) in rows])
    assert M.shape[0] == M.shape[1] > 1
    assert np.allclose(M.T @ M, np.eye(len(cols)), atol=1e-12)


def test_product_coupling_of_rank_zero_is_the_scalar_rule():
    for tsa2, tsb2, tsa, tsb, ts, tk in [(1, 1, 1, 1, 0, 2), (2, 1, 0, 1, 1, 2), (1, 2, 1, 0, 1, 1), (2, 2, 2, 2, 2, 2)]:
        got = su2.product_coupling(tsa2, tsb2, ts, tsa, tsb, ts, tk, tk, 0)
        assert abs(got - su2.scalar_coupling(tsa2, tsb2, tsa, tsb, ts, tk)) < 1e-13


@pytest.mark.parametrize("dn1,tk1,dn2,tk2,tk", [(0, 0, 1, 1, 1), (1, 1, 1, 1, 0), (1, 1, 1, 1, 2), (1, 1, -1, 1, 2),
                                                (0, 2, 0, 2, 2), (2, 0, -1, 1, 1), (-1, 1, 0, 2, 3)])
def test_product_operator_against_the_fock_space(dn1, tk1, dn2, tk2, tk):
    """[A^k1 x B^k2]^k of a two-orbital block operator A and a one-orbital
    site operator B (the renormalisation step of spin-adapted DMRG), built
    component by component on the Fock space with the Jordan-Wigner sign of
    B passing the block's electrons, against product_operator on the coupled
    multiplets of block x site."""
    nl, nr = 2, 1
    rng = np.random.default_rng(40 + 7 * dn1 + 3 * tk1 + tk)
    left, right = su2.multiplets(nl), su2.multiplets(nr)
    sec1 = [(M.n, M.tS, M.dim) for M in left]
    sec2 = [(M.n, M.tS, M.dim) for M in right]
    t1, A = block_tensor(left, nl, dn1, tk1, rng)
    t2, B = block_tensor(right, nr, dn2, tk2, rng)
    full_l = DetSpace.full(nl)
    nL = np.bitwise_count(full_l.dets.astype(np.uint64)).astype(int)
    p2 = abs(dn2) % 2
    sign = np.diag((-1.0) ** (p2 * nL))
    X = {}
    for tq in range(-tk, tk + 1, 2):
        X[tq] = sum(su2.clebsch_gordan(tk1, q1, tk2, tq - q1, tk, tq) * np.kron(B[tq - q1], A[q1] @ sign)
                    for q1 in range(-tk1, tk1 + 1, 2) if abs(tq - q1) <= tk2)
    rule = su2.product_operator(sec1, sec2, t1, t2, tk1, tk2, tk, p2)
    checked = 0
    for n in range(0, 2 * (nl + nr) + 1):
        n2 = n + dn1 + dn2
        if not 0 <= n2 <= 2 * (nl + nr):
            continue
        for tJ in range(n % 2, 2 * (nl + nr) + 1, 2):
            kb = su2.coupled_basis(left, right, n, tJ)
            if not kb:
                continue
            for tJ2 in range(n2 % 2, 2 * (nl + nr) + 1, 2):
                bb = su2.coupled_basis(left, right, n2, tJ2)
                if not bb or not su2._triangle(tJ, tk, tJ2):
                    continue
                tM = tJ
                Pk, sk = su2.coupled_vectors(left, right, nl, nr, n, tJ, tM, kb)
                for tq in range(-tk, tk + 1, 2):
                    tM2 = tM + tq
                    cg = su2.clebsch_gordan(tJ, tM, tk, tq, tJ2, tM2) if abs(tM2) <= tJ2 else 0.0
                    if abs(cg) < 1e-12:
                        continue
                    Pb, sb = su2.coupled_vectors(left, right, nl, nr, n2, tJ2, tM2, bb)
                    brute = Pb.T @ X[tq][np.ix_(np.asarray(sb.dets), np.asarray(sk.dets))] @ Pk / cg
                    want = np.zeros_like(brute)
                    for c2, (ia2, al2, ib2, be2) in enumerate(bb):
                        for c, (ia, al, ib, be) in enumerate(kb):
                            blk = rule.get(((ia2, ib2, tJ2), (ia, ib, tJ)))
                            if blk is not None:
                                want[c2, c] = blk[al2 * sec2[ib2][2] + be2, al * sec2[ib][2] + be]
                    assert np.allclose(brute, want, atol=1e-11)
                    checked += int(np.abs(brute).max() > 1e-3)
    assert checked >= 3


def test_renormalised_operator_against_the_fock_space():
    """A block operator times a site operator, coupled (product_operator) and
    projected onto a truncated spin-adapted basis of the enlarged block
    (rotate_operator), against the reduced elements of the Fock-space
    product between the kept multiplets (random orthonormal combinations of
    the coupled states of each (N, S), fewer than all)."""
    nl, nr = 2, 1
    dn1, tk1, dn2, tk2, tk = 1, 1, 0, 2, 1
    rng = np.random.default_rng(77)
    left, right = su2.multiplets(nl), su2.multiplets(nr)
    sec1 = [(M.n, M.tS, M.dim) for M in left]
    sec2 = [(M.n, M.tS, M.dim) for M in right]
    t1, A = block_tensor(left, nl, dn1, tk1, rng)
    t2, B = block_tensor(right, nr, dn2, tk2, rng)
    full_l = DetSpace.full(nl)
    nL = np.bitwise_count(full_l.dets.astype(np.uint64)).astype(int)
    sign = np.diag((-1.0) ** ((abs(dn2) % 2) * nL))
    X = {tq: sum(su2.clebsch_gordan(tk1, q1, tk2, tq - q1, tk, tq) * np.kron(B[tq - q1], A[q1] @ sign)
                 for q1 in range(-tk1, tk1 + 1, 2) if abs(tq - q1) <= tk2)
         for tq in range(-tk, tk + 1, 2)}
    blocks = su2.product_operator(sec1, sec2, t1, t2, tk1, tk2, tk, abs(dn2) % 2)
    # coupled sectors (i1, i2, 2S), numbered as the library does, grouped by (N, 2S)
    cs = [(i1, i2, ts) for i1, (_, s1, _) in enumerate(sec1) for i2, (_, s2, _) in enumerate(sec2)
          for ts in range(abs(s1 - s2), s1 + s2 + 1, 2)]
    groups = sorted({(sec1[i1][0] + sec2[i2][0], ts) for i1, i2, ts in cs})
    group_of = [groups.index((sec1[i1][0] + sec2[i2][0], ts)) for i1, i2, ts in cs]
    U, proj = {}, {}
    for g, (n, ts) in enumerate(groups):
        members = [c for c in range(len(cs)) if group_of[c] == g]
        dim = sum(sec1[cs[c][0]][2] * sec2[cs[c][1]][2] for c in members)
        keep = max(1, dim - 1) if dim > 1 else 1
        U[g] = np.linalg.qr(rng.normal(size=(dim, dim)))[0][:, :keep]
        r = 0
        for c in members:
            d = sec1[cs[c][0]][2] * sec2[cs[c][1]][2]
            proj[c] = U[g][r:r + d]
            r += d
    keyed = {(cs.index(k2), cs.index(k)): v for (k2, k), v in blocks.items()}
    got = su2.rotate_operator(keyed, proj, group_of)

    def kept_vectors(g, tM):
        n, ts = groups[g]
        basis = su2.coupled_basis(left, right, n, ts)  # (ia, al, ib, be), (ia, ib) outer: the coupled sectors in order
        P, space = su2.coupled_vectors(left, right, nl, nr, n, ts, tM, basis)
        return P @ U[g], space

    checked = 0
    for (g2, g), o in got.items():
        (n2, ts2), (n, ts) = groups[g2], groups[g]
        V, sk = kept_vectors(g, ts)
        for tq in range(-tk, tk + 1, 2):
            tM2 = ts + tq
            if abs(tM2) > ts2:
                continue
            cg = su2.clebsch_gordan(ts, ts, tk, tq, ts2, tM2)
            if abs(cg) < 1e-12:
                continue
            V2, sb = kept_vectors(g2, tM2)
            brute = V2.T @ X[tq][np.ix_(np.asarray(sb.dets), np.asarray(sk.dets))] @ V / cg
            assert np.allclose(brute, o, atol=1e-11)
            checked += 1
    assert checked >= 5


@pytest.mark.parametrize("K,nl,n,tS", [(4, 2, 4, 0), (4, 2, 4, 2), (4, 2, 3, 1), (4, 2, 5, 3)])
def test_window_hamiltonian_as_scalar_products(K, nl, n, tS):
    """The window Hamiltonian expanded into scalar products of left unit
    tensors and right partner operators (window_pairs), contracted block by
    block with the spin-adapted rule (contract_scalar_products, the
    contraction the library runs), equals the spin-adapted H_eff by its
    definition (heff_su2, whose spectrum is the full-CI spectrum of that
    spin)."""
    h, eri = make_integrals(K, K)
    left, right = su2.multiplets(nl), su2.multiplets(K - nl)
    lsec = [(M.n, M.tS, M.dim) for M in left]
    rsec = [(M.n, M.tS, M.dim) for M in right]
    pairs = su2.window_pairs(h, eri, left, right, nl, K - nl)
    # ranks 0, 1/2 and 1 (doubled 0, 1, 2): a term of H moves at most two
    # electrons' worth of spin across the cut; higher-rank unit tensors get
    # no partner
    assert {p[1] for p in pairs} == {0, 1, 2}
    m, basis = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS)
    rng = np.random.default_rng(5 + n + tS)
    psi_flat = rng.normal(size=len(basis))
    blocks = su2.coupled_blocks(lsec, rsec, n, tS)
    psi = {k: np.zeros((lsec[k[0]][2], rsec[k[1]][2])) for k in blocks}
    for c, (ia, al, ib, be) in enumerate(basis):
        psi[(ia, ib)][al, be] = psi_flat[c]
    got = su2.contract_scalar_products(lsec, rsec, n, tS, psi, pairs)
    got_flat = np.array([got[(ia, ib)][al, be] for (ia, al, ib, be) in basis])
    ref = m @ psi_flat
    assert np.abs(ref).max() > 1e-2
    assert np.allclose(got_flat, ref, atol=1e-10)
