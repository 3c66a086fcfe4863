"""Spin adaptation (SU(2)) of the two-site window -- TEST INFRASTRUCTURE ONLY.

The paper's production runs use spin-adapted DMRG (bond dimensions counted in
multiplets, D_SU(2); Numerical procedure section, Fig. 2-3).  This module
holds the plain definitions that a spin-adapted sigma has to reproduce:

* Spins are passed doubled (tj = 2j), so that half-integers stay integers.
* clebsch_gordan(tj1, tm1, tj2, tm2, tJ, tM) = <j1 m1; j2 m2 | J M>, Racah's
  closed formula with the Condon-Shortley phase (<j1 j1; j2 J-j1 | J J> > 0).
* wigner_6j(tj1, tj2, tj3, tj4, tj5, tj6) = {j1 j2 j3; j4 j5 j6}, Racah's
  closed formula (a sum over one index of factorial ratios).
* Multiplet bases of a block of orbitals: for every particle number N and
  spin S, the highest-weight states (S_z = S, S_+ psi = 0) span the
  multiplets; the other components follow by the lowering operator,
  |S M-1> = S_- |S M> / sqrt(S(S+1) - M(M-1)) (the Condon-Shortley
  convention).  `multiplets(n_orb, rng=None, keep=None)` builds them for a
  block's Fock space, all of them or a random subset of each (N, S).
* Reduced matrix elements, with the convention of the Wigner-Eckart theorem
  written with a Clebsch-Gordan coefficient:
      <a' S' M'| T^k_q |a S M> = <S M; k q | S' M'> <a' S' || T^k || a S>.
* The coupled basis of two blocks (left orbitals first in the Jordan-Wigner
  order, so a product of block states is the concatenated determinant with
  no sign): |(a S_a, b S_b) S M> = sum <S_a M_a; S_b M_b | S M> |a M_a>|b M_b>.
* heff_su2: the spin-adapted effective Hamiltonian of the window, the plain
  definition <c'| H |c> over coupled states c of total spin S at one M (the
  reduced matrix does not depend on M).
* scalar_coupling: the matrix element of the scalar product
  [A^k x B^k]^0 = sum_q <k q; k -q | 0 0> A_q B_-q between coupled states,
  for unit reduced elements of A (left block) and B (right block), without
  the fermion sign (-1)^(p(B) N_a):
      (-1)^(S_a + S_b' + S + k) sqrt((2 S_a' + 1)(2 S_b' + 1) / (2k + 1))
          {S_a S_b S; S_b' S_a' k}.
  A spin-adapted sigma is a sum of such scalar products of left and right
  (enlarged-block) tensor operators of rank 0, 1/2 and 1, each a product of
  reduced block matrices weighted by this coefficient, which is what the
  grouped block GEMMs would execute.
* window_pairs: the window Hamiltonian written as scalar products of left
  unit tensors and their right partner operators (an expansion over the
  left block's operator space), the input contract_scalar_products needs
  to apply H_eff.
* rotate_operator: the renormalisation's projection of those blocks onto
  the kept multiplets of each new (N, S) sector, O' = U^T X U by sector.
* wigner_9j and product_coupling / product_operator: the reduced blocks of
  a coupled product [A^k1 x B^k2]^k of operators on two subsystems (a block
  operator times a site operator: the renormalisation step that builds the
  enlarged block's tensor operators), weighted by
      sqrt((2S + 1)(2k + 1)(2S_a' + 1)(2S_b' + 1)) {S_a' S_a k1; S_b' S_b k2; S' S k}
  and the fermion sign (-1)^(p(B) N_a).

Pins (tests/test_oracle_su2.py): Clebsch-Gordan orthonormality, the closed
form for j2 = 1/2 and the eigenvectors of J^2 built from explicit spin
matrices; the 6j orthogonality relation and the special value with a zero
entry; scalar_coupling against the explicit Clebsch-Gordan sum that defines
it; multiplet bases against S^2, S_+ and the sector dimensions; heff_su2 at
complete bases against the full-CI eigenvalues of spin S (states of the
(N, 2S_z = 2S) sector with <S^2> = S(S+1), from oracle.fock), and at two
values of M; the scalar-product rule (with fermion signs) against the
operator built component by component on the Fock space; the 9j symbol
against its reduction to a 6j symbol when one entry is zero and against the
orthogonality of the recoupling matrix it defines; product_operator against
the coupled product built component by component on the Fock space, for
ranks 0, 1/2, 1 and 3/2 and particle changes 0, +-1, 2 (a dropped (2S + 1)
factor and a bra/ket exchange in the 9j symbol each fail it), and at k = 0
against scalar_coupling; product_operator followed by rotate_operator onto
a truncated spin-adapted basis of block x site against the reduced elements
of the Fock-space product between the kept multiplets; window_pairs
contracted by contract_scalar_products against heff_su2 (four windows of
four orbitals split 2 | 2; a phase error in the recoupling rule fails it).
"""
from math import factorial, sqrt

import numpy as np

from .fock import DetSpace


# ---- angular momentum algebra (doubled spins) --------------------------------
def _f(t2):
    """factorial of t2 / 2 (t2 even, >= 0)."""
    assert t2 % 2 == 0 and t2 >= 0, t2
    return factorial(t2 // 2)


def _triangle(ta, tb, tc):
    return abs(ta - tb) <= tc <= ta + tb and (ta + tb + tc) % 2 == 0


def clebsch_gordan(tj1, tm1, tj2, tm2, tJ, tM):
    """<j1 m1; j2 m2 | J M> (arguments doubled), Racah's formula."""
    if tm1 + tm2 != tM or not _triangle(tj1, tj2, tJ):
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    if (tj1 + tm1) % 2 or (tj2 + tm2) % 2 or (tJ + tM) % 2:
        return 0.0
    pre = (tJ + 1) * _f(tJ + tj1 - tj2) * _f(tJ - tj1 + tj2) * _f(tj1 + tj2 - tJ) / _f(tj1 + tj2 + tJ + 2)
    pre *= _f(tJ + tM) * _f(tJ - tM) * _f(tj1 - tm1) * _f(tj1 + tm1) * _f(tj2 - tm2) * _f(tj2 + tm2)
    s = 0.0
    for k in range(0, (tj1 + tj2 + tJ) // 2 + 1):
        d = (2 * k, tj1 + tj2 - tJ - 2 * k, tj1 - tm1 - 2 * k, tj2 + tm2 - 2 * k,
             tJ - tj2 + tm1 + 2 * k, tJ - tj1 - tm2 + 2 * k)
        if min(d) < 0:
            continue
        den = 1
        for x in d:
            den *= _f(x)
        s += (-1) ** k / den
    return sqrt(pre) * s


def _delta(ta, tb, tc):
    return sqrt(_f(ta + tb - tc) * _f(ta - tb + tc) * _f(-ta + tb + tc) / _f(ta + tb + tc + 2))


def wigner_6j(tj1, tj2, tj3, tj4, tj5, tj6):
    """{j1 j2 j3; j4 j5 j6} (arguments doubled), Racah's formula."""
    if not (_triangle(tj1, tj2, tj3) and _triangle(tj1, tj5, tj6) and _triangle(tj4, tj2, tj6)
            and _triangle(tj4, tj5, tj3)):
        return 0.0
    pre = _delta(tj1, tj2, tj3) * _delta(tj1, tj5, tj6) * _delta(tj4, tj2, tj6) * _delta(tj4, tj5, tj3)
    lo = max(tj1 + tj2 + tj3, tj1 + tj5 + tj6, tj4 + tj2 + tj6, tj4 + tj5 + tj3)
    hi = min(tj1 + tj2 + tj4 + tj5, tj2 + tj3 + tj5 + tj6, tj3 + tj1 + tj6 + tj4)
    s = 0.0
    for t2 in range(lo, hi + 1, 2):
        den = (_f(t2 - tj1 - tj2 - tj3) * _f(t2 - tj1 - tj5 - tj6) * _f(t2 - tj4 - tj2 - tj6)
               * _f(t2 - tj4 - tj5 - tj3) * _f(tj1 + tj2 + tj4 + tj5 - t2)
               * _f(tj2 + tj3 + tj5 + tj6 - t2) * _f(tj3 + tj1 + tj6 + tj4 - t2))
        s += (-1) ** (t2 // 2) * _f(t2 + 2) / den
    return pre * s


def scalar_coupling(tSa2, tSb2, tSa, tSb, tS, tk):
    """<(a' S_a', b' S_b') S M | [A^k x B^k]^0 | (a S_a, b S_b) S M> for unit
    reduced elements, without the fermion sign (closed form in the module
    docstring; primed spins first)."""
    ph = (tSa + tSb2 + tS + tk) // 2
    return (-1) ** ph * sqrt((tSa2 + 1) * (tSb2 + 1) / (tk + 1)) * wigner_6j(tSa, tSb, tS, tSb2, tSa2, tk)


def wigner_9j(tj1, tj2, tj3, tj4, tj5, tj6, tj7, tj8, tj9):
    """{j1 j2 j3; j4 j5 j6; j7 j8 j9} (arguments doubled) as the sum over x of
    (-1)^(2x) (2x + 1) {j1 j4 j7; j8 j9 x} {j2 j5 j8; j4 x j6} {j3 j6 j9; x j1 j2},
    the standard reduction of a 9j symbol to 6j symbols over the common
    index x (its range: the triangles (j1, j9, x), (j8, j4, x), (j2, j6, x))."""
    lo = max(abs(tj1 - tj9), abs(tj4 - tj8), abs(tj2 - tj6))
    hi = min(tj1 + tj9, tj4 + tj8, tj2 + tj6)
    s = 0.0
    for tx in range(lo, hi + 1, 2):
        s += ((-1) ** tx * (tx + 1) * wigner_6j(tj1, tj4, tj7, tj8, tj9, tx)
              * wigner_6j(tj2, tj5, tj8, tj4, tx, tj6) * wigner_6j(tj3, tj6, tj9, tx, tj1, tj2))
    return s


def product_coupling(tSa2, tSb2, tS2, tSa, tSb, tS, tk1, tk2, tk):
    """<(a' S_a', b' S_b') S' || [A^k1 x B^k2]^k || (a S_a, b S_b) S> for unit
    reduced elements of A (first subsystem) and B (second), in the
    Clebsch-Gordan convention of the reduced elements and without the
    fermion sign:
        sqrt((2S + 1)(2k + 1)(2S_a' + 1)(2S_b' + 1)) {S_a' S_a k1; S_b' S_b k2; S' S k}.
    (The tensor-product theorem for operators on two subsystems, restated
    from the 3j convention <j'||T||j>_3j = sqrt(2j' + 1) <j'||T||j>_CG; the
    phases (-1)^(2k) of that conversion cancel since k1 + k2 + k is an
    integer.  With k = 0 it is scalar_coupling.)"""
    return (sqrt((tS + 1) * (tk + 1) * (tSa2 + 1) * (tSb2 + 1))
            * wigner_9j(tSa2, tSa, tk1, tSb2, tSb, tk2, tS2, tS, tk))


def product_operator(sec1, sec2, t1, t2, tk1, tk2, tk, parity2):
    """Reduced blocks of [A^k1 x B^k2]^k on the coupled multiplets of two
    subsystems (the renormalisation of a block operator times a site
    operator).  sec1, sec2: the sectors (N, 2S, d) of the subsystems; t1, t2:
    reduced blocks {(out, in): matrix} of A and B; parity2: fermion parity of
    B (it passes the ket's N_1 electrons of the first subsystem).  A coupled
    sector is (i1, i2, 2S) with multiplets (alpha1, alpha2), alpha1 slowest;
    returns {((i1', i2', 2S'), (i1, i2, 2S)): matrix}."""
    out = {}
    for (i1p, i1), a in t1.items():
        for (i2p, i2), b in t2.items():
            n1, ts1 = sec1[i1][0], sec1[i1][1]
            ts2 = sec2[i2][1]
            tsa2, tsb2 = sec1[i1p][1], sec2[i2p][1]
            sign = -1.0 if (parity2 and n1 % 2) else 1.0
            for tS in range(abs(ts1 - ts2), ts1 + ts2 + 1, 2):
                for tS2 in range(abs(tsa2 - tsb2), tsa2 + tsb2 + 1, 2):
                    c = product_coupling(tsa2, tsb2, tS2, ts1, ts2, tS, tk1, tk2, tk)
                    if c == 0.0:
                        continue
                    key = ((i1p, i2p, tS2), (i1, i2, tS))
                    out[key] = out.get(key, 0.0) + sign * c * np.kron(a, b)
    return out


def rotate_operator(blocks, proj, group_of):
    """The renormalised reduced blocks: for coupled sectors cs grouped into
    new sectors g (group_of[cs], or -1 for a sector kept out) with kept
    multiplets spanned by the columns of proj[cs] (d_cs x D_g, the rows of
    U_g that belong to cs), O[g', g] = sum over blocks X[cs', cs] of
    proj[cs']^T X[cs', cs] proj[cs].  blocks: {(cs', cs): matrix};
    returns {(g', g): matrix}."""
    out = {}
    for (c2, c), x in blocks.items():
        g2, g = group_of[c2], group_of[c]
        if g2 < 0 or g < 0:
            continue
        y = proj[c2].T @ x @ proj[c]
        out[(g2, g)] = out.get((g2, g), 0.0) + y
    return out


# ---- multiplet bases of a block of orbitals ----------------------------------
def _sector(n_orb, n, t2m):
    try:
        return DetSpace.sector(n_orb, n, t2m)
    except ValueError:
        return None


def _s_plus(space_from, space_to):
    """S_+ = sum_i a+_{i up} a_{i dn} from (N, 2M) to (N, 2M + 2) (dense)."""
    m = np.zeros((space_to.dim, space_from.dim))
    for i in range(space_from.K):
        m += space_from.string_matrix([(2 * i, True), (2 * i + 1, False)], space_to).toarray()
    return m


class Multiplet:
    """The multiplets of one (N, S) of a block: vec[tM] is the (sector dim x
    D) matrix whose column alpha is the state |alpha S M> in the block's
    (N, 2M) determinant sector space[tM]."""

    def __init__(self, n, tS, space, vec):
        self.n, self.tS, self.space, self.vec = n, tS, space, vec

    @property
    def dim(self):
        return next(iter(self.vec.values())).shape[1]


def multiplets(n_orb, rng=None, keep=None):
    """All multiplets of a block of n_orb orbitals, by (N, S): the
    highest-weight states of each (N, 2S_z = 2S) sector (null space of S_+),
    then lowered.  With rng and keep, only min(keep, count) random orthonormal
    combinations of each (N, S) are kept (a truncated spin-adapted basis)."""
    out = []
    for n in range(0, 2 * n_orb + 1):
        for tS in range(n % 2, min(n, 2 * n_orb - n) + 1, 2):
            top = _sector(n_orb, n, tS)
            if top is None:
                continue
            up = _sector(n_orb, n, tS + 2)
            if up is None:
                hw = np.eye(top.dim)
            else:
                sp_ = _s_plus(top, up)
                u, sv, vt = np.linalg.svd(sp_)
                rank = int(np.sum(sv > 1e-10))
                hw = vt[rank:].T
            if hw.shape[1] == 0:
                continue
            if rng is not None and keep is not None:
                q, _ = np.linalg.qr(rng.normal(size=(hw.shape[1], hw.shape[1])))
                hw = hw @ q[:, :min(keep, hw.shape[1])]
            vec, space = {tS: hw}, {tS: top}
            cur, tM = hw, tS
            while tM > -tS:
                lower = _sector(n_orb, n, tM - 2)
                smin = _s_plus(lower, space[tM]).T  # S_- = S_+^T
                norm = sqrt((tS / 2) * (tS / 2 + 1) - (tM / 2) * (tM / 2 - 1))
                cur = smin @ cur / norm
                tM -= 2
                vec[tM], space[tM] = cur, lower
            out.append(Multiplet(n, tS, space, vec))
    return out


# ---- coupled states of two blocks and the spin-adapted H_eff -----------------
def coupled_basis(left, right, n, tS):
    """The coupled states (a, alpha, b, beta) of total N = n and spin S."""
    out = []
    for ia, A in enumerate(left):
        for ib, B in enumerate(right):
            if A.n + B.n != n or not _triangle(A.tS, B.tS, tS):
                continue
            for al in range(A.dim):
                for be in range(B.dim):
                    out.append((ia, al, ib, be))
    return out


def coupled_vectors(left, right, n_left, n_right, n, tS, tM, basis):
    """Fock vectors (columns) of the coupled states in the (n, 2M) sector of
    the n_left + n_right orbitals: sum_{M_a+M_b=M} CG |a M_a> |b M_b>, the
    left determinant in the low bits."""
    space = DetSpace.sector(n_left + n_right, n, tM)
    P = np.zeros((space.dim, len(basis)))
    shift = np.int64(2 * n_left)
    for c, (ia, al, ib, be) in enumerate(basis):
        A, B = left[ia], right[ib]
        for tMa in range(-A.tS, A.tS + 1, 2):
            tMb = tM - tMa
            if abs(tMb) > B.tS:
                continue
            cg = clebsch_gordan(A.tS, tMa, B.tS, tMb, tS, tM)
            if cg == 0.0:
                continue
            va, vb = A.vec[tMa][:, al], B.vec[tMb][:, be]
            da, db = A.space[tMa].dets, B.space[tMb].dets
            full = (da[:, None] | (db[None, :] << shift)).ravel()
            amp = (va[:, None] * vb[None, :]).ravel()
            P[space.index(full), c] += cg * amp
    return P, space


def heff_su2(h, eri, left, right, n_left, n_right, n, tS, tM=None):
    """The spin-adapted effective Hamiltonian <c'|H|c> over the coupled states
    of total spin S (at M = tM / 2, default S): the plain definition.
    Returns (matrix, basis)."""
    tM = tS if tM is None else tM
    basis = coupled_basis(left, right, n, tS)
    P, space = coupled_vectors(left, right, n_left, n_right, n, tS, tM, basis)
    H = space.hamiltonian(h, eri).toarray()
    return P.T @ H @ P, basis


def window_pairs(h, eri, left, right, n_left, n_right):
    """The window Hamiltonian as a sum of scalar products [U^k x V^k]^0 of a
    left and a right tensor operator, for complete multiplet bases of both
    blocks (an expansion over the left operator space, written out):

    * H on the n_left + n_right orbitals in the product basis |l>|r> (left
      determinant in the low bits) is sum over left basis states of
      |l'><l| (x) R(l', l), with R(l', l) = <l'| H |l> the right-block
      operator;
    * in the multiplet basis of the left block, |a' M'><a M| =
      sum over k of (2k + 1) / (2S_a' + 1) <S_a M; k q | S_a' M'> U^k_q,
      U^k the unit tensor with reduced element 1 between (a', alpha') and
      (a, alpha) (orthogonality of the Clebsch-Gordan coefficients over M);
    * so H = sum over (a' alpha', a alpha, k) of sum_q U^k_q W^k_q, and
      V^k_-q = W^k_q / <k q; k -q | 0 0> makes each term the scalar
      product [U^k x V^k]^0; V^k's reduced blocks on the right multiplets
      follow from one non-zero Clebsch-Gordan coefficient each.

    The products are taken in the product basis itself, so no fermion sign
    is added (parity 0).  Returns pairs (1, 2k, 0, {(a', a): unit block},
    {(b', b): reduced block of V^k}) for contract_scalar_products."""
    K = n_left + n_right
    H = DetSpace.full(K).hamiltonian(h, eri).toarray()
    dl, dr = 1 << (2 * n_left), 1 << (2 * n_right)
    H4 = H.reshape(dr, dl, dr, dl)  # [r', l', r, l]: index = l + dl r

    def state_vectors(mults, n_orb):
        full = DetSpace.full(n_orb)
        out = {}
        for i, M in enumerate(mults):
            for tM in range(-M.tS, M.tS + 1, 2):
                V = np.zeros((full.dim, M.dim))
                V[full.index(M.space[tM].dets)] = M.vec[tM]
                out[(i, tM)] = V
        return out

    lv, rv = state_vectors(left, n_left), state_vectors(right, n_right)
    pairs = []
    for ia2, A2 in enumerate(left):
        for ia, A in enumerate(left):
            for al2 in range(A2.dim):
                for al in range(A.dim):
                    for tk in range(abs(A2.tS - A.tS), A2.tS + A.tS + 1, 2):
                        V = {}
                        for tM in range(-A.tS, A.tS + 1, 2):
                            for tM2 in range(-A2.tS, A2.tS + 1, 2):
                                tq = tM2 - tM
                                if abs(tq) > tk:
                                    continue
                                cg = clebsch_gordan(A.tS, tM, tk, tq, A2.tS, tM2)
                                if cg == 0.0:
                                    continue
                                R = np.einsum("a,xayb,b->xy", lv[(ia2, tM2)][:, al2], H4, lv[(ia, tM)][:, al])
                                w = (tk + 1) / (A2.tS + 1) * cg / clebsch_gordan(tk, tq, tk, -tq, 0, 0)
                                V[-tq] = V.get(-tq, 0.0) + w * R
                        B = {}
                        for ib2, B2 in enumerate(right):
                            for ib, B1 in enumerate(right):
                                if not _triangle(B1.tS, tk, B2.tS):
                                    continue
                                pick = next(((tMb, tq) for tMb in range(-B1.tS, B1.tS + 1, 2)
                                             for tq in range(-tk, tk + 1, 2)
                                             if tq in V and abs(tMb + tq) <= B2.tS
                                             and abs(clebsch_gordan(B1.tS, tMb, tk, tq, B2.tS, tMb + tq)) > 1e-8),
                                            None)
                                if pick is None:
                                    continue
                                tMb, tq = pick
                                cg = clebsch_gordan(B1.tS, tMb, tk, tq, B2.tS, tMb + tq)
                                blk = rv[(ib2, tMb + tq)].T @ V[tq] @ rv[(ib, tMb)] / cg
                                if np.abs(blk).max() > 1e-13:
                                    B[(ib2, ib)] = blk
                        if B:
                            unit = np.zeros((A2.dim, A.dim))
                            unit[al2, al] = 1.0
                            pairs.append((1.0, tk, 0, {(ia2, ia): unit}, B))
    return pairs


def sigma_su2(h, eri, left, right, n_left, n_right, n, tS, psi):
    """H_eff psi for the reduced (spin-adapted) window vector psi."""
    m, _ = heff_su2(h, eri, left, right, n_left, n_right, n, tS)
    return m @ psi


# ---- the spin-adapted contraction ------------------------------------------
def coupled_blocks(left_sectors, right_sectors, n, tS):
    """The blocks (ia, ib) of a spin-adapted window vector: left sector ia =
    (N_a, 2S_a, d_a) and right sector ib with N_a + N_b = n and S in
    S_a x S_b; each block is a d_a x d_b matrix."""
    return [(ia, ib) for ia, (na, tsa, _) in enumerate(left_sectors)
            for ib, (nb, tsb, _) in enumerate(right_sectors)
            if na + nb == n and _triangle(tsa, tsb, tS)]


def contract_scalar_products(left_sectors, right_sectors, n, tS, psi, pairs):
    """sigma = sum over pairs (c, tk, parity_b, A, B) of c [A^k x B^k]^0 psi on
    the coupled blocks: A maps left sectors (blocks A[(ia2, ia)] of reduced
    matrix elements), B right sectors, psi and the result are dicts
    {(ia, ib): d_a x d_b matrix}.  Block by block:
        sigma[ia2, ib2] += c (-1)^(parity_b N_a) scalar_coupling(...)
                           A[ia2, ia] psi[ia, ib] B[ib2, ib]^T."""
    blocks = set(coupled_blocks(left_sectors, right_sectors, n, tS))
    out = {k: np.zeros((left_sectors[k[0]][2], right_sectors[k[1]][2])) for k in blocks}
    for c, tk, pb, A, B in pairs:
        for (ia2, ia), a in A.items():
            for (ib2, ib), b in B.items():
                if (ia, ib) not in blocks or (ia2, ib2) not in blocks:
                    continue
                coef = scalar_coupling(left_sectors[ia2][1], right_sectors[ib2][1], left_sectors[ia][1],
                                       right_sectors[ib][1], tS, tk)
                if coef == 0.0:
                    continue
                sign = -1.0 if (pb and left_sectors[ia][0] % 2) else 1.0
                out[(ia2, ib2)] += c * sign * coef * (a @ psi[(ia, ib)] @ b.T)
    return out
