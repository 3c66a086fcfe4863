"""Determinant (Fock) space, the ab initio Hamiltonian and full CI.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain definitions:

* Spin-orbitals in Jordan-Wigner order P = 2*i + s (s = 0 up, 1 down), i.e.
  (0up, 0dn, 1up, 1dn, ...), following the local basis of the Method section
  (|0>, |up>, |dn>, |updn>) with |updn> = a+_{i up} a+_{i dn} |vac>.
* A determinant is the bit string n (bit P set = P occupied) and stands for
  prod_{P ascending} (a+_P)^{n_P} |vac>; hence
  a_Q |n> = (-1)^{sum_{R<Q} n_R} |n - e_Q>, and likewise for a+_P.
  The site occupation n_i in {0,1,2,3} is exactly the 2-bit field of site i,
  so the integer of a determinant is sum_i n_i 4^i.
* H = sum_{pq,s} h_pq a+_{ps} a_{qs}
      + 1/2 sum_{pqrs,st} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
  (chemists' notation, the "model Hamiltonian" of the Method section with
  ab initio integrals).  With E_pq = sum_s a+_{ps} a_{qs} this equals
  sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - delta_qr E_ps), the form used
  below; tests pin it against the raw four-operator sum.
* FCI: lowest eigenvalue of H on the determinants with fixed (N, 2Sz).

* Reduced density matrices (transition form, <bra| . |ket>):
      gamma_pq   = sum_s <a+_{ps} a_{qs}>            = <E_pq>
      Gamma_pqrs = sum_{s,t} <a+_{ps} a+_{rt} a_{st} a_{qs}> = <E_pq E_rs> - delta_qr <E_ps>
  so that <bra|H|ket> = sum h_pq gamma_pq + 1/2 sum (pq|rs) Gamma_pqrs, i.e.
  gamma and Gamma / 2 are the derivatives of <bra|H|ket> with respect to the
  integral entries (each entry an independent input).

* Total spin: s_squared(space, v) = <S^2> from S_+ and S_z (definition in
  its docstring).  With the spin-summed 2-RDM above, any state of fixed N
  has <S^2> = -N (N - 4) / 4 - 1/2 sum_pq Gamma_pqqp (tests pin this
  identity on random vectors).

Pins: tests/test_oracle_fock.py (closed forms: g=0 orbital sums, two-site
Hubbard, K=1; [H,N]=[H,Sz]=0 on the full Fock space; the raw spin-orbital
Hamiltonian on tiny spaces); tests/test_oracle_rdm.py (single-determinant
closed form, contraction against the raw Hamiltonian, finite differences of
the raw Hamiltonian, trace and permutation identities).
"""
from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


class DetSpace:
    """Sorted list of determinants (int64 bit strings over 2K spin-orbitals)."""

    def __init__(self, n_orb, dets):
        self.K = int(n_orb)
        self.dets = np.asarray(np.sort(dets), dtype=np.int64)
        self.dim = len(self.dets)
        self._epq = {}

    @classmethod
    def sector(cls, n_orb, n_elec, two_sz):
        K = n_orb
        na, nb = (n_elec + two_sz) // 2, (n_elec - two_sz) // 2
        if (n_elec + two_sz) % 2 or na < 0 or nb < 0 or na > K or nb > K:
            raise ValueError("invalid sector")
        dets = []
        for ua in combinations(range(K), na):
            ma = sum(1 << (2 * i) for i in ua)
            for ub in combinations(range(K), nb):
                dets.append(ma | sum(1 << (2 * i + 1) for i in ub))
        return cls(K, np.array(dets, dtype=np.int64))

    @classmethod
    def full(cls, n_orb):
        return cls(n_orb, np.arange(1 << (2 * n_orb), dtype=np.int64))

    def index(self, dets):
        dets = np.asarray(dets, dtype=np.int64)
        pos = np.searchsorted(self.dets, dets)
        pos = np.minimum(pos, self.dim - 1)
        ok = self.dets[pos] == dets
        return np.where(ok, pos, -1)

    # ---- elementary operators -------------------------------------------
    def apply_string(self, ops, dets=None):
        """Apply an operator string to determinants.

        ops: list of (P, dagger) applied right-to-left as written, i.e. the
        operator product ops[0] ops[1] ... ops[-1].  Returns (new_dets,
        sign, alive) for every input determinant.
        """
        d = self.dets.copy() if dets is None else np.asarray(dets, np.int64).copy()
        sign = np.ones(len(d), dtype=np.int64)
        alive = np.ones(len(d), dtype=bool)
        for (P, dag) in reversed(ops):
            bit = np.int64(1) << np.int64(P)
            occ = (d & bit) != 0
            below = _popcount(d & (bit - 1))
            if dag:
                alive &= ~occ
                d = d | bit
            else:
                alive &= occ
                d = d & ~bit
            sign *= np.where(below % 2 == 1, -1, 1)
        return d, sign, alive

    def string_matrix(self, ops, target=None):
        """Sparse matrix of an operator string from this space to `target`."""
        target = self if target is None else target
        nd, sg, al = self.apply_string(ops)
        cols = np.nonzero(al)[0]
        rows = target.index(nd[cols])
        keep = rows >= 0
        return sp.csr_matrix((sg[cols][keep].astype(np.float64),
                              (rows[keep], cols[keep])),
                             shape=(target.dim, self.dim))

    def epq(self, p, q):
        key = (p, q)
        if key not in self._epq:
            m = self.string_matrix([(2 * p, True), (2 * q, False)])
            m = m + self.string_matrix([(2 * p + 1, True), (2 * q + 1, False)])
            self._epq[key] = m.tocsr()
        return self._epq[key]

    def number_op(self):
        return sp.diags(_popcount(self.dets).astype(np.float64))

    def sz2_op(self):
        mup = np.int64(sum(1 << (2 * i) for i in range(self.K)))
        up = _popcount(self.dets & mup)
        dn = _popcount(self.dets & (mup << np.int64(1)))
        return sp.diags((up - dn).astype(np.float64))

    # ---- Hamiltonian --------------------------------------------------------
    def hamiltonian(self, h, eri, e_core=0.0):
        """Sparse H on this space (spin-free E_pq form)."""
        K = self.K
        H = sp.csr_matrix((self.dim, self.dim))
        hp = h - 0.5 * np.einsum("prrq->pq", eri)
        for p in range(K):
            for q in range(K):
                if hp[p, q] != 0.0:
                    H = H + hp[p, q] * self.epq(p, q)
        for p in range(K):
            for q in range(K):
                F = sp.csr_matrix((self.dim, self.dim))
                for r in range(K):
                    for s in range(K):
                        if eri[p, q, r, s] != 0.0:
                            F = F + eri[p, q, r, s] * self.epq(r, s)
                H = H + 0.5 * (self.epq(p, q) @ F)
        if e_core:
            H = H + e_core * sp.identity(self.dim)
        return H.tocsr()

    def hamiltonian_matvec(self, h, eri):
        """Return a function c -> H c that never forms H (for larger K)."""
        K = self.K
        hp = h - 0.5 * np.einsum("prrq->pq", eri)
        E = [[self.epq(p, q) for q in range(K)] for p in range(K)]
        G = eri.reshape(K * K, K * K)

        def mv(c):
            c = np.asarray(c, dtype=np.float64).ravel()
            Ec = np.stack([E[r][s] @ c for r in range(K) for s in range(K)])
            W = G @ Ec
            out = np.zeros_like(c)
            for p in range(K):
                for q in range(K):
                    out += E[p][q] @ (hp[p, q] * c + 0.5 * W[p * K + q])
            return out
        return mv


def raw_hamiltonian(space, h, eri):
    """H built literally from spin-orbital four-operator strings (tiny K)."""
    K = space.K
    H = sp.csr_matrix((space.dim, space.dim))
    for p in range(K):
        for q in range(K):
            for s in (0, 1):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * space.string_matrix(
                        [(2 * p + s, True), (2 * q + s, False)])
    for p in range(K):
        for q in range(K):
            for r in range(K):
                for s_ in range(K):
                    g = eri[p, q, r, s_]
                    if g == 0.0:
                        continue
                    for a in (0, 1):
                        for b in (0, 1):
                            H = H + 0.5 * g * space.string_matrix(
                                [(2 * p + a, True), (2 * r + b, True),
                                 (2 * s_ + b, False), (2 * q + a, False)])
    return H.tocsr()


def fci(n_orb, n_elec, two_sz, h, eri, nroots=1, dense_limit=6000):
    """Lowest eigenpair(s) of H in the (N, 2Sz) determinant sector."""
    space = DetSpace.sector(n_orb, n_elec, two_sz)
    if space.dim <= dense_limit:
        H = space.hamiltonian(h, eri).toarray()
        w, v = np.linalg.eigh(H)
        return w[:nroots], v[:, :nroots], space
    mv = space.hamiltonian_matvec(h, eri)
    op = spla.LinearOperator((space.dim, space.dim), matvec=mv, dtype=np.float64)
    rng = np.random.default_rng(0)
    w, v = spla.eigsh(op, k=max(nroots, 2), which="SA", tol=1e-12,
                      v0=rng.normal(size=space.dim), maxiter=5000)
    o = np.argsort(w)
    return w[o][:nroots], v[:, o][:, :nroots], space


def s_squared(space, vec):
    """<S^2> of a vector of the (N, 2Sz) sector `space`, from the spin-orbital
    definition S^2 = S_- S_+ + S_z (S_z + 1), S_+ = sum_i a+_{i up} a_{i dn},
    S_- = S_+^T: S_+ maps the sector into (N, 2Sz + 2), and
    <S_- S_+> = |S_+ v|^2.  Normalised by |v|^2."""
    vec = np.asarray(vec, dtype=np.float64)
    n_elec = int(_popcount(space.dets[:1])[0])
    mup = np.int64(sum(1 << (2 * i) for i in range(space.K)))
    d0 = space.dets[:1]
    two_sz = int(_popcount(d0 & mup)[0] - _popcount(d0 & (mup << np.int64(1)))[0])
    sz = two_sz / 2.0
    norm2 = float(vec @ vec)
    val = sz * (sz + 1.0) * norm2
    try:
        target = DetSpace.sector(space.K, n_elec, two_sz + 2)
    except ValueError:
        return val / norm2
    w = np.zeros(target.dim)
    for i in range(space.K):
        w += space.string_matrix([(2 * i, True), (2 * i + 1, False)], target) @ vec
    return (val + float(w @ w)) / norm2


def rdm12(space, bra, ket):
    """Transition 1- and 2-RDM of two vectors of `space` (definitions above).

    Returns gamma (K, K) and Gamma (K, K, K, K) with
    gamma[p, q] = <bra|E_pq|ket> and
    Gamma[p, q, r, s] = <bra|E_pq E_rs|ket> - delta_qr <bra|E_ps|ket>.
    """
    K = space.K
    bra = np.asarray(bra, dtype=np.float64).ravel()
    ket = np.asarray(ket, dtype=np.float64).ravel()
    # <bra|E_pq = (E_qp|bra>)^T since E_pq^T = E_qp
    B = np.stack([space.epq(q, p) @ bra for p in range(K) for q in range(K)])
    C = np.stack([space.epq(r, s) @ ket for r in range(K) for s in range(K)])
    gamma = (B @ ket).reshape(K, K)
    Gamma = (B @ C.T).reshape(K, K, K, K)
    for q in range(K):
        Gamma[:, q, q, :] -= gamma
    return gamma, Gamma
