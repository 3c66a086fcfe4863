"""Block-sparse renormalised operators and the two-site sigma (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  This is the standard ab initio DMRG sigma step
(White-Martin 1999; Chan-Head-Gordon 2002), which the paper runs as its
"DMRG matrix and tensor algebra" (Hardware specific implementations) on the
MPS of eq. (1).  It is written here as plainly as possible: block operators
are dicts of dense sector blocks, an enlarged block (renormalised block plus
one site) is built explicitly from Kronecker products, and the sigma is the
sum of the partition terms below applied to psi.  Nothing is fused.

Spin-orbitals p = 2*i + s; t_pq = h_ij delta_{s s'}; and
V_pqrs = (ps|qr) delta_{s_p s_s} delta_{s_q s_r}, so that
H = sum t_pq a+_p a_q + 1/2 sum V_pqrs a+_p a+_q a_r a_s.
For a cut of the orbitals into a left part Lt and a right part Rt
(Lt first in Jordan-Wigner order):

  H = H^Lt (x) 1 + 1 (x) H^Rt
    + sum_{p in Lt} [a+_p S_p - a_p S_p^+]
    + sum_{m in Rt} [T_m a_m - T_m^+ a+_m]
    + sum_{p<q in Lt} [a+_p a+_q P_pq + a_q a_p P_pq^+]
    + sum_{p,q in Lt} a+_p a_q Q_pq
  S_p  = sum_{l in Rt} t_pl a_l + sum_{k,l,m in Rt} V_pklm a+_k a_l a_m
  T_m  = sum_{i,j,k in Lt} V_ijkm a+_i a+_j a_k
  P_pq = sum_{k,l in Rt} V_pqkl a_k a_l
  Q_pq = sum_{k,l in Rt} (V_pklq - V_pkql) a+_k a_l

A matrix element <l' r'| O_Lt O_Rt |l r> is O_Lt[l',l] O_Rt[r',r]
(-1)^{parity(O_Rt) N(l)} (Jordan-Wigner string of the ket's left part).

Left blocks (sites 0..j-1) keep H, a+_p, a+_p a+_q, a+_p a_q for p, q inside
and T_m for every m outside; right blocks (sites j..K-1) keep H, a+_m for m
inside and S_p, P_pq, Q_pq for p, q outside.  Enlarging a block by one site
and projecting with the site tensor gives the next block (the renormalisation
recursion); at the two-site window the enlarged blocks Lt = L + site i and
Rt = site i+1 + R enter the partition above.

Quantum numbers: left blocks use the bond label (N, 2Sz of the left part);
right blocks use their own (N, 2Sz); both are related by Q_tot.

Pins: equals the plain projection P^T H P psi of projection.py to 1e-12
(relative) at K <= 8 over several windows (tests/test_oracle_blocksparse.py).
"""
import numpy as np

QN = ((0, 0), (1, 1), (1, -1), (2, 0))


# --------------------------------------------------------------------------
# site operators (basis |0>, |up>, |dn>, |updn> = a+_up a+_dn |0>)
def _site_ops():
    cu = np.zeros((4, 4))
    cu[1, 0] = 1.0
    cu[3, 2] = 1.0
    cd = np.zeros((4, 4))
    cd[2, 0] = 1.0
    cd[3, 1] = -1.0
    return {0: cu, 1: cd}


SITE_CDAG = _site_ops()
SITE_C = {s: m.T.copy() for s, m in SITE_CDAG.items()}
I4 = np.eye(4)
SITE_N = np.array([0, 1, 1, 2])


def spin_orbital_integrals(h, eri):
    """t (2K x 2K) and V (2K)^4 in the convention of the module docstring."""
    K = h.shape[0]
    M = 2 * K
    sp = np.arange(M) % 2
    orb = np.arange(M) // 2
    t = h[orb[:, None], orb[None, :]] * (sp[:, None] == sp[None, :])
    # V_pqrs = (ps|qr) d(s_p,s_s) d(s_q,s_r)
    V = eri[orb[:, None, None, None], orb[None, None, None, :],
            orb[None, :, None, None], orb[None, None, :, None]]
    V = V * (sp[:, None, None, None] == sp[None, None, None, :])
    V = V * (sp[None, :, None, None] == sp[None, None, :, None])
    return np.ascontiguousarray(t), np.ascontiguousarray(V)


# --------------------------------------------------------------------------
class Basis:
    """Sorted list of sectors (qn -> dim)."""

    def __init__(self, sectors):
        sectors = sorted((tuple(q), int(d)) for q, d in sectors)
        self.qn = [q for q, d in sectors]
        self.dim = [d for q, d in sectors]
        self.idx = {q: k for k, q in enumerate(self.qn)}

    def __len__(self):
        return len(self.qn)


class Op:
    """Block-sparse real matrix with a definite quantum-number change dq."""

    def __init__(self, dq, blocks=None):
        self.dq = (int(dq[0]), int(dq[1]))
        self.blocks = {} if blocks is None else blocks

    @property
    def parity(self):
        return self.dq[0] % 2

    @property
    def T(self):
        return Op((-self.dq[0], -self.dq[1]),
                  {(b, a): m.T.copy() for (a, b), m in self.blocks.items()})

    def scaled(self, c):
        return Op(self.dq, {k: c * m for k, m in self.blocks.items()})

    def add_(self, other, c=1.0):
        if other is None or not other.blocks:
            return self
        assert other.dq == self.dq, (other.dq, self.dq)
        for k, m in other.blocks.items():
            if k in self.blocks:
                self.blocks[k] = self.blocks[k] + c * m
            else:
                self.blocks[k] = c * m
        return self

    def __add__(self, other):
        out = Op(self.dq, dict(self.blocks))
        return out.add_(other)

    def norm(self):
        return float(np.sqrt(sum(np.sum(m * m) for m in self.blocks.values())))


EMPTY = Op((0, 0))  # stands for an operator with no allowed blocks


class Stack:
    """A fixed list of operators, stacked per block so that linear
    combinations cost one tensordot per block (same sums as lincomb)."""

    def __init__(self, ops):
        self.n = len(ops)
        per = {}
        for k, o in enumerate(ops):
            if o is None or not o.blocks:
                continue
            for key, m in o.blocks.items():
                per.setdefault(key, []).append((k, m))
        self.keys = {}
        for key, lst in per.items():
            idx = np.array([k for k, m in lst])
            self.keys[key] = (idx, np.stack([m for k, m in lst]))

    def comb(self, coeffs, dq):
        coeffs = np.asarray(coeffs, dtype=np.float64)
        out = Op(dq)
        if not np.any(coeffs):
            return out
        for key, (idx, st) in self.keys.items():
            c = coeffs[idx]
            if np.any(c):
                out.blocks[key] = np.tensordot(c, st, axes=1)
        return out


def lincomb(ops, coeffs, dq):
    """sum_k coeffs[k] ops[k] (all with change dq); zero entries skipped."""
    out = Op(dq)
    for o, c in zip(ops, coeffs):
        if c != 0.0 and o is not None and o.blocks:
            out.add_(o, c)
    return out


def qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def qsub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def site_dq(m):
    """Quantum-number change of a 4x4 site matrix (assumed definite)."""
    nz = np.argwhere(np.abs(m) > 0)
    if len(nz) == 0:
        return None
    r, c = nz[0]
    return qsub(QN[r], QN[c])


# --------------------------------------------------------------------------
class Enlarged:
    """Product basis block (x) site (left) or site (x) block (right)."""

    def __init__(self, basis, side):
        self.side = side
        self.base = basis
        groups = {}
        if side == "left":
            for a, q in enumerate(basis.qn):
                for n in range(4):
                    groups.setdefault(qadd(q, QN[n]), []).append((a, n))
        else:
            for n in range(4):
                for a, q in enumerate(basis.qn):
                    groups.setdefault(qadd(QN[n], q), []).append((n, a))
        self.qn = sorted(groups)
        self.idx = {q: k for k, q in enumerate(self.qn)}
        self.offset = {}
        self.dim = []
        for k, q in enumerate(self.qn):
            o = 0
            for item in groups[q]:
                self.offset[item] = (k, o)
                o += basis.dim[item[0] if side == "left" else item[1]]
            self.dim.append(o)

    def kron(self, X, y, coef=1.0, out=None):
        """Enlarged operator of (X on the block) and (y on the site).

        left:  [(l',n'),(l,n)] = X[l',l] y[n',n] (-1)^{par(y) N(l)}
        right: [(n',r'),(n,r)] = y[n',n] X[r',r] (-1)^{par(X) N(n)}
        X=None means the block identity.
        """
        base = self.base
        if X is None:
            xdq = (0, 0)
            xblocks = {(a, a): np.eye(base.dim[a]) for a in range(len(base))}
        else:
            xdq = X.dq
            xblocks = X.blocks
        ydq = site_dq(y)
        if ydq is None or not xblocks:
            return out if out is not None else None
        dq = qadd(xdq, ydq)
        if out is None:
            out = Op(dq)
        assert out.dq == dq, (out.dq, dq)
        ypar = ydq[0] % 2
        xpar = xdq[0] % 2
        nz = np.argwhere(np.abs(y) > 0)
        for (a, b), m in xblocks.items():
            for (n1, n0) in nz:
                v = coef * y[n1, n0]
                if self.side == "left":
                    if ypar and (base.qn[b][0] % 2):
                        v = -v
                    kr, orow = self.offset[(a, n1)]
                    kc, ocol = self.offset[(b, n0)]
                else:
                    if xpar and (SITE_N[n0] % 2):
                        v = -v
                    kr, orow = self.offset[(n1, a)]
                    kc, ocol = self.offset[(n0, b)]
                blk = out.blocks.get((kr, kc))
                if blk is None:
                    blk = np.zeros((self.dim[kr], self.dim[kc]))
                    out.blocks[(kr, kc)] = blk
                blk[orow:orow + m.shape[0], ocol:ocol + m.shape[1]] += v * m
        return out


def _acc(ops, key, op):
    if op is None or not op.blocks:
        return
    if key in ops and ops[key] is not None:
        ops[key].add_(op)
    else:
        ops[key] = op


# --------------------------------------------------------------------------
def enlarge_left(env, j, t, V):
    """Operators of Lambda' = Lambda + site j from those of Lambda (sites < j).

    env: {"basis": Basis, "H": Op, ("C",p): Op, ("A",p,q): Op, ("B",p,q): Op,
          ("T",m): Op}.  Returns (Enlarged, ops on the enlarged basis).
    Each term is written as (block part)(site part) in Jordan-Wigner order;
    the reordering signs are stated next to each line.
    """
    E = Enlarged(env["basis"], "left")
    M = t.shape[0]
    inner = list(range(2 * j))
    site = [2 * j, 2 * j + 1]
    outer = list(range(2 * j + 2, M))
    cd, c = SITE_CDAG, SITE_C
    g = lambda key: env.get(key) or EMPTY
    out = {}
    # a+_p
    for p in inner:
        out[("C", p)] = E.kron(g(("C", p)), I4)
    for p in site:
        out[("C", p)] = E.kron(None, cd[p % 2])
    # a+_p a+_q (p<q)
    for p in inner:
        for q in inner:
            if p < q:
                out[("A", p, q)] = E.kron(g(("A", p, q)), I4)
        for q in site:
            out[("A", p, q)] = E.kron(g(("C", p)), cd[q % 2])
    out[("A", site[0], site[1])] = E.kron(None, cd[0] @ cd[1])
    # a+_p a_q
    for p in inner:
        for q in inner:
            out[("B", p, q)] = E.kron(g(("B", p, q)), I4)
        for q in site:
            out[("B", p, q)] = E.kron(g(("C", p)), c[q % 2])
            # a+_q a_p = - a_p a+_q
            out[("B", q, p)] = E.kron(g(("C", p)).T, cd[q % 2], coef=-1.0)
    for p in site:
        for q in site:
            out[("B", p, q)] = E.kron(None, cd[p % 2] @ c[q % 2])
    # T_m for m outside Lambda'
    Aops = {(p, q): g(("A", p, q)) for p in inner for q in inner if p < q}
    Bops = {(p, q): g(("B", p, q)) for p in inner for q in inner}
    Cops = {p: g(("C", p)) for p in inner}
    Akeys, Bkeys = list(Aops), list(Bops)
    Ast = Stack([Aops[k] for k in Akeys])
    Bst = Stack([Bops[k] for k in Bkeys])
    Cst = Stack([Cops[p] for p in inner])
    CTst = Stack([Cops[p].T for p in inner])
    for m in outer:
        sm = m % 2
        dqT = (1, 1 if sm == 0 else -1)
        T = Op(qadd(dqT, (0, 0)))
        if g(("T", m)) is not None:
            T.add_(E.kron(g(("T", m)), I4) or Op(dqT))
        for k in site:
            # (i,j in Lambda, k on site): a+_i a+_j a_k, i<j with V_ijkm - V_jikm
            X = Ast.comb([V[p, q, k, m] - V[q, p, k, m] for (p, q) in Akeys],
                         qsub(dqT, site_dq(c[k % 2])))
            if X.blocks:
                T.add_(E.kron(X, c[k % 2]))
        for jj in site:
            # (i in Lambda, j on site, k in Lambda): a+_i a+_j a_k = -a+_i a_k a+_j
            X = Bst.comb([-V[p, jj, q, m] for (p, q) in Bkeys],
                         qsub(dqT, site_dq(cd[jj % 2])))
            if X.blocks:
                T.add_(E.kron(X, cd[jj % 2]))
            # (i on site, j,k in Lambda): a+_i a+_j a_k = +a+_j a_k a+_i
            X = Bst.comb([V[jj, p, q, m] for (p, q) in Bkeys],
                         qsub(dqT, site_dq(cd[jj % 2])))
            if X.blocks:
                T.add_(E.kron(X, cd[jj % 2]))
        for a_ in site:
            for b_ in site:
                # (i in Lambda; j,k on site): a+_i (a+_j a_k)
                y = cd[a_ % 2] @ c[b_ % 2]
                if site_dq(y) is not None:
                    X = Cst.comb([V[p, a_, b_, m] for p in inner], qsub(dqT, site_dq(y)))
                    if X.blocks:
                        T.add_(E.kron(X, y))
                # (j in Lambda; i,k on site): a+_i a+_j a_k = -a+_j a+_i a_k
                if site_dq(y) is not None:
                    X = Cst.comb([-V[a_, p, b_, m] for p in inner], qsub(dqT, site_dq(y)))
                    if X.blocks:
                        T.add_(E.kron(X, y))
                # (k in Lambda; i,j on site): a+_i a+_j a_k = +a_k a+_i a+_j
                y2 = cd[a_ % 2] @ cd[b_ % 2]
                if site_dq(y2) is not None:
                    X = CTst.comb([V[a_, b_, p, m] for p in inner], qsub(dqT, site_dq(y2)))
                    if X.blocks:
                        T.add_(E.kron(X, y2))
        ysss = np.zeros((4, 4))
        for a_ in site:
            for b_ in site:
                for d_ in site:
                    ysss += V[a_, b_, d_, m] * (cd[a_ % 2] @ cd[b_ % 2] @ c[d_ % 2])
        if site_dq(ysss) is not None:
            T.add_(E.kron(None, ysss))
        out[("T", m)] = T
    # H of Lambda'
    H = Op((0, 0))
    if g("H") is not None and g("H").blocks:
        H.add_(E.kron(g("H"), I4))
    hs = _site_hamiltonian(j, t, V)
    H.add_(E.kron(None, hs))
    X = Op((0, 0))   # sum_{p in Lambda} a+_p S^site_p
    for p in inner:
        Sp = sum(t[p, l] * c[l % 2] for l in site)
        for k in site:
            for l in site:
                for m in site:
                    Sp = Sp + V[p, k, l, m] * (cd[k % 2] @ c[l % 2] @ c[m % 2])
        if Cops[p] is not None and site_dq(Sp) is not None:
            X.add_(E.kron(Cops[p], Sp))
    H.add_(X).add_(X.T)
    Y = Op((0, 0))   # sum_{m on site} T^Lambda_m a_m
    for m in site:
        if g(("T", m)) is not None and g(("T", m)).blocks:
            Y.add_(E.kron(g(("T", m)), c[m % 2]))
    H.add_(Y).add_(Y.T)
    Z = Op((0, 0))   # sum_{p<q in Lambda} a+_p a+_q P^site_pq
    for (p, q), A in Aops.items():
        Pp = V[p, q, site[0], site[1]] * (c[0] @ c[1]) + V[p, q, site[1], site[0]] * (c[1] @ c[0])
        if A is not None and A.blocks and site_dq(Pp) is not None:
            Z.add_(E.kron(A, Pp))
    H.add_(Z).add_(Z.T)
    for (p, q), B in Bops.items():   # sum_{p,q in Lambda} a+_p a_q Q^site_pq
        Qs = np.zeros((4, 4))
        for k in site:
            for l in site:
                Qs += (V[p, k, l, q] - V[p, k, q, l]) * (cd[k % 2] @ c[l % 2])
        if B is not None and B.blocks and site_dq(Qs) is not None:
            H.add_(E.kron(B, Qs))
    out["H"] = H
    return E, {k: v for k, v in out.items() if v is not None}


def enlarge_right(env, j, t, V):
    """Operators of R' = site j + R from those of R (sites > j)."""
    E = Enlarged(env["basis"], "right")
    M = t.shape[0]
    inner = list(range(2 * j + 2, M))
    site = [2 * j, 2 * j + 1]
    outer = list(range(0, 2 * j))
    cd, c = SITE_CDAG, SITE_C
    g = lambda key: env.get(key) or EMPTY
    Cops = {m: g(("C", m)) for m in inner}
    Cst = Stack([Cops[m] for m in inner])
    CTst = Stack([Cops[m].T for m in inner])
    out = {}
    for m in inner:
        out[("C", m)] = E.kron(Cops[m], I4) if Cops[m] is not None else None
    for m in site:
        out[("C", m)] = E.kron(None, cd[m % 2])

    def dqa(m):  # change of a_m
        return (-1, -1 if m % 2 == 0 else 1)

    def dqc(m):
        return (1, 1 if m % 2 == 0 else -1)

    def Pget(p, q):
        if p < q:
            return g(("P", p, q)), 1.0
        return g(("P", q, p)), -1.0

    for p in outer:
        dqS = dqa(p)
        S = Op(dqS)
        if g(("S", p)) is not None and g(("S", p)).blocks:
            S.add_(E.kron(g(("S", p)), I4))
        for l in site:
            if t[p, l] != 0.0:
                S.add_(E.kron(None, c[l % 2], coef=t[p, l]))
        for k in site:  # a+_k (sum_{lm in R} V_pklm a_l a_m) = a+_k P_pk
            P, sg = Pget(p, k)
            if P is not None and P.blocks:
                S.add_(E.kron(P, cd[k % 2], coef=sg))
        for x in site:  # a_x Q_px
            Q = g(("Q", p, x))
            if Q is not None and Q.blocks:
                S.add_(E.kron(Q, c[x % 2]))
        for k in site:
            for l in site:
                # (k,l on site, m in R): a+_k a_l a_m
                y = cd[k % 2] @ c[l % 2]
                if site_dq(y) is not None:
                    X = CTst.comb([V[p, k, l, m] for m in inner],
                                qsub(dqS, site_dq(y)))
                    if X.blocks:
                        S.add_(E.kron(X, y))
                # (k on site, l in R, m on site): a+_k a_l a_m = -a+_k a_m a_l
                y = cd[k % 2] @ c[l % 2]
                if site_dq(y) is not None:
                    X = CTst.comb([-V[p, k, m, l] for m in inner],
                                qsub(dqS, site_dq(y)))
                    if X.blocks:
                        S.add_(E.kron(X, y))
                # (k in R; l,m on site): a+_k a_l a_m = +a_l a_m a+_k
                y = c[k % 2] @ c[l % 2]
                if site_dq(y) is not None:
                    X = Cst.comb([V[p, m, k, l] for m in inner],
                                qsub(dqS, site_dq(y)))
                    if X.blocks:
                        S.add_(E.kron(X, y))
        ysss = np.zeros((4, 4))
        for k in site:
            for l in site:
                for m in site:
                    ysss += V[p, k, l, m] * (cd[k % 2] @ c[l % 2] @ c[m % 2])
        if site_dq(ysss) is not None:
            S.add_(E.kron(None, ysss))
        out[("S", p)] = S
    for p in outer:
        for q in outer:
            # Q_pq with W_kl = V_pklq - V_pkql
            dqQ = qsub(dqc(q), dqc(p))   # opposite of a+_p a_q
            Q = Op(dqQ)
            if g(("Q", p, q)) is not None and g(("Q", p, q)).blocks:
                Q.add_(E.kron(g(("Q", p, q)), I4))
            W = lambda k, l: V[p, k, l, q] - V[p, k, q, l]
            for k in site:
                X = CTst.comb([W(k, l) for l in inner],
                            qsub(dqQ, site_dq(cd[k % 2])))
                if X.blocks:
                    Q.add_(E.kron(X, cd[k % 2]))
            for l in site:  # a+_k a_l = -a_l a+_k
                X = Cst.comb([-W(k, l) for k in inner],
                            qsub(dqQ, site_dq(c[l % 2])))
                if X.blocks:
                    Q.add_(E.kron(X, c[l % 2]))
            ys = np.zeros((4, 4))
            for k in site:
                for l in site:
                    ys += W(k, l) * (cd[k % 2] @ c[l % 2])
            if site_dq(ys) is not None:
                Q.add_(E.kron(None, ys))
            out[("Q", p, q)] = Q
            if p < q:
                dqP = qadd(dqa(p), dqa(q))
                P = Op(dqP)
                if g(("P", p, q)) is not None and g(("P", p, q)).blocks:
                    P.add_(E.kron(g(("P", p, q)), I4))
                for k in site:  # a_k a_l
                    X = CTst.comb([V[p, q, k, l] for l in inner],
                                qsub(dqP, site_dq(c[k % 2])))
                    if X.blocks:
                        P.add_(E.kron(X, c[k % 2]))
                for l in site:  # a_k a_l = -a_l a_k
                    X = CTst.comb([-V[p, q, k, l] for k in inner],
                                qsub(dqP, site_dq(c[l % 2])))
                    if X.blocks:
                        P.add_(E.kron(X, c[l % 2]))
                ys = V[p, q, site[0], site[1]] * (c[0] @ c[1]) + V[p, q, site[1], site[0]] * (c[1] @ c[0])
                if site_dq(ys) is not None:
                    P.add_(E.kron(None, ys))
                out[("P", p, q)] = P
    # H of R'
    H = Op((0, 0))
    if g("H") is not None and g("H").blocks:
        H.add_(E.kron(g("H"), I4))
    H.add_(E.kron(None, _site_hamiltonian(j, t, V)))
    X = Op((0, 0))  # sum_{p on site} a+_p S^R_p
    for p in site:
        Sp = g(("S", p))
        if Sp is not None and Sp.blocks:
            X.add_(E.kron(Sp, cd[p % 2]))
    H.add_(X).add_(X.T)
    Y = Op((0, 0))  # sum_{m in R} T^site_m a_m
    for a_ in site:
        for b_ in site:
            for d_ in site:
                y = cd[a_ % 2] @ cd[b_ % 2] @ c[d_ % 2]
                if site_dq(y) is None:
                    continue
                Xs = CTst.comb([V[a_, b_, d_, m] for m in inner],
                             qsub((0, 0), site_dq(y)))
                if Xs.blocks:
                    Y.add_(E.kron(Xs, y))
    H.add_(Y).add_(Y.T)
    P = g(("P", site[0], site[1]))
    if P is not None and P.blocks:
        Z = E.kron(P, cd[0] @ cd[1])
        H.add_(Z).add_(Z.T)
    for p in site:
        for q in site:
            Q = g(("Q", p, q))
            if Q is not None and Q.blocks:
                H.add_(E.kron(Q, cd[p % 2] @ c[q % 2]))
    out["H"] = H
    return E, {k: v for k, v in out.items() if v is not None}


def _site_hamiltonian(j, t, V):
    cd, c = SITE_CDAG, SITE_C
    s = [2 * j, 2 * j + 1]
    hs = np.zeros((4, 4))
    for p in s:
        for q in s:
            hs += t[p, q] * (cd[p % 2] @ c[q % 2])
    for p in s:
        for q in s:
            for r in s:
                for u in s:
                    hs += 0.5 * V[p, q, r, u] * (cd[p % 2] @ cd[q % 2] @ c[r % 2] @ c[u % 2])
    return hs


# --------------------------------------------------------------------------
def _project_left(E, ops, site_blocks, bond_next):
    """O'[r',r] = A^T O A with A rows ordered as the enlarged sector."""
    newb = Basis([((s[0], s[1]), s[2]) for s in bond_next])
    Amat = {}
    for k, q in enumerate(E.qn):
        if q not in newb.idx:
            continue
        ri = newb.idx[q]
        Amat[k] = (ri, np.zeros((E.dim[k], newb.dim[ri])))
    for (a, n), blk in site_blocks.items():
        k, o = E.offset[(a, n)]
        if k in Amat:
            Amat[k][1][o:o + blk.shape[0], :] = blk
    env = {"basis": newb}
    for key, op in ops.items():
        new = Op(op.dq)
        for (kr, kc), m in op.blocks.items():
            if kr in Amat and kc in Amat:
                rr, Ar = Amat[kr]
                cc, Ac = Amat[kc]
                new.blocks[(rr, cc)] = Ar.T @ m @ Ac
        env[key] = new
    return env


def _project_right(E, ops, site_blocks, bond_this, bond_next, q_tot):
    """O'[l',l] = B O B^T; right blocks use their own quantum numbers."""
    own = lambda s: (q_tot[0] - s[0], q_tot[1] - s[1])
    newb = Basis([(own(s), s[2]) for s in bond_this])
    nxt = [own(s) for s in bond_next]
    nxt_basis = E.base
    Bmat = {}
    for li, s in enumerate(bond_this):
        q = own(s)
        if q not in E.idx:
            continue
        k = E.idx[q]
        Bmat[k] = (newb.idx[q], np.zeros((s[2], E.dim[k])))
    for (li, n), blk in site_blocks.items():
        q = own(bond_this[li])
        k = E.idx[q]
        # column r of the block: right sector of bond_next with bond label Q_l + Q_n
        rq = (bond_this[li][0] + QN[n][0], bond_this[li][1] + QN[n][1])
        rown = (q_tot[0] - rq[0], q_tot[1] - rq[1])
        a = nxt_basis.idx[rown]
        kk, o = E.offset[(n, a)]
        assert kk == k
        Bmat[k][1][:, o:o + blk.shape[1]] = blk
    env = {"basis": newb}
    for key, op in ops.items():
        new = Op(op.dq)
        for (kr, kc), m in op.blocks.items():
            if kr in Bmat and kc in Bmat:
                rr, Br = Bmat[kr]
                cc, Bc = Bmat[kc]
                new.blocks[(rr, cc)] = Br @ m @ Bc.T
        env[key] = new
    return env


def left_environment(mps, t, V, upto):
    """Block operators of sites 0..upto-1 at bond `upto`."""
    env = {"basis": Basis([((0, 0), 1)]), "H": Op((0, 0))}
    for j in range(upto):
        E, ops = enlarge_left(env, j, t, V)
        env = _project_left(E, ops, mps.sites[j], mps.bonds[j + 1])
    return env


def right_environment(mps, t, V, start):
    """Block operators of sites start..K-1 at bond `start` (own quantum numbers)."""
    K = mps.n_orb
    q_tot = (mps.n_elec, mps.two_sz)
    env = {"basis": Basis([((0, 0), 1)]), "H": Op((0, 0))}
    for j in range(K - 1, start - 1, -1):
        E, ops = enlarge_right(env, j, t, V)
        env = _project_right(E, ops, mps.sites[j], mps.bonds[j], mps.bonds[j + 1], q_tot)
    return env


class BlockSparseSigma:
    """sigma = H_eff psi at window (i, i+1) through the partition above."""

    def __init__(self, mps, h, eri, left_env=None, right_env=None):
        self.mps = mps
        self.t, self.V = spin_orbital_integrals(np.asarray(h), np.asarray(eri))
        i = mps.window
        self.Lenv = left_env if left_env is not None else left_environment(mps, self.t, self.V, i)
        self.Renv = right_env if right_env is not None else right_environment(mps, self.t, self.V, i + 2)
        self.EL, self.OL = enlarge_left(self.Lenv, i, self.t, self.V)
        self.ER, self.OR = enlarge_right(self.Renv, i + 1, self.t, self.V)
        self.q_tot = (mps.n_elec, mps.two_sz)
        self.terms = self._terms()

    def _terms(self):
        i = self.mps.window
        Lt = list(range(0, 2 * i + 2))
        Rt = list(range(2 * i + 2, self.t.shape[0]))
        OL, OR = self.OL, self.OR
        terms = [(1.0, OL["H"], None), (1.0, None, OR["H"])]
        for p in Lt:
            C, S = OL.get(("C", p)), OR.get(("S", p))
            if C is not None and S is not None:
                terms.append((1.0, C, S))
                terms.append((-1.0, C.T, S.T))
        for m in Rt:
            T, C = OL.get(("T", m)), OR.get(("C", m))
            if T is not None and C is not None:
                terms.append((1.0, T, C.T))
                terms.append((-1.0, T.T, C))
        for p in Lt:
            for q in Lt:
                if p < q:
                    A, P = OL.get(("A", p, q)), OR.get(("P", p, q))
                    if A is not None and P is not None:
                        terms.append((1.0, A, P))
                        terms.append((1.0, A.T, P.T))
                B, Q = OL.get(("B", p, q)), OR.get(("Q", p, q))
                if B is not None and Q is not None:
                    terms.append((1.0, B, Q))
        return [tm for tm in terms
                if (tm[1] is None or tm[1].blocks) and (tm[2] is None or tm[2].blocks)]

    # psi <-> enlarged-sector matrices
    def to_matrix(self, psi):
        i, EL, ER, q_tot = self.mps.window, self.EL, self.ER, self.q_tot
        bl = self.mps.bonds[i]
        out = {}
        for (li, n1, n2), blk in psi.items():
            ql = (bl[li][0] + QN[n1][0], bl[li][1] + QN[n1][1])
            rbond = (ql[0] + QN[n2][0], ql[1] + QN[n2][1])
            rown = (q_tot[0] - rbond[0], q_tot[1] - rbond[1])
            ra = ER.base.idx[rown]
            kl, ol = EL.offset[(li, n1)]
            kr, orr = ER.offset[(n2, ra)]
            if kl not in out:
                out[kl] = (kr, np.zeros((EL.dim[kl], ER.dim[kr])))
            assert out[kl][0] == kr
            out[kl][1][ol:ol + blk.shape[0], orr:orr + blk.shape[1]] = blk
        return out

    def from_matrix(self, mat, template):
        i, EL, ER, q_tot = self.mps.window, self.EL, self.ER, self.q_tot
        bl = self.mps.bonds[i]
        out = {}
        for (li, n1, n2), shape in template.items():
            ql = (bl[li][0] + QN[n1][0], bl[li][1] + QN[n1][1])
            rbond = (ql[0] + QN[n2][0], ql[1] + QN[n2][1])
            rown = (q_tot[0] - rbond[0], q_tot[1] - rbond[1])
            ra = ER.base.idx[rown]
            kl, ol = EL.offset[(li, n1)]
            kr, orr = ER.offset[(n2, ra)]
            if kl in mat:
                out[(li, n1, n2)] = mat[kl][1][ol:ol + shape[0], orr:orr + shape[1]].copy()
            else:
                out[(li, n1, n2)] = np.zeros(shape)
        return out

    def apply_matrix(self, Psi, terms=None):
        EL, ER = self.EL, self.ER
        sig = {}
        for (coef, XL, XR) in (self.terms if terms is None else terms):
            rpar = XR.parity if XR is not None else 0
            for kl, (kr, P) in Psi.items():
                if XL is None:
                    rows = [(kl, None)]
                else:
                    rows = [(a, m) for (a, b), m in XL.blocks.items() if b == kl]
                if XR is None:
                    cols = [(kr, None)]
                else:
                    cols = [(a, m) for (a, b), m in XR.blocks.items() if b == kr]
                if not rows or not cols:
                    continue
                s = coef * (-1.0 if (rpar and EL.qn[kl][0] % 2) else 1.0)
                for (ka, ml) in rows:
                    T = P if ml is None else ml @ P
                    for (kb, mr) in cols:
                        U = T if mr is None else T @ mr.T
                        if ka not in sig:
                            sig[ka] = (kb, np.zeros((EL.dim[ka], ER.dim[kb])))
                        sig[ka][1][...] += s * U
        return sig

    def apply(self, psi):
        tmpl = {k: v.shape for k, v in psi.items()}
        return self.from_matrix(self.apply_matrix(self.to_matrix(psi)), tmpl)

    def diagonal(self, template):
        """diag(H_eff) in psi blocks (template: {(l, n1, n2): shape}).

        A product X_L (x) X_R of the partition reaches a diagonal element
        <l r|X_L X_R|l r> only if both factors keep their quantum numbers
        (dq = 0, hence even parity and no Jordan-Wigner sign); the element is
        then X_L[l, l] X_R[r, r].  Summed over the terms of the partition.
        Pin: equals the diagonal of the dense P^T H P (projection.py) at
        small sizes (tests/test_oracle_blocksparse.py)."""
        EL, ER = self.EL, self.ER
        out = self.to_matrix({k: np.zeros(shape) for k, shape in template.items()})
        for (coef, XL, XR) in self.terms:
            if (XL is not None and XL.dq != (0, 0)) or (XR is not None and XR.dq != (0, 0)):
                continue
            for kl, (kr, D) in out.items():
                if XL is None:
                    dl = np.ones(EL.dim[kl])
                else:
                    blk = XL.blocks.get((kl, kl))
                    if blk is None:
                        continue
                    dl = np.diag(blk)
                if XR is None:
                    dr = np.ones(ER.dim[kr])
                else:
                    blk = XR.blocks.get((kr, kr))
                    if blk is None:
                        continue
                    dr = np.diag(blk)
                D += coef * np.outer(dl, dr)
        return self.from_matrix(out, template)

