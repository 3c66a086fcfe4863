"""The MPS of eq. (1) as Fock vectors, and the projected H_eff (plain definition).

TEST INFRASTRUCTURE ONLY.  For a two-site window (i, i+1):

* |l> (l a state of bond i) is the contraction of the left-canonical tensors
  A_0 ... A_{i-1} (eq. (1) restricted to sites 0..i-1), a vector over the
  occupations of sites 0..i-1;
* |r> (bond i+2) is the contraction of the right-canonical tensors
  B_{i+2} ... B_{K-1};
* the column (l, n1, n2, r) of the isometry P is the determinant-space vector
  |l> (x) |n1> (x) |n2> (x) |r>.  With determinants written as
  prod_{P ascending} a+_P |vac> the product of disjoint, ordered parts is the
  plain concatenation of occupations, so no sign enters.
* H_eff = P^T H P (the Galerkin projection), and sigma = H_eff psi.

At the small sizes where this is used (K <= 8) the full 4^K Fock vector of
P psi fits in memory.  Pins: P^T P = 1, Hermiticity of H_eff, and
lambda_min(H_eff) = E_FCI when the bond spaces are complete
(tests/test_oracle_projection.py).
"""
import numpy as np

from .fock import DetSpace

_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _state_offsets(bond):
    offs, o = [], 0
    for s in bond:
        offs.append(o)
        o += s[2]
    return offs, o


def left_states(mps, i):
    """Matrix (4^i, D_i): column = bond-i state as a vector over sites 0..i-1."""
    cur = np.ones((1, 1))  # (configs, states) at bond 0
    for b in range(i):
        left, right = mps.bonds[b], mps.bonds[b + 1]
        loffs, _ = _state_offsets(left)
        roffs, Dr = _state_offsets(right)
        ncfg = cur.shape[0]
        new = np.zeros((ncfg * 4, Dr))
        for (li, n), blk in mps.sites[b].items():
            q = (left[li][0] + _QN[n][0], left[li][1] + _QN[n][1])
            ri = [k for k, s in enumerate(right) if (s[0], s[1]) == q][0]
            dl, dr = blk.shape
            # config index of the extended part: old + n * 4^b
            rows = np.arange(ncfg) + n * ncfg
            new[rows, roffs[ri]:roffs[ri] + dr] += cur[:, loffs[li]:loffs[li] + dl] @ blk
        cur = new
    return cur


def right_states(mps, i):
    """Matrix (4^(K-i-2), D_{i+2}) over occupations of sites i+2..K-1."""
    K = mps.n_orb
    cur = np.ones((1, 1))  # (configs of sites > b, states at bond b+1)
    for b in range(K - 1, i + 1, -1):
        left, right = mps.bonds[b], mps.bonds[b + 1]
        loffs, Dl = _state_offsets(left)
        roffs, _ = _state_offsets(right)
        ncfg = cur.shape[0]
        new = np.zeros((ncfg * 4, Dl))
        for (li, n), blk in mps.sites[b].items():
            q = (left[li][0] + _QN[n][0], left[li][1] + _QN[n][1])
            ri = [k for k, s in enumerate(right) if (s[0], s[1]) == q][0]
            dl, dr = blk.shape
            # prepend site b: new config = n + 4 * old
            rows = n + 4 * np.arange(ncfg)
            new[rows, loffs[li]:loffs[li] + dl] += cur[:, roffs[ri]:roffs[ri] + dr] @ blk.T
        cur = new
    return cur


def psi_to_fock(mps, psi):
    """Full Fock vector (length 4^K, indexed by the determinant integer)."""
    i, K = mps.window, mps.n_orb
    L, R = left_states(mps, i), right_states(mps, i)
    loffs, DL = _state_offsets(mps.bonds[i])
    roffs, DR = _state_offsets(mps.bonds[i + 2])
    T = np.zeros((DL, 4, 4, DR))
    for (li, n1, n2), blk in psi.items():
        q = (mps.bonds[i][li][0] + _QN[n1][0] + _QN[n2][0],
             mps.bonds[i][li][1] + _QN[n1][1] + _QN[n2][1])
        ri = [k for k, s in enumerate(mps.bonds[i + 2]) if (s[0], s[1]) == q][0]
        T[loffs[li]:loffs[li] + blk.shape[0], n1, n2, roffs[ri]:roffs[ri] + blk.shape[1]] = blk
    # Phi[ld, n1, n2, rd]; determinant integer = ld + n1 4^i + n2 4^(i+1) + rd 4^(i+2)
    Phi = np.einsum("xl,labr,yr->xaby", L, T, R, optimize=True)
    return np.ascontiguousarray(Phi.transpose(3, 2, 1, 0)).reshape(-1)


def fock_to_psi(mps, vec):
    """P^T applied to a full Fock vector; returns psi blocks."""
    i, K = mps.window, mps.n_orb
    L, R = left_states(mps, i), right_states(mps, i)
    loffs, DL = _state_offsets(mps.bonds[i])
    roffs, DR = _state_offsets(mps.bonds[i + 2])
    Phi = np.asarray(vec).reshape(4 ** (K - i - 2), 4, 4, 4 ** i).transpose(3, 2, 1, 0)
    T = np.einsum("xl,xaby,yr->labr", L, Phi, R, optimize=True)
    out = {}
    for (li, n1, n2), blk in psi_template(mps).items():
        q = (mps.bonds[i][li][0] + _QN[n1][0] + _QN[n2][0],
             mps.bonds[i][li][1] + _QN[n1][1] + _QN[n2][1])
        ri = [k for k, s in enumerate(mps.bonds[i + 2]) if (s[0], s[1]) == q][0]
        out[(li, n1, n2)] = T[loffs[li]:loffs[li] + blk[0], n1, n2,
                              roffs[ri]:roffs[ri] + blk[1]].copy()
    return out


def psi_template(mps):
    """{(l, n1, n2): (d_l, d_r)} for every allowed psi block."""
    i = mps.window
    right = {(s[0], s[1]): s[2] for s in mps.bonds[i + 2]}
    out = {}
    for li, s in enumerate(mps.bonds[i]):
        for n1 in range(4):
            for n2 in range(4):
                q = (s[0] + _QN[n1][0] + _QN[n2][0], s[1] + _QN[n1][1] + _QN[n2][1])
                if q in right:
                    out[(li, n1, n2)] = (s[2], right[q])
    return out


class ProjectedHamiltonian:
    """sigma = P^T H P psi with H the sparse sector Hamiltonian (K <= 8)."""

    def __init__(self, mps, h, eri):
        self.mps = mps
        self.space = DetSpace.sector(mps.n_orb, mps.n_elec, mps.two_sz)
        self.H = self.space.hamiltonian(h, eri)

    def apply(self, psi):
        full = psi_to_fock(self.mps, psi)
        c = full[self.space.dets]
        out = np.zeros_like(full)
        out[self.space.dets] = self.H @ c
        return fock_to_psi(self.mps, out)

    def dense(self):
        """Dense H_eff in the packed psi order of psi_template (sorted keys)."""
        tmpl = psi_template(self.mps)
        keys = sorted(tmpl)
        sizes = [tmpl[k][0] * tmpl[k][1] for k in keys]
        n = sum(sizes)
        cols = []
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            cols.append(_flatten(self.apply(_unflatten(e, keys, tmpl)), keys))
        return np.array(cols).T, keys


def _flatten(psi, keys):
    return np.concatenate([psi[k].ravel() for k in keys])


def _unflatten(vec, keys, tmpl):
    out, o = {}, 0
    for k in keys:
        dl, dr = tmpl[k]
        out[k] = vec[o:o + dl * dr].reshape(dl, dr)
        o += dl * dr
    return out
