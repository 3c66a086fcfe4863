"""Writes the stored oracle sigmas used by tests/test_gpu_parity_large.py.

At 22 and 36 orbitals the block-sparse oracle needs 10-60 s per window to
build its environments, too slow to run inside the GPU test session, so its
results are stored here.  This script calls only ``oracle`` (the
normal/complementary sigma and diag(H_eff), pinned on the CPU against the
plain definition P^T H P) and the seeded generators in ``synthetic``; no
value comes from the HIP library.

    python tests/golden/make_sigma_golden.py          # rewrites every file

Each file sigma_<name>.npz holds the packed sigma and diag(H_eff) of the
window (psi layout of the library), the packed psi it was computed from (so
that the test can check that the generators still produce the same input),
and the case parameters.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.blocksparse import BlockSparseSigma  # noqa: E402
from oracle.projection import psi_template  # noqa: E402
from synthetic import make_integrals, make_mps, pack_psi  # noqa: E402

# name: (K, N, 2Sz, D, window, integral seed, MPS seed)
CASES = {
    "k22_n22_sz0_d48_w10": (22, 22, 0, 48, 10, 22, 1022),
    "k22_n22_sz4_d48_w10": (22, 22, 4, 48, 10, 22, 1022),
    "k36_n54_sz0_d24_w17": (36, 54, 0, 24, 17, 36, 1036),
    "k36_n54_sz4_d24_w17": (36, 54, 4, 24, 17, 36, 1036),
    "k36_n54_sz0_d20_w8": (36, 54, 0, 20, 8, 36, 1036),
}


def make(name):
    K, N, tsz, D, i, iseed, mseed = CASES[name]
    t0 = time.time()
    h, eri = make_integrals(K, iseed)
    m = make_mps(K, N, tsz, D, i, mseed)
    b = BlockSparseSigma(m, h, eri)
    sig = b.apply(m.psi)
    dia = b.diagonal(psi_template(m))
    np.savez(os.path.join(HERE, f"sigma_{name}.npz"),
             case=np.array([K, N, tsz, D, i, iseed, mseed], dtype=np.int64),
             psi=pack_psi(m.bonds, i, m.psi),
             sigma=pack_psi(m.bonds, i, sig),
             diag=pack_psi(m.bonds, i, dia))
    print(f"{name}: psi {m.psi_size()} elements, {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or CASES):
        make(n)
