"""Shared test helpers: run the library on synthetic inputs, compare with the oracle."""
import numpy as np

from synthetic import make_integrals, make_mps, mps_arrays, pack_psi, unpack_psi


def case(K, N, tsz, D, window, iseed=None, mseed=None):
    h, eri = make_integrals(K, K if iseed is None else iseed)
    m = make_mps(K, N, tsz, D, window, (1000 + K) if mseed is None else mseed)
    return h, eri, m


def lib_load(ctx, h, eri, m):
    ctx.build_ops(m.window, h=h, eri=eri, n_elec=m.n_elec, two_sz=m.two_sz,
                  mps_arrays=mps_arrays(m))
    n = ctx.psi_size()
    assert n == m.psi_size(), (n, m.psi_size())
    return n


def lib_sigma_flat(ctx, psi_flat, precision="fp64"):
    import torch
    psi = torch.from_numpy(np.ascontiguousarray(psi_flat)).cuda()
    out = torch.empty_like(psi)
    ctx.sigma(psi, out, precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def lib_sigma(ctx, h, eri, m, precision="fp64"):
    lib_load(ctx, h, eri, m)
    flat = pack_psi(m.bonds, m.window, m.psi)
    return unpack_psi(m.bonds, m.window, lib_sigma_flat(ctx, flat, precision))


def rel_err(a, b):
    num = np.sqrt(sum(np.sum((a[k] - b[k]) ** 2) for k in b))
    den = np.sqrt(sum(np.sum(b[k] ** 2) for k in b))
    return num / den


def max_abs(a, b):
    return max(float(np.max(np.abs(a[k] - b[k]))) if b[k].size else 0.0 for k in b)
