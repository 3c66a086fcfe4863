"""Seeded synthetic inputs shared by the CPU oracle and the GPU library tests.

This package only draws random numbers and lays them out in the documented
exchange formats (integral arrays, block-sparse MPS tensors, spin-adapted
sectors and reduced operator blocks in `synthetic.su2`).  It contains
none of the DMRG arithmetic: no operators, no Hamiltonian application, no
renormalisation.  Both the oracle and the library consume what it produces.
"""
from .integrals import make_integrals
from .mps import (SITE_QN, RandomMPS, make_mps, pack_site, pack_psi,
                  unpack_psi, psi_block_list, site_block_list, mps_arrays)

__all__ = ["make_integrals", "SITE_QN", "RandomMPS", "make_mps", "pack_site",
           "pack_psi", "unpack_psi", "psi_block_list", "site_block_list", "mps_arrays"]
