"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only draws random numbers and lays out structure (sector tables,
block shapes).  It holds none of the DMRG arithmetic: no Hamiltonian action, no
contraction, no eigensolver.  Everything here is passed *as data* to both sides.
"""

from .integrals import make_integrals, hubbard_integrals  # noqa: F401
from .sectors import SITE_QN, bond_sector_tables, site_shifts  # noqa: F401
from .mps import random_right_canonical_mps, random_left_canonical_mps  # noqa: F401
from .blocks import (  # noqa: F401
    random_env, random_site_ops, random_psi, two_site_blocks, random_site_tensor,
)
