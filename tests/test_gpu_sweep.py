"""Full GPU two-site sweeps against FCI exact diagonalisation (oracle)."""

import numpy as np
import pytest

from oracle import fock
from synth import make_integrals

pytestmark = pytest.mark.gpu

TOL_E = 1e-10  # Ha, FP64 target for sweep energies


def _run(K, M, sweeps, seed=0, max_iter=120):
    from paper_2310_03920_amd.dmrg import DMRG
    h, g = make_integrals(K, seed=seed)
    d = DMRG(h, g, K, 0, M, seed=seed + 1, device="cuda", tol=1e-9, max_iter=max_iter)
    d.run(sweeps)
    return h, g, d


def test_config1_sweep_middle_step_equals_fci(device):
    """8 orbitals, 8 electrons, 2Sz=0, M=64, 6 sweeps: at sites (3,4) both blocks are
    complete (4^3 = 64 states), so that step's energy is E_FCI in every pass; every
    step is variational."""
    print("[sweep K=8 M=64]", flush=True)
    h, g, d = _run(8, 64, 6)
    e_fci = fock.fci_energy(h, g, 8, 0)
    for rec in d.log:
        assert rec["energy"] >= e_fci - TOL_E, rec
        if rec["i"] == 3:
            assert abs(rec["energy"] - e_fci) < TOL_E, (rec, e_fci)
    for k in (3, 5):
        assert sum(m for _, m in d.bonds[k]) == 64
    print("final", d.log[-1]["energy"], "fci", e_fci, flush=True)


def test_untruncated_sweep_every_step_equals_fci(device):
    """6 orbitals with M=64: the sweep never truncates (every bond keeps its full
    Schmidt-rank bound), so every step after the first gives E_FCI.  The first
    step is the exception: its right block (4 sites, 256 states) is spanned only
    by the random initial MPS's 16 states across bond 2."""
    print("[sweep K=6 M=64 untruncated]", flush=True)
    h, g, d = _run(6, 64, 3, seed=4)
    e_fci = fock.fci_energy(h, g, 6, 0)
    assert d.log[0]["energy"] >= e_fci - TOL_E
    errs = [abs(r["energy"] - e_fci) for r in d.log[1:]]
    assert max(errs) < TOL_E, errs


def test_sweep_energies_bitwise_repeatable(device):
    print("[sweep repeat]", flush=True)
    _, _, d1 = _run(6, 16, 2, seed=2)
    _, _, d2 = _run(6, 16, 2, seed=2)
    assert [r["energy"] for r in d1.log] == [r["energy"] for r in d2.log]
