"""Sweeps with the NC->CN switched MPO on the GPU (Sec. II.B.2).

The switch changes the bond operators (complementary pairs on the left of every
cut right of the middle), not the Hamiltonian, so every quantity the sweep
produces must be the NC one: the config-1 middle step is E_FCI in every pass
(both blocks complete), every step is variational, and the step energies equal
those of the NC sweep from the same initial MPS.
"""

import pytest

from oracle import fock
from synth import make_integrals

pytestmark = pytest.mark.gpu

TOL_E = 1e-10


def test_switched_mpo_sweep_matches_fci_and_the_nc_sweep(device):
    from paper_2310_03920_amd.dmrg import DMRG
    K, M = 8, 64
    print(f"[partition] K={K} M={M}, NC vs NC->CN at cut {K // 2}", flush=True)
    h, g = make_integrals(K, seed=0)
    runs = {}
    for sw in (None, K // 2):
        d = DMRG(h, g, K, 0, M, seed=1, device="cuda", tol=1e-9, max_iter=120, mpo_switch=sw)
        d.run(6)
        runs[sw] = d
    e_fci = fock.fci_energy(h, g, K, 0)
    d_nc, d_sw = runs[None], runs[K // 2]
    assert max(len(c) for c in d_sw.mpo.cuts) < max(len(c) for c in d_nc.mpo.cuts)
    for rec in d_sw.log:
        assert rec["energy"] >= e_fci - TOL_E, rec
        if rec["i"] == 3:
            assert abs(rec["energy"] - e_fci) < TOL_E, (rec, e_fci)
    assert len(d_sw.log) == len(d_nc.log)
    diffs = [abs(a["energy"] - b["energy"]) for a, b in zip(d_sw.log, d_nc.log)]
    print(f"[partition] max |E_switch - E_nc| per step = {max(diffs):.2e}", flush=True)
    assert max(diffs) < 1e-9


def test_switched_mpo_truncated_sweep_matches_the_nc_sweep(device):
    """10 orbitals at M=40: every bond right of the first few is truncated, so the
    sweep's states depend on the SVD splits; the same initial MPS gives the same
    step energies with either partition (the operator is the same), and every
    step stays above E_FCI."""
    from paper_2310_03920_amd.dmrg import DMRG
    K, M = 10, 40
    print(f"[partition] K={K} M={M} truncated, NC vs NC->CN at cut {K // 2}", flush=True)
    h, g = make_integrals(K, seed=7)
    e_fci = fock.fci_energy(h, g, K, 0)
    logs = []
    for sw in (None, K // 2):
        d = DMRG(h, g, K, 0, M, seed=2, device="cuda", tol=1e-9, max_iter=150, mpo_switch=sw)
        d.run(4)
        logs.append(d.log)
    assert len(logs[0]) == len(logs[1])
    diffs = [abs(a["energy"] - b["energy"]) for a, b in zip(*logs)]
    print(f"[partition] max |E_switch - E_nc| per step = {max(diffs):.2e}; "
          f"final {logs[1][-1]['energy']:.10f} (FCI {e_fci:.10f})", flush=True)
    assert max(diffs) < 1e-8
    assert min(r["energy"] for r in logs[1]) > e_fci - TOL_E
