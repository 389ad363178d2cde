"""GPU two-site sweeps against the oracle's sweep (Sec. II.A.2), step by step.

Both start from the same seeded right-canonical MPS (synth) and the same
integrals.  The GPU path runs its own plans, environments, sigma-vectors,
Davidson and truncating split; the oracle takes H_eff := P^T H P (no MPO), a
library eigensolver and its own split.  Compared per site step: the energy, the
discarded weight, the new bond's sector table and its kept singular values --
quantities that do not depend on the gauge of the eigenvector or of the SVD.
The cases truncate: bond 4 of the 8-orbital chain has 256 states.
"""

import numpy as np
import pytest

from oracle import sweep as osw
from synth import bond_sector_tables, make_integrals, random_right_canonical_mps

pytestmark = pytest.mark.gpu

TOL_E = 1e-10      # Ha
TOL_W = 1e-9       # discarded weight
TOL_S = 1e-8       # kept singular values


@pytest.mark.parametrize("K,M,passes", [(8, 64, 6), (8, 16, 4), (8, 32, 3)])
def test_gpu_sweep_matches_oracle_sweep(device, K, M, passes):
    from paper_2310_03920_amd.dmrg import DMRG
    print(f"[sweep vs oracle] K={K} M={M} passes={passes}", flush=True)
    h, g = make_integrals(K, seed=0)
    bonds = bond_sector_tables(K, K, 0, M)
    tensors = random_right_canonical_mps(bonds, 1)
    ref = osw.sweep(osw.FockHeff(h, g, K, 0), bonds, tensors, M, passes)
    print(f"[sweep vs oracle] oracle done: {len(ref)} steps, E_last {ref[-1]['energy']:.12f}", flush=True)
    d = DMRG(h, g, K, 0, M, device="cuda", tol=1e-11, max_iter=400,
             bonds=[list(b) for b in bonds], tensors=[dict(t) for t in tensors])
    d.run(passes)
    got = d.log
    assert [(r["pass"], r["i"]) for r in got] == [(r["pass"], r["i"]) for r in ref]
    worst = {"E": 0.0, "w": 0.0, "s": 0.0}
    for a, b in zip(got, ref):
        assert a["rnorm"] < 1e-10, a
        worst["E"] = max(worst["E"], abs(a["energy"] - b["energy"]))
        worst["w"] = max(worst["w"], abs(a["discarded"] - b["discarded"]))
        assert a["bond"] == b["bond"], (a["pass"], a["i"])
        worst["s"] = max(worst["s"], float(np.max(np.abs(np.array(a["kept_s"]) - np.array(b["kept_s"])))))
    print(f"[sweep vs oracle] max |dE| {worst['E']:.2e}, |dw| {worst['w']:.2e}, |ds| {worst['s']:.2e}", flush=True)
    assert worst["E"] <= TOL_E
    assert worst["w"] <= TOL_W
    assert worst["s"] <= TOL_S
    assert max(r["discarded"] for r in ref) > 1e-6  # the case really truncates
