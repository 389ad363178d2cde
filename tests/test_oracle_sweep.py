"""Pins of the oracle's two-site sweep and its truncation (Sec. II.A.2) against facts
that do not come from the oracle itself: the singular value decomposition of the
whole two-site matrix with no symmetry blocking (Eckart-Young), exact
reconstruction without truncation, canonical conditions, FCI energies where the
bases are complete, the variational bound, and the P^T H P definition of H_eff
against the renormalised-operator contraction with the MPO as data."""

from math import comb

import numpy as np
import pytest

from oracle import contract, fock
from oracle import mps as omps
from oracle import sweep as osw
from synth import bond_sector_tables, make_integrals, random_right_canonical_mps
from synth.blocks import random_psi


def _bonds(K, M, i):
    b = bond_sector_tables(K, K, 0, M)
    return b[i], b[i + 2]


def _dense_matrix(psi, lb, rb):
    d = omps.dense_two_site(psi, lb, rb)
    return d.reshape(d.shape[0] * 4, 4 * d.shape[3])


def _recombine(canon, centre, lb, mb, rb, direction):
    if direction == 0:
        return osw.merge(canon, centre, lb, mb, rb)
    return osw.merge(centre, canon, lb, mb, rb)


@pytest.mark.parametrize("direction", [0, 1])
def test_split_without_truncation_reconstructs_psi(direction):
    lb, rb = _bonds(6, 16, 2)
    psi = random_psi(lb, rb, np.random.default_rng(4))
    nb, canon, centre, disc, ks = osw.split(psi, lb, rb, 10 ** 6, direction)
    back = _recombine(canon, centre, lb, nb, rb, direction)
    for k, blk in psi.items():
        np.testing.assert_allclose(back.get(k, 0 * blk), blk, atol=1e-12)
    assert disc == 0.0
    # canonical: A^T A = I (direction 0) / B B^T = I (direction 1) per new sector
    for q, (_, m) in enumerate(nb):
        if direction == 0:
            gram = sum(a.T @ a for (il, s1, qq), a in canon.items() if qq == q)
        else:
            gram = sum(b @ b.T for (qq, s2, ir), b in canon.items() if qq == q)
        np.testing.assert_allclose(gram, np.eye(m), atol=1e-12)


@pytest.mark.parametrize("direction,M", [(0, 5), (1, 9), (0, 23)])
def test_kept_spectrum_is_the_top_m_of_the_unblocked_svd(direction, M):
    """The symmetry blocks of psi are the diagonal blocks of one matrix, so its
    singular values (computed on the dense matrix, no blocking) are the union of the
    blocks' values: the split must keep exactly the M largest of them, discard the
    rest's squared sum, and the truncated tensor must be the best rank-M
    approximation (Eckart-Young)."""
    lb, rb = _bonds(6, 16, 2)
    psi = random_psi(lb, rb, np.random.default_rng(7))
    nrm = np.sqrt(sum(float((b * b).sum()) for b in psi.values()))
    psi = {k: b / nrm for k, b in psi.items()}
    s = np.linalg.svd(_dense_matrix(psi, lb, rb), compute_uv=False)
    assert s[M - 1] > s[M] * (1 + 1e-6)  # a gap at the cut: the kept set is unique
    nb, canon, centre, disc, ks = osw.split(psi, lb, rb, M, direction)
    assert sum(m for _, m in nb) == M
    np.testing.assert_allclose(ks, s[:M], rtol=1e-12)
    np.testing.assert_allclose(disc, float((s[M:] ** 2).sum()), rtol=1e-10, atol=1e-15)
    trunc = _recombine(canon, centre, lb, nb, rb, direction)
    err = _dense_matrix(psi, lb, rb) - _dense_matrix(trunc, lb, rb)
    np.testing.assert_allclose(float((err ** 2).sum()), disc, rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(float((_dense_matrix(trunc, lb, rb) ** 2).sum()), float((s[:M] ** 2).sum()),
                               rtol=1e-12)


def test_selection_orders_equal_values_by_sector_and_index():
    # exact tie across sectors: the lexicographically smaller (N, 2Sz) sector first
    sv = {(2, 2): np.array([0.5, 0.1]), (2, 0): np.array([0.5, 0.1]), (1, 1): np.array([0.3])}
    assert osw.select(sv, 1)[0] == {(2, 0): 1}
    assert osw.select(sv, 2)[0] == {(2, 0): 1, (2, 2): 1}
    kept, disc = osw.select(sv, 3)
    assert kept == {(2, 0): 1, (2, 2): 1, (1, 1): 1}
    np.testing.assert_allclose(disc, 0.02, rtol=1e-14)
    # a difference far below the tie tolerance is a tie: the sector order decides
    sv = {(2, 0): np.array([0.5]), (2, 2): np.array([0.5 + 1e-13])}
    assert osw.select(sv, 1)[0] == {(2, 0): 1}
    # a real gap is not a tie
    sv = {(2, 0): np.array([0.5]), (2, 2): np.array([0.5 + 1e-6])}
    assert osw.select(sv, 1)[0] == {(2, 2): 1}
    # zeros of a full factor are candidates too (kept when fewer than M are non-zero)
    sv = {(0, 0): np.array([1.0, 0.0]), (1, 1): np.array([0.0])}
    assert osw.select(sv, 3)[0] == {(0, 0): 2, (1, 1): 1}


def _sweep(K, M, passes, heff=None, seed=0, mps_seed=1):
    h, g = make_integrals(K, seed=seed)
    bonds = bond_sector_tables(K, K, 0, M)
    tensors = random_right_canonical_mps(bonds, mps_seed)
    heff = heff or osw.FockHeff(h, g, K, 0)
    return h, g, osw.sweep(heff, bonds, tensors, M, passes)


def test_complete_bases_give_fci_at_every_step_after_the_first():
    """6 orbitals, M = 64: no bond is truncated (every Schmidt rank is at most 64),
    so once the first step has replaced the random MPS's right block every step is
    E_FCI."""
    h, g, log = _sweep(6, 64, 2)
    e_fci = fock.fci_energy(h, g, 6, 0)
    assert log[0]["energy"] >= e_fci - 1e-10
    for r in log[1:]:
        assert abs(r["energy"] - e_fci) < 1e-10, r
        assert r["discarded"] == 0.0


def test_middle_step_of_the_8_orbital_chain_is_fci():
    """8 orbitals, M = 64: at sites (3, 4) both blocks hold 4^3 = 64 states, a complete
    basis, so that step is E_FCI in every pass although bond 4 (256 states) is
    truncated; every step is variational."""
    h, g, log = _sweep(8, 64, 2)
    e_fci = fock.fci_energy(h, g, 8, 0)
    mids = [r for r in log if r["i"] == 3]
    assert len(mids) == 2
    for r in log:
        assert r["energy"] >= e_fci - 1e-10
    for r in mids:
        assert abs(r["energy"] - e_fci) < 1e-10, r
    # the complete blocks have the full sector dimensions C(3, a) C(3, b)
    for r in log:
        if r["i"] in (2, 4) and r["pass"] == 0:
            k = r["i"] + 1
            n = 3 if k == 3 else 5
            full = {(na + nb, na - nb): comb(n, na) * comb(n, nb) for na in range(n + 1) for nb in range(n + 1)
                    if 0 <= 4 - na <= 8 - n and 0 <= 4 - nb <= 8 - n}
            if k == 3:
                assert dict(r["bond"]) == full
    assert any(r["discarded"] > 1e-6 for r in log)   # bond 4 is truncated


def test_truncated_sweep_is_variational_and_discards_weight():
    h, g, log = _sweep(6, 8, 3)
    e_fci = fock.fci_energy(h, g, 6, 0)
    for r in log:
        assert r["energy"] >= e_fci - 1e-10
        assert sum(m for _, m in r["bond"]) <= 8
    assert max(r["discarded"] for r in log) > 1e-6


def test_mpo_form_of_heff_gives_the_same_sweep_as_the_fock_definition():
    """The renormalised-operator contraction with the NC MPO passed as data and
    environments built from the MPS equals H_eff := P^T H P step by step, in a
    truncated sweep (pins the dense-environment form and the MPO values together)."""
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    K, M = 6, 8
    h, g = make_integrals(K, seed=0)
    mpo = build_nc_mpo(h, g)
    W = [contract.dense_mpo(site_entries(mpo, k), len(mpo.dq[k]), len(mpo.dq[k + 1])) for k in range(K)]
    _, _, ref = _sweep(K, M, 2)
    _, _, got = _sweep(K, M, 2, heff=osw.MpoHeff(W))
    assert len(ref) == len(got)
    for a, b in zip(ref, got):
        assert abs(a["energy"] - b["energy"]) < 1e-10, (a["i"], a["energy"], b["energy"])
        assert abs(a["discarded"] - b["discarded"]) < 1e-10
        assert a["bond"] == b["bond"]
