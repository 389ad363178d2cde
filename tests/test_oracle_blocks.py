"""Pins of the block-by-block host sigma-vector (oracle.blocks): it equals the dense
single-sum definition (itself pinned by Kronecker brute force), its restrictions to
middle-bond subsets and output column blocks add up to the whole, and its own count
of block-product work equals an independent count and the plan's."""

import numpy as np
import pytest

from oracle import blocks, contract
from oracle import mps as omps
from synth import bond_sector_tables, make_integrals
from synth.blocks import random_env, random_psi
from test_oracle_pins import _tiny_operands


def _dense(sig, lb, rb):
    return omps.dense_two_site(sig, lb, rb)


def _nc_problem(K=6, M=16, i=2, seed=3):
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    m = build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, M)
    lb, rb = b[i], b[i + 2]
    rng = np.random.default_rng(seed)
    Ldq, Rdq = [tuple(x) for x in m.dq[i]], [tuple(x) for x in m.dq[i + 2]]
    L, R = random_env(lb, Ldq, rng), random_env(rb, Rdq, rng)
    psi = random_psi(lb, rb, rng)
    return m, b, i, lb, rb, L, R, site_entries(m, i), site_entries(m, i + 1), psi


def test_blocks_match_dense_definition_on_random_operands():
    lb, rb, L, R, W1e, W2e, psi, D, Dm = _tiny_operands()
    ref = contract.heff_apply(contract.dense_env(L, lb), contract.dense_mpo(W1e, D, Dm),
                              contract.dense_mpo(W2e, Dm, D), contract.dense_env(R, rb),
                              omps.dense_two_site(psi, lb, rb))
    got = _dense(blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi), lb, rb)
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_blocks_match_dense_definition_with_the_nc_mpo():
    m, b, i, lb, rb, L, R, W1e, W2e, psi = _nc_problem()
    ref = contract.heff_apply(contract.dense_env(L, lb), contract.dense_mpo(W1e, len(m.dq[i]), len(m.dq[i + 1])),
                              contract.dense_mpo(W2e, len(m.dq[i + 1]), len(m.dq[i + 2])), contract.dense_env(R, rb),
                              omps.dense_two_site(psi, lb, rb))
    got = _dense(blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi), lb, rb)
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_restrictions_add_up_to_the_whole():
    m, b, i, lb, rb, L, R, W1e, W2e, psi = _nc_problem()
    full = _dense(blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi), lb, rb)
    nb = len(m.dq[i + 1])
    parts = [list(range(r, nb, 3)) for r in range(3)]
    tot, fl = 0.0, [0.0]
    for p in parts:
        tot = tot + _dense(blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi, bsel=p, flops=fl), lb, rb)
    np.testing.assert_allclose(tot, full, atol=1e-12 * np.abs(full).max())
    whole = [0.0]
    blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi, flops=whole)
    assert fl[0] == whole[0]
    cols = sorted({(s2, ir) for (_, _, s2, ir) in psi})[::2]
    sub = blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi, cols=cols)
    assert {(k[2], k[3]) for k in sub} <= set(cols)
    ro, _ = omps.bond_offsets(rb)
    lo, _ = omps.bond_offsets(lb)
    for (il, s1, s2, ir), blk in sub.items():
        ref = full[lo[il]:lo[il] + blk.shape[0], s1, s2, ro[ir]:ro[ir] + blk.shape[1]]
        np.testing.assert_allclose(blk, ref, atol=1e-12 * np.abs(full).max())


@pytest.mark.parametrize("i", [1, 3, 5])
def test_flop_count_equals_independent_and_plan_counts(i):
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    from test_host_lib import _count_flops
    K, M = 8, 64
    m = build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, M)
    lb, rb = b[i], b[i + 2]
    rng = np.random.default_rng(1)
    Ldq, Rdq = [tuple(x) for x in m.dq[i]], [tuple(x) for x in m.dq[i + 2]]
    W1e, W2e = site_entries(m, i), site_entries(m, i + 1)
    fl = [0.0]
    blocks.heff_apply(lb, rb, random_env(lb, Ldq, rng), W1e, W2e, random_env(rb, Rdq, rng),
                      random_psi(lb, rb, rng), flops=fl)
    assert fl[0] == pytest.approx(_count_flops(lb, rb, Ldq, Rdq, W1e, W2e), rel=1e-12)
    plan = X.HeffPlan(lb, rb, m.dq[i], m.dq[i + 1], m.dq[i + 2], W1e, W2e)
    assert fl[0] == pytest.approx(plan.info.flops_useful, rel=1e-12)


def test_middle_bond_part_plans_split_the_work_of_the_whole():
    """Plans restricted to b = p (mod n) split the useful block-product work of the
    whole plan exactly (every product belongs to one b), and each part's count equals
    the block-sparse oracle's own count over the same b; bad part options are refused."""
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    K, M, i, n = 8, 64, 3, 5
    m = build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, M)
    lb, rb = b[i], b[i + 2]
    W1e, W2e = site_entries(m, i), site_entries(m, i + 1)
    args = (lb, rb, m.dq[i], m.dq[i + 1], m.dq[i + 2], W1e, W2e)
    whole = X.HeffPlan(*args).info.flops_useful
    rng = np.random.default_rng(2)
    Ldq, Rdq = [tuple(x) for x in m.dq[i]], [tuple(x) for x in m.dq[i + 2]]
    L, R, psi = random_env(lb, Ldq, rng), random_env(rb, Rdq, rng), random_psi(lb, rb, rng)
    parts = 0.0
    for p in range(n):
        fp = X.HeffPlan(*args, b_part=p, b_nparts=n).info.flops_useful
        fl = [0.0]
        blocks.heff_apply(lb, rb, L, W1e, W2e, R, psi, bsel=range(p, len(m.dq[i + 1]), n), flops=fl)
        assert fp == pytest.approx(fl[0], rel=1e-12)
        parts += fp
    assert parts == pytest.approx(whole, rel=1e-12)
    with pytest.raises(RuntimeError, match="b_part"):
        X.HeffPlan(*args, b_part=5, b_nparts=5)
    with pytest.raises(RuntimeError, match="sigma-vector plans only"):
        X.EnvPlan(0, b[i], b[i + 1], m.dq[i], m.dq[i + 1], W1e, b_part=1, b_nparts=2)


@pytest.mark.parametrize("i", [2, 3])
def test_merged_intermediates_change_tiles_not_work(i):
    """Merging first-round intermediates that share their psi-side tasks leaves the
    block-product work (executed and useful) unchanged and cuts the tile count; the
    stacked operand copies enlarge the workspace."""
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    K, M = 8, 64
    m = build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, M)
    args = (b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], site_entries(m, i), site_entries(m, i + 1))
    sep = X.HeffPlan(*args, t_merge_off=1).info
    mer = X.HeffPlan(*args).info
    assert mer.flops_apply == sep.flops_apply
    assert mer.flops_useful == sep.flops_useful
    assert mer.n_tiles < sep.n_tiles
    assert mer.ws_bytes > sep.ws_bytes
    multi = X.HeffPlan(*args, n_roots=2).info  # several roots: intermediates stay separate
    assert multi.flops_apply == pytest.approx(2 * sep.flops_apply, rel=1e-12)
