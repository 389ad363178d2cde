"""Host-only checks of the C-ABI library and the product's host logic (no GPU)."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fock
from paper_2310_03920_amd import _lib as X
from paper_2310_03920_amd import mpo as M
from synth import bond_sector_tables, hubbard_integrals, make_integrals
from synth.blocks import two_site_blocks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "heffx.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(hx_\w+)\s*\(", hdr, re.M))
    assert names, "no declarations parsed"
    lib = ctypes.CDLL(X.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(X.EXPORTED)


@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_nc_mpo_densifies_to_fock_hamiltonian(K):
    h, g = make_integrals(K, seed=K + 20)
    m = M.build_nc_mpo(h, g)
    dets = fock.all_dets(K)
    Hf = fock.hamiltonian(h, g, dets).toarray()
    p = fock.product_index(dets, K)
    Hp = np.zeros_like(Hf)
    Hp[np.ix_(p, p)] = Hf
    np.testing.assert_allclose(M.densify(m), Hp, atol=1e-12)


def test_nc_mpo_sparse_hamiltonian_prunes_to_minimal_bond():
    h, g = hubbard_integrals(5, 1.0, 3.0)
    m = M.build_nc_mpo(h, g)
    assert max(len(c) for c in m.cuts) == 6
    dets = fock.all_dets(5)
    Hf = fock.hamiltonian(h, g, dets).toarray()
    p = fock.product_index(dets, 5)
    Hp = np.zeros_like(Hf)
    Hp[np.ix_(p, p)] = Hf
    np.testing.assert_allclose(M.densify(m), Hp, atol=1e-13)


def test_nc_mpo_bond_dimension_grows_quadratically():
    """NC partition: normal pair operators on the left give D ~ 8 k^2."""
    K = 12
    m = M.build_nc_mpo(*make_integrals(K, seed=1))
    D = [len(c) for c in m.cuts]
    for k in (3, 4, 5, 6):
        assert 6 * k * k < D[k] < 10 * k * k + 4 * K + 8


@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_switched_mpo_densifies_to_fock_hamiltonian_at_every_switch(K):
    """NC bond operators up to cut c and CN ones after it (Sec. II.B.2): the same
    operator for every switch position c, including pure CN (c = 0)."""
    h, g = make_integrals(K, seed=K + 30)
    dets = fock.all_dets(K)
    Hf = fock.hamiltonian(h, g, dets).toarray()
    p = fock.product_index(dets, K)
    Hp = np.zeros_like(Hf)
    Hp[np.ix_(p, p)] = Hf
    for c in range(K + 1):
        np.testing.assert_allclose(M.densify(M.build_mpo(h, g, switch=c)), Hp, atol=1e-12, err_msg=str(c))


def test_switched_mpo_entries_conserve_quantum_numbers_and_parity():
    """Every nonzero element (s', s) of an entry W[a, b] changes (N, 2Sz) by exactly
    dq(b) - dq(a) and flips parity by parity(b) - parity(a): the bond labels that
    the plans rely on are consistent with the site operators."""
    K = 6
    qn = np.array(M.SITE_QN)
    par = np.array([0, 1, 1, 0])
    h, g = make_integrals(K, seed=2)
    for c in (None, 0, 2, 3, 5):
        m = M.build_mpo(h, g, switch=c)
        for k in range(K):
            s = m.sites[k]
            for a, b, w in zip(s.rows, s.cols, s.mats):
                sp, ss = np.nonzero(w)
                assert (qn[sp] - qn[ss] == m.dq[k + 1][b] - m.dq[k][a]).all(), (c, k)
                assert ((par[sp] + par[ss]) % 2 == (m.parity[k + 1][b] + m.parity[k][a]) % 2).all(), (c, k)


def test_switched_mpo_bond_dimension_follows_the_smaller_side():
    """With the switch at the middle cut, bonds right of it hold the normal pairs of
    the right block: D ~ 8 (K - k)^2 there instead of 8 k^2."""
    K = 12
    h, g = make_integrals(K, seed=1)
    nc = [len(c) for c in M.build_nc_mpo(h, g).cuts]
    sw = [len(c) for c in M.build_mpo(h, g, switch=K // 2).cuts]
    assert sw[:K // 2 + 1] == nc[:K // 2 + 1]
    for k in range(K // 2 + 1, K - 1):
        r = K - k
        assert 6 * r * r < sw[k] < 10 * r * r + 4 * K + 8, (k, sw[k])
    assert max(sw) < 0.5 * max(nc)


def test_plans_build_on_the_switched_mpo_with_less_work_right_of_the_switch():
    """Host plan validation (quantum-number conservation of every task) passes at
    every site of the switched MPO; the same site step does less work right of the
    switch than with NC operators there."""
    K = 8
    h, g = make_integrals(K, seed=0)
    nc, sw = M.build_nc_mpo(h, g), M.build_mpo(h, g, switch=K // 2)
    b = bond_sector_tables(K, K, 0, 32)
    for i in range(K - 1):
        f = []
        for m in (nc, sw):
            args = (b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                    M.site_entries(m, i + 1))
            f.append(X.HeffPlan(*args).info.flops_apply)
            X.HeffVjpPlan(*args)
            X.EnvPlan(0, b[i], b[i + 1], m.dq[i], m.dq[i + 1], M.site_entries(m, i))
            X.EnvPlan(1, b[i + 1], b[i], m.dq[i + 1], m.dq[i], M.site_entries(m, i))
        if i + 2 <= K // 2:
            assert f[1] == f[0]
        if i >= K // 2:
            assert f[1] < f[0]


def test_plans_built_on_concurrent_threads_equal_sequential_builds():
    """The sweep builds the next sigma-vector plan on a worker thread while the
    environment plan is built on the caller's: the host builder is reentrant, so
    plans built at the same time on several threads equal those built one by one."""
    from concurrent.futures import ThreadPoolExecutor
    K = 10
    m = M.build_mpo(*make_integrals(K, seed=3), switch=K // 2)
    b = bond_sector_tables(K, K, 0, 48)

    def build(i):
        p = X.HeffPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                       M.site_entries(m, i + 1), split_kseg_min=64)
        e = X.EnvPlan(0, b[i], b[i + 1], m.dq[i], m.dq[i + 1], M.site_entries(m, i), split_kseg_min=64)
        return [(x.info.flops_apply, x.info.n_tasks, x.info.n_tiles, x.info.table_bytes, x.info.ws_bytes)
                for x in (p, e)]

    seq = [build(i) for i in range(K - 1)]
    with ThreadPoolExecutor(max_workers=4) as ex:
        par = list(ex.map(build, list(range(K - 1)) * 2))
    assert par == seq + seq


def test_psi_layout_matches_block_enumeration():
    """Blocks are ordered by column block (s2, ir) and then (il, s1), so every
    column block is one contiguous dense matrix."""
    b = bond_sector_tables(8, 8, 0, 64)
    lb, rb = X.Bond(b[3]), X.Bond(b[5])
    keys, off = X.psi_layout(lb, rb)
    assert sorted(keys) == sorted(two_site_blocks(b[3], b[5]))
    assert keys == sorted(keys, key=lambda k: (k[2], k[3], k[0], k[1]))
    sizes = [b[3][k[0]][1] * b[5][k[3]][1] for k in keys]
    np.testing.assert_array_equal(np.diff(off), sizes)
    assert off[-1] == 4900


def test_plan_rejects_site_matrix_breaking_conservation():
    lb = X.Bond([((0, 0), 2), ((1, 1), 3)])
    rb = X.Bond([((1, 1), 2), ((2, 0), 2)])
    bad = np.zeros((4, 4))
    bad[1, 0] = 1.0  # empty -> alpha: shift (1, 1)
    with pytest.raises(RuntimeError, match="conservation"):
        X.HeffPlan(lb, rb, [(0, 0)], [(0, 0)], [(0, 0)], [(0, 0, bad)], [(0, 0, np.eye(4))])


def test_plan_rejects_unsorted_bond():
    lb = X.Bond([((1, 1), 2), ((0, 0), 3)])
    rb = X.Bond([((1, 1), 2)])
    with pytest.raises(RuntimeError, match="increasing"):
        X.HeffPlan(lb, rb, [(0, 0)], [(0, 0)], [(0, 0)], [(0, 0, np.eye(4))], [(0, 0, np.eye(4))])


def _count_flops(lbond, rbond, Ldq, Rdq, W1, W2):
    """Independent count of 2 m n k over the two block-GEMM rounds, counting only
    intermediate blocks (il, s1, s2', r') that the second round reads."""
    lidx = {q: i for i, (q, _) in enumerate(lbond)}
    ridx = {q: i for i, (q, _) in enumerate(rbond)}
    SQ = M.SITE_QN
    left, right = {}, {}
    for a, b, op in W1:
        for so in range(4):
            for si in range(4):
                if op[so, si] != 0:
                    left.setdefault(b, {}).setdefault((so, si), set()).add(a)
    for b, c, op in W2:
        for so in range(4):
            for si in range(4):
                if op[so, si] != 0:
                    right.setdefault(b, {}).setdefault((so, si), set()).add(c)
    psi = two_site_blocks(lbond, rbond)
    fl = 0.0
    for b in set(left) & set(right):
        read = set()
        for (so, si), as_ in left[b].items():
            dq = Ldq[next(iter(as_))]
            for il, (q, _) in enumerate(lbond):
                if (q[0] + dq[0], q[1] + dq[1]) in lidx:
                    read.add((il, si))
        tb = set()
        for (so, si), cs in right[b].items():
            dq = Rdq[next(iter(cs))]
            for (il, s1, s2, ir) in psi:
                if s2 != si or (il, s1) not in read:
                    continue
                q = rbond[ir][0]
                irp = ridx.get((q[0] + dq[0], q[1] + dq[1]))
                if irp is None:
                    continue
                fl += 2.0 * lbond[il][1] * rbond[ir][1] * rbond[irp][1]
                tb.add((il, s1, so, irp))
        for (il, s1, s2p, irp) in tb:
            for (so, si), as_ in left[b].items():
                if si != s1:
                    continue
                dq = Ldq[next(iter(as_))]
                q = lbond[il][0]
                ilp = lidx.get((q[0] + dq[0], q[1] + dq[1]))
                if ilp is None:
                    continue
                fl += 2.0 * lbond[ilp][1] * lbond[il][1] * rbond[irp][1]
    return fl


def test_plan_flop_count_matches_independent_count():
    K, M_ = 8, 64
    h, g = make_integrals(K, seed=0)
    m = M.build_nc_mpo(h, g)
    b = bond_sector_tables(K, K, 0, M_)
    for i in (1, 3, 5):
        W1, W2 = M.site_entries(m, i), M.site_entries(m, i + 1)
        p = X.HeffPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], W1, W2)
        ref = _count_flops(b[i], b[i + 2], [tuple(x) for x in m.dq[i]], [tuple(x) for x in m.dq[i + 2]], W1, W2)
        assert p.info.flops_useful == pytest.approx(ref, rel=1e-12)
        assert p.info.flops_useful <= p.info.flops_apply < 1.1 * p.info.flops_useful
        assert p.info.psi_nnz == sum(b[i][k[0]][1] * b[i + 2][k[3]][1] for k in two_site_blocks(b[i], b[i + 2]))


def test_plan_split_k_keeps_flops():
    K = 8
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 64)
    args = (b[3], b[5], m.dq[3], m.dq[4], m.dq[5], M.site_entries(m, 3), M.site_entries(m, 4))
    p1 = X.HeffPlan(*args)
    p2 = X.HeffPlan(*args, split_kseg_min=8)
    assert p2.info.n_tiles > p1.info.n_tiles
    assert p2.info.flops_apply == pytest.approx(p1.info.flops_apply, rel=1e-12)


def test_plan_chunking_keeps_flops():
    K = 8
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 64)
    args = (b[3], b[5], m.dq[3], m.dq[4], m.dq[5], M.site_entries(m, 3), M.site_entries(m, 4))
    p1 = X.HeffPlan(*args)
    p2 = X.HeffPlan(*args, t_budget_bytes=64 * 1024)
    assert p1.info.n_chunks == 1 and p2.info.n_chunks > 4
    assert p2.info.flops_apply == pytest.approx(p1.info.flops_apply, rel=1e-12)


def _small_plans():
    K = 8
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 32)
    return [X.HeffPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                       M.site_entries(m, i + 1)) for i in (1, 3, 4)]


def test_batch_plan_concatenates_instances():
    ps = _small_plans()
    B = X.BatchPlan(ps)
    assert B.info.flops_apply == pytest.approx(sum(p.info.flops_apply for p in ps), rel=1e-12)
    assert B.info.n_tiles == sum(p.info.n_tiles for p in ps)
    assert B.info.psi_nnz == sum(p.info.psi_nnz for p in ps)
    assert B.info.ws_bytes == sum(p.info.ws_bytes for p in ps)
    po = np.cumsum([0] + [p.info.psi_nnz for p in ps])[:-1]
    lo = np.cumsum([0] + [p.info.in_nnz for p in ps])[:-1]
    ro = np.cumsum([0] + [p.info.in2_nnz for p in ps])[:-1]
    assert B.offsets == [(int(a), int(b), int(c)) for a, b, c in zip(po, lo, ro)]


def test_batch_plan_merges_chunked_instances_round_by_round():
    """Instances split into different numbers of intermediate chunks merge into one
    plan with all their work and tiles; the merged sequence is as long as the longest
    instance's (one launch per round and form), not the sum."""
    K = 8
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 64)
    args = (b[3], b[5], m.dq[3], m.dq[4], m.dq[5], M.site_entries(m, 3), M.site_entries(m, 4))
    ps = [X.HeffPlan(*args, t_budget_bytes=64 * 1024), X.HeffPlan(*args, t_budget_bytes=256 * 1024),
          X.HeffPlan(*args)]
    chunks = [p.info.n_chunks for p in ps]
    assert chunks[0] > chunks[1] > 1 and chunks[2] == 1
    B = X.BatchPlan(ps)
    assert B.info.n_chunks == chunks[0]
    assert B.info.flops_apply == pytest.approx(sum(p.info.flops_apply for p in ps), rel=1e-12)
    assert B.info.n_tiles == sum(p.info.n_tiles for p in ps)
    assert B.info.ws_bytes == sum(p.info.ws_bytes for p in ps)
    with pytest.raises(RuntimeError, match="sigma-vector plan"):
        X.BatchPlan([X.EnvPlan(0, b[3], b[4], m.dq[3], m.dq[4], M.site_entries(m, 3))])


def test_vjp_plan_builds_for_every_site_of_the_nc_mpo():
    """The adjoint plan exists wherever the forward plan does; its work includes
    the recomputed first round plus four more block-GEMM rounds."""
    K = 8
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 32)
    for i in range(K - 1):
        args = (b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i), M.site_entries(m, i + 1))
        f = X.HeffPlan(*args)
        v = X.HeffVjpPlan(*args)
        assert v.info.psi_nnz == f.info.psi_nnz and v.info.in_nnz == f.info.in_nnz
        assert v.info.flops_apply > 2.0 * f.info.flops_apply


def test_autotune_coordinate_search_finds_separable_minimum():
    from paper_2310_03920_amd import autotune as A
    cost = {"kernel_variant": {0: 3.0, 1: 1.0, 2: 2.0, 3: 1.5, 4: 2.5, 5: 1.2, 6: 1.1},
            "split_kseg_min": {512: 0.6, 1024: 0.5, 2048: 0.7, 4096: 0.9},
            "t_budget_bytes": {1 << 29: 0.3, 1 << 30: 0.2, 1 << 31: 0.1}}
    calls = []

    def timer(o):
        calls.append(o)
        if o["kernel_variant"] == 2:
            return None  # a rejected candidate never wins
        return sum(cost[k][v] for k, v in o.items())

    best, seen = A.coordinate_search(timer)
    assert best == {"kernel_variant": 1, "split_kseg_min": 1024, "t_budget_bytes": 1 << 31}
    # start + the other values of each axis, no repeats
    assert len(calls) == len(seen) == 1 + sum(len(v) - 1 for _, v in A.AXES)
    assert all(c["kernel_variant"] != 3 for c in calls)  # the removed persistent variant is not searched


def test_removed_persistent_variant_is_rejected():
    K, i = 4, 1
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 16)
    with pytest.raises(RuntimeError, match="persistent workgroups"):
        X.HeffPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                   M.site_entries(m, i + 1), kernel_variant=3)


def test_autotune_signature_depends_on_shape():
    from paper_2310_03920_amd import autotune as A
    K = 8
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 32)
    w = [X.MpoSite.from_entries(M.site_entries(m, i)) for i in (3, 4)]
    s1 = A.signature(b[3], b[5], m.dq[3], m.dq[4], m.dq[5], *w)
    s2 = A.signature(b[3], b[5], m.dq[3], m.dq[4], m.dq[5], *w)
    b2 = bond_sector_tables(K, K, 0, 40)
    s3 = A.signature(b2[3], b2[5], m.dq[3], m.dq[4], m.dq[5], *w)
    assert s1 == s2 != s3


def test_psi1_layout_groups_site_blocks_by_right_sector():
    b = bond_sector_tables(8, 8, 0, 64)
    lb, rb = X.Bond(b[3]), X.Bond(b[4])
    keys, off = X.psi1_layout(lb, rb)
    skeys, soff = X.site_layout(lb, rb)
    assert sorted(keys) == sorted(skeys) and off[-1] == soff[-1]
    assert keys == sorted(keys, key=lambda k: (k[2], k[0], k[1]))
    np.testing.assert_array_equal(np.diff(off), [b[3][k[0]][1] * b[4][k[2]][1] for k in keys])
