"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
closed forms, textbook special cases, brute force on tiny inputs, invariants, and
the one energy the paper prints (Listing 1)."""

import json
import os

import numpy as np
import pytest

from oracle import contract, davidson, fock, holstein, mps
from synth import (bond_sector_tables, hubbard_integrals, make_integrals,
                   random_left_canonical_mps, random_right_canonical_mps)
from synth.blocks import random_env, random_psi, random_site_ops, random_site_tensor, two_site_blocks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SITE_N, SITE_S = (0, 1, 1, 2), (0, 1, -1, 0)  # (N, 2Sz) of [empty, alpha, beta, alpha-beta]


# ---------------------------------------------------------------- Fock space

def test_canonical_anticommutation():
    K = 2
    dets = fock.all_dets(K)
    ops = {}
    for j in range(2 * K):
        ops[(j, True)] = fock.op_matrix(dets, [(j, True)]).toarray()
        ops[(j, False)] = fock.op_matrix(dets, [(j, False)]).toarray()
    eye = np.eye(len(dets))
    for i in range(2 * K):
        for j in range(2 * K):
            a, ad = ops[(i, False)], ops[(j, True)]
            np.testing.assert_allclose(a @ ad + ad @ a, eye * (i == j), atol=0)
            b = ops[(j, False)]
            np.testing.assert_allclose(a @ b + b @ a, 0 * eye, atol=0)
        np.testing.assert_allclose(ops[(i, True)], ops[(i, False)].T, atol=0)


def test_listing1_site_matrices_are_jordan_wigner_site_operators():
    """The printed on-site matrices equal a+_alpha, a_alpha, a+_beta, a_beta of one
    orbital in the determinant convention (alpha before beta)."""
    dets = fock.all_dets(1)  # bit0 = alpha, bit1 = beta -> [0, a, b, ab] = site basis order
    printed = {
        (0, True): [[0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0]],
        (0, False): [[0, 1, 0, 0], [0, 0, 0, 0], [0, 0, 0, 1], [0, 0, 0, 0]],
        (1, True): [[0, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [0, -1, 0, 0]],
        (1, False): [[0, 0, 1, 0], [0, 0, 0, -1], [0, 0, 0, 0], [0, 0, 0, 0]],
    }
    for (j, dag), m in printed.items():
        np.testing.assert_array_equal(fock.op_matrix(dets, [(j, dag)]).toarray(), np.array(m, float))


@pytest.mark.parametrize("K,N,twosz", [(3, 3, 1), (3, 2, 0), (2, 2, 0)])
def test_hamiltonian_matches_term_by_term_bruteforce(K, N, twosz):
    h, g = make_integrals(K, seed=11)
    d = fock.sector_dets(K, N, twosz)
    A = fock.hamiltonian(h, g, d).toarray()
    B = fock.hamiltonian_bruteforce(h, g, d).toarray()
    np.testing.assert_allclose(A, B, atol=1e-13)
    np.testing.assert_allclose(A, A.T, atol=1e-13)


def test_hamiltonian_conserves_n_and_sz():
    K = 3
    h, g = make_integrals(K, seed=3)
    dets = fock.all_dets(K)
    H = fock.hamiltonian(h, g, dets).tocoo()
    na = lambda x: fock.popcount(x & 0b010101)  # noqa: E731
    nb = lambda x: fock.popcount(x & 0b101010)  # noqa: E731
    r, c = dets[H.row], dets[H.col]
    keep = np.abs(H.data) > 1e-14
    assert np.all(na(r[keep]) == na(c[keep])) and np.all(nb(r[keep]) == nb(c[keep]))


@pytest.mark.parametrize("K,N,twosz", [(3, 3, 1), (3, 2, 0)])
def test_rdms_match_operator_products_traces_and_energy(K, N, twosz):
    """The E-form 2-RDM equals the four-operator definition term by term; its pair
    trace is N(N-1), tr(gamma) = N; and <v|H|v> = sum h gamma + 1/2 sum g Gamma with H
    assembled term by term, for integrals with no symmetry (so a transposed index
    or a dropped delta term fails)."""
    import itertools
    dets = fock.sector_dets(K, N, twosz)
    rng = np.random.default_rng(K * 10 + N)
    v = rng.standard_normal(len(dets))
    v /= np.linalg.norm(v)
    G = fock.two_rdm(v, dets, K)
    gam = fock.one_rdm(v, dets, K)
    B = np.zeros_like(G)
    for p, q, r, s in itertools.product(range(K), repeat=4):
        for si in range(2):
            for ti in range(2):
                op = fock.op_matrix(dets, [(2 * p + si, True), (2 * r + ti, True), (2 * s + ti, False),
                                           (2 * q + si, False)])
                B[p, q, r, s] += v @ (op @ v)
    np.testing.assert_allclose(G, B, atol=1e-13)
    assert abs(np.einsum("pprr->", G) - N * (N - 1)) < 1e-12
    assert abs(np.trace(gam) - N) < 1e-12
    h = rng.standard_normal((K, K))
    g = rng.standard_normal((K, K, K, K))
    H = fock.hamiltonian_bruteforce(h, g, dets)
    assert abs(v @ (H @ v) - (np.sum(h * gam) + 0.5 * np.sum(g * G))) < 1e-12


def test_noninteracting_closed_form():
    K, N = 6, 6
    h, _ = make_integrals(K, seed=5)
    eps = np.linalg.eigvalsh(h)
    for twosz in (0, 2):
        na, nb = (N + twosz) // 2, (N - twosz) // 2
        e = fock.fci_energy(h, np.zeros((K,) * 4), N, twosz)
        assert abs(e - (eps[:na].sum() + eps[:nb].sum())) < 1e-11


def test_single_orbital_doubly_occupied():
    h = np.array([[-0.7]])
    g = np.full((1, 1, 1, 1), 0.45)
    assert abs(fock.fci_energy(h, g, 2, 0) - (2 * -0.7 + 0.45)) < 1e-14


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.5, 1.0), (1.0, 0.0)])
def test_hubbard_dimer_closed_form(t, U):
    h, g = hubbard_integrals(2, t, U)
    e = fock.fci_energy(h, g, 2, 0)
    assert abs(e - (U / 2 - np.sqrt(U * U / 4 + 4 * t * t))) < 1e-12


def test_listing1_hubbard_holstein_printed_energy():
    ref = json.load(open(os.path.join(GOLDEN, "listing1_hubbard_holstein.json")))
    e, dim = holstein.ground_energy(n_sites=ref["n_sites_elec"], n_ph=ref["n_ph"], U=ref["U"],
                                    omega=ref["omega"], g=ref["g"], n_elec=ref["n_elec"],
                                    twosz=ref["twosz"])
    assert dim == 36 * 11 ** 4
    assert abs(e - ref["energy"]) < 0.5 * 10 ** (-ref["printed_digits"])


# ---------------------------------------------------------------- MPS / P^T H P

def _embedding(K, M, i, seed=0):
    h, g = make_integrals(K, seed=seed)
    bonds = bond_sector_tables(K, K, 0, M)
    left = random_left_canonical_mps(bonds, seed + 1)
    right = random_right_canonical_mps(bonds, seed + 2)
    emb = mps.Embedding(h, g, K, 0, left[:i], right[i + 2:], bonds, i)
    return h, g, bonds, emb


def test_embedding_is_isometry_and_hermitian():
    K, M, i = 6, 8, 2
    _, _, bonds, emb = _embedding(K, M, i)
    keys = two_site_blocks(bonds[i], bonds[i + 2])
    P = emb.embedding_matrix(keys)
    np.testing.assert_allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-13)
    Hm = emb.heff_matrix(keys)
    np.testing.assert_allclose(Hm, Hm.T, atol=1e-12)


def test_embedding_apply_matches_matrix():
    K, M, i = 6, 8, 1
    _, _, bonds, emb = _embedding(K, M, i)
    keys = two_site_blocks(bonds[i], bonds[i + 2])
    rng = np.random.default_rng(0)
    psi = random_psi(bonds[i], bonds[i + 2], rng)
    dense = mps.dense_two_site(psi, bonds[i], bonds[i + 2])
    sig = mps.two_site_blocks_from_dense(emb.apply(dense), bonds[i], bonds[i + 2], keys)
    vec = np.concatenate([psi[k].ravel() for k in keys])
    ref = emb.heff_matrix(keys) @ vec
    got = np.concatenate([sig[k].ravel() for k in keys])
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_complete_basis_two_site_space_gives_fci():
    """K=6 with M=16: bonds 2 and 4 hold complete bases (4^2 = 16 states), so the
    middle two-site space is the whole sector and H_eff's lowest eigenvalue is E_FCI."""
    K, M, i = 6, 16, 2
    h, g, bonds, emb = _embedding(K, M, i)
    assert sum(m for _, m in bonds[i]) == 16 and sum(m for _, m in bonds[i + 2]) == 16
    keys = two_site_blocks(bonds[i], bonds[i + 2])
    w = np.linalg.eigvalsh(emb.heff_matrix(keys))
    assert abs(w[0] - fock.fci_energy(h, g, K, 0)) < 1e-11


@pytest.mark.slow
def test_config1_middle_step_dimension_and_fci():
    """8 orbitals, 8 electrons, M=64: bonds 3 and 5 are complete (64 = 4^3 states),
    the middle two-site space has the FCI dimension 4900, and E0(H_eff) = E_FCI."""
    from math import comb
    K, M, i = 8, 64, 3
    h, g, bonds, emb = _embedding(K, M, i)
    for b in (bonds[3], bonds[5]):
        assert sum(m for _, m in b) == 64
    for q, m in bonds[3]:
        na, nb = (q[0] + q[1]) // 2, (q[0] - q[1]) // 2
        assert m == comb(3, na) * comb(3, nb)
    keys = two_site_blocks(bonds[i], bonds[i + 2])
    assert len(keys) == 196
    assert sum(bonds[i][k[0]][1] * bonds[i + 2][k[3]][1] for k in keys) == 4900 == comb(8, 4) ** 2
    w = np.linalg.eigvalsh(emb.heff_matrix(keys))
    assert abs(w[0] - fock.fci_energy(h, g, K, 0)) < 1e-10


# ---------------------------------------------------------------- contractions

def _tiny_operands(seed=0):
    rng = np.random.default_rng(seed)
    lb = [((0, 0), 1), ((1, -1), 2), ((1, 1), 2), ((2, 0), 3)]
    rb = [((1, 1), 2), ((2, 0), 2), ((3, 1), 1), ((3, -1), 2)]
    dqs = [(0, 0), (1, 1), (-1, -1), (1, -1), (0, 2), (-1, 1)]
    L = random_env(lb, dqs, rng)
    mid = [(0, 0), (1, 1), (-1, 1), (0, 0), (2, 0), (0, -2)]
    R = random_env(rb, dqs, rng)
    W1 = random_site_ops(dqs, mid, rng)
    W2 = random_site_ops(mid, dqs, rng)
    psi = random_psi(lb, rb, rng)
    return lb, rb, L, R, W1, W2, psi, len(dqs), len(mid)


def test_sigma_einsum_matches_kron_bruteforce():
    lb, rb, L, R, W1e, W2e, psi, D, Dm = _tiny_operands()
    Ld, Rd = contract.dense_env(L, lb), contract.dense_env(R, rb)
    W1, W2 = contract.dense_mpo(W1e, D, Dm), contract.dense_mpo(W2e, Dm, D)
    P = mps.dense_two_site(psi, lb, rb)
    s = contract.heff_apply(Ld, W1, W2, Rd, P)
    H = contract.heff_matrix_kron(Ld, W1, W2, Rd)
    np.testing.assert_allclose(s.ravel(), H @ P.ravel(), atol=1e-12)
    d = contract.heff_diag(Ld, W1, W2, Rd)
    np.testing.assert_allclose(d.ravel(), np.diag(H), atol=1e-12)


def test_sigma_identity_mpo_reduces_to_matrix_products():
    rng = np.random.default_rng(4)
    lb = [((0, 0), 3), ((1, 1), 2)]
    rb = [((1, 1), 2), ((2, 0), 4), ((2, 2), 1)]
    L = random_env(lb, [(0, 0)], rng)
    R = random_env(rb, [(0, 0)], rng)
    W = [(0, 0, np.eye(4))]
    psi = random_psi(lb, rb, rng)
    s = contract.heff_apply(contract.dense_env(L, lb), contract.dense_mpo(W, 1, 1),
                            contract.dense_mpo(W, 1, 1), contract.dense_env(R, rb),
                            mps.dense_two_site(psi, lb, rb))
    lo, _ = mps.bond_offsets(lb)
    ro, _ = mps.bond_offsets(rb)
    for (il, s1, s2, ir), blk in psi.items():
        ref = L[0]["blocks"][il] @ blk @ R[0]["blocks"][ir].T
        got = s[lo[il]:lo[il] + blk.shape[0], s1, s2, ro[ir]:ro[ir] + blk.shape[1]]
        np.testing.assert_allclose(got, ref, atol=1e-13)


def test_env_updates_match_kron_bruteforce():
    rng = np.random.default_rng(7)
    lb = [((0, 0), 2), ((1, 1), 2), ((1, -1), 1)]
    nb = [((1, 1), 2), ((2, 0), 3), ((1, -1), 2), ((2, 2), 1)]
    dqs = [(0, 0), (1, 1), (-1, 1)]
    mid = [(0, 0), (1, -1), (0, 2)]
    L = contract.dense_env(random_env(lb, dqs, rng), lb)
    W = contract.dense_mpo(random_site_ops(dqs, mid, rng), len(dqs), len(mid))
    A = mps.dense_site_tensor(random_site_tensor(lb, nb, rng), lb, nb)
    Lp = contract.env_update_left(L, W, A)
    Am = A.reshape(-1, A.shape[2])
    for b in range(len(mid)):
        ref = sum(Am.T @ np.kron(L[a], W[a, b]) @ Am for a in range(len(dqs)))
        np.testing.assert_allclose(Lp[b], ref, atol=1e-12)
    R = contract.dense_env(random_env(nb, mid, rng), nb)
    Bt = mps.dense_site_tensor(random_site_tensor(lb, nb, rng), lb, nb)
    Rp = contract.env_update_right(R, W, Bt)
    Bm = Bt.reshape(Bt.shape[0], -1)
    for a in range(len(dqs)):
        ref = sum(Bm @ np.kron(W[a, b], R[b]) @ Bm.T for b in range(len(mid)))
        np.testing.assert_allclose(Rp[a], ref, atol=1e-12)


def test_sigma_rows_match_dense_definition():
    lb, rb, L, R, W1e, W2e, psi, D, Dm = _tiny_operands(seed=2)
    s = contract.heff_apply(contract.dense_env(L, lb), contract.dense_mpo(W1e, D, Dm),
                            contract.dense_mpo(W2e, Dm, D), contract.dense_env(R, rb),
                            mps.dense_two_site(psi, lb, rb))
    lo, _ = mps.bond_offsets(lb)
    ro, _ = mps.bond_offsets(rb)
    rows = [(il, s1, x) for il, (_, m) in enumerate(lb) for s1 in range(4) for x in range(m)]
    got = contract.sigma_rows(lb, rb, L, W1e, W2e, R, psi, rows)
    for (il, s1, x), acc in got.items():
        full = np.zeros((4, s.shape[3]))
        for (s2, ir), vec in acc.items():
            full[s2, ro[ir]:ro[ir] + len(vec)] += vec
        np.testing.assert_allclose(full, s[lo[il] + x, s1], atol=1e-12)


def test_one_site_sigma_matches_kron_bruteforce_and_identity_mpo():
    rng = np.random.default_rng(8)
    A, B, Dl, Dr = 3, 4, 5, 6
    L, W, R = rng.standard_normal((A, Dl, Dl)), rng.standard_normal((A, B, 4, 4)), rng.standard_normal((B, Dr, Dr))
    psi = rng.standard_normal((Dl, 4, Dr))
    s = contract.heff1_apply(L, W, R, psi)
    np.testing.assert_allclose(s.ravel(), contract.heff1_matrix_kron(L, W, R) @ psi.ravel(), atol=1e-11)
    # identity MPO: sigma[:, s, :] = L psi[:, s, :] R^T
    s1 = contract.heff1_apply(L[:1], np.eye(4)[None, None], R[:1], psi)
    for t in range(4):
        np.testing.assert_allclose(s1[:, t, :], L[0] @ psi[:, t, :] @ R[0].T, atol=1e-12)


@pytest.mark.parametrize("K,i", [(5, 2), (6, 2), (6, 3)])
def test_one_site_embedding_complete_basis_gives_fci(K, i):
    """Where bond i spans the whole left space and bond i+1 the whole right space
    (centre sites: i >= (K-2)/2 and i <= K/2), the one-site P^T H P holds the ground
    state: its lowest eigenvalue is the FCI energy, and P is an isometry."""
    h, g = make_integrals(K, seed=4)
    tsz = K % 2
    bonds = bond_sector_tables(K, K, tsz, 10 ** 6)
    left = random_left_canonical_mps(bonds, 3)
    right = random_right_canonical_mps(bonds, 4)
    emb = mps.Embedding1(h, g, K, tsz, left[:i], right[i + 1:], bonds, i)
    lb, rb = bonds[i], bonds[i + 1]
    lo, Dl = mps.bond_offsets(lb)
    ro, Dr = mps.bond_offsets(rb)
    cols = []
    for il, (ql, ml) in enumerate(lb):
        for s_ in range(4):
            for ir, (qr, mr) in enumerate(rb):
                if (ql[0] + SITE_N[s_], ql[1] + SITE_S[s_]) != tuple(qr):
                    continue
                for x in range(ml):
                    for y in range(mr):
                        e = np.zeros((Dl, 4, Dr))
                        e[lo[il] + x, s_, ro[ir] + y] = 1.0
                        cols.append(emb.to_fock(e))
    P = np.array(cols).T
    np.testing.assert_allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-10)
    w = np.linalg.eigvalsh(P.T @ (emb.H @ P))
    assert w[0] == pytest.approx(fock.fci_energy(h, g, K, tsz), abs=1e-10)


def _dense_random_operands(seed):
    """Dense random operands (no symmetry) of a tiny two-site problem."""
    rng = np.random.default_rng(seed)
    A, Bm, Dl, Dr = 3, 4, 5, 6  # left ops, mid ops, left dim, right dim
    return (rng.standard_normal((A, Dl, Dl)), rng.standard_normal((A, Bm, 4, 4)),
            rng.standard_normal((Bm, 2, 4, 4)), rng.standard_normal((2, Dr, Dr)),
            rng.standard_normal((Dl, 4, 4, Dr)), rng.standard_normal((Dl, 4, 4, Dr)))


@pytest.mark.parametrize("seed", [0, 1])
def test_vjp_is_adjoint_of_each_linear_slot(seed):
    """sigma is linear in each operand X, so <dX, V> must equal <g, sigma(X -> V)>
    for any V: pins every index and term of the VJP against heff_apply."""
    L, W1, W2, R, psi, g = _dense_random_operands(seed)
    gL, gW1, gW2, gR, gpsi = contract.heff_vjp(L, W1, W2, R, psi, g)
    rng = np.random.default_rng(100 + seed)
    args = [L, W1, W2, R, psi]
    for slot, grad in zip(range(5), (gL, gW1, gW2, gR, gpsi)):
        V = rng.standard_normal(args[slot].shape)
        a2 = list(args)
        a2[slot] = V
        lhs = np.sum(grad * V)
        rhs = np.sum(g * contract.heff_apply(*a2))
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-10), slot


def test_vjp_psi_is_transpose_of_kron_matrix():
    lb, rb, L, R, W1e, W2e, psi, D, Dm = _tiny_operands(seed=3)
    Ld, Rd = contract.dense_env(L, lb), contract.dense_env(R, rb)
    W1, W2 = contract.dense_mpo(W1e, D, Dm), contract.dense_mpo(W2e, Dm, D)
    P = mps.dense_two_site(psi, lb, rb)
    g = np.random.default_rng(9).standard_normal(P.shape)
    gpsi = contract.heff_vjp(Ld, W1, W2, Rd, P, g)[4]
    H = contract.heff_matrix_kron(Ld, W1, W2, Rd)
    np.testing.assert_allclose(gpsi.ravel(), H.T @ g.ravel(), atol=1e-12)


def test_energy_gradient_matches_central_differences():
    """E = <psi|H_eff|psi>: dE/dX from the VJP with g = psi (plus H psi for psi
    itself) against central differences, step 1e-5, along random directions."""
    L, W1, W2, R, psi, _ = _dense_random_operands(5)
    args = [L, W1, W2, R, psi]
    sigma = contract.heff_apply(*args)
    grads = list(contract.heff_vjp(*args, psi))
    grads[4] = grads[4] + sigma

    def energy(a):
        return float(np.sum(a[4] * contract.heff_apply(*a)))

    rng = np.random.default_rng(6)
    h = 1e-5
    for slot in range(5):
        V = rng.standard_normal(args[slot].shape)
        ap, am = list(args), list(args)
        ap[slot] = args[slot] + h * V
        am[slot] = args[slot] - h * V
        fd = (energy(ap) - energy(am)) / (2 * h)
        assert np.sum(grads[slot] * V) == pytest.approx(fd, rel=1e-6), slot


def test_vjp_euler_identity():
    """Degree-1 homogeneity in each operand: <dX, X> = <g, sigma> for all five."""
    L, W1, W2, R, psi, g = _dense_random_operands(2)
    ref = np.sum(g * contract.heff_apply(L, W1, W2, R, psi))
    for grad, x in zip(contract.heff_vjp(L, W1, W2, R, psi, g), (L, W1, W2, R, psi)):
        assert np.sum(grad * x) == pytest.approx(ref, rel=1e-12)


# ---------------------------------------------------------------- Davidson

def test_davidson_step_invariants_and_solve():
    rng = np.random.default_rng(1)
    n = 60
    A = rng.standard_normal((n, n))
    H = 0.5 * (A + A.T) + np.diag(np.arange(n, dtype=float))
    d = np.diag(H).copy()
    V, _ = np.linalg.qr(rng.standard_normal((n, 4)))
    V = V.T
    theta, rnorm, x, hx, t, tnorm = davidson.step(V, V @ H, d)
    assert abs(theta - x @ H @ x) < 1e-12 and abs(np.linalg.norm(x) - 1) < 1e-13
    np.testing.assert_allclose(V @ t, 0, atol=1e-13)
    assert abs(np.linalg.norm(t) - 1) < 1e-13
    assert abs(rnorm - np.linalg.norm(H @ x - theta * x)) < 1e-12
    e, xs, nmv, rn = davidson.solve(lambda v: H @ v, rng.standard_normal(n), d, tol=1e-10, kmax=8)
    assert rn < 1e-10
    assert abs(e - np.linalg.eigvalsh(H)[0]) < 1e-12


def test_env_rows_match_dense_updates():
    """Selected rows of both environment updates, from the block formats, equal the
    dense definitions (themselves pinned by Kronecker brute force above)."""
    rng = np.random.default_rng(9)
    lb = [((0, 0), 2), ((1, 1), 2), ((1, -1), 1)]
    nb = [((1, 1), 2), ((2, 0), 3), ((1, -1), 2), ((2, 2), 1)]
    dqs = [(0, 0), (1, 1), (-1, 1)]
    mid = [(0, 0), (1, -1), (0, 2)]
    Le = random_env(lb, dqs, rng)
    We = random_site_ops(dqs, mid, rng)
    At = random_site_tensor(lb, nb, rng)
    W = contract.dense_mpo(We, len(dqs), len(mid))
    Lp = contract.env_update_left(contract.dense_env(Le, lb), W, mps.dense_site_tensor(At, lb, nb))
    no, _ = mps.bond_offsets(nb)
    rows = [(b, iq, m) for b in range(len(mid)) for iq, (_, d) in enumerate(nb) for m in range(d)]
    got = contract.env_rows_left(lb, nb, Le, We, At, rows)
    for (b, iq, m), acc in got.items():
        full = np.zeros(Lp.shape[2])
        for iqn, vec in acc.items():
            full[no[iqn]:no[iqn] + len(vec)] += vec
        np.testing.assert_allclose(full, Lp[b, no[iq] + m], atol=1e-12)
    Re = random_env(nb, mid, rng)
    Bt = random_site_tensor(lb, nb, rng)
    Rp = contract.env_update_right(contract.dense_env(Re, nb), W, mps.dense_site_tensor(Bt, lb, nb))
    lo, _ = mps.bond_offsets(lb)
    rows = [(a, iq, m) for a in range(len(dqs)) for iq, (_, d) in enumerate(lb) for m in range(d)]
    got = contract.env_rows_right(nb, lb, Re, We, Bt, rows)
    for (a, iq, m), acc in got.items():
        full = np.zeros(Rp.shape[2])
        for iqn, vec in acc.items():
            full[lo[iqn]:lo[iqn] + len(vec)] += vec
        np.testing.assert_allclose(full, Rp[a, lo[iq] + m], atol=1e-12)
