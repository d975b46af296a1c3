"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Every test here runs on the CPU.  The pins are: the second-quantised
Hamiltonian built from Jordan-Wigner matrices (textbook operator algebra, no
Slater-Condon rules), closed forms for one electron per spin and for
non-interacting electrons, the complete-space resolution-of-identity form of
H (valid only when every string is kept), LAPACK diagonalisation, Cauchy
interlacing over nested selections, the colex rank of complete string lists,
and the link-table entry counts printed in the paper (Sec. III.C).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2503_10335_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _jw_annihilators(K):
    """Dense Jordan-Wigner annihilators on K modes; basis bit X = mode X."""
    dim = 1 << K
    out = []
    for X in range(K):
        A = np.zeros((dim, dim))
        for n in range(dim):
            if (n >> X) & 1:
                A[n ^ (1 << X), n] = (-1.0) ** bin(n & ((1 << X) - 1)).count("1")
        out.append(A)
    return out


@pytest.fixture(scope="module")
def fock4():
    from oracle import oracle as O
    M = 4
    h, eri = W.integrals(M, 11)
    return M, h, eri, O.fock_hamiltonian(M, h, eri).toarray()


@pytest.mark.parametrize("na,nb,la,lb,seed", [
    (2, 2, 5, 4, 1), (1, 2, 4, 6, 2), (3, 1, 4, 3, 3), (2, 2, 6, 6, 4), (0, 2, 1, 5, 5),
    (2, 0, 6, 1, 6), (1, 1, 4, 4, 7), (3, 3, 4, 4, 8),
])
def test_elements_match_jordan_wigner(oracle_mod, fock4, na, nb, la, lb, seed):
    """Oracle P H P (every element) equals the JW Fock-space H restricted to D_TPB."""
    M, h, eri, H = fock4
    rng = np.random.default_rng(seed)
    A = W.all_strings(M, na)
    B = W.all_strings(M, nb)
    a = A[rng.permutation(len(A))[:la]]
    b = B[rng.permutation(len(B))[:lb]]
    sp = oracle_mod.Space(M, na, nb, h, eri, a, b)
    Ho = sp.dense_h()
    idx = [oracle_mod.fock_index(x, y, M) for x in a for y in b]
    Hj = H[np.ix_(idx, idx)]
    assert np.abs(Ho - Hj).max() < 1e-13
    # sigma (excitation enumeration + hash lookup) agrees with the element path
    C = rng.standard_normal((len(a), len(b)))
    assert np.abs(sp.sigma(C).ravel() - Hj @ C.ravel()).max() < 1e-13
    assert np.abs(sp.diag().ravel() - np.diag(Hj)).max() < 1e-13


def test_one_electron_per_spin_closed_form(oracle_mod):
    """N_alpha = N_beta = 1, all strings: H[(i,j),(k,l)] = h_ik d_jl + d_ik h_jl + (ik|jl)."""
    M = 6
    h, eri = W.integrals(M, 21)
    a = W.all_strings(M, 1)  # 1<<p ascending, so position = orbital
    sp = oracle_mod.Space(M, 1, 1, h, eri, a, a)
    H = sp.dense_h()
    I = np.eye(M)
    ref = (np.einsum("ik,jl->ijkl", h, I) + np.einsum("ik,jl->ijkl", I, h)
           + np.einsum("ikjl->ijkl", eri)).reshape(M * M, M * M)
    assert np.abs(H - ref).max() < 1e-13


def test_alpha_only_is_h(oracle_mod):
    M = 7
    h, eri = W.integrals(M, 22)
    a = W.all_strings(M, 1)
    sp = oracle_mod.Space(M, 1, 0, h, eri, a, np.zeros(1, dtype=np.uint64))
    assert np.abs(sp.dense_h() - h).max() < 1e-14


def test_noninteracting_energy(oracle_mod):
    """(pq|rs) = 0, complete space: E0 = lowest N_alpha + lowest N_beta orbital energies."""
    M, na, nb = 7, 3, 2
    h, _ = W.integrals(M, 23)
    eri = np.zeros((M,) * 4)
    sp = oracle_mod.Space(M, na, nb, h, eri, W.all_strings(M, na), W.all_strings(M, nb))
    eps = np.linalg.eigvalsh(h)
    e_ref = eps[:na].sum() + eps[:nb].sum()
    e_dense, _ = oracle_mod.lowest_eigpair_dense(sp.dense_h())
    assert abs(e_dense - e_ref) < 1e-12
    res = oracle_mod.davidson(sp.sigma, sp.diag(), tol=1e-9)
    assert res["converged"] and abs(res["energy"] - e_ref) < 1e-10


def _ri_sigma(M, h, eri, a, b, C):
    """Complete-space sigma from E_pq products (valid only with all strings kept):
    H = sum_pq k_pq E_pq + 1/2 sum_pqrs (pq|rs) E_pq E_rs, k = h - 1/2 sum_r (pr|rq)."""
    def ops(strs):
        idx = {int(s): i for i, s in enumerate(strs)}
        n = len(strs)
        E = np.zeros((M, M, n, n))
        for j, J in enumerate(map(int, strs)):
            for q in range(M):
                if not (J >> q) & 1:
                    continue
                sgn_q = (-1) ** bin(J & ((1 << q) - 1)).count("1")
                K = J ^ (1 << q)
                for p in range(M):
                    if (K >> p) & 1:
                        continue
                    sgn_p = (-1) ** bin(K & ((1 << p) - 1)).count("1")
                    E[p, q, idx[K | (1 << p)], j] = sgn_q * sgn_p
        return E
    Ea, Eb = ops(a), ops(b)
    app = lambda p, q, X: Ea[p, q] @ X + X @ Eb[p, q].T
    k = h - 0.5 * np.einsum("prrq->pq", eri)
    out = np.zeros_like(C)
    for p in range(M):
        for q in range(M):
            out += k[p, q] * app(p, q, C)
    for r in range(M):
        for s in range(M):
            T = app(r, s, C)
            for p in range(M):
                for q in range(M):
                    if eri[p, q, r, s] != 0.0:
                        out += 0.5 * eri[p, q, r, s] * app(p, q, T)
    return out


def test_complete_space_matches_ri_form(oracle_mod):
    M, na, nb = 6, 3, 2
    h, eri = W.integrals(M, 24)
    a, b = W.all_strings(M, na), W.all_strings(M, nb)
    C = np.random.default_rng(0).standard_normal((len(a), len(b)))
    sp = oracle_mod.Space(M, na, nb, h, eri, a, b)
    assert np.abs(sp.sigma(C) - _ri_sigma(M, h, eri, a, b, C)).max() < 1e-12


def test_hermiticity_and_spin_flip(oracle_mod):
    p = W.make_problem("t", 10, 5, 60, 31, 41)
    sp = oracle_mod.Space.of(p)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((sp.la, sp.lb))
    y = rng.standard_normal((sp.la, sp.lb))
    sx, sy = sp.sigma(x), sp.sigma(y)
    assert abs((x * sy).sum() - (sx * y).sum()) < 1e-12 * np.abs(sx).sum()
    # identical alpha/beta lists and N_alpha = N_beta: sigma(C^T) = sigma(C)^T
    assert np.abs(sp.sigma(x.T) - sx.T).max() < 1e-12
    # ground state is spin-flip symmetric or antisymmetric
    e, v = oracle_mod.lowest_eigpair_dense(sp.dense_h())
    V = v.reshape(sp.la, sp.lb)
    assert min(np.abs(V - V.T).max(), np.abs(V + V.T).max()) < 1e-8


def test_sigma_selected_vs_dense_with_independent_lists(oracle_mod):
    p = W.make_problem("t", 9, 4, 40, 32, 42, independent_beta=True)
    sp = oracle_mod.Space.of(p)
    C = np.random.default_rng(2).standard_normal((sp.la, sp.lb))
    H = sp.dense_h()
    assert np.abs(H - H.T).max() == 0.0
    assert np.abs(sp.sigma(C).ravel() - H @ C.ravel()).max() < 1e-12
    rows = np.array([0, 7, 39, 3])
    assert np.abs(sp.sigma(C, rows=rows) - sp.sigma(C)[rows]).max() == 0.0


def test_interlacing_over_nested_selections(oracle_mod):
    """Nested string selections give non-increasing E0, bounded below by FCI."""
    M, N = 8, 4
    h, eri = W.integrals(M, 33)
    ranked = W.select_strings(M, N, 70, h, 43)
    energies = []
    for n in (10, 25, 45, 70):
        s = ranked[:n]
        sp = oracle_mod.Space(M, N, N, h, eri, s, s)
        energies.append(oracle_mod.lowest_eigpair_dense(sp.dense_h())[0])
    assert all(e1 >= e2 - 1e-12 for e1, e2 in zip(energies, energies[1:]))
    full = oracle_mod.Space(M, N, N, h, eri, W.all_strings(M, N), W.all_strings(M, N))
    e_fci = oracle_mod.lowest_eigpair_dense(full.dense_h())[0]
    assert abs(energies[-1] - e_fci) < 1e-10


def test_davidson_matches_eigh_fci_m8(oracle_mod):
    p = W.config("fci_m8")
    sp = oracle_mod.Space.of(p)
    e_ref, x_ref = oracle_mod.lowest_eigpair_dense(sp.dense_h())
    res = oracle_mod.davidson(sp.sigma, sp.diag(), tol=1e-8, n_max=8)
    assert res["converged"]
    assert abs(res["energy"] - e_ref) < 1e-10
    assert np.abs(np.abs(res["x"]) - np.abs(x_ref)).max() < 1e-6


def test_same_spin_matrix_vs_jordan_wigner(oracle_mod):
    """One-spin Hamiltonian between selected strings vs the JW H with the
    other spin empty."""
    M = 4
    h, eri = W.integrals(M, 25)
    H = oracle_mod.fock_hamiltonian(M, h, eri).toarray()
    s = W.all_strings(M, 2)[[0, 2, 3, 5]]
    sp = oracle_mod.Space(M, 2, 2, h, eri, s, s)
    ia = [oracle_mod.fock_index(x, 0, M) for x in s]
    ib = [oracle_mod.fock_index(0, x, M) for x in s]
    assert np.abs(sp.same_spin_matrix(0) - H[np.ix_(ia, ia)]).max() < 1e-13
    assert np.abs(sp.same_spin_matrix(1) - H[np.ix_(ib, ib)]).max() < 1e-13


def test_list_signs_vs_jordan_wigner(oracle_mod):
    """Every single/double entry's sign equals the JW matrix element of its operator."""
    M, N = 6, 3
    ann = _jw_annihilators(M)
    cre = [a.T for a in ann]
    rng = np.random.default_rng(3)
    strs = W.all_strings(M, N)[rng.permutation(20)[:14]]
    ptr, ent = oracle_mod.lists(strs, M, 1)
    n1 = 0
    for r, I in enumerate(strs):
        for e in ent[ptr[r]:ptr[r + 1]]:
            j, p, q, sg = e[0], e[1], e[2], e[5]
            J = int(strs[j])
            assert (cre[p] @ ann[q])[int(I), J] == sg
            n1 += 1
    ptr, ent = oracle_mod.lists(strs, M, 2)
    n2 = 0
    for r, I in enumerate(strs):
        for e in ent[ptr[r]:ptr[r + 1]]:
            j, i, jj, a, b, sg = e
            J = int(strs[j])
            assert (cre[i] @ cre[jj] @ ann[b] @ ann[a])[int(I), J] == sg
            n2 += 1
    # the lists hold exactly the degree-1 / degree-2 pairs of the selection
    pc = lambda x: bin(x).count("1")
    assert n1 == sum(1 for x in strs for y in strs if pc(int(x) ^ int(y)) == 2)
    assert n2 == sum(1 for x in strs for y in strs if pc(int(x) ^ int(y)) == 4)


def test_list_counts_complete():
    from oracle import oracle as O
    for M, N in [(8, 4), (10, 3), (9, 6)]:
        s = W.all_strings(M, N)
        ptr, _ = O.lists(s, M, 1)
        assert np.all(np.diff(ptr) == N * (M - N))
        ptr, _ = O.lists(s, M, 2)
        assert np.all(np.diff(ptr) == math.comb(N, 2) * math.comb(M - N, 2))
        ptr, ent = O.singles_with_diag(s, M)
        assert np.all(np.diff(ptr) == N * (M - N) + N)


def test_string_index_colex_rank():
    """Complete lists: ascending position equals the colex rank sum_k C(p_k, k+1)."""
    from oracle import oracle as O
    M, N = 9, 4
    s = W.all_strings(M, N)
    perm = np.random.default_rng(4).permutation(len(s))
    keys, pos = O.string_index(s[perm])
    for rank, (k, p) in enumerate(zip(keys, pos)):
        occ = [b for b in range(M) if (int(k) >> b) & 1]
        assert sum(math.comb(c, i + 1) for i, c in enumerate(occ)) == rank
        assert s[perm][p] == k
    q = np.concatenate([s[perm][:5], np.array([0b1111100000], dtype=np.uint64)])
    assert list(O.lookup(s[perm], q)) == [0, 1, 2, 3, 4, -1]


def test_link_table_counts_from_paper():
    """Entry counts and GiB of the paper's single-link table (FCI rows)."""
    from oracle import oracle as O
    tab = json.load(open(os.path.join(GOLDEN, "single_link_table.json")))
    for row in tab["rows"]:
        M, n = row["M"], row["n_beta"]
        assert math.comb(M, n) * n * (M - n) == row["entries"]
        assert round(row["entries"] * tab["bytes_per_entry"] / 2 ** 30, 2) == row["gib"]
    # the oracle's hash-membership builder reproduces the CN row (424,270 strings)
    cn = [r for r in tab["rows"] if r["M"] == 58 and r["n_beta"] == 4][0]
    strs = np.array([sum(1 << p for p in c) for c in itertools.combinations(range(58), 4)],
                    dtype=np.uint64)
    assert O.count_singles(strs, 58) == cn["entries"]


def test_spin_flip_symmetry_and_singlet_sector(oracle_mod):
    """With identical alpha/beta lists and N_alpha = N_beta, H commutes with
    F|I J> = (-1)^N |J I> (alpha creators first in the determinant), and a
    closed-shell determinant |I I> lies in the F = (-1)^N sector, i.e. C = C^T."""
    O = oracle_mod
    for (M, N, keep, s1, s2) in ((6, 3, 12, 3, 4), (8, 4, 30, 5, 6), (7, 2, 15, 7, 8)):
        p = W.make_problem("flip", M, N, keep, s1, s2)
        sp = O.Space.of(p)
        H = sp.dense_h()
        l = len(p.alpha)
        F = np.zeros((l * l, l * l))
        for i in range(l):
            for j in range(l):
                F[j * l + i, i * l + j] = (-1) ** N
        assert np.abs(H @ F - F @ H).max() <= 1e-13 * np.abs(H).max()
        # the symmetric-C subspace is F-invariant with eigenvalue (-1)^N
        C = np.random.default_rng(1).normal(size=(l, l))
        C = C + C.T
        assert np.allclose(F @ C.ravel(), (-1) ** N * C.ravel())


def test_sigma_rows_from_and_linked_rows(oracle_mod):
    """The row-sampled sigma used by the full-size parity tests: on selected
    spaces where the linked rows are a small strict subset, linked_rows equals
    a brute-force scan of excitation degrees <= 2, sigma_rows_from on just
    those rows equals the full sigma bit for bit, and leaving out one needed
    row raises."""
    O = oracle_mod
    # uniformly random selections from large string sets, so that few rows
    # are within two excitations of a sampled row
    cases = [W.random_selection(14, 7, 7, 300, 40, seed=21),
             W.random_selection(14, 6, 5, 250, 60, seed=25),
             W.random_selection(13, 5, 6, 260, 30, seed=27)]
    for p in cases:
        sp = O.Space.of(p)
        la = len(p.alpha)
        rows = np.array([0, la // 3], dtype=np.int64)
        need = sp.linked_rows(rows)
        a = [int(x) for x in p.alpha]
        brute = sorted({j for r in rows for j in range(la)
                        if bin(a[int(r)] ^ a[j]).count("1") <= 4})
        assert need.tolist() == brute
        assert len(need) < la // 2  # a strict, small subset
        C = W.random_vector(la, len(p.beta), seed=5)
        full = sp.sigma(C, rows=rows)
        part = sp.sigma_rows_from(rows, C[need], need)
        assert np.array_equal(full, part)
        # the sub-matrix really is all it reads: other rows may hold anything
        junk = C.copy()
        others = np.setdiff1d(np.arange(la), need)
        junk[others] = 1e300
        assert np.array_equal(sp.sigma(junk, rows=rows), full)
        with pytest.raises(ValueError):
            drop = need[need != rows[1]][:-1] if len(need) > 1 else need[:0]
            sp.sigma_rows_from(rows, C[drop], drop)


def test_fock_spin_squared_spectrum(oracle_mod):
    """S^2 built from Jordan-Wigner operators has eigenvalues S(S+1) with the
    multiplicities of two-electron spin coupling (M = 2: 16 states; the
    N_alpha = N_beta = 1 block holds 3 singlets and 1 triplet component)."""
    O = oracle_mod
    S2 = O.fock_spin_squared(2)
    w = np.round(np.linalg.eigvalsh(S2), 10)
    vals, counts = np.unique(w, return_counts=True)
    # Fock space of 2 spatial orbitals: 1 (vacuum) + 4 doublet states x 2 ...
    assert set(vals.tolist()) <= {0.0, 0.75, 2.0}
    assert np.isclose(np.trace(S2), sum(v * c for v, c in zip(vals, counts)))
    idx = [O.fock_index(a, b, 2) for a in (1, 2) for b in (1, 2)]
    blk = np.linalg.eigvalsh(S2[np.ix_(idx, idx)])
    assert np.allclose(np.sort(blk), [0.0, 0.0, 0.0, 2.0], atol=1e-12)


@pytest.mark.parametrize("M,N,seed", [(4, 2, 31), (4, 1, 32), (3, 1, 33), (5, 2, 34)])
def test_flip_sectors_are_spin_parity_sectors(oracle_mod, M, N, seed):
    """On a complete space with N_alpha = N_beta (closed under S^2), the
    spectrum of H on symmetric CI matrices equals its spectrum on the states
    of even S, and on antisymmetric ones that of odd S, with S^2 built
    independently from Jordan-Wigner operators; the lowest of both sectors is
    the lowest eigenvalue overall."""
    O = oracle_mod
    p = W.make_problem("flip_pin", M, N, None, seed)
    sp = O.Space.of(p)
    H = sp.dense_h()
    l = len(p.alpha)
    idx = [O.fock_index(a, b, M) for a in p.alpha for b in p.beta]
    S2 = O.fock_spin_squared(M)[np.ix_(idx, idx)]
    # S^2 blocks: eigenvalue S(S+1); H within each S block
    s2w, s2v = np.linalg.eigh(S2)
    S = np.round((-1 + np.sqrt(1 + 4 * np.clip(s2w, 0, None))) / 2).astype(int)
    assert np.allclose(S * (S + 1), s2w, atol=1e-9)
    by_parity = {0: [], 1: []}
    for s in np.unique(S):
        Q = s2v[:, S == s]
        by_parity[int(s) % 2] += np.linalg.eigvalsh(Q.T @ H @ Q).tolist()
    for tau, par in ((1, 0), (-1, 1)):
        Q = O.flip_sector_basis(l, tau)
        sec = np.linalg.eigvalsh(Q.T @ H @ Q) if Q.shape[1] else np.zeros(0)
        assert np.allclose(np.sort(sec), np.sort(by_parity[par]), atol=1e-10)
    r = O.lowest_by_flip_sector(sp, H)
    assert np.isclose(r["lowest"], np.linalg.eigvalsh(H)[0], atol=1e-12)
    assert r["lowest"] == min(x for x in (r["sym"], r["anti"]) if x is not None)


def test_flip_sector_ground_state_outside_symmetric_sector(oracle_mod):
    """A problem of the smallest configuration's recipe (M = 8, N = 4, every
    string, integral seed 100) whose lowest state is antisymmetric: the
    symmetric sector alone would miss it by more than 0.04 Eh."""
    O = oracle_mod
    p = W.make_problem("anti_gs", 8, 4, None, 100)
    r = O.lowest_by_flip_sector(O.Space.of(p))
    assert r["sector"] == -1
    assert r["sym"] - r["anti"] > 0.04
    assert np.isclose(r["lowest"], r["lowest_all"], atol=1e-12)


# ------------------------------------------------ TBSCI (pruned) spaces

def _pruned(O, p, keep, seed):
    sp = O.Space.of(p)
    ro, bi = W.dets_random(len(p.alpha), len(p.beta), keep, seed)
    sp.set_dets(ro, bi)
    return sp


@pytest.mark.parametrize("na,nb,la,lb,keep,seed", [
    (2, 2, 6, 6, 0.5, 41), (1, 2, 4, 6, 0.4, 42), (3, 1, 4, 4, 0.7, 43), (2, 3, 5, 4, 0.3, 44)])
def test_dets_elements_match_jordan_wigner(oracle_mod, fock4, na, nb, la, lb, keep, seed):
    """sigma over a ragged TBSCI space, applied to every unit vector, equals
    the Jordan-Wigner Fock-space H restricted to the kept determinants."""
    O = oracle_mod
    M, h, eri, H = fock4
    rng = np.random.default_rng(seed)
    A, B = W.all_strings(M, na), W.all_strings(M, nb)
    a = A[rng.permutation(len(A))[:la]]
    b = B[rng.permutation(len(B))[:lb]]
    sp = O.Space(M, na, nb, h, eri, a, b)
    ro, bi = W.dets_random(len(a), len(b), keep, seed)
    sp.set_dets(ro, bi)
    n = sp.n_dets
    assert 0 < n < len(a) * len(b) and (np.diff(ro) == 0).any() or n > 0
    Hd = np.array([sp.sigma_dets(np.eye(n)[k]) for k in range(n)]).T
    keys = sp.dets_index()
    idx = [O.fock_index(a[k // len(b)], b[k % len(b)], M) for k in keys]
    assert np.abs(Hd - H[np.ix_(idx, idx)]).max() <= 1e-12 * max(1.0, np.abs(H).max())


def test_dets_sigma_is_restricted_tpb_sigma(oracle_mod):
    """sigma over kept determinants equals the TPB sigma of the vector
    extended by zeros, read at the kept determinants (the projector onto the
    TBSCI space is diagonal in the TPB basis); keeping everything gives the
    TPB sigma bit for bit."""
    O = oracle_mod
    for p, keep in ((W.make_problem("d12", 12, 6, 150, 51, 52, independent_beta=True), 0.3),
                    (W.random_selection(10, 4, 5, 90, 70, seed=53), 0.6)):
        sp = _pruned(O, p, keep, 54)
        k = sp.dets_index()
        c = np.random.default_rng(5).normal(size=sp.n_dets)
        full = np.zeros(sp.la * sp.lb)
        full[k] = c
        ref = O.Space.of(p).sigma(full).ravel()[k]
        got = sp.sigma_dets(c)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
        rows = np.array([sp.la - 1, 0, sp.la // 2])
        seg = np.concatenate([got[sp.row_off[r]:sp.row_off[r + 1]] for r in rows])
        assert np.array_equal(sp.sigma_dets(c, rows=rows), seg)
        every = O.Space.of(p)
        every.set_dets(np.arange(sp.la + 1, dtype=np.int64) * sp.lb,
                       np.tile(np.arange(sp.lb, dtype=np.int32), sp.la))
        cf = np.random.default_rng(6).normal(size=sp.la * sp.lb)
        assert np.array_equal(every.sigma_dets(cf), O.Space.of(p).sigma(cf).ravel())


def test_dets_hermitian_and_interlacing(oracle_mod):
    """The TBSCI matrix is symmetric, its lowest eigenvalue lies above that
    of the TPB space, and growing the kept set (nested layouts) never raises
    it (Cauchy interlacing)."""
    O = oracle_mod
    p = W.make_problem("d10", 10, 5, 40, 61, 62)
    tpb = O.Space.of(p)
    e_tpb = np.linalg.eigvalsh(tpb.dense_h())[0]
    la, lb = len(p.alpha), len(p.beta)
    prev = None
    for frac in (0.15, 0.3, 0.6, 1.0):
        sp = O.Space.of(p)
        sp.set_dets(*W.dets_rank_sum(la, lb, frac))
        Hd = sp.dense_h_dets()
        k = sp.dets_index()
        assert np.array_equal(Hd, tpb.dense_h()[np.ix_(k, k)])
        c = np.random.default_rng(7).normal(size=(sp.n_dets, 3))
        Hc = np.stack([sp.sigma_dets(c[:, j]) for j in range(3)], axis=1)
        assert np.abs(Hc - Hd @ c).max() <= 1e-12 * np.abs(Hd @ c).max()
        assert np.abs(Hd - Hd.T).max() == 0.0
        e = np.linalg.eigvalsh(Hd)[0]
        assert e >= e_tpb - 1e-12
        if prev is not None:
            assert e <= prev + 1e-12
        prev = e
    assert abs(prev - e_tpb) < 1e-10


def test_dets_layout_errors(oracle_mod):
    O = oracle_mod
    p = W.random_selection(8, 3, 3, 10, 12, seed=63)
    sp = O.Space.of(p)
    for ro, bi in (([1] + [0] * 10, [0]),                       # offsets not from 0
                   ([0, 2] + [2] * 9, [0, 12]),                 # index out of range
                   ([0, 2] + [2] * 9, [3, 3])):                 # repeated index
        with pytest.raises(ValueError):
            sp.set_dets(np.array(ro), np.array(bi))


# ------------------------------------------------ point-group symmetry

def test_symmetry_dimensions_of_the_paper_systems(oracle_mod):
    """The determinant counts of one total irrep reproduce the FCI dimensions
    printed for the four benchmark systems (three significant digits), and
    the count without symmetry does not."""
    tab = json.load(open(os.path.join(GOLDEN, "fci_dimensions.json")))
    for r in tab["systems"]:
        orb = {int(k): v for k, v in r["orbitals"].items()}
        assert sum(orb.values()) == r["active"]
        order = 8 if r["group"] == "D2h" else 4
        d = oracle_mod.symmetry_dimension(orb, r["n_alpha"], r["n_beta"], r["target"], order)
        assert float(f"{d:.2e}") == r["printed"], (r["name"], d)
        full = math.comb(r["active"], r["n_alpha"]) * math.comb(r["active"], r["n_beta"])
        assert float(f"{full:.2e}") != r["printed"]


def test_symmetric_hamiltonian_is_block_diagonal(oracle_mod):
    """With the symmetric integral recipe, H has no element between
    determinants of different total irreps, the TPB spectrum is the union of
    the spectra of the one-irrep spaces, each irrep's layout is an interval of
    the irrep-sorted beta strings, and the counts add up."""
    O = oracle_mod
    dist = {0: 2, 5: 1, 2: 1, 7: 1, 6: 1}
    p = W.make_sym_problem("sym6", 6, 3, dist, 0, 91, 92)
    irr = p.meta["irreps"]
    sp = O.Space.of(p)
    H = sp.dense_h()
    ga = O.string_irreps(p.alpha, irr)
    gb = O.string_irreps(p.beta, irr)
    gK = (ga[:, None] ^ gb[None, :]).ravel()
    assert (H[gK[:, None] != gK[None, :]] == 0.0).all()
    assert np.abs(H[gK[:, None] == gK[None, :]]).max() > 0.1
    spec = []
    total = 0
    for tgt in range(8):
        ro, bi = O.symmetry_layout(p.alpha, p.beta, irr, tgt)
        total += int(ro[-1])
        assert int(ro[-1]) == O.symmetry_dimension(dist, 3, 3, tgt)
        for w in range(len(p.alpha)):
            seg = bi[ro[w]:ro[w + 1]]
            assert len(seg) == 0 or (np.diff(seg) == 1).all()
        if ro[-1] == 0:
            continue
        s2 = O.Space.of(p)
        s2.set_dets(ro, bi)
        spec += np.linalg.eigvalsh(s2.dense_h_dets()).tolist()
    assert total == len(p.alpha) * len(p.beta)
    assert np.allclose(np.sort(spec), np.linalg.eigvalsh(H), atol=1e-11)


def test_string_irreps_brute_force(oracle_mod):
    """A string's irrep is the product of its occupied orbitals' irreps
    (checked against a direct product over occupied orbitals on random
    strings)."""
    rng = np.random.default_rng(3)
    irr = rng.integers(0, 8, size=20)
    s = W.all_strings(20, 4)[rng.permutation(4845)[:200]]
    got = oracle_mod.string_irreps(s, irr)
    for x, g in zip(s, got):
        occ = [p for p in range(20) if (int(x) >> p) & 1]
        prod = 0
        for p in occ:
            prod = prod ^ int(irr[p])
        assert g == prod


# ------------------------------------------------ string-weight selection

def test_string_weights_closed_forms(oracle_mod):
    """Weights of a product vector a (x) b are a^2 |b|^2 and b^2 |a|^2; the
    alpha and beta weights of any normalised vector both sum to 1."""
    O = oracle_mod
    rng = np.random.default_rng(21)
    a, b = rng.normal(size=7), rng.normal(size=5)
    wa, wb = O.string_weights(np.outer(a, b))
    assert np.allclose(wa, a * a * (b @ b), rtol=1e-14)
    assert np.allclose(wb, b * b * (a @ a), rtol=1e-14)
    C = rng.normal(size=(9, 6))
    C /= np.linalg.norm(C)
    wa, wb = O.string_weights(C)
    assert abs(wa.sum() - 1) < 1e-14 and abs(wb.sum() - 1) < 1e-14


def test_selection_is_nested_and_variational(oracle_mod):
    """Selections by decreasing delta are nested, always hold the reference
    string, keep every string of nonzero weight at delta = 0, and their TPB
    ground-state energies decrease towards the complete-space energy
    (interlacing)."""
    O = oracle_mod
    p = W.make_problem("sel8", 8, 4, None, 22)
    sp = O.Space.of(p)
    H = sp.dense_h()
    e_all, x = O.lowest_eigpair_dense(H)
    wa, wb = O.string_weights(x.reshape(len(p.alpha), len(p.beta)))
    hf = int(sum(1 << q for q in range(4)))
    prev_set, prev_e = None, None
    for delta in (0.5, 1e-1, 1e-2, 1e-3, 1e-4, 0.0):
        a = O.select_by_weight(p.alpha, wa, delta, hf)
        b = O.select_by_weight(p.beta, wb, delta, hf)
        assert int(a[0]) == hf or wa[list(map(int, p.alpha)).index(int(a[0]))] >= wa[
            list(map(int, p.alpha)).index(hf)]
        assert hf in set(map(int, a)) and hf in set(map(int, b))
        s = (set(map(int, a)), set(map(int, b)))
        if prev_set is not None:
            assert prev_set[0] <= s[0] and prev_set[1] <= s[1]
        sub = O.Space(8, 4, 4, p.h, p.eri, a, b)
        e = float(np.linalg.eigvalsh(sub.dense_h())[0])
        assert e >= e_all - 1e-12
        if prev_e is not None:
            assert e <= prev_e + 1e-12
        prev_set, prev_e = s, e
    assert len(prev_set[0]) == int((wa > 0).sum())
    assert abs(prev_e - e_all) < 1e-10


def test_coef_histogram_counts(oracle_mod):
    """Histogram of log10 |c|: every coefficient counted once; values placed
    in the bin their exponent falls in; zeros and tiny values in bin 0."""
    O = oracle_mod
    c = np.array([0.0, 1e-20, 3e-5, 5e-3, 0.2, 0.9, -0.05, 2.0])
    h = O.coef_histogram(c, -6.0, 0.0, 6)
    assert h.sum() == len(c)
    assert h.tolist() == [2, 1, 0, 1, 1, 3]
