"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer structures (sorted index, lookups, excitation lists, phases) must
match bit for bit; FP64 sigma to 1e-12 relative (norm-wise and max-wise);
FP64 energies to 1e-8 Eh; FP32 sigma to 2e-5 relative (FP32 rounding of
sums of a few thousand terms).
"""
import ctypes
import math

import numpy as np
import pytest

from paper_2503_10335_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2503_10335_amd import tbsci as T
    T.load()
    return T, O, torch


def _problems():
    return {
        "fci_m8": W.config("fci_m8"),
        "rand_m8_3_4": W.random_selection(8, 3, 4, 37, 53, seed=11),
        "rand_m10_5_5": W.random_selection(10, 5, 5, 130, 97, seed=12),
        "rand_m12_4_6": W.random_selection(12, 4, 6, 300, 257, seed=13),
        "ranked_m12": W.make_problem("ranked_m12", 12, 6, 500, 14, 24),
        "ranked_m11_indep": W.make_problem("ranked_m11", 11, 5, 200, 15, 25, independent_beta=True),
        "empty_alpha": W.random_selection(6, 0, 3, 1, 20, seed=16),
        "full_alpha": W.random_selection(5, 5, 2, 1, 10, seed=17),
        "one_by_one": W.random_selection(7, 3, 3, 1, 1, seed=18),
        "m1": W.random_selection(1, 1, 0, 1, 1, seed=19),
    }


PROBS = _problems()


def _rel(a, b):
    n = np.linalg.norm(b)
    return (np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a),
            np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(PROBS))
def test_index_and_lookup(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    for spin, strs, n in ((0, p.alpha, p.n_alpha), (1, p.beta, p.n_beta)):
        keys, pos = ctx.string_index(spin)
        rk, rp = O.string_index(strs)
        assert np.array_equal(keys, rk) and np.array_equal(pos, rp)
        q = W.all_strings(p.M, n)
        if len(q) > 5000:
            q = q[:5000]
        got = ctx.lookup(spin, torch.from_numpy(q.view(np.int64)).cuda()).cpu().numpy()
        assert np.array_equal(got, O.lookup(strs, q))
    ctx.close()


@pytest.mark.parametrize("name", list(PROBS))
def test_excitation_lists_bit_exact(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    for spin, strs in ((0, p.alpha), (1, p.beta)):
        ptr, ent = ctx.get_list(spin, 1)
        rptr, rent = O.singles_with_diag(strs, p.M)
        assert np.array_equal(ptr, rptr)
        assert np.array_equal(ent, rent)
        ptr, ent = ctx.get_list(spin, 2)
        rptr, rent = O.lists(strs, p.M, 2)
        assert np.array_equal(ptr, rptr)
        assert np.array_equal(ent, rent)
    ctx.close()


@pytest.mark.parametrize("name", ["fci_m8", "rand_m8_3_4", "ranked_m11_indep", "full_alpha"])
def test_same_spin_operator(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    sp = O.Space.of(p)
    for spin, l in ((0, len(p.alpha)), (1, len(p.beta))):
        if l > 250:
            continue
        ptr, col, val = ctx.get_list(spin, 3)
        A = np.zeros((l, l))
        for i in range(l):
            assert col[ptr[i]] == i  # diagonal first
            for e in range(ptr[i], ptr[i + 1]):
                A[i, col[e]] += val[e]
        assert np.abs(A - sp.same_spin_matrix(spin)).max() < 1e-13
    ctx.close()


@pytest.mark.parametrize("name", list(PROBS))
def test_diag(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    d = ctx.diag().cpu().numpy()
    ref = O.Space.of(p).diag()
    assert np.abs(d - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    ctx.close()


@pytest.mark.parametrize("name", list(PROBS))
def test_sigma_fp64(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    C = W.random_vector(ctx.l_alpha, ctx.l_beta, seed=7)
    S = ctx.sigma(torch.from_numpy(C).cuda()).cpu().numpy()
    ref = O.Space.of(p).sigma(C)
    nrm, mx = _rel(S, ref)
    assert nrm <= 1e-12 and mx <= 1e-12, (nrm, mx)
    ctx.close()


@pytest.mark.parametrize("name", ["fci_m8", "rand_m8_3_4", "ranked_m11_indep", "empty_alpha",
                                  "full_alpha"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sigma_terms_separately(env, name, prec):
    """Each of the three terms against the oracle: A_a C and C A_b^T from the
    oracle's dense same-spin matrices, the opposite-spin term as the rest."""
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    sp = O.Space.of(p)
    C = W.random_vector(ctx.l_alpha, ctx.l_beta, seed=5)
    full = sp.sigma(C)
    ta = sp.same_spin_matrix(0) @ C
    tb = C @ sp.same_spin_matrix(1).T
    refs = {1: ta, 2: tb, 4: full - ta - tb, 7: full}
    pr = T.TBSCI_FP64 if prec == "fp64" else T.TBSCI_FP32
    Cd = torch.from_numpy(C).cuda()
    if pr == T.TBSCI_FP32:
        Cd = Cd.float()
    tol = 1e-12 if prec == "fp64" else 2e-5
    scale = np.linalg.norm(full)
    for mask, ref in refs.items():
        got = ctx.sigma_terms(Cd, mask, precision=pr).double().cpu().numpy()
        err = np.linalg.norm(got - ref) / scale
        assert err <= tol, (mask, err)
    ctx.close()


@pytest.mark.parametrize("name", ["fci_m8", "rand_m12_4_6", "ranked_m12", "one_by_one"])
def test_sigma_fp32(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    C = W.random_vector(ctx.l_alpha, ctx.l_beta, seed=8)
    S = ctx.sigma(torch.from_numpy(C).float().cuda(), precision=T.TBSCI_FP32).cpu().double().numpy()
    ref = O.Space.of(p).sigma(C)
    nrm, mx = _rel(S, ref)
    assert nrm <= 2e-5 and mx <= 2e-5, (nrm, mx)
    ctx.close()


def test_sigma_fp64_selected_m16_sampled_rows(env):
    """The 3,000 x 3,000 selected M=16 space, oracle on sampled rows."""
    T, O, torch = env
    p = W.config("sel_m16")
    ctx = T.Context.from_problem(p)
    C = W.random_vector(ctx.l_alpha, ctx.l_beta, seed=7)
    S = ctx.sigma(torch.from_numpy(C).cuda()).cpu().numpy()
    rows = np.array([0, 1, 17, 1500, 2998, 2999])
    ref = O.Space.of(p).sigma(C, rows=rows)
    nrm, mx = _rel(S[rows], ref)
    assert nrm <= 1e-12 and mx <= 1e-12, (nrm, mx)
    # Hermiticity at full size
    Y = W.random_vector(ctx.l_alpha, ctx.l_beta, seed=9)
    SY = ctx.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    assert abs((C * SY).sum() - (S * Y).sum()) <= 1e-12 * np.abs(S).sum()
    # identical alpha/beta lists: sigma(C^T) = sigma(C)^T
    ST = ctx.sigma(torch.from_numpy(np.ascontiguousarray(C.T)).cuda()).cpu().numpy()
    assert np.abs(ST - S.T).max() <= 1e-12 * np.abs(S).max()
    ctx.close()


@pytest.mark.parametrize("name", ["fci_m8", "rand_m10_5_5", "ranked_m11_indep"])
def test_davidson_fp64_vs_dense(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    sp = O.Space.of(p)
    if sp.n_det <= 6000:
        e_ref, _ = O.lowest_eigpair_dense(sp.dense_h())
    else:
        # residual 1e-9: the energy error is ~|r|^2/gap ~ 1e-16 Eh, far
        # below the 1e-8 Eh of the check, while 1e-10 takes the oracle's
        # plain collapse restart thousands of iterations on this space
        res = O.davidson(sp.sigma, sp.diag(), tol=1e-9, n_max=12)
        assert res["converged"]
        e_ref = res["energy"]
    info, X = ctx.davidson(tol_resid=1e-8, n_max=8)
    assert info["converged"] == 1 and info["status"] == 0
    assert abs(info["energy"] - e_ref) < 1e-8
    x = X.cpu().numpy().ravel()
    assert abs(np.linalg.norm(x) - 1) < 1e-10
    # residual recomputed by the oracle
    r = sp.sigma(x).ravel() - info["energy"] * x
    assert np.linalg.norm(r) < 2e-8
    ctx.close()


@pytest.mark.parametrize("name", ["fci_m8", "ranked_m12"])
def test_davidson_mixed(env, name):
    T, O, torch = env
    p = PROBS[name]
    ctx = T.Context.from_problem(p)
    ref, _ = ctx.davidson(tol_resid=1e-8)
    info, X = ctx.davidson(precision=T.TBSCI_MIXED, tol_resid=1e-4)
    assert info["converged"] == 1
    assert info["iters_fp32"] > 0 and info["iters_fp64"] > 0
    assert abs(info["energy"] - ref["energy"]) < 1e-6
    ctx.close()


def test_davidson_guess_and_vector(env):
    """A start vector from the caller: the converged eigenvector as guess
    converges at once to the same energy; a zero guess is rejected; the
    returned vector has unit norm, its largest entry positive, and the
    oracle residual of the stated energy."""
    T, O, torch = env
    p = PROBS["ranked_m12"]
    ctx = T.Context.from_problem(p)
    sp = O.Space.of(p)
    info, X = ctx.davidson(tol_resid=1e-9, n_max=8, max_iter=400)
    assert info["status"] == 0
    x = X.cpu().numpy().ravel()
    assert abs(np.linalg.norm(x) - 1) < 1e-12
    k = int(np.argmax(np.abs(x)))
    assert x[k] > 0
    assert np.linalg.norm(sp.sigma(x).ravel() - info["energy"] * x) < 5e-9
    # warm start (scaled, to exercise the normalisation of the guess)
    info2, X2 = ctx.davidson(tol_resid=1e-9, n_max=8, guess=3.0 * X)
    # at most two iterations and the final FP64 energy check
    assert info2["status"] == 0 and info2["iters"] <= 4 and info2["sector"] == 0
    assert abs(info2["energy"] - info["energy"]) < 1e-10
    assert np.abs(X2.cpu().numpy() - X.cpu().numpy()).max() < 1e-8
    with pytest.raises(T.TbsciError) as ei:
        ctx.davidson(guess=torch.zeros_like(X))
    assert ei.value.code == T.TBSCI_E_INVAL and "zero" in str(ei.value)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_davidson_both_flip_sectors(env, prec):
    """Identical lists whose lowest state is antisymmetric (M = 8, N = 4,
    every string, integral seed 100): the default solve returns the lowest
    eigenvalue of the oracle's dense P H P over both sectors, reports sector
    -1, the symmetric sector's lowest as energy_other, and an antisymmetric
    eigenvector; a solve restricted to one sector returns that sector's
    lowest state; lean storage gives the same energies."""
    T, O, torch = env
    p = W.make_problem("anti_gs", 8, 4, None, 100)
    ref = O.lowest_by_flip_sector(O.Space.of(p))
    assert ref["sector"] == -1
    pr = T.TBSCI_FP64 if prec == "fp64" else T.TBSCI_MIXED
    tol_e = 1e-8 if prec == "fp64" else 1e-6
    ctx = T.Context.from_problem(p)
    for storage in (T.TBSCI_STORE_FULL, T.TBSCI_STORE_LEAN):
        info, X = ctx.davidson(tol_resid=1e-8 if prec == "fp64" else 1e-5, n_max=6,
                               max_iter=400, precision=pr, storage=storage)
        assert info["status"] == 0 and info["converged"] == 1
        assert info["lean"] == (1 if storage == T.TBSCI_STORE_LEAN else 0)
        assert info["sector"] == -1
        assert abs(info["energy"] - ref["lowest"]) < tol_e
        assert abs(info["energy_other"] - ref["sym"]) < tol_e
        assert abs(info["energy_fp64_check"] - info["energy"]) < 1e-9
        x = X.cpu().numpy()
        assert np.abs(x + x.T).max() < 1e-10
        for sec, key in ((1, "sym"), (-1, "anti")):
            i1, X1 = ctx.davidson(tol_resid=1e-8 if prec == "fp64" else 1e-5, n_max=6,
                                  max_iter=400, precision=pr, storage=storage, sector=sec)
            assert i1["status"] == 0 and i1["sector"] == sec
            assert abs(i1["energy"] - ref[key]) < tol_e
            assert np.isnan(i1["energy_other"])
            x1 = X1.cpu().numpy()
            assert np.abs(x1 - sec * x1.T).max() < 1e-10
    ctx.close()


@pytest.mark.parametrize("n_max", [2, 3, 8])
def test_davidson_lean_storage(env, n_max):
    """Lean storage (2 n_max + 3 vectors: collapse restart, the image of the
    correction in a vector of the collapsed basis, H_KK recomputed) against
    dense diagonalisation on a space with independent lists and on a
    complete one, FP64 and mixed; the fresh FP64 energy check agrees with
    the reported energy."""
    T, O, torch = env
    for name in ("rand_m8_3_4", "fci_m8"):
        p = PROBS[name]
        e_ref = O.lowest_by_flip_sector(O.Space.of(p))["lowest"]
        ctx = T.Context.from_problem(p)
        info, X = ctx.davidson(tol_resid=1e-8, n_max=n_max, max_iter=2000,
                               storage=T.TBSCI_STORE_LEAN)
        assert info["status"] == 0 and info["lean"] == 1
        assert abs(info["energy"] - e_ref) < 1e-8
        assert abs(info["energy_fp64_check"] - info["energy"]) < 1e-10
        im, _ = ctx.davidson(tol_resid=1e-5, n_max=n_max, max_iter=2000,
                             precision=T.TBSCI_MIXED, storage=T.TBSCI_STORE_LEAN,
                             want_vector=False)
        assert im["status"] == 0 and abs(im["energy"] - e_ref) < 1e-6
        assert abs(im["energy_fp64_check"] - im["energy"]) < 1e-8
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_davidson_subspace_start(env, prec):
    """A start from the subspace of the strings with the smallest same-spin
    diagonal (solved first, per spin-flip sector) reaches the same lowest
    state as the diagonal start, against dense references over both sectors
    (identical lists with an antisymmetric ground state, and independent
    lists), with the sector kept."""
    T, O, torch = env
    pr = T.TBSCI_FP64 if prec == "fp64" else T.TBSCI_MIXED
    tol_r, tol_e = (1e-8, 1e-8) if prec == "fp64" else (1e-5, 1e-6)
    for p, k in ((W.make_problem("anti_gs", 8, 4, None, 100), 20),
                 (PROBS["rand_m8_3_4"], 0)):
        ref = O.lowest_by_flip_sector(O.Space.of(p))
        ctx = T.Context.from_problem(p)
        info, X = ctx.davidson(tol_resid=tol_r, max_iter=600, precision=pr, subspace_guess=k)
        assert info["status"] == 0 and abs(info["energy"] - ref["lowest"]) < tol_e
        if ref["sector"]:
            assert info["sector"] == ref["sector"]
            assert abs(info["energy_other"] - ref["sym"]) < tol_e
            x = X.cpu().numpy()
            assert np.abs(x - ref["sector"] * x.T).max() < 1e-9
        ctx.close()
    # TBSCI spaces do not take subspace starts
    ctx = T.Context.from_problem(PROBS["rand_m8_3_4"])
    ctx.set_dets(*W.dets_random(37, 53, 0.5, 3))
    with pytest.raises(T.TbsciError) as ei:
        ctx.davidson(subspace_guess=0)
    assert ei.value.code == T.TBSCI_E_INVAL
    ctx.close()


def test_davidson_option_errors(env):
    """guess_kind must match the guess pointer; an empty antisymmetric
    sector (one string per spin) and out-of-range options are rejected."""
    T, O, torch = env
    p = PROBS["fci_m8"]
    ctx = T.Context.from_problem(p)
    X = torch.zeros((ctx.l_alpha, ctx.l_beta), dtype=torch.float64, device="cuda")
    X[0, 0] = 1.0
    info = T.DavidsonInfo()
    lib = T.load()
    for kw, guess in ((dict(guess_kind=T.TBSCI_GUESS_USER), None),
                      (dict(guess_kind=T.TBSCI_GUESS_DIAG), X),
                      (dict(sector=2), None), (dict(storage=5), None)):
        o = T.make_opts(**kw)
        rc = lib.tbsci_davidson(ctx.handle, ctypes.byref(o),
                                ctypes.c_void_p(guess.data_ptr()) if guess is not None else None,
                                None, ctypes.byref(info), None)
        assert rc == T.TBSCI_E_INVAL, kw
    ctx.close()
    one = W.random_selection(7, 3, 3, 1, 1, seed=18)
    one.beta = one.alpha.copy()
    c1 = T.Context.from_problem(one)
    with pytest.raises(T.TbsciError) as ei:
        c1.davidson(sector=-1)
    assert ei.value.code == T.TBSCI_E_INVAL
    i1, _ = c1.davidson()
    assert i1["status"] == 0 and i1["sector"] == 1 and np.isnan(i1["energy_other"])
    c1.close()


@pytest.mark.parametrize("shape", [(3200, 40), (40, 3200)])
def test_sigma_chunked_sweeps(env, shape):
    """More than 3072 strings of one spin: that spin's same-spin sweep runs
    in source chunks (one pass per chunk of 3072 strings); FP64 and FP32
    sigma against the oracle."""
    T, O, torch = env
    la, lb = shape
    p = W.random_selection(14, 7, 7, la, lb, seed=31)
    ctx = T.Context.from_problem(p)
    C = np.random.default_rng(5).normal(size=(la, lb))
    ref = O.Space.of(p).sigma(C, nthreads=16)
    Cg = torch.from_numpy(C).cuda()
    got = ctx.sigma(Cg).cpu().numpy()
    e, m = _rel(got, ref)
    assert e <= 1e-12 and m <= 1e-12
    got32 = ctx.sigma(Cg.float(), precision=T.TBSCI_FP32).double().cpu().numpy()
    assert _rel(got32, ref)[0] <= 2e-5
    ctx.close()


def _shell_alpha(M, N):
    """The lowest string (orbitals 0..N-1) and all of its single excitations."""
    ref = (1 << N) - 1
    out = [ref] + [ref ^ (1 << i) ^ (1 << a) for i in range(N) for a in range(N, M)]
    return np.array(out, dtype=np.uint64)


def test_sigma_global_fragments_many_links(env):
    """An alpha string with more links than the slab kernel's LDS fragments
    take (the reference string of a single-excitation shell at M = 20 has 100
    singles plus 10 occupations, 28 k-steps): the opposite-spin term reads its
    integral fragments from global memory, whole FP64 row in LDS.  FP64 and
    FP32 sigma against the oracle."""
    T, O, torch = env
    M, N = 20, 10
    h, eri = W.integrals(M, 41)
    rng = np.random.default_rng(42)
    B = W.all_strings(M, N)
    beta = np.ascontiguousarray(B[rng.permutation(len(B))[:60]])
    p = W.Problem("shell_m20", M, N, N, h, eri, _shell_alpha(M, N), beta)
    ptr, _ = O.lists(p.alpha, M, 1)
    assert int(np.diff(ptr).max()) + N == 110
    ctx = T.Context.from_problem(p)
    C = np.random.default_rng(5).normal(size=(len(p.alpha), len(p.beta)))
    ref = O.Space.of(p).sigma(C, nthreads=16)
    Cg = torch.from_numpy(C).cuda()
    e, m = _rel(ctx.sigma(Cg).cpu().numpy(), ref)
    assert e <= 1e-12 and m <= 1e-12
    got32 = ctx.sigma(Cg.float(), precision=T.TBSCI_FP32).double().cpu().numpy()
    assert _rel(got32, ref)[0] <= 2e-5
    ctx.close()


@pytest.mark.parametrize("shape", [(24, 18000), (16, 21000), (10, 45000)])
def test_sigma_global_fragments_long_rows(env, shape):
    """Beta lists too long for the slab kernel's LDS (an FP64 row of 18000,
    21000 or 45000 strings plus FP64 fragments): FP64 sigma reads its
    fragments from global memory, with the whole FP64 row in LDS (18000) or
    the row split between LDS and global atomics (21000, 45000).  FP32 sigma:
    fragments in LDS (18000; they are half the size), or from global memory
    with a whole FP32 row in LDS (21000) or a split FP32 row (45000).  Eight
    alpha rows, first and last included, against the oracle."""
    T, O, torch = env
    la, lb = shape
    p = W.random_selection(18, 9, 9, la, lb, seed=43)
    ctx = T.Context.from_problem(p)
    C = np.random.default_rng(6).normal(size=(la, lb))
    rows = np.unique(np.r_[0, la - 1, np.random.default_rng(7).choice(la, 6, replace=False)])
    ref = O.Space.of(p).sigma(C, rows=rows, nthreads=16)
    Cg = torch.from_numpy(C).cuda()
    e, m = _rel(ctx.sigma(Cg).cpu().numpy()[rows], ref)
    assert e <= 1e-12 and m <= 1e-12
    got32 = ctx.sigma(Cg.float(), precision=T.TBSCI_FP32).double().cpu().numpy()[rows]
    assert _rel(got32, ref)[0] <= 2e-5
    ctx.close()


def test_executed_mfma_flops_accounting(env):
    """The executed-flop count the benchmark reports for the MFMA
    opposite-spin kernel, recomputed from the oracle's alpha link lists: per
    alpha row, the link count padded to whole k-steps (4 links; chunks of 16
    in the FP32 slab kernel) x the folded pairs padded to 16 x the beta
    strings padded to the 16-column slab x 2."""
    T, O, torch = env
    p = PROBS["rand_m12_4_6"]
    ctx = T.Context.from_problem(p)
    ptr, _ = O.singles_with_diag(p.alpha, p.M)
    K = np.diff(ptr)
    P = p.M * (p.M + 1) // 2
    rows16 = 16 * ((P + 15) // 16)
    cols = 16 * ((len(p.beta) + 15) // 16)
    for prec, pad in ((T.TBSCI_FP64, 4), (T.TBSCI_FP32, 16)):
        kp = int(np.sum(pad * ((K + pad - 1) // pad)))
        assert ctx.mfma_flops(prec) == 2.0 * kp * rows16 * cols
    ctx.close()


def test_sigma_direct_fallback(env):
    """A shape neither MFMA kernel takes in FP64: M = 23 (P = 276, so the V
    row offsets of the global-fragment kernel would not fit 16 bits) with all
    253 two-electron alpha strings (44 links each) and 7000 beta strings (the
    FP64 fragments and row overflow LDS): the opposite-spin term runs in the
    direct double-sum kernel.  FP32 takes the slab kernel with 18 M-tiles.
    Six alpha rows against the oracle."""
    T, O, torch = env
    p = W.random_selection(23, 2, 4, 253, 7000, seed=47)
    assert len(p.alpha) == 253 and len(p.beta) == 7000
    ctx = T.Context.from_problem(p)
    # the executed-flop count names the kernel: the direct kernel's is the
    # plain double sum over all alpha and beta links
    na = int(np.diff(O.singles_with_diag(p.alpha, p.M)[0]).sum())
    nb = int(np.diff(O.singles_with_diag(p.beta, p.M)[0]).sum())
    assert ctx.mfma_flops(T.TBSCI_FP64) == 2.0 * na * nb
    C = np.random.default_rng(8).normal(size=(ctx.l_alpha, ctx.l_beta))
    rows = np.array([0, 17, 100, 181, 222, 252])
    ref = O.Space.of(p).sigma(C, rows=rows, nthreads=16)
    Cg = torch.from_numpy(C).cuda()
    e, m = _rel(ctx.sigma(Cg).cpu().numpy()[rows], ref)
    assert e <= 1e-12 and m <= 1e-12
    got32 = ctx.sigma(Cg.float(), precision=T.TBSCI_FP32).double().cpu().numpy()[rows]
    assert _rel(got32, ref)[0] <= 2e-5
    ctx.close()
