"""GPU parity of the hole-pair same-spin sweep (tbsci_set_same_spin with
TBSCI_SAME_SPIN_HOLE) through the C ABI.

The same-spin terms A_a C and C A_b^T against the oracle's Slater-Condon
same-spin matrices (FP64 to 1e-12 of |sigma|, FP32 to 2e-5), whole sigma
against the oracle, the hole-pair and CSR methods against each other, lists
of more than 64 strings per hole string (the 128-entry kernel), a spin with
fewer than two electrons (keeps CSR), a space whose products take several
column windows and a beta sweep in blocks (sampled rows), bitwise
repeatability, and a Davidson solve.
"""
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


def _shell(M, N, nb, seed):
    """Alpha: the lowest string and every string within two excitations of
    it (its hole strings hold up to C(M-N+2, 2) strings); beta: random."""
    ref = (1 << N) - 1
    A = W.all_strings(M, N)
    keep = [int(s) for s in A if bin(int(s) ^ ref).count("1") <= 4]
    rng = np.random.default_rng(seed)
    beta = np.ascontiguousarray(A[np.sort(rng.permutation(len(A))[:nb])])
    h, eri = W.integrals(M, seed)
    return W.Problem(f"shell_m{M}", M, N, N, h, eri, np.array(sorted(keep), dtype=np.uint64),
                     beta)


PROBS = {
    "fci_m8": lambda: W.config("fci_m8"),
    "rand_m8_3_4": lambda: W.random_selection(8, 3, 4, 37, 53, seed=11),
    "rand_m10_5_5": lambda: W.random_selection(10, 5, 5, 130, 97, seed=12),
    "rand_m12_4_6": lambda: W.random_selection(12, 4, 6, 300, 257, seed=13),
    "ranked_m12": lambda: W.make_problem("ranked_m12", 12, 6, 500, 14, 24),
    "one_alpha": lambda: W.random_selection(7, 1, 3, 7, 35, seed=18),
    # hole strings of up to C(12, 2) = 66 strings: the 128-entry kernel
    "shell_m20": lambda: _shell(20, 10, 40, 61),
}


def _rel(a, b):
    n = np.linalg.norm(b)
    return (np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a),
            np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(PROBS))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hole_terms_vs_oracle(env, name, prec):
    T, O, torch = env
    p = PROBS[name]()
    print(f"hole terms: {name} {len(p.alpha)} x {len(p.beta)} {prec}", flush=True)
    ctx = T.Context.from_problem(p)
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_HOLE)
    sp = O.Space.of(p)
    C = W.random_vector(ctx.l_alpha, ctx.l_beta, seed=5)
    full = sp.sigma(C, nthreads=16)
    ta = sp.same_spin_matrix(0) @ C
    tb = C @ sp.same_spin_matrix(1).T
    refs = {1: ta, 2: tb, 7: full}
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
    # whole sigma through tbsci_sigma, and the CSR method on the same context
    got = ctx.sigma(Cd, precision=pr).double().cpu().numpy()
    assert np.linalg.norm(got - full) / scale <= tol
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_CSR)
    csr = ctx.sigma(Cd, precision=pr).double().cpu().numpy()
    assert np.linalg.norm(got - csr) / scale <= tol
    ctx.close()


def test_hole_windows_and_beta_blocks(env):
    """The complete M = 16, N = 8 space (12,870 strings per spin, 360,360
    hole-string entries per spin): the products of one sweep take several
    column windows of the 2 GiB buffer, and the beta sweep runs in two
    blocks of alpha rows (10,240 and 2,630 columns).  Eight sampled rows,
    first and last included, against the oracle, FP64 and FP32; FP64 equal
    to the CSR method's to 1e-12; the same-spin terms of two runs bitwise
    equal."""
    T, O, torch = env
    p = W.make_problem("fci_m16", 16, 8, None, 1006)
    ctx = T.Context.from_problem(p)
    # the automatic method (the default) takes the hole-pair sweep here: a
    # dense string set (45 strings per hole string) in a space of 1.66e8
    # determinants; its executed MFMA work is 8008 hole strings x a 48 x 48
    # padded block x 12,880 padded columns x 2
    for k in (0, 1):
        assert T.tbsci_timing_executed_flops(ctx.handle, k) == 2.0 * 8008 * 48 * 48 * 12880
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_HOLE)
    la = ctx.l_alpha
    C = np.random.default_rng(9).normal(size=(la, ctx.l_beta))
    rows = np.unique(np.r_[0, la - 1, np.random.default_rng(10).choice(la, 6, replace=False)])
    ref = O.Space.of(p).sigma(C, rows=rows, nthreads=16)
    Cg = torch.from_numpy(C).cuda()
    S1 = ctx.sigma(Cg).cpu().numpy()
    e, m = _rel(S1[rows], ref)
    assert e <= 1e-12 and m <= 1e-12, (e, m)
    # the hole-pair sweeps have no atomics: the same-spin terms repeat bit
    # for bit (the opposite-spin term does only in the reproducible mode)
    T1 = ctx.sigma_terms(Cg, 3).cpu().numpy()
    T2 = ctx.sigma_terms(Cg, 3).cpu().numpy()
    assert np.array_equal(T1.view(np.uint8), T2.view(np.uint8))
    got32 = ctx.sigma(Cg.float(), precision=T.TBSCI_FP32).double().cpu().numpy()[rows]
    assert _rel(got32, ref)[0] <= 2e-5
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_CSR)
    csr = ctx.sigma(Cg).cpu().numpy()
    e, m = _rel(S1, csr)
    assert e <= 1e-12 and m <= 1e-12, (e, m)
    ctx.close()


def test_hole_davidson(env):
    """A Davidson solve with the hole-pair sweeps reaches the CSR solve's
    energy (1e-8 Eh), FP64 and mixed."""
    T, O, torch = env
    p = PROBS["rand_m10_5_5"]()
    ctx = T.Context.from_problem(p)
    ref = ctx.davidson(tol_resid=1e-8)[0]
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_HOLE)
    a = ctx.davidson(tol_resid=1e-8)[0]
    b = ctx.davidson(precision=T.TBSCI_MIXED, tol_resid=1e-8)[0]
    assert a["converged"] == 1 and b["converged"] == 1
    assert abs(a["energy"] - ref["energy"]) < 1e-8
    assert abs(b["energy"] - ref["energy"]) < 1e-8
    ctx.close()


def test_same_spin_method_errors(env):
    """An unknown method is refused; a small space keeps CSR under the
    automatic method (its executed sweep work is 2 x entries x columns)
    and takes the hole-pair sweep when asked."""
    T, O, torch = env
    p = PROBS["fci_m8"]()
    ctx = T.Context.from_problem(p)
    with pytest.raises(T.TbsciError):
        ctx.set_same_spin(3)
    csr = T.tbsci_timing_executed_flops(ctx.handle, 0)
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_HOLE)
    # 28 hole strings of 15 strings each: 16 x 16 padded blocks, 70 columns -> 80
    assert T.tbsci_timing_executed_flops(ctx.handle, 0) == 2.0 * 28 * 16 * 16 * 80
    ctx.set_same_spin(T.TBSCI_SAME_SPIN_AUTO)
    assert T.tbsci_timing_executed_flops(ctx.handle, 0) == csr
    ctx.close()


def test_hole_with_reproducible_mode(env):
    """A context on the hole-pair sweeps (the complete M = 16 space, taken
    by the automatic method) in the reproducible mode: two whole sigma
    builds bitwise equal, and equal to the default mode's to 1e-12."""
    T, O, torch = env
    p = W.make_problem("fci_m16", 16, 8, None, 1006)
    ctx = T.Context.from_problem(p)
    Cg = torch.from_numpy(np.random.default_rng(12).normal(size=(ctx.l_alpha,
                                                                  ctx.l_beta))).cuda()
    ref = ctx.sigma(Cg).cpu().numpy()
    ctx.set_deterministic(True)
    a = ctx.sigma(Cg).cpu().numpy()
    b = ctx.sigma(Cg).cpu().numpy()
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    e, m = _rel(a, ref)
    assert e <= 1e-12 and m <= 1e-12, (e, m)
    ctx.close()
