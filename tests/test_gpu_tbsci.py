"""GPU parity of TBSCI spaces (determinant-level pruning, Sec. II.A) through
the C ABI, against the oracle's sigma over the kept determinants (both
membership tests of Algorithm 1):

* compact sigma in FP64 (1e-12 relative) and FP32 (2e-5) on ragged random
  layouts (empty rows, empty columns, single entries), on a staircase layout
  of energy-ranked strings and on the layout that keeps everything;
* the compact diagonal against the oracle's restricted diagonal (1e-13);
* Davidson in FP64 against dense diagonalisation of the oracle's restricted
  matrix (1e-8 Eh) and mixed within 1e-6 of it, with the compact eigenvector
  checked by the oracle's sigma; flip sectors on symmetric layouts of
  identical lists;
* sampled rows of a full-size layout (M = 16, 3000 x 3000 strings, about a
  third of the TPB space kept);
* layout errors and entry points that take whole TPB spaces only.
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


def _layouts():
    return {
        "rand_m9_ragged": (W.random_selection(9, 4, 3, 70, 60, seed=71),
                           lambda la, lb: W.dets_random(la, lb, 0.35, 72)),
        "rand_m8_sparse": (W.random_selection(8, 3, 4, 40, 50, seed=73),
                           lambda la, lb: W.dets_random(la, lb, 0.05, 74)),
        "ranked_m12_stair": (W.make_problem("st12", 12, 6, 130, 75, 76, independent_beta=True),
                             lambda la, lb: W.dets_rank_sum(la, lb, 0.3)),
        "fci_m8_all": (W.config("fci_m8"),
                       lambda la, lb: (np.arange(la + 1, dtype=np.int64) * lb,
                                       np.tile(np.arange(lb, dtype=np.int32), la))),
    }


LAYOUTS = _layouts()


def _ctx_and_oracle(T, O, name):
    p, lay = LAYOUTS[name]
    ro, bi = lay(len(p.alpha), len(p.beta))
    ctx = T.Context.from_problem(p)
    ctx.set_dets(ro, bi)
    sp = O.Space.of(p)
    sp.set_dets(ro, bi)
    assert ctx.n_det == sp.n_dets == int(ro[-1])
    return p, ctx, sp


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b)), \
        float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_tbsci_sigma_and_diag(env, name):
    T, O, torch = env
    p, ctx, sp = _ctx_and_oracle(T, O, name)
    c = np.random.default_rng(3).normal(size=ctx.n_det)
    ref = sp.sigma_dets(c)
    S = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    r2, rm = _rel(S, ref)
    assert r2 <= 1e-12 and rm <= 1e-12, (r2, rm)
    S32 = ctx.sigma(torch.from_numpy(c).float().cuda(), precision=T.TBSCI_FP32)
    r2, rm = _rel(S32.double().cpu().numpy(), ref)
    assert r2 <= 2e-5, r2
    D = ctx.diag().cpu().numpy()
    dref = O.Space.of(p).diag().ravel()[sp.dets_index()]
    assert np.abs(D - dref).max() <= 1e-13 * np.abs(dref).max()
    # back to the whole TPB space
    ctx.set_dets()
    assert ctx.n_det == len(p.alpha) * len(p.beta)
    ctx.close()


@pytest.mark.parametrize("name", ["rand_m9_ragged", "ranked_m12_stair"])
def test_tbsci_davidson_vs_dense(env, name):
    T, O, torch = env
    p, ctx, sp = _ctx_and_oracle(T, O, name)
    Hd = sp.dense_h_dets()
    e_ref = float(np.linalg.eigvalsh(Hd)[0])
    info, X = ctx.davidson(tol_resid=1e-8, n_max=8, max_iter=1000)
    assert info["status"] == 0 and abs(info["energy"] - e_ref) < 1e-8
    x = X.cpu().numpy()
    assert x.shape == (ctx.n_det,) and abs(np.linalg.norm(x) - 1) < 1e-10
    assert np.linalg.norm(sp.sigma_dets(x) - info["energy"] * x) < 5e-8
    im, _ = ctx.davidson(tol_resid=1e-5, n_max=8, max_iter=1000, precision=T.TBSCI_MIXED,
                         want_vector=False)
    assert im["status"] == 0 and abs(im["energy"] - e_ref) < 1e-6
    # a compact guess: the eigenvector converges at once
    i2, _ = ctx.davidson(tol_resid=1e-8, guess=X, want_vector=False)
    assert i2["iters"] <= 4 and abs(i2["energy"] - e_ref) < 1e-9
    ctx.close()


def test_tbsci_symmetric_layout_keeps_flip_sectors(env):
    """Identical lists and a layout closed under (w, u) -> (u, w): both
    spin-flip sectors are solved and the lowest over the kept space is
    returned; an asymmetric layout solves without sectors."""
    T, O, torch = env
    p = W.make_problem("sym10", 10, 5, 60, 77, 78)
    la = len(p.alpha)
    ro, bi = W.dets_rank_sum(la, la, 0.4)  # symmetric staircase: w/la + u/la <= t
    ctx = T.Context.from_problem(p)
    ctx.set_dets(ro, bi)
    sp = O.Space.of(p)
    sp.set_dets(ro, bi)
    e_ref = float(np.linalg.eigvalsh(sp.dense_h_dets())[0])
    info, X = ctx.davidson(tol_resid=1e-8, max_iter=1000)
    assert info["status"] == 0 and info["sector"] in (1, -1) and not np.isnan(info["energy_other"])
    assert abs(info["energy"] - e_ref) < 1e-8
    ro2, bi2 = W.dets_random(la, la, 0.5, 79)
    ctx.set_dets(ro2, bi2)
    sp2 = O.Space.of(p)
    sp2.set_dets(ro2, bi2)
    i2, _ = ctx.davidson(tol_resid=1e-8, max_iter=1000, want_vector=False)
    assert i2["sector"] == 0
    assert abs(i2["energy"] - np.linalg.eigvalsh(sp2.dense_h_dets())[0]) < 1e-8
    ctx.close()


def test_tbsci_full_size_sampled_rows(env):
    """M = 16, N = 8, 3000 x 3000 energy-ranked strings with the staircase
    layout keeping about a third of the 9.0e6 determinants: FP64 sigma on 12
    seeded alpha rows against the oracle."""
    T, O, torch = env
    p = W.config("sel_m16")
    la, lb = len(p.alpha), len(p.beta)
    ro, bi = W.dets_rank_sum(la, lb, 0.33)
    ctx = T.Context.from_problem(p)
    ctx.set_dets(ro, bi)
    sp = O.Space.of(p)
    sp.set_dets(ro, bi)
    c = np.random.default_rng(9).normal(size=ctx.n_det)
    c /= np.linalg.norm(c)
    S = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    rows = np.sort(np.random.default_rng(10).choice(la, size=12, replace=False))
    ref = sp.sigma_dets(c, rows=rows, nthreads=16)
    got = np.concatenate([S[ro[r]:ro[r + 1]] for r in rows])
    r2, rm = _rel(got, ref)
    assert r2 <= 1e-12 and rm <= 1e-11, (r2, rm)
    ctx.close()


def test_tbsci_errors(env):
    T, O, torch = env
    p = W.random_selection(8, 3, 3, 10, 12, seed=80)
    ctx = T.Context.from_problem(p)
    bad = [([1] + [0] * 10, [0]), ([0, 2] + [2] * 9, [0, 12]), ([0, 2] + [2] * 9, [3, 3]),
           ([0] * 11, [])]
    for ro, bi in bad:
        with pytest.raises(T.TbsciError) as ei:
            ctx.set_dets(np.array(ro, dtype=np.int64), np.array(bi, dtype=np.int32))
        assert ei.value.code == T.TBSCI_E_INVAL
    assert ctx.n_det == 10 * 12  # the failed calls left the TPB space
    ctx.set_dets(*W.dets_random(10, 12, 0.5, 81))
    C = torch.zeros(ctx.n_det, dtype=torch.float64, device="cuda")
    S = torch.zeros_like(C)
    with pytest.raises(T.TbsciError):
        T.tbsci_sigma_noalloc(ctx.handle, C, S)
    with pytest.raises(T.TbsciError):
        T.tbsci_sigma_batch([ctx.handle, ctx.handle], [C, C], [S, S])
    ctx.close()
