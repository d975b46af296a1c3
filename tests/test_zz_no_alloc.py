"""GPU test of tbsci_sigma_noalloc through the C ABI: its sigma against
tbsci_sigma's on the same inputs, FP64 to 1e-12 and FP32 to 2e-5 relative
(the kernels are shared; only the beta sweep's blocking differs), on two
calls in a row with the second space smaller than the first, and with a
space whose beta sweep needs several blocks of the 64 MiB static array."""
import numpy as np
import pytest

from paper_2503_10335_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_sigma_noalloc_matches_sigma():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10335_amd import tbsci as T
    T.load()
    # the first needs several workspace blocks (l_beta 6000: 96 KB of scratch
    # per alpha row, 699 rows fit, blocks of 512 rows), the second is smaller
    probs = [W.make_problem("noalloc_big", 16, 8, 6000, 41, 42),
             W.random_selection(10, 5, 4, 150, 180, seed=43)]
    for p in probs:
        ctx = T.Context.from_problem(p)
        C64 = torch.from_numpy(W.random_vector(ctx.l_alpha, ctx.l_beta, seed=3)).cuda()
        for prec, dt, tol in ((T.TBSCI_FP64, torch.float64, 1e-12),
                              (T.TBSCI_FP32, torch.float32, 2e-5)):
            C = C64.to(dt)
            ref = torch.empty_like(C)
            got = torch.full_like(C, float("nan"))
            T.tbsci_sigma(ctx.handle, C, ref, prec)
            T.tbsci_sigma_noalloc(ctx.handle, C, got, prec)
            torch.cuda.synchronize()
            r, g = ref.double().cpu().numpy(), got.double().cpu().numpy()
            assert np.isfinite(g).all()
            assert _rel(g, r) <= tol, (p.name, prec)
        ctx.close()
