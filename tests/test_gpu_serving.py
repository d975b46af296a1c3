"""GPU tests of the batched sigma / batched Davidson entry points and of the
serving loop, through the C ABI.

* grouped sigma: every problem of a mixed batch against the oracle (FP64
  1e-12 relative, FP32 2e-5) and against its own single launch;
* batched Davidson: energies against dense diagonalisation of the oracle
  Hamiltonian (1e-8 Eh), the same problem alone and inside a batch (1e-10
  Eh: the arithmetic of a problem does not depend on its batch), mixed
  precision against FP64 (1e-6 Eh);
* server: each request's result alone and in a mix of concurrent requests
  (1e-8 Eh, mixed precision both times), HBM budget never exceeded with
  requests queued behind it, small requests batched and large ones solo,
  per-request errors (invalid input, footprint above the budget, unknown
  ticket), cancellation on destroy.
"""
import math
import time

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


def _mix():
    return [
        W.config("fci_m8"),
        W.random_selection(8, 3, 4, 37, 53, seed=11),
        W.random_selection(10, 5, 5, 130, 97, seed=12),
        W.make_problem("ranked_m12", 12, 6, 400, 14, 24),
        W.make_problem("ranked_m10", 10, 5, 180, 31, 41),
        W.random_selection(7, 3, 3, 1, 1, seed=18),
        W.random_selection(12, 4, 6, 300, 257, seed=13),
    ]


def _dense_e0(O, p):
    """Lowest eigenvalue of the oracle's dense P H P (over both spin-flip
    sectors when the alpha and beta lists are identical)."""
    return O.lowest_by_flip_sector(O.Space.of(p))["lowest"]


def _ref_e0(T, O, p):
    """Dense diagonalisation of the oracle Hamiltonian for small spaces, else
    the single-problem FP64 solver (itself checked against the oracle)."""
    if len(p.alpha) * len(p.beta) <= 6000:
        return _dense_e0(O, p)
    ctx = T.Context.from_problem(p)
    r, _ = ctx.davidson(tol_resid=1e-8, n_max=8, max_iter=2000, want_vector=False)
    ctx.close()
    assert r["status"] == T.TBSCI_OK
    return r["energy"]


def test_sigma_batch_matches_oracle_and_single(env):
    T, O, torch = env
    probs = _mix()
    ctxs = [T.Context.from_problem(p) for p in probs]
    g = torch.Generator(device="cuda").manual_seed(5)
    Cs = [torch.randn((c.l_alpha, c.l_beta), dtype=torch.float64, device="cuda", generator=g)
          for c in ctxs]
    Sb = T.sigma_batch(ctxs, Cs)
    Sb32 = T.sigma_batch(ctxs, [C.float() for C in Cs], precision=T.TBSCI_FP32)
    for p, c, C, S, S32 in zip(probs, ctxs, Cs, Sb, Sb32):
        ref = O.Space.of(p).sigma(C.cpu().numpy())
        got = S.cpu().numpy()
        err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
        print(f"{p.name}: batch fp64 {err:.2e}", flush=True)
        assert err <= 1e-12
        single = c.sigma(C).cpu().numpy()
        assert np.abs(single - got).max() <= 1e-13 * max(np.abs(ref).max(), 1.0)
        e32 = np.linalg.norm(S32.double().cpu().numpy() - ref) / max(np.linalg.norm(ref), 1e-300)
        assert e32 <= 2e-5
    for c in ctxs:
        c.close()


def test_davidson_batch_energies(env):
    T, O, torch = env
    probs = _mix()
    ctxs = [T.Context.from_problem(p) for p in probs]
    res = T.davidson_batch(ctxs, tol_resid=1e-7, n_max=8, max_iter=400)
    for p, r in zip(probs, res):
        e0 = _ref_e0(T, O, p)
        print(f"{p.name}: batch E {r['energy']:.12f} dense {e0:.12f} iters {r['iters']}",
              flush=True)
        assert r["status"] == T.TBSCI_OK and r["converged"] == 1
        assert abs(r["energy"] - e0) <= 1e-8
    # the same problem alone in a batch of one
    alone = T.davidson_batch([ctxs[2]], tol_resid=1e-7, n_max=8, max_iter=400)[0]
    assert abs(alone["energy"] - res[2]["energy"]) <= 1e-10
    # against the single-problem solver
    single, _ = ctxs[2].davidson(tol_resid=1e-7, n_max=8, max_iter=400, want_vector=False)
    assert abs(single["energy"] - res[2]["energy"]) <= 1e-8
    # mixed precision: FP32 sigma phase, FP64 correction phase
    mixed = T.davidson_batch(ctxs, tol_resid=1e-6, n_max=8, max_iter=400,
                             precision=T.TBSCI_MIXED, fp32_switch_resid=1e-4)
    for p, r64, rm in zip(probs, res, mixed):
        assert rm["status"] == T.TBSCI_OK
        assert rm["iters_fp64"] >= 1
        assert abs(rm["energy"] - r64["energy"]) <= 1e-6
    for c in ctxs:
        c.close()


def test_davidson_batch_restart_n_max_2_and_3(env):
    T, O, torch = env
    p = W.make_problem("ranked_m10", 10, 5, 70, 31, 41)  # 4,900 determinants
    ctx = T.Context.from_problem(p)
    e0 = _dense_e0(O, p)
    for nmax in (2, 3):
        r = T.davidson_batch([ctx], tol_resid=1e-7, n_max=nmax, max_iter=2000)[0]
        assert r["status"] == T.TBSCI_OK
        assert abs(r["energy"] - e0) <= 1e-8
        s, _ = ctx.davidson(tol_resid=1e-7, n_max=nmax, max_iter=2000, want_vector=False)
        assert abs(s["energy"] - e0) <= 1e-8
    ctx.close()


def _wait(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(out)} requests unfinished")
        time.sleep(0.002)
    return out


def _serving_requests(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        M = int(rng.choice([8, 10, 12]))
        keep = min(int(rng.integers(20, 76)), math.comb(M, M // 2))  # dense-checkable
        reqs.append(W.make_problem(f"req{i}", M, M // 2, keep, 7000 + i, 8000 + i))
    return reqs


OPTS = dict(precision=2, tol_resid=1e-6, fp32_switch_resid=1e-4, n_max=8, max_iter=400)


def test_server_alone_vs_mix(env):
    T, O, torch = env
    reqs = _serving_requests(10, 3)
    # each request alone on a fresh server
    alone = []
    for p in reqs[:4]:
        srv = T.Server(hbm_budget_bytes=8 << 30, batch_ndet_threshold=1 << 40)
        t = srv.submit(p, **OPTS)
        alone.append(_wait(srv, [t])[t])
        srv.close()
    # all of them at once, with staggered arrivals
    srv = T.Server(hbm_budget_bytes=8 << 30, batch_ndet_threshold=1 << 40)
    tickets = []
    for p in reqs:
        tickets.append(srv.submit(p, **OPTS))
        time.sleep(0.003)
    res = _wait(srv, tickets)
    st = srv.stats()
    print(st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_batch"] >= 2  # requests shared rounds of the batched solver
    for a, t in zip(alone, tickets[:4]):
        r = res[t]
        print(f"alone {a['energy']:.12f} mix {r['energy']:.12f}", flush=True)
        assert a["status"] == T.TBSCI_OK and r["status"] == T.TBSCI_OK
        assert abs(a["energy"] - r["energy"]) <= 1e-8
    # every request against dense diagonalisation (mixed precision: 1e-6)
    for p, t in zip(reqs, tickets):
        assert res[t]["batched"] is True
        assert abs(res[t]["energy"] - _dense_e0(O, p)) <= 1e-6
    srv.close()


def test_server_budget_queueing_and_solo(env):
    T, O, torch = env
    # requests of one shape: their footprint bounds are equal
    reqs = [W.make_problem(f"u{i}", 10, 5, 60, 9100 + i, 9200 + i) for i in range(8)]
    big = W.make_problem("big_m12", 12, 6, 700, 77, 78)  # 490,000 determinants
    # smallest budget (in 25% steps) that admits one request: requests
    # above the whole budget are refused at submission
    budget = 1 << 20
    while True:
        srv = T.Server(hbm_budget_bytes=budget, batch_ndet_threshold=100_000)
        try:
            srv.submit(reqs[0], **OPTS)
            srv.close()
            break
        except T.TbsciError as e:
            assert e.code == T.TBSCI_E_NOMEM
            srv.close()
            budget = int(budget * 1.25)
    budget = int(budget * 1.3)
    srv = T.Server(hbm_budget_bytes=budget, batch_ndet_threshold=100_000)
    tickets = [srv.submit(p, **OPTS) for p in reqs]
    with pytest.raises(T.TbsciError) as ei:  # the big one cannot fit this budget at all
        srv.submit(big, **OPTS)
    assert ei.value.code == T.TBSCI_E_NOMEM
    res = _wait(srv, tickets)
    st = srv.stats()
    print(budget, st, flush=True)
    assert st["hbm_reserved_peak"] <= budget
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert max(r["queue_s"] for r in res.values()) > 0.0
    for p, t in zip(reqs, tickets):
        assert res[t]["status"] == T.TBSCI_OK
        assert res[t]["footprint_bytes"] <= budget
        assert abs(res[t]["energy"] - _dense_e0(O, p)) <= 1e-6
    srv.close()
    # a roomy server runs the big request solo beside the batch
    srv = T.Server(hbm_budget_bytes=16 << 30, batch_ndet_threshold=100_000)
    tb = srv.submit(big, **OPTS)
    ts = [srv.submit(p, **OPTS) for p in reqs[:3]]
    res = _wait(srv, [tb] + ts, timeout=300.0)
    assert res[tb]["batched"] is False and res[tb]["status"] == T.TBSCI_OK
    ctx = T.Context.from_problem(big)
    ref, _ = ctx.davidson(tol_resid=1e-6, n_max=8, max_iter=400, want_vector=False)
    ctx.close()
    assert abs(res[tb]["energy"] - ref["energy"]) <= 1e-6
    for t in ts:
        assert res[t]["batched"] is True
    srv.close()


def test_server_errors_and_cancel(env):
    T, O, torch = env
    srv = T.Server(hbm_budget_bytes=4 << 30, batch_ndet_threshold=1 << 40)
    p = W.config("fci_m8")
    bad_h = p.h.copy()
    bad_h[0, 1] += 1.0  # not symmetric
    with pytest.raises(T.TbsciError) as ei:
        T.tbsci_submit(srv._srv, p.M, p.n_alpha, p.n_beta, bad_h, p.eri, p.alpha, p.beta)
    assert ei.value.code == T.TBSCI_E_INVAL
    with pytest.raises(T.TbsciError) as ei:
        srv.poll(987654321)
    assert ei.value.code == T.TBSCI_E_NOTFOUND
    # a good request still runs after the failed submit
    t = srv.submit(p, **OPTS)
    r = _wait(srv, [t])[t]
    assert r["status"] == T.TBSCI_OK
    # destroy with work queued and running: returns, nothing hangs
    for q in _serving_requests(12, 5):
        srv.submit(q, **OPTS)
    srv.close()


def test_two_sector_slots_in_batch_and_server(env):
    """Batched and served solves of identical-list problems run their two
    spin-flip sectors in two slots at once and report one result: the lowest
    state (here antisymmetric: M = 8, N = 4, every string, integral seed
    100), the other sector's lowest as energy_other, the iterations of both;
    equal to the single solver's result."""
    T, O, torch = env
    p = W.make_problem("anti_gs", 8, 4, None, 100)
    ref = O.lowest_by_flip_sector(O.Space.of(p))
    ctx = T.Context.from_problem(p)
    other = T.Context.from_problem(W.random_selection(8, 3, 4, 37, 53, seed=11))
    single, _ = ctx.davidson(tol_resid=1e-8, want_vector=False)
    res = T.davidson_batch([ctx, other], tol_resid=1e-8)
    r = res[0]
    assert r["status"] == 0 and r["sector"] == -1
    assert abs(r["energy"] - ref["lowest"]) < 1e-8
    assert abs(r["energy_other"] - ref["sym"]) < 1e-8
    assert abs(r["energy"] - single["energy"]) < 1e-10
    assert r["iters"] >= 2 and res[1]["status"] == 0 and res[1]["sector"] == 0
    srv = T.Server()
    tk = srv.submit(p, tol_resid=1e-8)
    while (d := srv.poll(tk)) is None:
        time.sleep(0.01)
    assert d["status"] == 0 and d["batched"] and d["sector"] == -1
    assert abs(d["energy"] - ref["lowest"]) < 1e-8
    assert abs(d["energy_other"] - ref["sym"]) < 1e-8
    srv.close()
    ctx.close()
    other.close()
