"""C-ABI boundary checks that need no GPU: the library loads, exports every
function include/tbsci.h declares, and rejects bad inputs before any device
work (status codes, message, output untouched)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_10335_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tbsci_\w+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def T():
    from paper_2503_10335_amd import tbsci
    if not os.path.exists(tbsci.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    tbsci.load()
    return tbsci


def test_exports_every_declared_symbol(T):
    names = _declared()
    assert "tbsci_sigma" in names and "tbsci_create" in names and len(names) >= 12
    lib = ctypes.CDLL(T.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _create_rc(T, M, na, nb, h, eri, a, b):
    out = ctypes.c_void_p(12345)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p) if x is not None else None
    rc = T.load().tbsci_create(M, na, nb, p(h), p(eri), p(a), 0 if a is None else len(a), p(b),
                               0 if b is None else len(b), 0, ctypes.byref(out))
    return rc, out.value


@pytest.fixture(scope="module")
def good():
    return W.make_problem("v", 6, 3, 10, 3, 4)


def test_validation_errors(T, good):
    p = good
    h, eri, a, b = p.h, p.eri, p.alpha, p.beta
    cases = []
    cases.append(("M>64", (65, 3, 3, h, eri, a, b), "M must be"))
    cases.append(("M<1", (0, 3, 3, h, eri, a, b), "M must be"))
    bad = a.copy(); bad[2] = bad[1]
    cases.append(("duplicate", (6, 3, 3, h, eri, bad, b), "duplicate"))
    bad = a.copy(); bad[0] = np.uint64(0b111100)
    cases.append(("popcount", (6, 3, 3, h, eri, bad, b), "wrong number"))
    bad = b.copy(); bad[0] = np.uint64((1 << 6) | 0b11)
    cases.append(("bit>=M", (6, 3, 3, h, eri, a, bad), "at or above M"))
    hb = h.copy(); hb[0, 1] += 1e-6
    cases.append(("h asym", (6, 3, 3, hb, eri, a, b), "not symmetric"))
    eb = eri.copy(); eb[0, 1, 2, 3] += 1e-6
    cases.append(("eri asym", (6, 3, 3, h, eb, a, b), "8-fold"))
    eb = eri.copy(); eb[1, 1, 1, 1] = np.nan
    cases.append(("eri nan", (6, 3, 3, h, eb, a, b), "non-finite"))
    cases.append(("null h", (6, 3, 3, None, eri, a, b), "NULL"))
    cases.append(("null alpha", (6, 3, 3, h, eri, None, b), "NULL"))
    cases.append(("n>M", (6, 7, 3, h, eri, a, b), "electron counts"))
    for name, args, msg in cases:
        rc, out = _create_rc(T, *args)
        assert rc == T.TBSCI_E_INVAL, name
        assert out == 12345, name  # output untouched
        assert msg in T.last_error(), (name, T.last_error())


def test_null_handles_are_safe(T):
    lib = T.load()
    lib.tbsci_destroy(None)
    assert lib.tbsci_sigma(None, None, None, 0, None) == T.TBSCI_E_INVAL
    assert lib.tbsci_dims(None, None, None, None) == T.TBSCI_E_INVAL
    info = T.DavidsonInfo()
    assert lib.tbsci_davidson(None, None, None, None, ctypes.byref(info), None) == T.TBSCI_E_INVAL
    o = T.tbsci_davidson_default_opts()
    assert (o.n_max, o.max_iter, o.precision) == (8, 200, T.TBSCI_FP64)
    assert o.tol_resid == 1e-6 and o.fp32_switch_resid == 1e-4


def test_batch_and_server_null_and_invalid(T, good):
    lib = T.load()
    lib.tbsci_server_destroy(None)
    info = T.DavidsonInfo()
    assert lib.tbsci_poll(None, 1, ctypes.byref(info)) == T.TBSCI_E_INVAL
    assert lib.tbsci_server_stats(None, None) == T.TBSCI_E_INVAL
    assert lib.tbsci_request_times(None, 1, None, None, None, None) == T.TBSCI_E_INVAL
    t = ctypes.c_uint64(77)
    p = good
    ptr = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    assert lib.tbsci_submit(None, p.M, p.n_alpha, p.n_beta, ptr(p.h), ptr(p.eri), ptr(p.alpha),
                            len(p.alpha), ptr(p.beta), len(p.beta), None,
                            ctypes.byref(t)) == T.TBSCI_E_INVAL
    assert t.value == 77
    out = ctypes.c_void_p(5)
    assert lib.tbsci_server_create(0, 0, 10, ctypes.byref(out)) == T.TBSCI_E_INVAL
    assert "budget" in T.last_error() and out.value == 5
    assert lib.tbsci_server_create(0, 1 << 30, -1, ctypes.byref(out)) == T.TBSCI_E_INVAL
    # batched entry points: n out of range, NULL arrays; n == 0 is a no-op
    st = (ctypes.c_int * 1)()
    infos = (T.DavidsonInfo * 1)()
    assert lib.tbsci_davidson_batch(None, 65, None, infos, st, None) == T.TBSCI_E_INVAL
    assert lib.tbsci_davidson_batch(None, 1, None, infos, st, None) == T.TBSCI_E_INVAL
    assert lib.tbsci_davidson_batch(None, 0, None, None, None, None) == T.TBSCI_OK
    assert lib.tbsci_sigma_batch(None, -1, None, None, 0, None) == T.TBSCI_E_INVAL
    assert lib.tbsci_sigma_batch(None, 1, None, None, 0, None) == T.TBSCI_E_INVAL
