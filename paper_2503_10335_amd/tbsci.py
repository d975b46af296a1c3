"""Thin ctypes binding of libtbsci.so (declared in include/tbsci.h).

Argument marshalling only: every step of the sigma build, the solver and
the serving loop runs in the library's HIP kernels.  PyTorch provides the
device memory (tensors) and the streams.  There is no CPU fallback: if the
library is missing, loading fails with an error.

Functions named tbsci_* mirror the C entry points one to one; ``Context``
is a small convenience wrapper over them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime the library binds to (same soname)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtbsci.so")

TBSCI_OK = 0
TBSCI_PENDING = 1
TBSCI_E_INVAL = -1
TBSCI_E_NOMEM = -2
TBSCI_E_DEVICE = -3
TBSCI_E_NOTCONV = -4
TBSCI_E_NOTFOUND = -5
TBSCI_E_STATE = -6
TBSCI_FP64 = 0
TBSCI_FP32 = 1
TBSCI_MIXED = 2


class TbsciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tbsci error {code}: {msg}")
        self.code = code


TBSCI_GUESS_DIAG = 0
TBSCI_GUESS_USER = 1
TBSCI_GUESS_SUBSPACE = 2
TBSCI_STORE_AUTO = 0
TBSCI_STORE_FULL = 1
TBSCI_STORE_LEAN = 2
TBSCI_SAME_SPIN_AUTO, TBSCI_SAME_SPIN_CSR, TBSCI_SAME_SPIN_HOLE = 0, 1, 2


class DavidsonOpts(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int), ("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("guess_kind", ctypes.c_int), ("sector", ctypes.c_int), ("storage", ctypes.c_int),
                ("guess_strings", ctypes.c_int),
                ("tol_resid", ctypes.c_double), ("tol_energy", ctypes.c_double),
                ("fp32_switch_resid", ctypes.c_double), ("precond_floor", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("hbm_reserved", ctypes.c_size_t),
                ("hbm_reserved_peak", ctypes.c_size_t), ("submitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running_batched", ctypes.c_int64),
                ("running_solo", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("max_batch", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class DavidsonInfo(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("resid_norm", ctypes.c_double),
                ("energy_fp64_check", ctypes.c_double), ("energy_other", ctypes.c_double),
                ("iters", ctypes.c_int), ("iters_fp32", ctypes.c_int), ("iters_fp64", ctypes.c_int),
                ("converged", ctypes.c_int), ("sector", ctypes.c_int), ("lean", ctypes.c_int),
                ("t_total_s", ctypes.c_double), ("t_sigma_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libtbsci.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_10335_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, c_int, c_dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "tbsci_create": (c_int, [c_int, c_int, c_int, P, P, P, i64, P, i64, c_int, P]),
        "tbsci_destroy": (None, [P]),
        "tbsci_dims": (c_int, [P, P, P, P]),
        "tbsci_set_dets": (c_int, [P, P, P]),
        "tbsci_get_dets": (c_int, [P, P, P]),
        "tbsci_set_symmetry": (c_int, [P, P, c_int]),
        "tbsci_string_irreps": (c_int, [P, c_int, P]),
        "tbsci_string_weights": (c_int, [P, P, P, P, P]),
        "tbsci_select_strings": (c_int, [P, c_int, P, c_dbl, ctypes.c_uint64, P, P, P]),
        "tbsci_coef_histogram": (c_int, [P, P, c_dbl, c_dbl, c_int, P, P]),
        "tbsci_sigma": (c_int, [P, P, P, c_int, P]),
        "tbsci_sigma_terms": (c_int, [P, P, P, c_int, c_int, P]),
        "tbsci_sigma_noalloc": (c_int, [P, P, P, c_int, P]),
        "tbsci_diag": (c_int, [P, P, P]),
        "tbsci_davidson_default_opts": (None, [P]),
        "tbsci_davidson": (c_int, [P, P, P, P, P, P]),
        "tbsci_string_index": (c_int, [P, c_int, P, P]),
        "tbsci_lookup": (c_int, [P, c_int, P, i64, P, P]),
        "tbsci_list_size": (c_int, [P, c_int, c_int, P]),
        "tbsci_get_list": (c_int, [P, c_int, c_int, P, P, P]),
        "tbsci_timing_enable": (c_int, [P, c_int]),
        "tbsci_set_deterministic": (c_int, [P, c_int]),
        "tbsci_set_same_spin": (c_int, [P, c_int]),
        "tbsci_timing_read": (c_int, [P, c_int, c_int, P, P, P, P, P]),
        "tbsci_timing_executed_flops": (c_int, [P, c_int, c_int, P]),
        "tbsci_sigma_batch": (c_int, [P, c_int, P, P, c_int, P]),
        "tbsci_davidson_batch": (c_int, [P, c_int, P, P, P, P]),
        "tbsci_server_create": (c_int, [c_int, ctypes.c_size_t, i64, P]),
        "tbsci_server_destroy": (None, [P]),
        "tbsci_submit": (c_int, [P, c_int, c_int, c_int, P, P, P, i64, P, i64, P, P]),
        "tbsci_poll": (c_int, [P, ctypes.c_uint64, P]),
        "tbsci_request_times": (c_int, [P, ctypes.c_uint64, P, P, P, P]),
        "tbsci_server_stats": (c_int, [P, P]),
        "tbsci_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().tbsci_last_error().decode()


def _check(rc, allow=(TBSCI_OK,)):
    if rc not in allow:
        raise TbsciError(rc, last_error())
    return rc


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ---------------------------------------------------------------- raw calls

def tbsci_create(M, n_alpha, n_beta, h, eri, alpha, beta, device=0):
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    a = np.ascontiguousarray(alpha, dtype=np.uint64)
    b = np.ascontiguousarray(beta, dtype=np.uint64)
    out = ctypes.c_void_p()
    _check(load().tbsci_create(int(M), int(n_alpha), int(n_beta), _np_ptr(h), _np_ptr(eri),
                               _np_ptr(a), len(a), _np_ptr(b), len(b), int(device),
                               ctypes.byref(out)))
    return out


def tbsci_destroy(ctx):
    load().tbsci_destroy(ctx)


def tbsci_dims(ctx):
    la, lb, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().tbsci_dims(ctx, ctypes.byref(la), ctypes.byref(lb), ctypes.byref(nd)))
    return la.value, lb.value, nd.value


def tbsci_set_dets(ctx, row_off=None, beta_idx=None):
    if row_off is None and beta_idx is None:
        _check(load().tbsci_set_dets(ctx, None, None))
        return
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    bi = np.ascontiguousarray(beta_idx, dtype=np.int32)
    _check(load().tbsci_set_dets(ctx, _np_ptr(ro), _np_ptr(bi) if bi.size else None))


def tbsci_get_dets(ctx, l_alpha, n_det):
    ro = np.zeros(l_alpha + 1, dtype=np.int64)
    bi = np.zeros(max(n_det, 1), dtype=np.int32)
    _check(load().tbsci_get_dets(ctx, _np_ptr(ro), _np_ptr(bi)))
    return ro, bi[:n_det]


def tbsci_set_symmetry(ctx, orb_irrep, target_irrep):
    g = np.ascontiguousarray(orb_irrep, dtype=np.int32)
    _check(load().tbsci_set_symmetry(ctx, _np_ptr(g), int(target_irrep)))


def tbsci_string_irreps(ctx, spin, l):
    out = np.zeros(max(l, 1), dtype=np.int32)
    _check(load().tbsci_string_irreps(ctx, int(spin), _np_ptr(out)))
    return out[:l]


def tbsci_sigma(ctx, C, S, precision=TBSCI_FP64, stream=None):
    _check(load().tbsci_sigma(ctx, ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                              int(precision), _stream(stream)))


def tbsci_sigma_noalloc(ctx, C, S, precision=TBSCI_FP64, stream=None):
    _check(load().tbsci_sigma_noalloc(ctx, ctypes.c_void_p(C.data_ptr()),
                                      ctypes.c_void_p(S.data_ptr()), int(precision),
                                      _stream(stream)))


def tbsci_sigma_terms(ctx, C, S, precision=TBSCI_FP64, terms=7, stream=None):
    _check(load().tbsci_sigma_terms(ctx, ctypes.c_void_p(C.data_ptr()),
                                    ctypes.c_void_p(S.data_ptr()), int(precision), int(terms),
                                    _stream(stream)))


def tbsci_diag(ctx, D, stream=None):
    _check(load().tbsci_diag(ctx, ctypes.c_void_p(D.data_ptr()), _stream(stream)))


def tbsci_davidson_default_opts():
    o = DavidsonOpts()
    load().tbsci_davidson_default_opts(ctypes.byref(o))
    return o


def tbsci_davidson(ctx, opts=None, guess=None, C_out=None, stream=None):
    info = DavidsonInfo()
    rc = load().tbsci_davidson(ctx, ctypes.byref(opts) if opts is not None else None,
                               ctypes.c_void_p(guess.data_ptr()) if guess is not None else None,
                               ctypes.c_void_p(C_out.data_ptr()) if C_out is not None else None,
                               ctypes.byref(info), _stream(stream))
    _check(rc, allow=(TBSCI_OK, TBSCI_E_NOTCONV))
    return rc, info


def tbsci_string_index(ctx, spin, l):
    keys = np.zeros(l, dtype=np.uint64)
    pos = np.zeros(l, dtype=np.int32)
    _check(load().tbsci_string_index(ctx, int(spin), _np_ptr(keys), _np_ptr(pos)))
    return keys, pos


def tbsci_lookup(ctx, spin, queries, out, stream=None):
    _check(load().tbsci_lookup(ctx, int(spin), ctypes.c_void_p(queries.data_ptr()), queries.numel(),
                               ctypes.c_void_p(out.data_ptr()), _stream(stream)))


def tbsci_list_size(ctx, spin, kind):
    n = ctypes.c_int64()
    _check(load().tbsci_list_size(ctx, int(spin), int(kind), ctypes.byref(n)))
    return n.value


def tbsci_get_list(ctx, spin, kind, l):
    n = tbsci_list_size(ctx, spin, kind)
    ptr = np.zeros(l + 1, dtype=np.int64)
    if kind == 3:
        ent = np.zeros(max(n, 1), dtype=np.int32)
        val = np.zeros(max(n, 1), dtype=np.float64)
        _check(load().tbsci_get_list(ctx, int(spin), 3, _np_ptr(ptr), _np_ptr(ent), _np_ptr(val)))
        return ptr, ent[:n], val[:n]
    ent = np.zeros((max(n, 1), 6), dtype=np.int32)
    _check(load().tbsci_get_list(ctx, int(spin), int(kind), _np_ptr(ptr), _np_ptr(ent), None))
    return ptr, ent[:n]


TBSCI_N_KERNELS = 3


def tbsci_set_same_spin(ctx, method):
    _check(load().tbsci_set_same_spin(ctx, int(method)))


def tbsci_set_deterministic(ctx, enable=True):
    _check(load().tbsci_set_deterministic(ctx, 1 if enable else 0))


def tbsci_timing_enable(ctx, enable=True):
    _check(load().tbsci_timing_enable(ctx, 1 if enable else 0))


def tbsci_timing_read(ctx, kernel, precision=TBSCI_FP64):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    fl, by = ctypes.c_double(), ctypes.c_double()
    name = ctypes.c_char_p()
    _check(load().tbsci_timing_read(ctx, int(kernel), int(precision), ctypes.byref(ms),
                                    ctypes.byref(n), ctypes.byref(fl), ctypes.byref(by),
                                    ctypes.byref(name)))
    return dict(name=name.value.decode(), total_ms=ms.value, launches=n.value, flops=fl.value,
                bytes=by.value)


def tbsci_timing_executed_flops(ctx, kernel, precision=TBSCI_FP64):
    fl = ctypes.c_double()
    _check(load().tbsci_timing_executed_flops(ctx, int(kernel), int(precision),
                                              ctypes.byref(fl)))
    return fl.value


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * max(len(ptrs), 1))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def tbsci_sigma_batch(ctxs, Cs, Ss, precision=TBSCI_FP64, stream=None):
    n = len(ctxs)
    _check(load().tbsci_sigma_batch(_ptr_array([c.value for c in ctxs]), n,
                                    _ptr_array([C.data_ptr() for C in Cs]),
                                    _ptr_array([S.data_ptr() for S in Ss]), int(precision),
                                    _stream(stream)))


def tbsci_davidson_batch(ctxs, opts=None, stream=None):
    n = len(ctxs)
    infos = (DavidsonInfo * max(n, 1))()
    status = (ctypes.c_int * max(n, 1))()
    op = None
    if opts is not None:
        op = (DavidsonOpts * n)(*opts)
    _check(load().tbsci_davidson_batch(_ptr_array([c.value for c in ctxs]), n, op, infos, status,
                                       _stream(stream)))
    return [status[i] for i in range(n)], [infos[i] for i in range(n)]


def tbsci_server_create(device=0, hbm_budget_bytes=64 << 30, batch_ndet_threshold=2_000_000):
    out = ctypes.c_void_p()
    _check(load().tbsci_server_create(int(device), int(hbm_budget_bytes),
                                      int(batch_ndet_threshold), ctypes.byref(out)))
    return out


def tbsci_server_destroy(srv):
    load().tbsci_server_destroy(srv)


def tbsci_submit(srv, M, n_alpha, n_beta, h, eri, alpha, beta, opts=None):
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    a = np.ascontiguousarray(alpha, dtype=np.uint64)
    b = np.ascontiguousarray(beta, dtype=np.uint64)
    t = ctypes.c_uint64()
    _check(load().tbsci_submit(srv, int(M), int(n_alpha), int(n_beta), _np_ptr(h), _np_ptr(eri),
                               _np_ptr(a), len(a), _np_ptr(b), len(b),
                               ctypes.byref(opts) if opts is not None else None, ctypes.byref(t)))
    return t.value


def tbsci_poll(srv, ticket):
    """(status, info): status TBSCI_PENDING while not finished."""
    info = DavidsonInfo()
    rc = load().tbsci_poll(srv, ctypes.c_uint64(ticket), ctypes.byref(info))
    if rc == TBSCI_E_NOTFOUND:
        raise TbsciError(rc, last_error())
    return rc, info


def tbsci_request_times(srv, ticket):
    q, lat = ctypes.c_double(), ctypes.c_double()
    bt, fp = ctypes.c_int(), ctypes.c_int64()
    rc = load().tbsci_request_times(srv, ctypes.c_uint64(ticket), ctypes.byref(q),
                                    ctypes.byref(lat), ctypes.byref(bt), ctypes.byref(fp))
    _check(rc, allow=(TBSCI_OK, TBSCI_PENDING))
    if rc == TBSCI_PENDING:
        return None
    return dict(queue_s=q.value, latency_s=lat.value, batched=bool(bt.value),
                footprint_bytes=fp.value)


def tbsci_server_stats(srv):
    s = ServerInfo()
    _check(load().tbsci_server_stats(srv, ctypes.byref(s)))
    return s.as_dict()


def make_opts(n_max=8, max_iter=200, precision=TBSCI_FP64, tol_resid=1e-6, tol_energy=0.0,
              fp32_switch_resid=1e-4, precond_floor=1e-8, sector=0, storage=TBSCI_STORE_AUTO,
              guess_kind=TBSCI_GUESS_DIAG, guess_strings=0):
    o = tbsci_davidson_default_opts()
    o.n_max, o.max_iter, o.precision = n_max, max_iter, precision
    o.guess_kind, o.sector, o.storage = guess_kind, sector, storage
    o.guess_strings = guess_strings
    o.tol_resid, o.tol_energy = tol_resid, tol_energy
    o.fp32_switch_resid, o.precond_floor = fp32_switch_resid, precond_floor
    return o


class Server:
    """Serving loop on one device (tbsci_server_*)."""

    def __init__(self, device=0, hbm_budget_bytes=64 << 30, batch_ndet_threshold=2_000_000):
        self._srv = tbsci_server_create(device, hbm_budget_bytes, batch_ndet_threshold)

    def submit(self, prob, **opts):
        o = make_opts(**opts) if opts else None
        return tbsci_submit(self._srv, prob.M, prob.n_alpha, prob.n_beta, prob.h, prob.eri,
                            prob.alpha, prob.beta, o)

    def poll(self, ticket):
        rc, info = tbsci_poll(self._srv, ticket)
        if rc == TBSCI_PENDING:
            return None
        d = info.as_dict()
        d["status"] = rc
        d.update(tbsci_request_times(self._srv, ticket))
        return d

    def stats(self):
        return tbsci_server_stats(self._srv)

    def close(self):
        if getattr(self, "_srv", None):
            tbsci_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- wrapper

class Context:
    """One TPB problem resident on a GPU."""

    def __init__(self, M, n_alpha, n_beta, h, eri, alpha, beta, device=0):
        self.M, self.n_alpha, self.n_beta = int(M), int(n_alpha), int(n_beta)
        self.device = int(device)
        self._ctx = tbsci_create(M, n_alpha, n_beta, h, eri, alpha, beta, device)
        self.l_alpha, self.l_beta, self.n_det = tbsci_dims(self._ctx)

    @classmethod
    def from_problem(cls, prob, device=0):
        return cls(prob.M, prob.n_alpha, prob.n_beta, prob.h, prob.eri, prob.alpha, prob.beta,
                   device)

    def close(self):
        if getattr(self, "_ctx", None):
            tbsci_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ctx

    def _dev(self):
        return torch.device("cuda", self.device)

    def set_dets(self, row_off=None, beta_idx=None):
        """Restrict to a TBSCI space (compact vectors afterwards); no
        arguments: back to the whole TPB space."""
        tbsci_set_dets(self._ctx, row_off, beta_idx)
        self.l_alpha, self.l_beta, self.n_det = tbsci_dims(self._ctx)
        self.compact = row_off is not None

    def set_symmetry(self, orb_irrep, target_irrep):
        """Keep the determinants of one total irrep (compact vectors afterwards)."""
        tbsci_set_symmetry(self._ctx, orb_irrep, target_irrep)
        self.l_alpha, self.l_beta, self.n_det = tbsci_dims(self._ctx)
        self.compact = True

    def get_dets(self):
        return tbsci_get_dets(self._ctx, self.l_alpha, self.n_det)

    def string_irreps(self, spin):
        return tbsci_string_irreps(self._ctx, spin, self.l_alpha if spin == 0 else self.l_beta)

    def string_weights(self, C, stream=None):
        """(w_alpha, w_beta) device FP64 tensors of a CI vector's string weights."""
        wa = torch.empty(self.l_alpha, dtype=torch.float64, device=self._dev())
        wb = torch.empty(self.l_beta, dtype=torch.float64, device=self._dev())
        _check(load().tbsci_string_weights(self._ctx, ctypes.c_void_p(C.data_ptr()),
                                           ctypes.c_void_p(wa.data_ptr()),
                                           ctypes.c_void_p(wb.data_ptr()), _stream(stream)))
        return wa, wb

    def select_strings(self, spin, w, delta, ref_string, stream=None):
        """Strings of one spin whose weight exceeds delta x the reference's."""
        l = self.l_alpha if spin == 0 else self.l_beta
        out = np.zeros(max(l, 1), dtype=np.uint64)
        n = ctypes.c_int64()
        _check(load().tbsci_select_strings(self._ctx, int(spin), ctypes.c_void_p(w.data_ptr()),
                                           float(delta), ctypes.c_uint64(int(ref_string)),
                                           _np_ptr(out), ctypes.byref(n), _stream(stream)))
        return out[:n.value].copy()

    def coef_histogram(self, C, log10_lo=-12.0, log10_hi=0.0, nbins=24, stream=None):
        counts = np.zeros(nbins, dtype=np.int64)
        _check(load().tbsci_coef_histogram(self._ctx, ctypes.c_void_p(C.data_ptr()),
                                           float(log10_lo), float(log10_hi), int(nbins),
                                           _np_ptr(counts), _stream(stream)))
        return counts

    def _shape(self):
        return (self.n_det,) if getattr(self, "compact", False) else (self.l_alpha, self.l_beta)

    def set_same_spin(self, method):
        """TBSCI_SAME_SPIN_AUTO, _CSR or _HOLE for the two same-spin terms."""
        tbsci_set_same_spin(self._ctx, method)

    def set_deterministic(self, enable=True):
        """Bitwise-reproducible sigma for this context (alone or batched)."""
        tbsci_set_deterministic(self._ctx, enable)

    def mfma_flops(self, precision=TBSCI_FP64):
        """Flops one launch of the opposite-spin kernel executes (padded tiles)."""
        return tbsci_timing_executed_flops(self._ctx, 2, precision)

    def sigma(self, C, out=None, precision=TBSCI_FP64, stream=None):
        dt = torch.float64 if precision == TBSCI_FP64 else torch.float32
        if C.dtype != dt or not C.is_cuda or not C.is_contiguous() or C.numel() != self.n_det:
            raise ValueError("C must be a contiguous device tensor of n_det elements of the "
                             "precision's type")
        if out is None:
            out = torch.empty(self._shape(), dtype=dt, device=C.device)
        elif out.dtype != dt or not out.is_contiguous() or out.numel() != self.n_det:
            raise ValueError("out must be a contiguous tensor like C")
        tbsci_sigma(self._ctx, C, out, precision, stream)
        return out

    def sigma_terms(self, C, terms, precision=TBSCI_FP64, stream=None):
        dt = torch.float64 if precision == TBSCI_FP64 else torch.float32
        if C.dtype != dt or not C.is_cuda or not C.is_contiguous() or C.numel() != self.n_det:
            raise ValueError("C must be a contiguous device tensor of n_det elements")
        out = torch.empty(self._shape(), dtype=dt, device=C.device)
        tbsci_sigma_terms(self._ctx, C, out, precision, terms, stream)
        return out

    def diag(self, stream=None):
        D = torch.empty(self._shape(), dtype=torch.float64, device=self._dev())
        tbsci_diag(self._ctx, D, stream)
        return D

    def davidson(self, n_max=8, max_iter=200, precision=TBSCI_FP64, tol_resid=1e-6,
                 tol_energy=0.0, fp32_switch_resid=1e-4, precond_floor=1e-8, guess=None,
                 want_vector=True, sector=0, storage=TBSCI_STORE_AUTO, subspace_guess=None,
                 stream=None):
        """subspace_guess: None, or the strings per spin of a subspace solved
        first for the start vector (0 for the library's default size)."""
        if guess is not None:
            kind, k = TBSCI_GUESS_USER, 0
        elif subspace_guess is not None:
            kind, k = TBSCI_GUESS_SUBSPACE, int(subspace_guess)
        else:
            kind, k = TBSCI_GUESS_DIAG, 0
        o = make_opts(n_max, max_iter, precision, tol_resid, tol_energy, fp32_switch_resid,
                      precond_floor, sector, storage, kind, k)
        if guess is not None and (guess.dtype != torch.float64 or guess.numel() != self.n_det):
            raise ValueError("guess must be an FP64 device tensor of n_det elements")
        X = torch.empty(self._shape(), dtype=torch.float64,
                        device=self._dev()) if want_vector else None
        rc, info = tbsci_davidson(self._ctx, o, guess, X, stream)
        d = info.as_dict()
        d["status"] = rc
        return d, X

    def string_index(self, spin):
        return tbsci_string_index(self._ctx, spin, self.l_alpha if spin == 0 else self.l_beta)

    def lookup(self, spin, queries, stream=None):
        out = torch.empty(queries.numel(), dtype=torch.int32, device=queries.device)
        tbsci_lookup(self._ctx, spin, queries, out, stream)
        return out

    def get_list(self, spin, kind):
        return tbsci_get_list(self._ctx, spin, kind, self.l_alpha if spin == 0 else self.l_beta)


def selection_loop(prob, deltas, ref_string=None, symmetry=None, device=0, **davidson_opts):
    """String-weight selection (Sec. III.B): solve the problem's space for a
    reference vector, weigh its strings, and for each relative threshold
    delta solve the TPB space of the strings kept (all of its determinants,
    or those of the target irrep when `symmetry` = (orbital irreps, target)).
    The reference string defaults to the lowest orbitals occupied.  Returns
    the reference solve and one dict per delta (strings kept per spin,
    determinants, energy, iterations).  Argument marshalling and bookkeeping
    only: the solves, weights and thresholds run in the library."""
    if ref_string is None:
        ref_string = sum(1 << q for q in range(prob.n_alpha))
        ref_b = sum(1 << q for q in range(prob.n_beta))
    else:
        ref_b = ref_string
    ctx = Context.from_problem(prob, device)
    if symmetry is not None:
        ctx.set_symmetry(*symmetry)
    ref, X = ctx.davidson(**davidson_opts)
    wa, wb = ctx.string_weights(X)
    out = []
    for d in deltas:
        a = ctx.select_strings(0, wa, d, ref_string)
        b = ctx.select_strings(1, wb, d, ref_b)
        if prob.n_alpha == prob.n_beta and np.array_equal(prob.alpha, prob.beta):
            # one list for both spins (the union, heaviest first by alpha weight)
            seen = set(map(int, a))
            a = np.concatenate([a, np.array([x for x in b if int(x) not in seen],
                                            dtype=np.uint64)])
            b = a.copy()
        sub = Context(prob.M, prob.n_alpha, prob.n_beta, prob.h, prob.eri, a, b, device)
        if symmetry is not None:
            sub.set_symmetry(*symmetry)
        info, _ = sub.davidson(want_vector=False, **davidson_opts)
        out.append(dict(delta=d, n_alpha_strings=len(a), n_beta_strings=len(b),
                        n_det=sub.n_det, energy=info["energy"], status=info["status"],
                        iters=info["iters"], sector=info["sector"],
                        time_s=info["t_total_s"]))
        sub.close()
    ctx.close()
    return ref, X, out


def sigma_batch(contexts, Cs, precision=TBSCI_FP64, stream=None):
    """sigma of several contexts in shared launches; returns new tensors."""
    dt = torch.float64 if precision == TBSCI_FP64 else torch.float32
    outs = []
    for c, C in zip(contexts, Cs):
        if C.dtype != dt or not C.is_cuda or not C.is_contiguous() or C.numel() != c.n_det:
            raise ValueError("each C must be a contiguous device tensor of its n_det elements")
        outs.append(torch.empty((c.l_alpha, c.l_beta), dtype=dt, device=C.device))
    tbsci_sigma_batch([c.handle for c in contexts], Cs, outs, precision, stream)
    return outs


def davidson_batch(contexts, stream=None, **opts):
    """Lowest eigenvalues of several contexts solved in lock step."""
    o = [make_opts(**opts) for _ in contexts]
    status, infos = tbsci_davidson_batch([c.handle for c in contexts], o, stream)
    out = []
    for st, inf in zip(status, infos):
        d = inf.as_dict()
        d["status"] = st
        out.append(d)
    return out
