"""Plain FP64 CPU reference (the oracle) for the TPB sigma build and solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code
with the HIP library: the heavy loops live in ``tbsci_oracle.c`` (compiled
here with gcc), the rest is numpy.

Contents, each following the paper (arXiv 2503.10335):

* ``string_index`` -- sorted keys plus caller positions; membership by a
  Python dict (Sec. II.C: membership of a candidate string in the selected
  set, by hashing or by sorted binary search).
* ``lists`` -- same-spin single and double excitation lists between selected
  strings, built by pair scan and explicit operator application
  (Sec. II.C: the single- and double-excitation link tables of the selected
  beta strings; Sec. III.C: one entry = target index, two orbital indices and
  a sign).
* ``same_spin_matrix`` -- the same-spin Hamiltonian between selected strings,
  each element a generic Slater-Condon element of a single-spin determinant
  (Sec. II.C, categories [2,0]/[0,2] and the one-spin parts of [1,0]/[0,1]).
* ``sigma`` / ``diag`` / ``dense_h`` -- sigma = P H P C over the TPB space
  (Sec. II.A, Eq. TPB_Det and the beta-fastest index map; Sec. II.C,
  Slater-Condon rule and Algorithm 1's six categories).
* ``set_dets`` / ``sigma_dets`` / ``dense_h_dets`` -- the same over a TBSCI
  space: per alpha string w only the beta strings of its index set I_w
  (Sec. II.A), with the membership of both the output and every
  contributing determinant tested (Algorithm 1; its [0,2] loop writes only
  the first test).
* ``davidson`` -- a plain Davidson eigensolver with collapse restart
  (Sec. II.B, Davidson matrix-vector products; Sec. III.C, restart with a
  bounded number of stored vectors).
* ``string_irreps`` / ``symmetry_layout`` / ``symmetry_dimension`` -- the
  irrep of a string (product over occupied orbitals) and the determinants of
  one total irrep, as a TBSCI layout and as a count (Sec. II.A: only the
  symmetry-allowed determinants are kept, each I_w an interval of irrep-sorted
  beta strings; Table of the benchmark systems: their FCI dimensions).
* ``string_weights`` / ``select_by_weight`` / ``coef_histogram`` -- the
  weight of each string in a CI vector, the strings above a relative
  threshold of the Hartree-Fock string's weight, and the histogram of the
  coefficient magnitudes (Sec. III.B, the bitstring screening of SCI
  wavefunctions).
* ``lowest_by_flip_sector`` -- with identical alpha and beta lists, the
  lowest eigenvalue of P H P among symmetric and among antisymmetric CI
  matrices, and the lower of the two (the lowest eigenpair of Sec. II.B's
  diagonalisation, split by the alpha/beta exchange symmetry of H).
* ``fock_hamiltonian`` / ``fock_spin_squared`` -- brute-force Jordan-Wigner
  Fock-space Hamiltonian and total spin for tiny M, from the second-quantised
  operators, used only to pin the above.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tbsci_oracle.c")
_LIB = os.path.join(_HERE, "libtbsci_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64 = ctypes.c_int64
            lib.orc_space_new.restype = P
            lib.orc_space_new.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, i64, P,
                                          i64, ctypes.POINTER(ctypes.c_int)]
            lib.orc_space_free.argtypes = [P]
            lib.orc_sigma.argtypes = [P, P, P, P, P, P, i64, ctypes.c_int]
            lib.orc_sigma_rowmap.restype = ctypes.c_int
            lib.orc_sigma_rowmap.argtypes = [P, P, P, P, P, P, P, i64, ctypes.c_int]
            lib.orc_element.restype = ctypes.c_double
            lib.orc_element.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64]
            lib.orc_dense.argtypes = [P, P, P, P, ctypes.c_int]
            lib.orc_diag.argtypes = [P, P, P, P, P, i64, ctypes.c_int]
            lib.orc_lists.restype = i64
            lib.orc_lists.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, P, i64, P, P, ctypes.c_int]
            lib.orc_count_singles.restype = i64
            lib.orc_count_singles.argtypes = [P, i64, ctypes.c_int, ctypes.c_int]
            lib.orc_set_dets.restype = ctypes.c_int
            lib.orc_set_dets.argtypes = [P, P, P]
            lib.orc_sigma_dets.argtypes = [P, P, P, P, P, P, P, P, i64, ctypes.c_int]
            lib.orc_dense_dets.argtypes = [P, P, P, P, P, P, ctypes.c_int]
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class Space:
    """Hash-indexed TPB space with integrals; owns contiguous copies."""

    def __init__(self, M, n_alpha, n_beta, h, eri, alpha, beta):
        lib = _load()
        self.M, self.na, self.nb = int(M), int(n_alpha), int(n_beta)
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.alpha = np.ascontiguousarray(alpha, dtype=np.uint64)
        self.beta = np.ascontiguousarray(beta, dtype=np.uint64)
        st = ctypes.c_int(0)
        self._p = lib.orc_space_new(self.M, self.na, self.nb, _ptr(self.h), _ptr(self.eri),
                                    _ptr(self.alpha), len(self.alpha), _ptr(self.beta),
                                    len(self.beta), ctypes.byref(st))
        if st.value != 0:
            lib.orc_space_free(self._p)
            self._p = None
            raise ValueError("duplicate strings in a selected list")
        self.la, self.lb = len(self.alpha), len(self.beta)

    @classmethod
    def of(cls, prob):
        return cls(prob.M, prob.n_alpha, prob.n_beta, prob.h, prob.eri, prob.alpha, prob.beta)

    def __del__(self):
        if getattr(self, "_p", None):
            _load().orc_space_free(self._p)
            self._p = None

    @property
    def n_det(self):
        return self.la * self.lb

    def sigma(self, C, rows=None, nthreads=0):
        """sigma = P H P C; C is [la][lb] (or flat); rows selects output alpha rows."""
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(self.la, self.lb))
        if rows is None:
            out = np.empty((self.la, self.lb))
            _load().orc_sigma(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(C), _ptr(out),
                              None, 0, nthreads)
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            out = np.empty((len(rows), self.lb))
            _load().orc_sigma(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(C), _ptr(out),
                              _ptr(rows), len(rows), nthreads)
        return out

    def sigma_rows_from(self, rows, csub, c_rows, nthreads=0):
        """sigma on output rows ``rows`` with C supplied only on rows ``c_rows``
        (csub[i] = C[c_rows[i]]); every row linked to an output row must be
        supplied, else ValueError."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        csub = np.ascontiguousarray(csub, dtype=np.float64).reshape(len(c_rows), self.lb)
        slot = np.full(self.la, -1, dtype=np.int64)
        slot[np.asarray(c_rows, dtype=np.int64)] = np.arange(len(c_rows))
        out = np.empty((len(rows), self.lb))
        rc = _load().orc_sigma_rowmap(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(csub),
                                      _ptr(slot), _ptr(out), _ptr(rows), len(rows), nthreads)
        if rc != 0:
            raise ValueError("a needed row of C was not supplied")
        return out

    def linked_rows(self, rows):
        """Alpha rows reachable from ``rows`` by zero, one or two excitations."""
        need = set(int(r) for r in rows)
        for kind in (1, 2):
            ptr, ent = lists(self.alpha, self.M, kind, rows=rows)
            need.update(int(j) for j in ent[:, 0])
        return np.array(sorted(need), dtype=np.int64)

    # ------------------------------------------ determinant-level pruning

    def set_dets(self, row_off, beta_idx):
        """Keep only some determinants (Sec. II.A, the TBSCI space): alpha
        row w keeps the beta strings beta_idx[row_off[w]:row_off[w+1]] (caller
        indices).  Compact vectors list the kept determinants row by row in
        that order."""
        self.row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        self.beta_idx = np.ascontiguousarray(beta_idx, dtype=np.int32)
        if len(self.row_off) != self.la + 1:
            raise ValueError("row_off needs l_alpha + 1 entries")
        if _load().orc_set_dets(self._p, _ptr(self.row_off), _ptr(self.beta_idx)) != 0:
            raise ValueError("malformed determinant layout")

    @property
    def n_dets(self):
        return int(self.row_off[-1])

    def dets_index(self):
        """Position in the [l_alpha][l_beta] TPB layout of every kept
        determinant, in compact order."""
        w = np.repeat(np.arange(self.la, dtype=np.int64), np.diff(self.row_off))
        return w * self.lb + self.beta_idx.astype(np.int64)

    def sigma_dets(self, c, rows=None, nthreads=0):
        """sigma_K = sum_{L kept} H_KL c_L for every kept K (compact vectors);
        with rows, only the segments of those alpha rows, concatenated."""
        c = np.ascontiguousarray(c, dtype=np.float64).ravel()
        if c.size != self.n_dets:
            raise ValueError("c must have one entry per kept determinant")
        if rows is None:
            out = np.empty(self.n_dets)
            r, nr = None, 0
        else:
            r = np.ascontiguousarray(rows, dtype=np.int64)
            nr = len(r)
            out = np.empty(int(np.sum(self.row_off[r + 1] - self.row_off[r])))
        _load().orc_sigma_dets(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(self.row_off),
                               _ptr(self.beta_idx), _ptr(c), _ptr(out), _ptr(r), nr, nthreads)
        return out

    def dense_h_dets(self, nthreads=0):
        """Dense P H P over the kept determinants, element by element with the
        generic Slater-Condon rule (small spaces)."""
        n = self.n_dets
        if n > 6000:
            raise ValueError("dense H only for small spaces")
        H = np.empty((n, n))
        _load().orc_dense_dets(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(self.row_off),
                               _ptr(self.beta_idx), _ptr(H), nthreads)
        return H

    def diag(self, rows=None, nthreads=0):
        if rows is None:
            out = np.empty((self.la, self.lb))
            _load().orc_diag(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(out), None, 0,
                             nthreads)
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            out = np.empty((len(rows), self.lb))
            _load().orc_diag(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(out), _ptr(rows),
                             len(rows), nthreads)
        return out

    def element(self, Ia, Ib, Ja, Jb):
        return _load().orc_element(self._p, int(Ia), int(Ib), int(Ja), int(Jb))

    def dense_h(self, nthreads=0):
        n = self.n_det
        if n > 6000:
            raise ValueError("dense H only for small spaces")
        H = np.empty((n, n))
        _load().orc_dense(self._p, _ptr(self.alpha), _ptr(self.beta), _ptr(H), nthreads)
        return H

    def same_spin_matrix(self, spin):
        """Dense same-spin Hamiltonian A_spin between selected strings.

        Element (I, J) is <I|H|J> for a determinant holding electrons of one
        spin only (the other spin string empty), i.e. the one-spin part of H.
        """
        strs = self.alpha if spin == 0 else self.beta
        n = len(strs)
        A = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                if bin(int(strs[i]) ^ int(strs[j])).count("1") > 4:
                    continue
                if spin == 0:
                    A[i, j] = self.element(strs[i], 0, strs[j], 0)
                else:
                    A[i, j] = self.element(0, strs[i], 0, strs[j])
        return A


# ------------------------------------------------------------------ indices

def string_index(strings):
    """(keys ascending uint64, pos int32 caller index of each sorted key)."""
    s = np.asarray(strings, dtype=np.uint64)
    order = sorted(range(len(s)), key=lambda i: int(s[i]))
    return s[order].copy(), np.array(order, dtype=np.int32)


def lookup(strings, queries):
    """Caller index of each query string, or -1 (dict membership)."""
    d = {int(v): i for i, v in enumerate(np.asarray(strings, dtype=np.uint64))}
    return np.array([d.get(int(q), -1) for q in np.asarray(queries, dtype=np.uint64)],
                    dtype=np.int32)


def lists(strings, M, kind, rows=None, count_only=False):
    """Canonical same-spin excitation lists by pair scan.

    kind 1 (singles): per row I, entries (j, p, q, sign), I = a+_p a_q J,
    ordered by (p, q).  kind 2 (doubles): entries (j, i, jj, a, b, sign),
    I = a+_i a+_jj a_b a_a J, ordered by (i, jj, a, b).
    Returns (row_ptr int64[n+1], entries int32[total, 6]) or total if count_only.
    """
    lib = _load()
    s = np.ascontiguousarray(strings, dtype=np.uint64)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = len(s) if r is None else len(r)
    ptr = np.zeros(nr + 1, dtype=np.int64)
    tot = lib.orc_lists(_ptr(s), len(s), int(M), int(kind), _ptr(r), 0 if r is None else len(r),
                        _ptr(ptr), None, 1)
    if count_only:
        return tot
    ent = np.zeros((max(tot, 1), 6), dtype=np.int32)
    lib.orc_lists(_ptr(s), len(s), int(M), int(kind), _ptr(r), 0 if r is None else len(r),
                  _ptr(ptr), _ptr(ent), 0)
    return ptr, ent[:tot]


def singles_with_diag(strings, M, rows=None):
    """Singles lists with the occupation entries (p = q, p in I, j = I, sign
    +1) merged in, ordered by (p, q): the full set of E_pq links per row."""
    ptr, ent = lists(strings, M, 1, rows)
    s = np.asarray(strings, dtype=np.uint64)
    idx = range(len(s)) if rows is None else rows
    out_ptr = [0]
    out = []
    for r, ii in enumerate(idx):
        I = int(s[ii])
        row = [tuple(e) for e in ent[ptr[r]:ptr[r + 1]]]
        row += [(int(ii), p, p, 0, 0, 1) for p in range(M) if (I >> p) & 1]
        row.sort(key=lambda e: (e[1], e[2]))
        out.extend(row)
        out_ptr.append(len(out))
    return np.array(out_ptr, dtype=np.int64), np.array(out, dtype=np.int32).reshape(-1, 6)


def count_singles(strings, M, nthreads=0):
    """Number of single-excitation links inside a string set (hash membership)."""
    s = np.ascontiguousarray(strings, dtype=np.uint64)
    return int(_load().orc_count_singles(_ptr(s), len(s), int(M), nthreads))


# ------------------------------------------------------------------ solvers

def lowest_eigpair_dense(H):
    w, v = np.linalg.eigh(H)
    x = v[:, 0].copy()
    k = int(np.argmax(np.abs(x)))
    if x[k] < 0:
        x = -x
    return float(w[0]), x


def davidson(apply_h, diag, tol=1e-8, n_max=8, max_iter=500, guess=None, floor=1e-8):
    """Plain Davidson for the lowest eigenpair of a real symmetric operator.

    Guess: unit vector on the smallest diagonal element (first on ties).
    Preconditioner t = r / (theta - H_KK), denominators below ``floor`` in
    magnitude replaced by +-floor keeping the sign.  The correction is
    normalised, orthogonalised twice (Gram-Schmidt); if less than 1e-10 of
    its norm survives, the solve stops (no new direction).
    Restart: when the basis reaches n_max vectors it collapses to the Ritz
    vector.  Returns dict(energy, x, resid, iters, converged).
    """
    diag = np.asarray(diag, dtype=np.float64).ravel()
    n = diag.size
    if guess is None:
        x0 = np.zeros(n)
        x0[int(np.argmin(diag))] = 1.0
    else:
        x0 = np.asarray(guess, dtype=np.float64).ravel().copy()
        x0 /= np.linalg.norm(x0)
    V = [x0]
    W = [np.asarray(apply_h(x0), dtype=np.float64).ravel()]
    theta, x, rn = None, x0, np.inf
    for it in range(1, max_iter + 1):
        k = len(V)
        G = np.array([[V[i] @ W[j] for j in range(k)] for i in range(k)])
        G = 0.5 * (G + G.T)
        w, y = np.linalg.eigh(G)
        theta = float(w[0])
        yv = y[:, 0]
        x = sum(yv[i] * V[i] for i in range(k))
        Wx = sum(yv[i] * W[i] for i in range(k))
        r = Wx - theta * x
        rn = float(np.linalg.norm(r))
        if rn <= tol:
            return dict(energy=theta, x=_fix_sign(x), resid=rn, iters=it, converged=True)
        if k >= n_max:
            nx = np.linalg.norm(x)
            V, W = [x / nx], [Wx / nx]
        den = theta - diag
        small = np.abs(den) < floor
        den[small] = np.where(den[small] < 0, -floor, floor)
        t = r / den
        t /= np.linalg.norm(t)  # the stagnation test below is relative to |t|
        for _ in range(2):
            for v in V:
                t = t - (v @ t) * v
        nt = np.linalg.norm(t)
        if nt < 1e-10:
            return dict(energy=theta, x=_fix_sign(x), resid=rn, iters=it, converged=False)
        t /= nt
        V.append(t)
        W.append(np.asarray(apply_h(t), dtype=np.float64).ravel())
    return dict(energy=theta, x=_fix_sign(x), resid=rn, iters=max_iter, converged=False)


def _fix_sign(x):
    k = int(np.argmax(np.abs(x)))
    return -x if x[k] < 0 else x


# ------------------------------------------------- point-group symmetry

def string_irreps(strings, irreps):
    """Irrep of each string: the product (XOR of the labels) of the irreps
    of its occupied orbitals."""
    out = []
    for s in np.asarray(strings, dtype=np.uint64):
        g, v, p = 0, int(s), 0
        while v:
            if v & 1:
                g ^= int(irreps[p])
            v >>= 1
            p += 1
        out.append(g)
    return np.array(out, dtype=np.int32)


def symmetry_layout(alpha, beta, irreps, target):
    """The determinants of total irrep `target` as a TBSCI layout (Sec. II.A:
    the symmetry-allowed determinants, I_w = the beta strings whose irrep
    times that of alpha string w is the target): (row_off, beta_idx)."""
    ga, gb = string_irreps(alpha, irreps), string_irreps(beta, irreps)
    rows = [np.nonzero((gb ^ g) == target)[0] for g in ga]
    row_off = np.zeros(len(ga) + 1, dtype=np.int64)
    row_off[1:] = np.cumsum([len(r) for r in rows])
    beta_idx = (np.concatenate(rows) if rows else np.zeros(0)).astype(np.int32)
    return row_off, beta_idx


def symmetry_dimension(orbital_counts, n_alpha, n_beta, target, order=8):
    """Number of determinants of total irrep `target` with n_alpha and n_beta
    electrons in orbitals whose irreps are given as {label: count}: strings
    counted per irrep by adding one orbital at a time."""
    def per_irrep(n):
        c = [[0] * order for _ in range(n + 1)]
        c[0][0] = 1
        for g, k in orbital_counts.items():
            for _ in range(k):
                new = [row[:] for row in c]
                for j in range(n):
                    for x in range(order):
                        if c[j][x]:
                            new[j + 1][x ^ g] += c[j][x]
                c = new
        return c[n]
    a, b = per_irrep(n_alpha), per_irrep(n_beta)
    return sum(a[g] * b[g ^ target] for g in range(order))


# ------------------------------------------------ string-weight selection

def string_weights(C):
    """Weights of the alpha and beta strings of a CI matrix C [l_alpha][l_beta]:
    the sum of the squared coefficients of the determinants containing each
    string (Sec. III.B)."""
    C = np.asarray(C, dtype=np.float64)
    wa = np.array([sum(float(x) * float(x) for x in row) for row in C])
    wb = np.array([sum(float(x) * float(x) for x in col) for col in C.T])
    return wa, wb


def select_by_weight(strings, w, delta, ref_string):
    """The strings whose weight exceeds delta times the weight of the
    reference (Hartree-Fock) string, ranked heaviest first (ties: smaller
    string first); the reference string is always kept (Sec. III.B)."""
    strings = [int(x) for x in np.asarray(strings, dtype=np.uint64)]
    ref = strings.index(int(ref_string))
    thresh = delta * float(w[ref])
    keep = [i for i in range(len(strings)) if float(w[i]) > thresh or i == ref]
    keep.sort(key=lambda i: (-float(w[i]), strings[i]))
    return np.array([strings[i] for i in keep], dtype=np.uint64)


def coef_histogram(c, log10_lo, log10_hi, nbins):
    """Counts of the coefficients by log10 |c| in nbins equal bins over
    [log10_lo, log10_hi); smaller magnitudes (and zeros) in the first bin,
    larger in the last."""
    counts = [0] * nbins
    for x in np.asarray(c, dtype=np.float64).ravel():
        a = abs(float(x))
        b = 0
        if a > 0.0:
            t = (np.log10(a) - log10_lo) * nbins / (log10_hi - log10_lo)
            b = 0 if t < 0 else (nbins - 1 if t >= nbins else int(t))
        counts[b] += 1
    return np.array(counts, dtype=np.int64)


# ------------------------------------------------------ spin-flip sectors

def flip_sector_basis(l, tau):
    """Orthonormal basis (columns) of the CI matrices C [l][l] with
    C^T = tau C, as vectors of length l*l (row-major).  tau = +1: the unit
    matrices on the diagonal and (e_ij + e_ji)/sqrt 2 for i < j; tau = -1:
    (e_ij - e_ji)/sqrt 2 for i < j."""
    cols = []
    for i in range(l):
        for j in range(i, l):
            if i == j and tau < 0:
                continue
            v = np.zeros(l * l)
            if i == j:
                v[i * l + i] = 1.0
            else:
                v[i * l + j] = 1.0 / np.sqrt(2.0)
                v[j * l + i] = tau / np.sqrt(2.0)
            cols.append(v)
    return np.array(cols).T.reshape(l * l, len(cols))


def lowest_by_flip_sector(space, H=None):
    """Lowest eigenvalue of P H P in each spin-flip sector and overall.

    With the same strings in the same order for both spins (N_alpha =
    N_beta), the spin-orbital H commutes with the exchange of the alpha and
    beta strings of every determinant, so its eigenvectors can be taken as
    CI matrices that are symmetric (C^T = C) or antisymmetric (C^T = -C).
    Returns dict(sym=E+, anti=E- (None when l = 1), lowest=min, sector=+1 or
    -1 of the lowest); for different lists only 'lowest' (sector 0).
    Dense, for small spaces only."""
    if H is None:
        H = space.dense_h()
    e_all = float(np.linalg.eigvalsh(H)[0])
    same = (space.na == space.nb and space.la == space.lb
            and np.array_equal(space.alpha, space.beta))
    if not same:
        return dict(sym=None, anti=None, lowest=e_all, sector=0)
    l = space.la
    out = {}
    for tau, key in ((1, "sym"), (-1, "anti")):
        Q = flip_sector_basis(l, tau)
        out[key] = float(np.linalg.eigvalsh(Q.T @ H @ Q)[0]) if Q.shape[1] else None
    lo = out["sym"] if out["anti"] is None or out["sym"] <= out["anti"] else out["anti"]
    out["lowest"] = lo
    out["sector"] = 1 if lo == out["sym"] else -1
    out["lowest_all"] = e_all
    return out


# ------------------------------------------------------------ brute force

def fock_hamiltonian(M, h, eri):
    """Full Fock-space H (dimension 4^M) from Jordan-Wigner operators.

    Spin orbital index: alpha orbital p -> p, beta orbital p -> M+p.  The basis
    state with occupation bits n (bit X = spin orbital X) is the product of
    creators in ascending spin-orbital order acting on the vacuum, so
    a+_X |n> = (-1)^{sum_{Y<X} n_Y} |n + e_X>.
    H = sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs.
    Returns a scipy.sparse CSR matrix.
    """
    import scipy.sparse as sp

    K = 2 * M
    dim = 1 << K
    ann = []
    for X in range(K):
        rows, cols, vals = [], [], []
        for n in range(dim):
            if (n >> X) & 1:
                sign = -1.0 if bin(n & ((1 << X) - 1)).count("1") & 1 else 1.0
                rows.append(n ^ (1 << X))
                cols.append(n)
                vals.append(sign)
        ann.append(sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim)))
    cre = [a.T.tocsr() for a in ann]
    H = sp.csr_matrix((dim, dim))
    so = lambda p, s: p + s * M
    for s in range(2):
        for p in range(M):
            for q in range(M):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * (cre[so(p, s)] @ ann[so(q, s)])
    # two-body: precompute pair operators a+_ps a_qs for reuse
    for s in range(2):
        for t in range(2):
            for p in range(M):
                for q in range(M):
                    Lp = cre[so(p, s)]
                    for r in range(M):
                        for u in range(M):
                            v = eri[p, q, r, u]
                            if v == 0.0:
                                continue
                            H = H + (0.5 * v) * (Lp @ cre[so(r, t)] @ ann[so(u, t)] @ ann[so(q, s)])
    return H.tocsr()


def fock_spin_squared(M):
    """Total spin S^2 on the Fock space of M spatial orbitals (dimension
    4^M, same basis and Jordan-Wigner signs as fock_hamiltonian), from its
    textbook form S^2 = S_- S_+ + S_z (S_z + 1) with
    S_+ = sum_p a+_{p alpha} a_{p beta}, S_- = S_+^T and
    S_z = (1/2) sum_p (n_{p alpha} - n_{p beta}).  Returns a dense array."""
    K = 2 * M
    dim = 1 << K
    ann = []
    for X in range(K):
        A = np.zeros((dim, dim))
        for n in range(dim):
            if (n >> X) & 1:
                A[n ^ (1 << X), n] = -1.0 if bin(n & ((1 << X) - 1)).count("1") & 1 else 1.0
        ann.append(A)
    Sp = sum(ann[p].T @ ann[M + p] for p in range(M))
    Sz = 0.5 * sum(ann[p].T @ ann[p] - ann[M + p].T @ ann[M + p] for p in range(M))
    return Sp.T @ Sp + Sz @ (Sz + np.eye(dim))


def fock_index(alpha_str, beta_str, M):
    """Fock basis index of the determinant (alpha bits low, beta bits high)."""
    return int(alpha_str) | (int(beta_str) << M)
