"""Seeded synthetic inputs for TPB sigma builds and ground-state solves.

This module only draws inputs: one-electron integrals h, two-electron
integrals (pq|rs) in chemists' notation, and selected alpha/beta string
lists.  It holds none of the Hamiltonian arithmetic, so both the HIP path
and the CPU reference can be driven from the same inputs.

Recipe (the paper's molecular FCIDUMP files are not available, so these
stand in for them):

* h_pp = -1 + 2p/M (p is 0-based); off-diagonal h_pq ~ N(0, 0.05), mirrored.
* (pq|rs) = sum_{L<M} B^L_pq B^L_rs with B^L symmetric, entries ~ N(0, 0.15).
  This gives the 8-fold permutational symmetry of real orbitals and a
  positive semidefinite supermatrix.
* Draw order from ``numpy.random.default_rng(seed)``: the strict upper
  triangle of h row-major, then for L = 0..M-1 the upper triangle of B^L
  including the diagonal, row-major.
* String selection: every M-bit string with N set bits, enumerated in
  ascending integer order, gets one N(0, 0.1) noise draw; the score is the
  sum of occupied h_pp plus the noise; the ``n`` lowest scores are kept
  (ties broken by the smaller integer).  The kept list is returned in rank
  order, which is not sorted by integer value.

Strings are uint64 with bit p set when spatial orbital p is occupied.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np


def integrals(M: int, seed: int):
    """Return (h[M,M], eri[M,M,M,M]) float64 from the seeded recipe."""
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    for p in range(M):
        h[p, p] = -1.0 + 2.0 * p / M
    iu = np.triu_indices(M, 1)
    off = rng.normal(0.0, 0.05, size=len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    iu0 = np.triu_indices(M, 0)
    B = np.zeros((M, M, M))
    for L in range(M):
        v = rng.normal(0.0, 0.15, size=len(iu0[0]))
        B[L][iu0] = v
        B[L][(iu0[1], iu0[0])] = v
    eri = np.einsum("lpq,lrs->pqrs", B, B, optimize=True)
    # enforce exact 8-fold symmetry bitwise (einsum rounding can differ by 1 ulp)
    eri = (eri + eri.transpose(1, 0, 2, 3)) * 0.5
    eri = (eri + eri.transpose(0, 1, 3, 2)) * 0.5
    eri = (eri + eri.transpose(2, 3, 0, 1)) * 0.5
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


def all_strings(M: int, N: int) -> np.ndarray:
    """Every M-bit string with N set bits, ascending integer order."""
    if N == 0:
        return np.zeros(1, dtype=np.uint64)
    out = []
    for occ in itertools.combinations(range(M), N):
        v = 0
        for p in occ:
            v |= 1 << p
        out.append(v)
    out.sort()
    return np.array(out, dtype=np.uint64)


def _occ_matrix(strings: np.ndarray, M: int) -> np.ndarray:
    bits = np.arange(M, dtype=np.uint64)
    return ((strings[:, None] >> bits[None, :]) & np.uint64(1)).astype(np.float64)


def select_strings(M: int, N: int, n_keep: int, h: np.ndarray, seed: int,
                   noise_std: float = 0.1) -> np.ndarray:
    """Keep the n_keep lowest-scoring strings (rank order)."""
    cand = all_strings(M, N)
    rng = np.random.default_rng(seed)
    noise = rng.normal(0.0, noise_std, size=len(cand))
    score = _occ_matrix(cand, M) @ np.diag(h) + noise
    order = np.lexsort((cand, score))  # primary: score, ties: smaller integer
    n_keep = min(n_keep, len(cand))
    return np.ascontiguousarray(cand[order[:n_keep]])


@dataclass
class Problem:
    """One TPB eigenproblem: integrals plus selected alpha/beta strings."""
    name: str
    M: int
    n_alpha: int
    n_beta: int
    h: np.ndarray
    eri: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_det(self) -> int:
        return len(self.alpha) * len(self.beta)


def make_problem(name: str, M: int, N: int, n_keep: int | None, int_seed: int,
                 sel_seed: int | None = None, independent_beta: bool = False) -> Problem:
    """Closed-shell-count problem (N_alpha = N_beta = N).

    n_keep None keeps every string (FCI limit of the TPB space, strings in
    ascending integer order).  With ``independent_beta`` the beta list is
    drawn with its own noise (seed sel_seed + 1) instead of reusing alpha's.
    """
    h, eri = integrals(M, int_seed)
    if n_keep is None or n_keep >= math.comb(M, N):
        a = all_strings(M, N)
        b = a.copy()
    else:
        a = select_strings(M, N, n_keep, h, sel_seed)
        b = select_strings(M, N, n_keep, h, sel_seed + 1) if independent_beta else a.copy()
    return Problem(name, M, N, N, h, eri, a, b,
                   dict(int_seed=int_seed, sel_seed=sel_seed, n_keep=n_keep))


# ------------------------------------------------------ point-group symmetry
#
# Irreducible representations of the abelian point groups as integer labels
# whose product is their XOR (D2h: Ag 0, B1g 1, B2g 2, B3g 3, Au 4, B1u 5,
# B2u 6, B3u 7; C2v: A1 0, A2 1, B1 2, B2 3).

D2H = {"Ag": 0, "B1g": 1, "B2g": 2, "B3g": 3, "Au": 4, "B1u": 5, "B2u": 6, "B3u": 7}
C2V = {"A1": 0, "A2": 1, "B1": 2, "B2": 3}


def orbital_irreps(dist: dict, seed: int) -> np.ndarray:
    """Irrep label of each orbital: `dist` maps label -> number of orbitals;
    the labels are interleaved over the orbital index by a seeded shuffle (as
    energy-ordered molecular orbitals interleave their irreps)."""
    labels = np.array([g for g, k in sorted(dist.items()) for _ in range(k)], dtype=np.int32)
    return labels[np.random.default_rng(seed).permutation(len(labels))]


def integrals_sym(M: int, seed: int, irreps: np.ndarray, order: int = 8):
    """The integral recipe of ``integrals`` (same draws), made totally
    symmetric in the point group: h_pq = 0 unless orbitals p and q share an
    irrep, and B^L carries the irrep L mod `order`, keeping B^L_pq only where
    irrep(p) x irrep(q) is that irrep, so (pq|rs) = sum_L B^L_pq B^L_rs
    vanishes unless irrep(p) x irrep(q) x irrep(r) x irrep(s) is totally
    symmetric, and stays 8-fold symmetric and positive semidefinite."""
    irreps = np.asarray(irreps, dtype=np.int64)
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    for p in range(M):
        h[p, p] = -1.0 + 2.0 * p / M
    iu = np.triu_indices(M, 1)
    off = rng.normal(0.0, 0.05, size=len(iu[0]))
    off[irreps[iu[0]] != irreps[iu[1]]] = 0.0
    h[iu] = off
    h[(iu[1], iu[0])] = off
    iu0 = np.triu_indices(M, 0)
    B = np.zeros((M, M, M))
    for L in range(M):
        v = rng.normal(0.0, 0.15, size=len(iu0[0]))
        v[(irreps[iu0[0]] ^ irreps[iu0[1]]) != (L % order)] = 0.0
        B[L][iu0] = v
        B[L][(iu0[1], iu0[0])] = v
    eri = np.einsum("lpq,lrs->pqrs", B, B, optimize=True)
    eri = (eri + eri.transpose(1, 0, 2, 3)) * 0.5
    eri = (eri + eri.transpose(0, 1, 3, 2)) * 0.5
    eri = (eri + eri.transpose(2, 3, 0, 1)) * 0.5
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


def make_sym_problem(name: str, M: int, N: int, dist: dict, target: int, int_seed: int,
                     irrep_seed: int, n_keep: int | None = None, sel_seed: int | None = None,
                     order: int = 8) -> Problem:
    """A point-group-symmetric problem: orbital irreps from `dist`,
    symmetric integrals, every string (or the n_keep lowest-ranked ones), the
    same list for both spins sorted by (string irrep, integer value) so that
    the beta strings of each irrep are contiguous.  meta holds the orbital
    irreps and the target irrep of the determinants."""
    irreps = orbital_irreps(dist, irrep_seed)
    h, eri = integrals_sym(M, int_seed, irreps, order)
    s = all_strings(M, N) if n_keep is None else select_strings(M, N, n_keep, h, sel_seed)
    g = np.zeros(len(s), dtype=np.int64)
    for p in range(M):
        g ^= ((s >> np.uint64(p)) & np.uint64(1)).astype(np.int64) * int(irreps[p])
    s = np.ascontiguousarray(s[np.lexsort((s, g))])
    return Problem(name, M, N, N, h, eri, s, s.copy(),
                   dict(int_seed=int_seed, irreps=irreps, target=int(target), order=order,
                        n_keep=n_keep, sel_seed=sel_seed))


# The five workloads: FCI-limit M=8; selected M=16 (3,000 x 3,000);
# selected M=20 (20,000 x 20,000); FCI M=18 (48,620 x 48,620); serving mix.
CONFIGS = {
    "fci_m8": dict(M=8, N=4, n_keep=None, int_seed=1001),
    "sel_m16": dict(M=16, N=8, n_keep=3000, int_seed=1002, sel_seed=2002),
    "sel_m20": dict(M=20, N=10, n_keep=20000, int_seed=1003, sel_seed=2003),
    "fci_m18": dict(M=18, N=9, n_keep=None, int_seed=1004),
}


# A point-group-symmetric complete space: M = 14 orbitals with a D2h irrep
# distribution shaped like a diatomic's (Ag and B1u largest), N = 7 per spin,
# determinants of total irrep Ag (about 1/8 of the 3432 x 3432 TPB space).
SYM_CONFIGS = {
    "sym_m14": dict(M=14, N=7, dist={0: 3, 5: 3, 2: 2, 7: 2, 3: 1, 6: 1, 1: 1, 4: 1},
                    target=0, int_seed=1005, irrep_seed=3005),
}


def config(name: str) -> Problem:
    if name in SYM_CONFIGS:
        c = dict(SYM_CONFIGS[name])
        return make_sym_problem(name, c.pop("M"), c.pop("N"), c.pop("dist"), c.pop("target"),
                                **c)
    c = dict(CONFIGS[name])
    return make_problem(name, c.pop("M"), c.pop("N"), c.pop("n_keep"), **c)


def random_selection(M: int, na: int, nb: int, la: int, lb: int, seed: int,
                     int_seed: int | None = None) -> Problem:
    """Uniformly random (non energy-ranked) selections, for small tests."""
    rng = np.random.default_rng(seed)
    h, eri = integrals(M, seed if int_seed is None else int_seed)
    A = all_strings(M, na)
    B = all_strings(M, nb)
    a = A[rng.permutation(len(A))[:min(la, len(A))]]
    b = B[rng.permutation(len(B))[:min(lb, len(B))]]
    return Problem(f"rand_m{M}", M, na, nb, h, eri, np.ascontiguousarray(a),
                   np.ascontiguousarray(b), dict(seed=seed))


def dets_random(la: int, lb: int, keep: float, seed: int):
    """A ragged determinant layout: each (alpha row w, beta string u) kept
    with probability `keep` (seeded), so rows differ in length and some may be
    empty.  Returns (row_off int64[la+1], beta_idx int32, ascending in a row)."""
    rng = np.random.default_rng(seed)
    m = rng.random((la, lb)) < keep
    row_off = np.zeros(la + 1, dtype=np.int64)
    row_off[1:] = np.cumsum(m.sum(axis=1))
    beta_idx = np.nonzero(m)[1].astype(np.int32)
    return row_off, beta_idx


def dets_rank_sum(la: int, lb: int, frac: float):
    """Determinant layout that pairs important strings with important ones:
    with strings in rank order, (w, u) is kept when w / la + u / lb <= t, t
    chosen so that about `frac` of the TPB space is kept (a staircase of
    contiguous intervals; the structure of a weight-screened product space)."""
    t = float(np.sqrt(2.0 * frac)) if frac <= 0.5 else 2.0 - float(np.sqrt(2.0 * (1.0 - frac)))
    w = np.arange(la) / la
    n = np.clip(np.floor((t - w) * lb) + 1, 0, lb).astype(np.int64)
    row_off = np.zeros(la + 1, dtype=np.int64)
    row_off[1:] = np.cumsum(n)
    beta_idx = np.concatenate([np.arange(k, dtype=np.int32) for k in n]) if la else \
        np.zeros(0, dtype=np.int32)
    return row_off, beta_idx


def random_vector(n_alpha_rows: int, n_beta_cols: int, seed: int = 7) -> np.ndarray:
    """N(0,1) CI matrix [l_alpha][l_beta], normalised to unit 2-norm."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n_alpha_rows, n_beta_cols))
    C /= np.linalg.norm(C)
    return C


def random_vector_device(n_alpha_rows: int, n_beta_cols: int, seed: int = 7,
                         device="cuda:0", dtype=None):
    """N(0,1) CI matrix [l_alpha][l_beta] drawn on the device by torch's
    generator of that device (seeded), normalised to unit 2-norm: the input
    of the full-size sigma timings, where a host draw and copy of tens of
    GB would dominate the run."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    C = torch.randn((n_alpha_rows, n_beta_cols), generator=g, device=device,
                    dtype=dtype or torch.float64)
    C /= torch.linalg.vector_norm(C)
    return C


def serving_mix(n_requests: int = 512, seed: int = 5005, rate_per_s: float = 10.0):
    """Request stream: M uniform in {10,12,14,16}, N = M/2, string count
    log-uniform in [500, 4000] clamped to C(M, N), Poisson arrival times.

    Returns a list of dicts with keys M, N, n_keep, int_seed, sel_seed, t_arrive.
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n_requests):
        M = int(rng.choice([10, 12, 14, 16]))
        N = M // 2
        n = int(round(math.exp(rng.uniform(math.log(500), math.log(4000)))))
        n = min(n, math.comb(M, N))
        t += rng.exponential(1.0 / rate_per_s)
        out.append(dict(M=M, N=N, n_keep=n, int_seed=50000 + i, sel_seed=60000 + i,
                        t_arrive=t))
    return out


def serving_problem(req: dict) -> Problem:
    return make_problem(f"req_m{req['M']}_{req['n_keep']}", req["M"], req["N"],
                        req["n_keep"], req["int_seed"], req["sel_seed"])
