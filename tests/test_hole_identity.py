"""The hole-pair form of the same-spin operator, checked on the CPU.

The library's hole-pair sweep (tbsci_set_same_spin, TBSCI_SAME_SPIN_HOLE)
evaluates A_s = <I|H_s|J> for one spin's strings as

  A_s[I][J] = sum_{K in I and J} s(I; K) W[pair(I - K)][pair(J - K)] s(J; K)
  W[pr][qs] = (pq|rs) - (ps|rq)
            + (h_pq d_rs + h_rs d_pq - h_ps d_rq - h_rq d_ps) / (n - 1)

over the (n-2)-electron strings K, with s(Z; K) = <K| a_y a_x |Z> for
Z = K + {x < y} (the two-body part over ordered pairs; the one-body part
folded in through a+_p a_q = a+_p N a_q / (n - 1)).  Here that formula,
written with plain loops, must equal the oracle's Slater-Condon same-spin
matrix on complete and randomly selected string sets, both spins: a wrong
sign convention, a dropped exchange term or a wrong one-body fold changes
the singles, doubles or diagonal and fails.
"""
import numpy as np
import pytest

from paper_2503_10335_amd import workloads as W


def _hole_matrix(strs, n, M, h, eri):
    f = 1.0 / (n - 1)
    groups = {}
    for x, X in enumerate(strs):
        occ = [i for i in range(M) if (int(X) >> i) & 1]
        for j in range(1, n):
            for i in range(j):
                a, b = occ[i], occ[j]
                K = int(X) & ~(1 << a) & ~(1 << b)
                groups.setdefault(K, []).append((x, a, b, -1.0 if (i + j - 1) & 1 else 1.0))
    A = np.zeros((len(strs), len(strs)))
    for lst in groups.values():
        for (x, p, r, sx) in lst:
            for (y, q, s, sy) in lst:
                w = eri[p, q, r, s] - eri[p, s, r, q]
                w += f * ((h[p, q] if r == s else 0.0) + (h[r, s] if p == q else 0.0)
                          - (h[p, s] if r == q else 0.0) - (h[r, q] if p == s else 0.0))
                A[x, y] += sx * w * sy
    return A


@pytest.mark.parametrize("prob", [
    lambda: W.config("fci_m8"),
    lambda: W.random_selection(8, 3, 4, 37, 53, seed=11),
    lambda: W.random_selection(10, 5, 5, 130, 97, seed=12),
    lambda: W.random_selection(9, 2, 7, 30, 36, seed=21),
], ids=["fci_m8", "rand_m8_3_4", "rand_m10_5_5", "rand_m9_2_7"])
def test_hole_pair_form_equals_same_spin_matrix(prob):
    from oracle import oracle as O
    p = prob()
    sp = O.Space.of(p)
    M = p.M
    eri = p.eri.reshape(M, M, M, M)
    h = p.h.reshape(M, M)
    for spin, strs, n in ((0, p.alpha, p.n_alpha), (1, p.beta, p.n_beta)):
        ref = sp.same_spin_matrix(spin)
        got = _hole_matrix(strs, n, M, h, eri)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
