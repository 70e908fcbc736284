"""Structure of the finite-Taylor moments (CPU).

With q(x) = a x + b x^2 + e x^3 and e^{theta q(x)} = sum_k M_k(theta) x^k / k!,
M_k is a polynomial in theta: M_k = sum_m mu[k][m] theta^m.  The x^k
coefficient of (theta q)^m / m! needs m <= k <= 2m (3m with the cubic term),
so mu[k][m] vanishes outside ceil(k/2) <= m <= k (ceil(k/3) <= m <= k).  The
GPU kernels skip the multiply-adds on those zeros and bench.py counts
algorithmic flops over the same ranges.  These tests derive the pattern from
the definition, expanding the exponential in exact rational arithmetic, and
check that the recurrence the series is built from gives the same moments,
and that bench._moment_terms counts exactly the non-zero ones.
"""
import os
import sys
from fractions import Fraction
from math import factorial

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

K_MAX = 14  # orders up to n - 1 for the largest stencil (n = 15)


def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, x in enumerate(p):
        if x:
            for j, y in enumerate(q):
                out[i + j] += x * y
    return out


def _moments_by_definition(a, b, e, kmax):
    """mu[k][m] from e^{theta q} = sum_m theta^m q^m / m!: the x^k coefficient
    of q^m / m!, times k!."""
    q = [Fraction(0), a, b, e]
    mu = [[Fraction(0)] * (kmax + 1) for _ in range(kmax + 1)]
    qm = [Fraction(1)]
    for m in range(kmax + 1):
        for k in range(min(len(qm), kmax + 1)):
            mu[k][m] += qm[k] * factorial(k) / factorial(m)
        qm = _poly_mul(qm, q)[: kmax + 1]
    return mu


def _moments_by_recurrence(a, b, e, kmax):
    """The recurrence used by the series: d/dx e^{theta q} = theta q' e^{theta q}
    gives M_{k+1} = theta (a M_k + 2 b k M_{k-1} + 3 e k (k-1) M_{k-2})."""
    mu = [[Fraction(0)] * (kmax + 1) for _ in range(kmax + 1)]
    mu[0][0] = Fraction(1)
    for k in range(kmax):
        for m in range(1, kmax + 1):
            v = a * mu[k][m - 1]
            if k >= 1:
                v += 2 * b * k * mu[k - 1][m - 1]
            if k >= 2:
                v += 3 * e * k * (k - 1) * mu[k - 2][m - 1]
            mu[k + 1][m] = v
    return mu


GENERIC = (Fraction(7, 3), Fraction(-5, 11), Fraction(2, 13))


def test_recurrence_matches_definition():
    a, b, e = GENERIC
    assert _moments_by_recurrence(a, b, e, K_MAX) == _moments_by_definition(a, b, e, K_MAX)


def test_nonzero_range_without_cubic_term():
    a, b, _ = GENERIC
    mu = _moments_by_definition(a, b, Fraction(0), K_MAX)
    for k in range(K_MAX + 1):
        nz = [m for m in range(K_MAX + 1) if mu[k][m] != 0]
        assert nz == list(range((k + 1) // 2, k + 1)), (k, nz)


def test_nonzero_range_with_cubic_term():
    mu = _moments_by_definition(*GENERIC, K_MAX)
    for k in range(K_MAX + 1):
        nz = [m for m in range(K_MAX + 1) if mu[k][m] != 0]
        assert nz == list(range((k + 2) // 3, k + 1)), (k, nz)


def test_flop_model_counts_the_nonzero_moments():
    """bench._moment_terms: per order K the moments that can be non-zero, and
    the recurrence terms whose source moment can be non-zero."""
    import bench
    a, b, _ = GENERIC
    mu = _moments_by_definition(a, b, Fraction(0), K_MAX)
    for n in (3, 5, 7, 9, 11, 13, 15):
        for K, (entries, terms) in enumerate(bench._moment_terms(n), start=1):
            k = K - 1
            assert entries == sum(1 for m in range(K_MAX + 1) if mu[K][m] != 0), (n, K)
            want = 0
            for m in range(1, K + 1):
                if mu[K][m] == 0:
                    continue
                want += mu[k][m - 1] != 0
                want += k >= 1 and mu[k - 1][m - 1] != 0
            assert terms == want, (n, K)
