"""Brute-force and exact-arithmetic references used to pin the oracle.

Independent of both the oracle and the GPU path: permutation (Leibniz) sums,
perfect-matching sums (Appendix A, Eq. pf_def) and exact rational elimination.
"""
from __future__ import annotations

import itertools
from fractions import Fraction


def perm_sign(p) -> int:
    """Parity of a permutation given as a sequence of distinct ints, by cycle count."""
    p = list(p)
    seen = [False] * len(p)
    sign = 1
    for i in range(len(p)):
        if seen[i]:
            continue
        j, length = i, 0
        while not seen[j]:
            seen[j] = True
            j = p[j]
            length += 1
        if length % 2 == 0:
            sign = -sign
    return sign


def leibniz_det(a):
    """det A = sum over permutations of sign(p) prod_i A[i][p(i)]."""
    n = len(a)
    total = 0
    for p in itertools.permutations(range(n)):
        term = perm_sign(p)
        for i in range(n):
            term = term * a[i][p[i]]
        total += term
    return total


def perfect_matchings(elems):
    """All partitions of ``elems`` (even length) into pairs (i<j), first element paired first."""
    if not elems:
        yield []
        return
    first = elems[0]
    for idx in range(1, len(elems)):
        partner = elems[idx]
        rest = elems[1:idx] + elems[idx + 1:]
        for m in perfect_matchings(rest):
            yield [(first, partner)] + m


def matching_pf(a):
    """Eq. pf_def: sum over pairings alpha of sign(alpha) prod A[i_k][j_k]."""
    n = len(a)
    if n % 2:
        return 0
    total = 0
    for m in perfect_matchings(list(range(n))):
        flat = [x for pair in m for x in pair]
        term = perm_sign(flat)
        for i, j in m:
            term = term * a[i][j]
        total += term
    return total


def frac_matrix(a):
    return [[Fraction(int(x)) if not isinstance(x, Fraction) else x for x in row] for row in a]


def exact_det(a):
    """Exact determinant of a rational matrix by fraction-valued Gaussian elimination."""
    m = [row[:] for row in frac_matrix(a)]
    n = len(m)
    det = Fraction(1)
    for j in range(n):
        p = next((i for i in range(j, n) if m[i][j] != 0), None)
        if p is None:
            return Fraction(0)
        if p != j:
            m[j], m[p] = m[p], m[j]
            det = -det
        det *= m[j][j]
        for i in range(j + 1, n):
            f = m[i][j] / m[j][j]
            if f:
                for c in range(j, n):
                    m[i][c] -= f * m[j][c]
    return det


def exact_inverse(a):
    """Exact inverse of a nonsingular rational matrix (Gauss-Jordan on [A | I])."""
    m = [row[:] for row in frac_matrix(a)]
    n = len(m)
    aug = [m[i] + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for j in range(n):
        p = next(i for i in range(j, n) if aug[i][j] != 0)
        aug[j], aug[p] = aug[p], aug[j]
        piv = aug[j][j]
        aug[j] = [x / piv for x in aug[j]]
        for i in range(n):
            if i != j and aug[i][j] != 0:
                f = aug[i][j]
                aug[i] = [x - f * y for x, y in zip(aug[i], aug[j])]
    return [row[n:] for row in aug]


def matmul(a, b):
    return [[sum(a[i][t] * b[t][j] for t in range(len(b))) for j in range(len(b[0]))]
            for i in range(len(a))]


def transpose(a):
    return [list(r) for r in zip(*a)]


def add(a, b):
    return [[x + y for x, y in zip(r, s)] for r, s in zip(a, b)]


def sub(a, b):
    return [[x - y for x, y in zip(r, s)] for r, s in zip(a, b)]


def scale(a, s):
    return [[x * s for x in r] for r in a]


def eye(n):
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
