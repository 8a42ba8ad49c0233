"""SU(3) colour algebra by brute force (FP64).  Test infrastructure only.

Generators t^a = lambda^a / 2 (Gell-Mann matrices, Tr t^a t^b = delta^ab / 2),
structure constants from [t^a, t^b] = i f^abc t^c, i.e.
f^abc = -2 i Tr([t^a, t^b] t^c).

For one quark line with k gluons the colour basis is
X_sigma = (t^{a_sigma1} ... t^{a_sigmak})_{i jbar}, sigma a permutation of the
gluons, and the colour matrix is C_{sigma tau} = sum over all colour indices of
X_sigma X_tau^*, i.e. sum_a Tr(X_sigma X_tau^dagger), evaluated here by summing
explicitly over all 8^k gluon colours.
"""
import itertools
from fractions import Fraction

import numpy as np


def gell_mann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


T = gell_mann() / 2.0


def structure_constants():
    comm = np.einsum('aij,bjk->abik', T, T) - np.einsum('bij,ajk->abik', T, T)
    f = -2j * np.einsum('abij,cji->abc', comm, T)
    assert np.abs(f.imag).max() < 1e-14
    return f.real


F = structure_constants()


def orderings(k):
    """All permutations of range(k), lexicographic."""
    return list(itertools.permutations(range(k)))


def colour_tensor(sigma):
    """X_sigma as an array [8]*k + [3, 3] indexed by the colours of gluons 0..k-1."""
    k = len(sigma)
    letters = 'abcdefgh'[:k]
    # product t^{a_sigma1} t^{a_sigma2} ... with matrix indices chained
    idx = 'ijklmn'
    terms = []
    for pos, g in enumerate(sigma):
        terms.append(letters[g] + idx[pos] + idx[pos + 1])
    spec = ','.join(terms) + '->' + letters + idx[0] + idx[k]
    return np.einsum(spec, *([T] * k), optimize=True)


def colour_matrix(k):
    """C[sigma, tau] (float) over the k! orderings of k gluons."""
    perms = orderings(k)
    X = np.stack([colour_tensor(s).reshape(-1) for s in perms])
    C = X @ X.conj().T                       # C[a, b] = sum over all colours of X_a X_b^*
    assert np.abs(C.imag).max() < 1e-12
    return C.real


def colour_matrix_exact(k, max_den=1000):
    """C as Fractions, recovered from the brute-force floats (denominator search)."""
    C = colour_matrix(k)
    for den in range(1, max_den + 1):
        num = C * den
        if np.abs(num - np.round(num)).max() < 1e-9:
            return [[Fraction(int(round(v)), den) for v in row] for row in num], den
    raise ValueError('no small common denominator')
