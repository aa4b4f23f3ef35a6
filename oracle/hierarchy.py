"""Hierarchy index set of the HEOM (oracle).

Paper, Sec. II.B (text after Eq. HEOM_DB): ADOs are labelled by one
non-negative integer per exponential bath term, n = (n_j), j running over the
(mode s, term k) pairs; an index with a negative entry denotes the zero
operator and n +- e_j increments/decrements entry j.  The paper does not state
its truncation; the triangular set |n| = sum_j n_j <= L is used, ordered by
depth |n| and then ascending lexicographically within a depth.  Optionally the
set is filtered further by the total damping rate, sum_j n_j Re(nu_j) <= cut
(relative tolerance 1e-9), which keeps it closed under n -> n - e_j.
"""

from __future__ import annotations

import itertools

import numpy as np


def enumerate_ados(n_terms: int, depth: int):
    """All n in N^M with |n| <= L: list of tuples in (depth, lexicographic) order."""
    out = []
    for level in range(depth + 1):
        level_set = [n for n in itertools.product(range(level + 1), repeat=n_terms)
                     if sum(n) == level]
        out.extend(sorted(level_set))
    return out


class Hierarchy:
    """ADO list with neighbour maps.

    up[i, j]  = index of n_i + e_j, or -1 when that is outside the set;
    down[i, j] = index of n_i - e_j, or -1 when n_ij = 0.
    """

    def __init__(self, n_terms: int, depth: int, rates=None, rate_cut: float = 0.0):
        self.n_terms = n_terms
        self.depth = depth
        self.ados = enumerate_ados(n_terms, depth)
        if rate_cut > 0.0:
            r = np.asarray(rates, dtype=float)
            self.ados = [n for n in self.ados
                         if sum(k * x for k, x in zip(n, r)) <= rate_cut * (1.0 + 1e-9)]
        self.index = {n: i for i, n in enumerate(self.ados)}
        N = len(self.ados)
        self.n = np.array(self.ados, dtype=np.int64).reshape(N, n_terms)
        self.up = -np.ones((N, n_terms), dtype=np.int64)
        self.down = -np.ones((N, n_terms), dtype=np.int64)
        for i, n in enumerate(self.ados):
            for j in range(n_terms):
                m = list(n)
                m[j] += 1
                self.up[i, j] = self.index.get(tuple(m), -1)
                if n[j] > 0:
                    m[j] -= 2
                    self.down[i, j] = self.index[tuple(m)]

    def __len__(self):
        return len(self.ados)
