"""Seeded random hierarchies for kernel-level parity checks."""

from __future__ import annotations

import numpy as np


def random_hierarchy(n_traj: int, n_ado: int, d: int, seed: int = 0,
                     hermitian: bool = False, scale_by_depth=None):
    """Complex array of shape (n_traj, n_ado, d, d) with entries ~ N(0,1)+iN(0,1).

    hermitian=True symmetrises every matrix (A + A^H)/2.  scale_by_depth, if
    given, is a per-ADO factor multiplied in so that deep ADOs can be made
    small as they are in physical states.
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n_traj, n_ado, d, d)) + 1j * rng.standard_normal((n_traj, n_ado, d, d))
    if hermitian:
        x = 0.5 * (x + np.conj(np.swapaxes(x, -1, -2)))
    if scale_by_depth is not None:
        x = x * np.asarray(scale_by_depth)[None, :, None, None]
    return x
