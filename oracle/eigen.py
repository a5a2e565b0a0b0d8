"""Oracle of the symmetric eigensolve with the Hellmann-Feynman gradient
(Eq. adjoint_eig: dlambda/dA_ij = v_i v_j for a simple eigenpair): the
dense eigen-decomposition (a library routine, numpy.linalg.eigh) of the
assembled matrix, and the gradient written out on the pattern.

TEST INFRASTRUCTURE; nothing here is shared with the GPU path."""
from __future__ import annotations

import numpy as np


def smallest(a, k):
    """(k smallest eigenvalues ascending, eigenvectors (n, k))."""
    w, v = np.linalg.eigh(a.to_dense())
    return w[:k], v[:, :k]


def largest(a, k):
    w, v = np.linalg.eigh(a.to_dense())
    return w[-k:], v[:, -k:]


def grad(a, V, glam):
    """dL/dA on the pattern for dL/dlambda_j = glam[j]: sum_j glam_j v_j[i] v_j[l]."""
    rows = a.rows()
    g = np.zeros(a.nnz)
    for j in range(V.shape[1]):
        g += glam[j] * V[rows, j] * V[a.col, j]
    return g


def rect_poisson_eigs(mx, my, k):
    """Closed form of the 5-point Dirichlet operator (diag 4, off -1) on an
    mx x my grid: 4 sin^2(p pi / 2(mx+1)) + 4 sin^2(q pi / 2(my+1))."""
    p = np.arange(1, mx + 1)[:, None]
    q = np.arange(1, my + 1)[None, :]
    lam = 4 * np.sin(p * np.pi / (2 * (mx + 1))) ** 2 + 4 * np.sin(q * np.pi / (2 * (my + 1))) ** 2
    return np.sort(lam.reshape(-1))[:k]
