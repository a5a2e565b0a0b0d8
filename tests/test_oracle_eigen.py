"""Pins of the eigen oracle: the dense decomposition of the rectangular
Poisson operator against its closed form, and the Hellmann-Feynman gradient
against central differences (symmetric perturbations)."""
import numpy as np

import workloads as W
from oracle import eigen as OE


def test_rect_poisson_closed_form():
    a = W.poisson2d_rect(9, 7)
    w, v = OE.smallest(a, 6)
    assert np.allclose(w, OE.rect_poisson_eigs(9, 7, 6), rtol=1e-13, atol=0)
    wl, _ = OE.largest(a, 3)
    p = np.arange(1, 10)[:, None]
    q = np.arange(1, 8)[None, :]
    full = np.sort((4 * np.sin(p * np.pi / 20) ** 2 + 4 * np.sin(q * np.pi / 16) ** 2).reshape(-1))
    assert np.allclose(wl, full[-3:], rtol=1e-13, atol=0)


def test_hellmann_feynman_fd():
    """dlambda_j / d(A_il = A_li) = 2 v_i v_l (i != l), dlambda / dA_ii = v_i^2,
    checked by central differences of the dense eigenvalues."""
    r = np.random.default_rng(8)
    m = 6
    a = W.diffusion3d(m, np.exp(r.standard_normal(m ** 3)))
    k = 4
    w, V = OE.smallest(a, k)
    glam = r.standard_normal(k)
    g = OE.grad(a, V, glam)
    rows = a.rows()
    eps = 1e-6
    dense = a.to_dense()
    for kk in r.choice(a.nnz, 12, replace=False):
        i, l = rows[kk], a.col[kk]
        dp, dm = dense.copy(), dense.copy()
        dp[i, l] += eps
        dm[i, l] -= eps
        if i != l:
            dp[l, i] += eps
            dm[l, i] -= eps
        fd = (glam @ np.linalg.eigvalsh(dp)[:k] - glam @ np.linalg.eigvalsh(dm)[:k]) / (2 * eps)
        # the mirror entry (l, i) carries the same gradient
        an = g[kk] if i == l else 2 * g[kk]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (i, l, fd, an)
