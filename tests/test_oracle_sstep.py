"""Pins of the s-step CG oracle (no GPU).

In exact arithmetic s-step CG produces CG's iterates, whatever the basis: a
textbook CG in rational arithmetic (below, independent of the oracle's
basis, Gram matrix and coordinate recurrence) must agree exactly with the
oracle's run capped at every k, for every s.  In floating point the oracle
must solve like the C oracle's Jacobi-PCG."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import sstep


def _exact_cg(a, b, k):
    """k steps of textbook CG from x = 0 in rational arithmetic."""
    n = a.n
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for e in range(a.row_ptr[i], a.row_ptr[i + 1]):
            A[i][a.col[e]] = Fraction(a.val[e])
    x = [Fraction(0)] * n
    r = [Fraction(v) for v in b]
    p = list(r)
    rr = sum(v * v for v in r)
    for _ in range(k):
        ap = [sum(A[i][j] * p[j] for j in range(n)) for i in range(n)]
        alpha = rr / sum(u * v for u, v in zip(p, ap))
        x = [u + alpha * v for u, v in zip(x, p)]
        r = [u - alpha * v for u, v in zip(r, ap)]
        rr_new = sum(v * v for v in r)
        if rr_new == 0:
            break
        beta = rr_new / rr
        rr = rr_new
        p = [u + beta * v for u, v in zip(r, p)]
    return x


def _int_spd(n, seed):
    """Integer SPD matrix (diagonally dominant, random sparse pattern)."""
    r = np.random.default_rng(seed)
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(i):
            if r.random() < 0.4:
                M[i, j] = M[j, i] = -float(r.integers(1, 4))
    M += np.diag(np.abs(M).sum(axis=1) + r.integers(1, 3, n))
    rp = np.zeros(n + 1, np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(M[i])[0]
        cols += list(nz)
        vals += list(M[i, nz])
        rp[i + 1] = len(cols)
    return W.Csr(n, rp, np.array(cols, np.int32), np.array(vals))


@pytest.mark.parametrize("s", [2, 3, 4])
@pytest.mark.parametrize("make", [lambda: W.poisson2d(3), lambda: _int_spd(7, 1), lambda: _int_spd(9, 2)],
                         ids=["poisson3x3", "spd7", "spd9"])
def test_exact_arithmetic_iterates_are_cg(s, make):
    a = make()
    b = [Fraction(int(v)) for v in np.random.default_rng(a.n).integers(-5, 6, a.n)]
    if not any(b):
        b[0] = Fraction(1)
    for k in range(1, a.n + 1):
        res = sstep.sstep_cg(a, b, s=s, precond="none", rtol=0.0, max_iter=k, exact=True)
        ref = _exact_cg(a, b, k)
        assert list(res.x) == ref, (s, k)
        if res.status == sstep.OK:
            break
    # CG terminates in at most n steps: the oracle reports convergence with an
    # exactly zero residual
    res = sstep.sstep_cg(a, b, s=s, precond="none", rtol=0.0, exact=True)
    assert res.status == sstep.OK and res.iters <= a.n
    assert list(res.x) == _exact_cg(a, b, a.n)


@pytest.mark.parametrize("s", [2, 4])
@pytest.mark.parametrize("make", [lambda: W.poisson2d(20), lambda: W.diffusion3d(8, W.diffusion3d_kappa(8))],
                         ids=["poisson20", "diffusion8"])
def test_float_solves_like_jacobi_pcg(orc, s, make):
    """Against the C oracle's Jacobi-PCG: the solution to 1e-9 at rtol 1e-12,
    iteration counts within max(2, 2%), and the k-th iterate of a capped run
    at k = s (an outer boundary) and k = s + 1 (inside an outer step)."""
    a = make()
    b = np.random.default_rng(3).standard_normal(a.n)
    res = sstep.sstep_cg(a, b, s=s, precond="jacobi", rtol=1e-12)
    ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    assert res.status == sstep.OK
    assert np.linalg.norm(res.x - ref.x) / np.linalg.norm(ref.x) <= 1e-9
    assert abs(res.iters - ref.iters) <= max(2, 0.02 * ref.iters), (res.iters, ref.iters)
    for k in (s, s + 1):
        rk = sstep.sstep_cg(a, b, s=s, precond="jacobi", rtol=1e-14, max_iter=k)
        ck = orc.cg(a, b, precond="jacobi", rtol=1e-14, max_iter=k)
        assert rk.status == sstep.NOT_CONVERGED and rk.iters == k
        assert np.linalg.norm(rk.x - ck.x) / np.linalg.norm(ck.x) <= 1e-11, k


def test_change_of_basis_matches_the_chebyshev_recurrence():
    """A Y = Y B on the columns that stay inside the basis, for a random
    symmetric A: the recurrence T_{j+1} = 2 (A - I) T_j - T_{j-1} defines Y,
    and B must reproduce A times each non-final basis vector."""
    s = 3
    r = np.random.default_rng(0)
    n = 12
    M = r.standard_normal((n, n))
    A = (M + M.T) / 4
    p, q = r.standard_normal(n), r.standard_normal(n)
    Y = []
    for v0, length in ((p, s + 1), (q, s)):
        prev, cur = None, v0
        Y.append(cur)
        for j in range(1, length):
            t = A @ cur - cur
            nxt = t if j == 1 else 2 * t - prev
            prev, cur = cur, nxt
            Y.append(cur)
    Y = np.array(Y).T
    Bm = sstep.change_of_basis(s).astype(float)
    inside = [c for c in range(2 * s + 1) if c not in (s, 2 * s)]
    assert np.allclose((A @ Y)[:, inside], (Y @ Bm)[:, inside], rtol=1e-12, atol=1e-12)
