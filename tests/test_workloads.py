"""Invariants of the seeded input generators (no GPU)."""
import math

import numpy as np
import pytest

import workloads as W


def _canonical(a):
    assert a.row_ptr.dtype == np.int32 and a.col.dtype == np.int32 and a.val.dtype == np.float64
    assert a.row_ptr[0] == 0 and np.all(np.diff(a.row_ptr) >= 0) and a.row_ptr[-1] == len(a.col)
    assert np.all((a.col >= 0) & (a.col < a.n))
    rows = a.rows()
    same = rows[1:] == rows[:-1]
    assert np.all(a.col[1:][same] > a.col[:-1][same])


def _bit_symmetric(a):
    d = a.to_dense()
    return np.array_equal(d, d.T)


@pytest.mark.parametrize("m", [1, 2, 5, 64])
def test_poisson2d(m):
    a = W.poisson2d(m)
    _canonical(a)
    assert a.nnz == 5 * m * m - 4 * m
    if m <= 5:
        assert _bit_symmetric(a)


@pytest.mark.parametrize("m", [1, 2, 4, 7])
def test_diffusion3d(m):
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    _canonical(a)
    assert a.nnz == 7 * m ** 3 - 6 * m * m
    assert _bit_symmetric(a)
    # kappa == 1 -> standard 7-point Laplacian
    p = W.diffusion3d(m)
    assert np.array_equal(p.val[p.rows() == p.col], np.full(m ** 3, 6.0))
    assert set(np.unique(p.val[p.rows() != p.col])) <= {-1.0}


def test_diffusion3d_workload_sizes():
    # full-size closed form (not built here): n = 256^3, nnz = 7m^3 - 6m^2
    assert 7 * 256 ** 3 - 6 * 256 ** 2 == 117047296
    a, b = W.diffusion3d_workload(16)
    assert a.n == 4096 and len(b) == 4096


def test_upwind_m_matrix():
    a = W.diffusion3d(5, W.diffusion3d_kappa(5), velocity=10.0)
    _canonical(a)
    d = a.to_dense()
    off = d - np.diag(np.diag(d))
    assert np.all(off <= 0)
    assert np.all(np.diag(d) >= np.abs(off).sum(axis=1) - 1e-12)  # weak row dominance
    assert not _bit_symmetric(a)


def test_knn_laplacian():
    a, b = W.knn_system(0, n_lo=300, n_hi=400)
    _canonical(a)
    assert _bit_symmetric(a)
    deg = np.diff(a.row_ptr) - 1
    assert deg.min() >= 8 and deg.max() <= 60
    one = np.ones(a.n)
    assert np.abs(a.to_dense() @ one - 0.01).max() <= 1e-14 * deg.max() * 4
    assert len(b) == a.n


def test_aniso2d():
    m = 6
    for s in range(4):
        ratio, ang = W.aniso_params(s)
        assert 1.0 <= ratio <= 1000.0 and 0.0 <= ang < math.pi
        a = W.aniso2d(m, ratio, ang)
        _canonical(a)
        assert a.nnz == (3 * m - 2) ** 2
        assert _bit_symmetric(a)
        assert np.linalg.eigvalsh(a.to_dense()).min() > 0


def test_seeds_reproducible():
    assert np.array_equal(W.rng(2, 1).standard_normal(5), W.rng(2, 1).standard_normal(5))
    assert not np.array_equal(W.rng(2, 1).standard_normal(5), W.rng(2, 2).standard_normal(5))
