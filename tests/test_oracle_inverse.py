"""Pins of the inverse-problem oracle (Sec. "End-to-End: Inverse Coefficient
Learning") against facts that do not come from its own formulas: exactness
of the five-point operator on functions it reproduces, symmetry and
homogeneity in kappa, central finite differences of the loss, and Adam's
first step in closed form."""
import numpy as np
import pytest

import workloads as W
from oracle import inverse as OI


def _centres(m):
    c = (np.arange(m) + 0.5) / m
    x, y = np.meshgrid(c, c)
    return x.reshape(-1), y.reshape(-1)


def test_operator_exact_on_quadratic():
    """kappa = 1: interior rows of A applied to x^2 + y^2 give -Laplace = -4
    exactly (the five-point stencil is exact on quadratics)."""
    m = 9
    a = OI.assemble(np.ones(m * m), m)
    x, y = _centres(m)
    u = x * x + y * y
    r = a.to_dense() @ u
    ix, iy = np.arange(m * m) % m, np.arange(m * m) // m
    inner = (ix > 0) & (ix < m - 1) & (iy > 0) & (iy < m - 1)
    assert np.allclose(r[inner], -4.0, rtol=0, atol=1e-9)


def test_operator_exact_on_linear_with_wall():
    """kappa = g(y) only: -div(kappa grad x) = 0, and the half-cell wall
    treatment is exact for x, which vanishes on the wall x = 0; rows away
    from the other walls give 0."""
    m = 10
    _, y = _centres(m)
    kappa = 1.0 + 0.7 * np.cos(3.0 * y)
    a = OI.assemble(kappa, m)
    x, _ = _centres(m)
    r = a.to_dense() @ x
    ix, iy = np.arange(m * m) % m, np.arange(m * m) // m
    rows = (ix < m - 1) & (iy > 0) & (iy < m - 1)
    assert np.abs(r[rows]).max() <= 1e-10 * np.abs(a.val).max()


def test_operator_symmetric_homogeneous():
    m = 7
    r = np.random.default_rng(1)
    kappa = np.exp(r.standard_normal(m * m))
    a = OI.assemble(kappa, m)
    d = a.to_dense()
    assert np.array_equal(d, d.T)
    assert np.all(np.linalg.eigvalsh(d) > 0)
    b = OI.assemble(2.0 * kappa, m)
    assert np.allclose(b.val, 2.0 * a.val, rtol=1e-15, atol=0)


def test_loss_gradient_finite_differences(orc):
    """dL/dtheta (adjoint + chain rule) against central differences of the
    loss at h = 1e-6 on 12 entries."""
    m = 6
    kt, f = W.inverse_truth(m)
    u_obs = OI.observe(m, kt, f, rtol=1e-14)
    r = np.random.default_rng(2)
    theta = np.log(np.e - 1.0) + 0.3 * r.standard_normal(m * m)
    _, g, _ = OI.loss_and_grad(theta, m, u_obs, f, rtol=1e-14)
    h = 1e-6
    picks = r.choice(m * m, 12, replace=False)
    fd = []
    for k in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp, _, _ = OI.loss_and_grad(tp, m, u_obs, f, rtol=1e-14)
        lm, _, _ = OI.loss_and_grad(tm, m, u_obs, f, rtol=1e-14)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    assert np.linalg.norm(fd - g[picks]) <= 1e-6 * np.linalg.norm(g[picks])


def test_truth_fits_its_observation(orc):
    """At kappa = kappa* the misfit vanishes: the loss is the regulariser
    alone, and the data part of the gradient is zero."""
    m = 8
    kt, f = W.inverse_truth(m)
    u_obs = OI.observe(m, kt, f, rtol=1e-14)
    theta = np.log(np.expm1(kt))
    loss, g, u = OI.loss_and_grad(theta, m, u_obs, f, rtol=1e-14)
    reg, greg = OI.regulariser(kt, m)
    assert abs(loss - OI.REG * reg) <= 1e-12 * loss
    sig = 1.0 / (1.0 + np.exp(-theta))
    assert np.allclose(g, OI.REG * greg * sig, rtol=1e-6, atol=1e-12)


def test_adam_first_step_closed_form():
    """Adam's first step moves each coordinate by lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    st = {"t": 0, "m": np.zeros(4), "v": np.zeros(4)}
    th = OI.adam(np.zeros(4), g, st, lr=5e-2)
    assert np.allclose(th, -5e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_truth_field():
    kt, f = W.inverse_truth(64)
    assert kt.shape == (4096,) and np.all(f == 1.0)
    assert 0.5 < kt.min() < 0.51 and 1.49 < kt.max() < 1.5
    assert kt[0] == pytest.approx(1 + 0.5 * np.sin(np.pi / 64) ** 2)
