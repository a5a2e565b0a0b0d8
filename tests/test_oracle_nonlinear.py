"""Pins of the nonlinear-solve oracle (F(u) = A u + u^2 - f, Newton, one
adjoint solve): the diagonal case in closed form, and the gradient against
the paper's central finite differences (epsilon = 1e-5) on entries of A
and f."""
import numpy as np

import workloads as W
from oracle import nonlinear as ON


def test_diagonal_closed_form(orc):
    """A = diag(a): u_i = (-a_i + sqrt(a_i^2 + 4 f_i)) / 2, and for
    L = c.u: dL/df_i = c_i / (a_i + 2 u_i), dL/da_i = -u_i dL/df_i."""
    r = np.random.default_rng(3)
    n = 40
    a = W.from_dense(np.diag(r.uniform(1.0, 3.0, n)))
    f = r.uniform(0.1, 2.0, n)
    c = r.standard_normal(n)
    u, its = ON.newton(a, f)
    exact = (-a.val + np.sqrt(a.val ** 2 + 4 * f)) / 2
    assert np.allclose(u, exact, rtol=1e-13, atol=0) and its <= 8
    gA, gf = ON.gradients(a, u, c)
    assert np.allclose(gf, c / (a.val + 2 * u), rtol=1e-12, atol=0)
    assert np.allclose(gA, -u * gf, rtol=1e-12, atol=0)


def test_gradient_finite_differences(orc):
    m = 12
    p = W.poisson2d(m)
    a = p.with_values(p.val * (m + 1) ** 2)
    r = np.random.default_rng(4)
    f = 1.0 + 0.5 * r.standard_normal(a.n)
    c = r.standard_normal(a.n)
    u, its = ON.newton(a, f)
    assert its <= 8
    gA, gf = ON.gradients(a, u, c)
    eps = 1e-5

    def L(aa, ff):
        return c @ ON.newton(aa, ff)[0]

    ka = r.choice(a.nnz, 10, replace=False)
    fd = []
    for k in ka:
        vp, vm = a.val.copy(), a.val.copy()
        vp[k] += eps
        vm[k] -= eps
        fd.append((L(a.with_values(vp), f) - L(a.with_values(vm), f)) / (2 * eps))
    assert np.linalg.norm(np.array(fd) - gA[ka]) <= 1e-6 * np.linalg.norm(gA[ka])
    kf = r.choice(a.n, 10, replace=False)
    fd = []
    for k in kf:
        fp, fm = f.copy(), f.copy()
        fp[k] += eps
        fm[k] -= eps
        fd.append((L(a, fp) - L(a, fm)) / (2 * eps))
    assert np.linalg.norm(np.array(fd) - gf[kf]) <= 1e-6 * np.linalg.norm(gf[kf])
