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


# ---------------------------------------------------------------- general residuals

def _dense(a):
    import torch

    return torch.as_tensor(a.to_dense())


def test_general_oracle_reduces_to_the_semilinear_one(orc):
    """F(u; values, f) = A(values) u + u^2 - f through the general dense
    Newton (Jacobian by automatic differentiation) gives the semilinear
    oracle's u and its gradients w.r.t. f and every stored value."""
    import torch

    m = 8
    p = W.poisson2d(m)
    a = p.with_values(p.val * (m + 1) ** 2)
    r = np.random.default_rng(5)
    f = 1.0 + 0.5 * r.standard_normal(a.n)
    c = r.standard_normal(a.n)
    rows = torch.as_tensor(a.rows())
    cols = torch.as_tensor(a.col.astype(np.int64))

    def res(u, vals, ff):
        A = torch.zeros(a.n, a.n, dtype=torch.float64).index_put((rows, cols), vals)
        return A @ u + u * u - ff

    vt, ft = torch.as_tensor(a.val), torch.as_tensor(f)
    u, its = ON.newton_general(res, a.n, (vt, ft))
    u_ref, _ = ON.newton(a, f)
    assert np.allclose(u, u_ref, rtol=1e-12, atol=1e-14)
    (gv, gf), _ = ON.gradients_general(res, u, (vt, ft), c)
    gA_ref, gf_ref = ON.gradients(a, u_ref, c)
    assert np.allclose(gf, gf_ref, rtol=1e-10, atol=1e-14)
    assert np.allclose(gv, gA_ref, rtol=1e-10, atol=1e-14)


def test_general_oracle_cubic_closed_form():
    """F_i = a_i u_i + k u_i^3 - f_i with a scalar k inside the nonlinearity:
    u_i is the real root of the cubic, and for L = w.u
    dL/dk = -sum_i w_i u_i^3 / (a_i + 3 k u_i^2)."""
    import torch

    r = np.random.default_rng(6)
    n = 30
    av = r.uniform(1.0, 3.0, n)
    f = r.uniform(0.2, 2.0, n)
    w = r.standard_normal(n)
    k = torch.tensor(0.7, dtype=torch.float64)

    def res(u, kk):
        return torch.as_tensor(av) * u + kk * u ** 3 - torch.as_tensor(f)

    u, its = ON.newton_general(res, n, (k,))
    exact = np.array([max(np.roots([0.7, 0.0, av[i], -f[i]]).real[
        np.abs(np.roots([0.7, 0.0, av[i], -f[i]]).imag) < 1e-12]) for i in range(n)])
    assert np.allclose(u, exact, rtol=1e-13, atol=0) and its <= 10
    (gk,), _ = ON.gradients_general(res, u, (k,), w)
    assert np.isclose(float(gk), -np.sum(w * u ** 3 / (av + 0.7 * 3 * u ** 2)), rtol=1e-12)


def nl_diffusion(u, kap, f, m):
    """-div(kappa(u) grad u) - f on m x m cells (unit spacing, Dirichlet
    ghosts u = 0), face coefficient the mean of the two cells' kappa times
    (1 + (mean of the two cells' u)^2): a residual whose Jacobian has the
    5-point pattern and is not symmetric."""
    import torch

    U = u.reshape(m, m)
    K = kap.reshape(m, m)
    out = torch.zeros_like(U)
    for axis in (0, 1):
        for side in (-1, 1):
            Un = torch.roll(U, -side, dims=axis)
            Kn = torch.roll(K, -side, dims=axis)
            idx = torch.arange(m, device=U.device)
            edge = (idx == (0 if side < 0 else m - 1))
            edge = edge[:, None].expand(m, m) if axis == 0 else edge[None, :].expand(m, m)
            Un = torch.where(edge, torch.zeros_like(Un), Un)
            Kn = torch.where(edge, K, Kn)
            face = 0.5 * (K + Kn) * (1.0 + (0.5 * (U + Un)) ** 2)
            out = out + face * (U - Un)
    return out.reshape(-1) - f


def test_general_oracle_fd_on_nonlinear_diffusion():
    """dL/dkappa of L = w.u for the nonlinear diffusion residual against the
    paper's central differences at epsilon = 1e-5 (Eq. 7), on 8 cells."""
    import torch

    m = 7
    r = np.random.default_rng(7)
    kap = torch.as_tensor(np.exp(0.3 * r.standard_normal(m * m)))
    f = torch.as_tensor(1.0 + 0.3 * r.standard_normal(m * m))
    w = r.standard_normal(m * m)

    def res(u, kk, ff):
        return nl_diffusion(u, kk, ff, m)

    u, its = ON.newton_general(res, m * m, (kap, f))
    assert its <= 10
    (gk, gf), _ = ON.gradients_general(res, u, (kap, f), w)
    eps = 1e-5
    for j in r.choice(m * m, 8, replace=False):
        kp, km = kap.clone(), kap.clone()
        kp[j] += eps
        km[j] -= eps
        fd = (w @ ON.newton_general(res, m * m, (kp, f))[0] - w @ ON.newton_general(res, m * m, (km, f))[0]) / (2 * eps)
        assert abs(fd - gk[j]) <= 1e-6 * max(abs(gk[j]), 1e-3), (j, fd, gk[j])
