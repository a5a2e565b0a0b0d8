"""Oracle of the nonlinear solve with adjoint gradients (Sec. "Adjoint
Differentiation", paragraph "Nonlinear systems"): F(u) = A u + u^2 - f = 0,
the paper's listing example, by Newton from u = 0 with the C oracle's CG on
the Jacobian J = A + 2 diag(u); the gradient at the converged u from one
adjoint solve J^T lambda = dL/du: dL/df = lambda, dL/dA_ij = -lambda_i u_j.

General residuals F(u, *params) = 0 (same paragraph: the residual is any
differentiable function, the Jacobian dF/du is inverted by the solver and
the parameter gradient is -lambda^T dF/dparams): newton_general and
gradients_general take the residual as a torch callable on the CPU in
float64, form the dense Jacobian with torch.autograd.functional.jacobian and
solve with numpy.linalg.solve (tiny n).

TEST INFRASTRUCTURE; nothing here is shared with the GPU path."""
from __future__ import annotations

import numpy as np

import oracle


def jacobian(a, u):
    """J = A + 2 diag(u) (every row stores its diagonal)."""
    v = a.val.copy()
    for i in range(a.n):
        for k in range(a.row_ptr[i], a.row_ptr[i + 1]):
            if a.col[k] == i:
                v[k] += 2.0 * u[i]
    return a.with_values(v)


def newton(a, f, tol=1e-13, rtol=1e-14, max_newton=50):
    """(u, Newton steps)."""
    u = np.zeros(a.n)
    fn = np.linalg.norm(f)
    for it in range(max_newton + 1):
        F = oracle.spmv(a, u) + u * u - f
        if np.linalg.norm(F) <= tol * fn or it == max_newton:
            return u, it
        d = oracle.cg(jacobian(a, u), F, precond="jacobi", rtol=rtol).x
        u = u - d
    return u, max_newton


def gradients(a, u, gu, rtol=1e-14):
    """(dL/dA on the pattern, dL/df) at the converged u for dL/du = gu."""
    gA, lam, _ = oracle.adjoint(jacobian(a, u), u, gu, method="cg", precond="jacobi", rtol=rtol)
    return gA, lam


def _dense_jacobian(residual, u, params):
    import torch

    return torch.autograd.functional.jacobian(lambda uu: residual(uu, *params), u).numpy()


def newton_general(residual, n, params=(), tol=1e-13, max_newton=50):
    """(u, Newton steps): u with residual(u, *params) = 0 from u = 0, dense
    Newton (Jacobian by automatic differentiation, LU solve), stopping when
    ||F(u)|| <= tol ||F(0)||."""
    import torch

    u = torch.zeros(n, dtype=torch.float64)
    F = residual(u, *params).detach()
    f0 = float(torch.linalg.norm(F))
    for it in range(max_newton + 1):
        if float(torch.linalg.norm(F)) <= tol * f0 or it == max_newton:
            return u.numpy(), it
        J = _dense_jacobian(residual, u, params)
        d = np.linalg.solve(J, F.numpy())
        u = u - torch.as_tensor(d)
        F = residual(u, *params).detach()
    return u.numpy(), max_newton


def gradients_general(residual, u, params, gu):
    """dL/dparams for dL/du = gu at a root u: lambda = J^{-T} gu, then
    -lambda^T dF/dparams (one gradient per tensor in params; None for a
    parameter F does not depend on)."""
    import torch

    ut = torch.as_tensor(u, dtype=torch.float64)
    J = _dense_jacobian(residual, ut, [p.detach() for p in params])
    lam = np.linalg.solve(J.T, np.asarray(gu, dtype=np.float64))
    leaves = [p.detach().clone().requires_grad_(True) for p in params]
    F = residual(ut, *leaves)
    grads = torch.autograd.grad(F, leaves, grad_outputs=-torch.as_tensor(lam), allow_unused=True)
    return [None if g is None else g.numpy() for g in grads], lam
