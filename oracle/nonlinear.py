"""Oracle of the nonlinear solve with adjoint gradients (Sec. "Adjoint
Differentiation", paragraph "Nonlinear systems"): F(u) = A u + u^2 - f = 0,
the paper's listing example, by Newton from u = 0 with the C oracle's CG on
the Jacobian J = A + 2 diag(u); the gradient at the converged u from one
adjoint solve J^T lambda = dL/du: dL/df = lambda, dL/dA_ij = -lambda_i u_j.

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
