"""Nonlinear solves with the adjoint gradient (Sec. "Adjoint
Differentiation", paragraph "Nonlinear systems"; the paper's listing solves
F(u) = A u + u^2 - f = 0 by Newton).

Semilinear residuals F(u) = A u + g(u) - f with an elementwise g: the Newton
Jacobian J = A + diag(g'(u)) keeps A's pattern, so every Newton step is one
library solve on J's values (A's values plus g'(u) on the diagonal).  The
backward (Eq. adjoint_master at the converged u) is one adjoint solve
J^T lambda = dL/du, after which dL/df = lambda and, since dF/dA_ij = u_j e_i,
dL/dA_ij = -lambda_i u_j on the pattern -- exactly the library's adjoint
output for J with x = u.  One autograd node; the forward's Newton steps are
not recorded."""
from __future__ import annotations

import warnings

import torch

from . import SparseCSR, _lib


def square(u):
    return u * u


def square_prime(u):
    return 2.0 * u


def diagonal_positions(pat) -> torch.Tensor:
    """Entry index of every row's diagonal (each row must have one)."""
    n = pat.n
    counts = (pat.row_ptr[1:] - pat.row_ptr[:-1]).to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(n, device=pat.device), counts)
    pos = torch.nonzero(pat.col.to(torch.int64) == rows).flatten()
    if pos.numel() != n:
        raise ValueError("every row needs a stored diagonal entry")
    return pos


class NewtonSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, f, pat, dpos, g, gp, kw):
        values = values.detach()
        f = f.detach()
        u = torch.zeros_like(f)
        fn0 = float(torch.linalg.norm(f))
        lin = _lib.make_opts(method="auto", precond="jacobi", rtol=kw["lin_rtol"])
        its, converged = 0, False
        J = values.clone()
        for its in range(kw["max_newton"] + 1):
            F = _lib.spmv(pat, values, u) + g(u) - f
            if float(torch.linalg.norm(F)) <= kw["tol"] * fn0:
                converged = True
                break
            if its == kw["max_newton"]:
                break
            J = values.clone()
            J[dpos] += gp(u)
            d, _, st = _lib.solve(pat, J, F, lin)
            if st != _lib.OK:
                warnings.warn(f"Newton step {its}: linear solve status {_lib.status_string(st)}", RuntimeWarning)
            u = u - d
        if not converged:
            warnings.warn(f"Newton did not converge in {kw['max_newton']} steps", RuntimeWarning)
        J = values.clone()
        J[dpos] += gp(u)
        ctx.pat, ctx.kw, ctx.converged = pat, kw, converged
        ctx.newton_steps = its
        ctx.save_for_backward(J, u)
        return u

    @staticmethod
    def backward(ctx, gu):
        J, u = ctx.saved_tensors
        if not ctx.converged:
            raise RuntimeError("backward through a Newton solve that did not converge")
        opts = _lib.make_opts(method="auto", precond="jacobi", rtol=ctx.kw["lin_rtol"])
        gA, lam, _, st = _lib.adjoint(ctx.pat, J, u, gu.contiguous(), opts, want_gA=ctx.needs_input_grad[0])
        if st != _lib.OK:
            warnings.warn(f"adjoint solve finished with status {_lib.status_string(st)}", RuntimeWarning)
        return (gA if ctx.needs_input_grad[0] else None), (lam if ctx.needs_input_grad[1] else None), \
            None, None, None, None, None


def newton_solve(A: SparseCSR, f: torch.Tensor, g=square, g_prime=square_prime, *, tol: float = 1e-12,
                 lin_rtol: float = 1e-12, max_newton: int = 50, info: dict | None = None) -> torch.Tensor:
    """u with A u + g(u) = f (default g(u) = u^2, the paper's example), by
    Newton from u = 0; differentiable in A's values and f.  tol bounds
    ||F(u)|| / ||f||; lin_rtol is each linear solve's relative tolerance.
    `info`, if given, receives the number of Newton steps."""
    if not hasattr(A, "_dpos"):
        A._dpos = diagonal_positions(A.pattern)
    kw = dict(tol=tol, lin_rtol=lin_rtol, max_newton=max_newton)
    u = NewtonSolveFn.apply(A.values, f, A.pattern, A._dpos, g, g_prime, kw)
    if info is not None:
        info["newton_steps"] = u.grad_fn.newton_steps if u.grad_fn is not None else None
    return u
