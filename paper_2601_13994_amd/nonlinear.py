"""Nonlinear solves with the adjoint gradient (Sec. "Adjoint
Differentiation", paragraph "Nonlinear systems"; the paper's listing solves
F(u) = A u + u^2 - f = 0 by Newton).

Two entry points.  newton_solve: the semilinear form below, with the
Jacobian written down.  newton_solve_residual: any residual F(u, *params)
given as a torch callable whose Jacobian dF/du lies on a given sparsity
pattern (each F_i depends only on the u_j of row i's stored columns), with
parameters anywhere in it; the Jacobian's values are recovered from one
forward-mode product per color of hsla_pattern_colors, and the backward is
one adjoint solve J^T lambda = dL/du followed by the vector-Jacobian product
dL/dparams = -lambda^T dF/dparams through the residual (implicit function
theorem, Eq. adjoint_master).

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


# ---------------------------------------------------------------------------
# General residuals
# ---------------------------------------------------------------------------

class PatternJacobian:
    """Values, in the pattern's entry order, of a Jacobian whose sparsity
    lies on `pat`: J v_c for the indicator v_c of each color c of a column
    coloring in which columns sharing a row differ holds J_ij at row i for
    the single column j of color c stored in row i (Curtis, Powell and
    Reid)."""

    def __init__(self, pat):
        self.pat = pat
        self.colors, self.ncolors = pat.colors()
        counts = (pat.row_ptr[1:] - pat.row_ptr[:-1]).to(torch.int64)
        self.rows = torch.repeat_interleave(torch.arange(pat.n, device=pat.device), counts)
        self.key = self.colors.to(torch.int64)[pat.col.to(torch.int64)]

    def values(self, fn, u: torch.Tensor) -> torch.Tensor:
        import torch.autograd.forward_ad as fwAD

        jv = torch.empty((self.ncolors, u.numel()), dtype=u.dtype, device=u.device)
        with fwAD.dual_level():
            for c in range(self.ncolors):
                v = (self.colors == c).to(u.dtype)
                jv[c] = fwAD.unpack_dual(fn(fwAD.make_dual(u, v))).tangent
        return jv[self.key, self.rows].contiguous()


def _newton_general(jac, kw, residual, u0, params):
    """Newton on residual(u, *params) = 0 with the colored Jacobian; returns
    (u, J's values at u, steps, converged).  Runs outside autograd (forward
    mode carries the Jacobian products)."""
    dparams = tuple(p.detach() if isinstance(p, torch.Tensor) else p for p in params)

    def F(uu):
        return residual(uu, *dparams)

    pat = jac.pat
    u = u0.detach().clone()
    lin = _lib.make_opts(method=kw["method"], precond=kw["precond"], rtol=kw["lin_rtol"])
    r = F(u)
    r0 = float(torch.linalg.norm(r))
    its, converged = 0, r0 == 0.0
    for its in range(kw["max_newton"] + 1):
        if converged or float(torch.linalg.norm(r)) <= kw["tol"] * r0:
            converged = True
            break
        if its == kw["max_newton"]:
            break
        J = jac.values(F, u)
        d, _, st = _lib.solve(pat, J, r.contiguous(), lin)
        if st != _lib.OK:
            warnings.warn(f"Newton step {its}: linear solve status {_lib.status_string(st)}", RuntimeWarning)
        u = u - d
        r = F(u)
    if not converged:
        warnings.warn(f"Newton did not converge in {kw['max_newton']} steps", RuntimeWarning)
    return u, jac.values(F, u), its, converged


class ImplicitRootFn(torch.autograd.Function):
    """The root u of residual(u, *params) = 0 as a function of params
    (implicit function theorem): the forward passes the converged u through;
    the backward solves J^T lambda = dL/du once and returns
    -lambda^T dF/dparams from one vector-Jacobian product of the residual."""

    @staticmethod
    def forward(ctx, jac, kw, residual, u, J, converged, *params):
        ctx.jac, ctx.kw, ctx.residual, ctx.converged, ctx.J = jac, kw, residual, converged, J
        ctx.param_is_tensor = [isinstance(p, torch.Tensor) for p in params]
        ctx.params_nontensor = [None if isinstance(p, torch.Tensor) else p for p in params]
        ctx.save_for_backward(u, *[p for p in params if isinstance(p, torch.Tensor)])
        return u.clone()

    @staticmethod
    def backward(ctx, gu):
        if not ctx.converged:
            raise RuntimeError("backward through a Newton solve that did not converge")
        u, *tparams = ctx.saved_tensors
        opts = _lib.make_opts(method=ctx.kw["method"], precond=ctx.kw["precond"], rtol=ctx.kw["lin_rtol"])
        _, lam, _, st = _lib.adjoint(ctx.jac.pat, ctx.J, u, gu.contiguous(), opts, want_gA=False)
        if st != _lib.OK:
            warnings.warn(f"adjoint solve finished with status {_lib.status_string(st)}", RuntimeWarning)
        it = iter(tparams)
        params = [next(it) if t else v for t, v in zip(ctx.param_is_tensor, ctx.params_nontensor)]
        need = [i for i, p in enumerate(params) if isinstance(p, torch.Tensor) and ctx.needs_input_grad[6 + i]]
        grads = [None] * len(params)
        if need:
            with torch.enable_grad():
                leaves = [p.detach().requires_grad_(i in need) if isinstance(p, torch.Tensor) else p
                          for i, p in enumerate(params)]
                Fu = ctx.residual(u.detach(), *leaves)
                got = torch.autograd.grad(Fu, [leaves[i] for i in need], grad_outputs=-lam, allow_unused=True)
            for i, g in zip(need, got):
                grads[i] = g
        return (None, None, None, None, None, None, *grads)


def newton_solve_residual(residual, params=(), *, pattern, u0: torch.Tensor | None = None, tol: float = 1e-12,
                          lin_rtol: float = 1e-12, max_newton: int = 50, method: str = "auto",
                          precond: str = "jacobi", info: dict | None = None) -> torch.Tensor:
    """u with residual(u, *params) = 0, by Newton from u0 (default 0) until
    ||F(u)|| <= tol ||F(u0)||; differentiable in every tensor in params.

    residual: a torch callable (float64 vectors on the GPU) built from
    operations that support forward-mode differentiation (elementwise torch
    ops, SparseCSR.mv, ...).  pattern: a Pattern that holds the sparsity of
    dF/du (every row's diagonal stored when precond is "jacobi").  Each
    Newton step assembles J's values from ncolors Jacobian-vector products
    and runs one library solve (method "auto": CG when J is symmetric, else
    BiCGStab).  `info`, if given, receives the Newton steps and the number of
    colors."""
    if not hasattr(pattern, "_newton_jac"):
        pattern._newton_jac = PatternJacobian(pattern)
    jac = pattern._newton_jac
    kw = dict(tol=tol, lin_rtol=lin_rtol, max_newton=max_newton, method=method, precond=precond)
    if u0 is None:
        u0 = torch.zeros(pattern.n, dtype=torch.float64, device=pattern.device)
    with torch.no_grad():
        u, J, steps, converged = _newton_general(jac, kw, residual, u0, params)
    u = ImplicitRootFn.apply(jac, kw, residual, u, J, converged, *params)
    if info is not None:
        info["newton_steps"] = steps
        info["colors"] = jac.ncolors
    return u
