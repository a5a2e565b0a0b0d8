"""Symmetric eigensolve with the Hellmann-Feynman gradient (Sec. "Adjoint
Differentiation", paragraph "Eigenvalue problems", Eq. adjoint_eig: for a
simple eigenpair A v = lambda v, ||v|| = 1, dlambda/dA_ij = v_i v_j on the
pattern; Table tab:gradient, the .eigsh entry point).

The k smallest eigenpairs of a symmetric positive definite A come from
Lanczos with full reorthogonalisation on A^{-1} (shift-invert at 0): every
Lanczos step is one library CG solve, so the well-separated large
eigenvalues 1/lambda of A^{-1} converge in a few dozen steps where Lanczos on
A would need hundreds.  The largest eigenpairs use Lanczos on A (one library
SpMV per step).  Ritz vectors are refined into Rayleigh quotients with the
library SpMV and checked by their residuals ||A v - lambda v||.  The backward
of the eigenvalues is one on-pattern outer-product launch
(hsla_outer_on_pattern) over the k eigenvectors; eigenvector gradients
(which need a deflated solve per pair) are not provided."""
from __future__ import annotations

import warnings

import torch

from . import SparseCSR, _lib


def _lanczos(apply, n, k, device, tol, max_steps, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    q = torch.randn(n, generator=g, dtype=torch.float64).to(device)
    q /= torch.linalg.norm(q)
    Q = torch.empty((max_steps + 1, n), dtype=torch.float64, device=device)
    Q[0] = q
    alpha, beta = [], []
    theta = S = None
    m = 0
    for j in range(max_steps):
        w = apply(Q[j])
        a = float(Q[j] @ w)
        w = w - a * Q[j] - (beta[-1] * Q[j - 1] if j > 0 else 0.0)
        for _ in range(2):  # full reorthogonalisation, twice
            w = w - Q[: j + 1].T @ (Q[: j + 1] @ w)
        b = float(torch.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        m = j + 1
        if m >= k and (m % 4 == 0 or b == 0.0 or m == max_steps):
            T = torch.diag(torch.tensor(alpha, dtype=torch.float64))
            if m > 1:
                off = torch.tensor(beta[: m - 1], dtype=torch.float64)
                T = T + torch.diag(off, 1) + torch.diag(off, -1)
            theta, S = torch.linalg.eigh(T)
            res = b * S[-1, :].abs()
            top = torch.argsort(theta, descending=True)[:k]
            if bool((res[top] <= tol * theta[top].abs()).all()) or b == 0.0:
                break
        if b == 0.0:
            break
        Q[j + 1] = w / b
    top = torch.argsort(theta, descending=True)[:k]
    return theta[top], Q[:m].T @ S[:, top].to(device), m


class EigshFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, pat, V):
        ctx.pat = pat
        ctx.save_for_backward(V)
        lam = torch.stack([V[:, j] @ _lib.spmv(pat, values.detach(), V[:, j].contiguous())
                           for j in range(V.shape[1])])
        return lam

    @staticmethod
    def backward(ctx, glam):
        (V,) = ctx.saved_tensors
        # dL/dA_ij = sum_j glam_j v_j[i] v_j[j]; the kernel forms -lam[row] x[col]
        lamv = (-(V * glam)).T.contiguous()
        x = V.T.contiguous()
        gA = _lib.outer_on_pattern(ctx.pat, lamv, x).sum(dim=0)
        return gA, None, None


def eigsh(A: SparseCSR, k: int = 6, which: str = "SA", tol: float = 1e-12, max_steps: int = 300,
          solve_rtol: float = 1e-14, seed: int = 0, info: dict | None = None):
    """(eigenvalues (k,), eigenvectors (n, k)) of symmetric A, the k smallest
    ("SA", A positive definite) or largest ("LA") in ascending order;
    eigenvalues are differentiable in A's values (Hellmann-Feynman).  `info`
    receives the Lanczos steps and the largest relative residual."""
    pat, vals = A.pattern, A.values.detach()
    n = A.n
    if which == "SA":
        opts = _lib.make_opts(method="cg", precond="jacobi", rtol=solve_rtol)

        def apply(q):
            x, _, st = _lib.solve(pat, vals, q.contiguous(), opts)
            if st != _lib.OK:
                warnings.warn(f"eigsh: inner solve status {_lib.status_string(st)}", RuntimeWarning)
            return x
    elif which == "LA":
        def apply(q):
            return _lib.spmv(pat, vals, q.contiguous())
    else:
        raise ValueError("which must be 'SA' or 'LA'")
    theta, V, steps = _lanczos(apply, n, k, vals.device, tol, min(max_steps, n), seed)
    V = V / torch.linalg.norm(V, dim=0)
    lam = EigshFn.apply(A.values, pat, V.contiguous())
    order = torch.argsort(lam.detach())
    lam, V = lam[order], V[:, order]
    if info is not None:
        R = torch.stack([_lib.spmv(pat, vals, V[:, j].contiguous()) for j in range(k)], 1) - V * lam.detach()
        info["lanczos_steps"] = steps
        info["max_rel_residual"] = float((torch.linalg.norm(R, dim=0) / lam.detach().abs()).max())
    return lam, V
