"""hsla: differentiable sparse Krylov solves on one MI355X.

The user-facing mirror of the paper's API (arXiv 2601.13994, Sec. "API" and
the appendix listing):

    A = SparseCSR(values, row_ptr, col, shape=(n, n))   # values (nnz,) or (B, nnz)
    x = A.solve(b)                                      # CG if A is symmetric, else BiCGStab
    loss(x).backward()                                  # adjoint gradients, one graph node

Every numerical step runs in libhsla.so (hand-written HIP for gfx950); this
package only marshals torch tensors into the C ABI.
"""
from __future__ import annotations

import warnings

import torch

from . import _lib
from ._lib import HslaError, Pattern

__all__ = ["SparseCSR", "SparseCSRList", "SolveFn", "SpMVFn", "HslaError", "Pattern", "from_coo"]


class SolveFn(torch.autograd.Function):
    """x = A(values)^{-1} b with the implicit-function adjoint (Eq.
    adjoint_master / adjoint_linear): the forward runs without building an
    autograd graph and stashes only (values, x); the backward solves
    A^T lambda = dL/dx once and returns dL/db = lambda and
    dL/dA_k = -lambda[row(k)] x[col(k)] on the pattern."""

    @staticmethod
    def forward(ctx, values, b, pat, opts_kw, allow_unconverged):
        opts = _lib.make_opts(**opts_kw)
        x, infos, st = _lib.solve(pat, values.detach(), b.detach(), opts)
        if st != _lib.OK:
            msg = f"solve finished with status {_lib.status_string(st)} ({infos[0] if len(infos) == 1 else ''})"
            warnings.warn(msg, RuntimeWarning, stacklevel=3)
        ctx.pat = pat
        ctx.opts_kw = {k: v for k, v in opts_kw.items() if k not in ("G", "GT", "x0")}
        ctx.opts_kw["precond"] = "jacobi" if opts_kw.get("precond") == "fsai" else opts_kw.get("precond", "jacobi")
        ctx.status = st
        ctx.allow_unconverged = allow_unconverged
        ctx.infos = infos
        ctx.save_for_backward(values, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        values, x = ctx.saved_tensors
        if ctx.status != _lib.OK and not ctx.allow_unconverged:
            raise RuntimeError("backward through a solve that did not converge (status "
                               f"{_lib.status_string(ctx.status)}); the adjoint would be biased. "
                               "Pass allow_unconverged=True to proceed anyway.")
        opts = _lib.make_opts(**ctx.opts_kw)
        want_gA = ctx.needs_input_grad[0]
        gA, gb, _, st = _lib.adjoint(ctx.pat, values.detach(), x, gx.contiguous(), opts, want_gA=want_gA)
        if st != _lib.OK:
            warnings.warn(f"adjoint solve finished with status {_lib.status_string(st)}", RuntimeWarning)
        return (gA if want_gA else None), (gb if ctx.needs_input_grad[1] else None), None, None, None


class SpMVFn(torch.autograd.Function):
    """y = A(values) x, differentiable in reverse mode (dL/dvalues_k =
    g[row(k)] x[col(k)] on the pattern, dL/dx = A^T g) and forward mode
    (d y = A dx + A(d values) x), so that residuals built from it can be
    differentiated with torch.autograd.forward_ad (the Jacobian products of
    the general Newton solve) and torch.autograd.grad (its adjoint
    gradient)."""

    @staticmethod
    def forward(values, x, A):
        return _lib.spmv(A.pattern, values.detach(), x.detach().contiguous())

    @staticmethod
    def setup_context(ctx, inputs, output):
        values, x, A = inputs
        ctx.A = A
        ctx.save_for_backward(values, x)
        ctx.save_for_forward(values, x)

    @staticmethod
    def backward(ctx, g):
        values, x = ctx.saved_tensors
        A = ctx.A
        g = g.contiguous()
        gv = _lib.outer_on_pattern(A.pattern, -g, x.detach()) if ctx.needs_input_grad[0] else None
        gx = A._transpose_mv(values.detach(), g) if ctx.needs_input_grad[1] else None
        return gv, gx, None

    @staticmethod
    def jvp(ctx, dvalues, dx, _):
        values, x = ctx.saved_tensors
        A = ctx.A
        out = None
        if dx is not None:
            out = _lib.spmv(A.pattern, values.detach(), dx.contiguous())
        if dvalues is not None:
            t = _lib.spmv(A.pattern, dvalues.contiguous(), x.detach().contiguous())
            out = t if out is None else out + t
        return out


class SparseCSR:
    """A square sparse matrix (or a batch sharing one pattern) in CSR form.

    values: float64 (nnz,) or (B, nnz); row_ptr: int32 (n+1,); col: int32 (nnz,),
    canonical (columns strictly increasing per row).  All on one GPU."""

    def __init__(self, values: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor, shape=None,
                 pattern: Pattern | None = None):
        self.values = values
        n = row_ptr.numel() - 1
        if shape is not None and (shape[-1] != n or shape[-2] != n):
            raise ValueError(f"shape {shape} does not match row_ptr (n = {n})")
        self.n = n
        self.pattern = pattern if pattern is not None else Pattern(row_ptr, col)

    @property
    def batch(self) -> int | None:
        return self.values.shape[0] if self.values.dim() == 2 else None

    @property
    def shape(self):
        return (self.n, self.n) if self.batch is None else (self.batch, self.n, self.n)

    def with_values(self, values: torch.Tensor) -> "SparseCSR":
        return SparseCSR(values, self.pattern.row_ptr, self.pattern.col, pattern=self.pattern)

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        """y = A x (not differentiable; SpMV in FP64)."""
        return _lib.spmv(self.pattern, self.values.detach(), x)

    __matmul__ = matvec

    def mv(self, x: torch.Tensor) -> torch.Tensor:
        """y = A x, differentiable in the values and x (reverse and forward
        mode; see SpMVFn)."""
        return SpMVFn.apply(self.values, x, self)

    def _transpose_mv(self, values: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
        """A^T g on the transpose pattern (built once per matrix)."""
        if not hasattr(self, "_tpat"):
            rpT, colT, src = self.pattern.transpose()
            self._tpat = Pattern(rpT, colT)
            self._tsrc = src.to(torch.int64)
        return _lib.spmv(self._tpat, values[..., self._tsrc].contiguous(), g)

    def solve(self, b: torch.Tensor, *, rtol: float = 1e-8, atol: float = 0.0, method: str = "auto",
              precond: str = "jacobi", max_iter: int = 0, check_every: int = 0, graph: bool = True,
              allow_unconverged: bool = False, G: torch.Tensor | None = None,
              GT: torch.Tensor | None = None) -> torch.Tensor:
        """x = A^{-1} b; differentiable w.r.t. values and b (one autograd node)."""
        opts_kw = dict(method=method, precond=precond, rtol=rtol, atol=atol, max_iter=max_iter,
                       check_every=check_every, graph=graph, G=G, GT=GT)
        return SolveFn.apply(self.values, b, self.pattern, opts_kw, allow_unconverged)

    def solve_info(self, b: torch.Tensor, **kw):
        """Non-differentiable solve returning (x, per-system info dicts, status)."""
        G, GT = kw.pop("G", None), kw.pop("GT", None)
        x0 = kw.pop("x0", None)
        opts = _lib.make_opts(G=G, GT=GT, x0=x0 is not None, **kw)
        return _lib.solve(self.pattern, self.values.detach(), b.detach(), opts, x0=x0)


def from_coo(values: torch.Tensor, row: torch.Tensor, col: torch.Tensor, n: int) -> SparseCSR:
    """CSR from COO triplets (the paper's storage).  Entries are sorted by
    (row, col) with a differentiable gather of the values; duplicates are
    rejected."""
    key = row.to(torch.int64) * n + col.to(torch.int64)
    order = torch.argsort(key, stable=True)
    k = key[order]
    if k.numel() > 1 and bool((k[1:] == k[:-1]).any()):
        raise ValueError("duplicate (row, col) entries")
    r = row.to(torch.int64)[order]
    counts = torch.bincount(r, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=row.device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    vals = values[..., order]
    return SparseCSR(vals, row_ptr.to(torch.int32), col.to(torch.int32)[order].contiguous(), shape=(n, n))


class SparseCSRList:
    """Matrices with distinct sparsity patterns and sizes (the paper's matrix
    list); solved together in one persistent launch, or, for large batches,
    by per-iteration kernels over all systems at once.  Each element is given
    as (values float64 (nnz_s,), row_ptr int32 (n_s+1,), col int32 (nnz_s,))
    tensors on one GPU; they are concatenated once here."""

    def __init__(self, mats):
        self.n = [int(rp.numel()) - 1 for _, rp, _ in mats]
        self.nnz = [int(c.numel()) for _, _, c in mats]
        dev = mats[0][1].device
        self.device = dev
        ro = [0]
        no = [0]
        for n, z in zip(self.n, self.nnz):
            ro.append(ro[-1] + n)
            no.append(no[-1] + z)
        self.row_off = torch.tensor(ro, dtype=torch.int64, device=dev)
        self.nnz_off = torch.tensor(no, dtype=torch.int64, device=dev)
        self.row_ptr = torch.cat([rp.to(torch.int32) for _, rp, _ in mats]).contiguous()
        self.col = torch.cat([c.to(torch.int32) for _, _, c in mats]).contiguous()
        self.values = torch.cat([v.to(torch.float64) for v, _, _ in mats]).contiguous()

    def __len__(self):
        return len(self.n)

    def split(self, v: torch.Tensor):
        return list(torch.split(v, self.n))

    def solve(self, bs, rtol: float = 1e-8, atol: float = 0.0, precond: str = "jacobi", max_iter: int = 0,
              persistent: bool | str = True):
        """Solves every system; `bs` is a list of right-hand sides or their
        concatenation.  persistent=False always takes the segmented
        per-iteration path (large batches take it anyway); "force" always the
        persistent launch.  Returns (list of x, infos, status)."""
        b = torch.cat(list(bs)) if isinstance(bs, (list, tuple)) else bs
        opts = _lib.make_opts(method="cg", precond=precond, rtol=rtol, atol=atol, max_iter=max_iter,
                              persistent=persistent)
        x, infos, st = _lib.solve_ragged(self.row_off, self.nnz_off, self.row_ptr, self.col, self.values, b, opts)
        return self.split(x), infos, st
