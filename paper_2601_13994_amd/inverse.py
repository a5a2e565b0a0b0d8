"""Inverse coefficient learning (Sec. "End-to-End: Inverse Coefficient
Learning"): recover kappa in -div(kappa grad u) = f on (0, 1)^2, u = 0 on the
boundary, from u_obs, with kappa = softplus(theta), the cell-centred
five-point operator assembled from kappa by differentiable torch ops on the
GPU, u = A(kappa).solve(f) through the library's adjoint (one autograd node,
no user-level autograd.Function) and Adam on ||u - u_obs||^2 plus a
1e-3 ||grad_h kappa||^2 / N smoothness term.

Discretisation (cells of size h = 1/m): the face between neighbouring cells
P and Q carries 2 kappa_P kappa_Q / (kappa_P + kappa_Q) / h^2; a boundary
face, h/2 from the cell centre where u = 0, carries 2 kappa_P / h^2;
(A u)_P = sum over faces of t (u_P - u_other).  The pattern is built once;
each step only recomputes the values."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import SparseCSR
from ._lib import Pattern

REG = 1e-3


class VarCoefPoisson2D:
    """The m x m cell-centred operator: fixed CSR pattern on the GPU and a
    differentiable map kappa (m*m,) -> CSR values."""

    def __init__(self, m: int, device):
        self.m, self.n = m, m * m
        self.device = torch.device(device)
        n = self.n
        idx = np.arange(n).reshape(m, m)  # [iy, ix]
        # value sources, concatenated: [diag (n), x faces (m*(m-1)), y faces ((m-1)*m)]
        nx = m * (m - 1)
        xface = np.arange(nx).reshape(m, m - 1)  # face between (iy, ix) and (iy, ix+1)
        yface = np.arange((m - 1) * m).reshape(m - 1, m)  # between (iy, ix) and (iy+1, ix)
        rows, cols, src = [], [], []
        for iy in range(m):
            for ix in range(m):
                p = idx[iy, ix]
                ent = [(p, p, p)]
                if iy > 0:
                    ent.append((p, p - m, n + nx + yface[iy - 1, ix]))
                if ix > 0:
                    ent.append((p, p - 1, n + xface[iy, ix - 1]))
                if ix + 1 < m:
                    ent.append((p, p + 1, n + xface[iy, ix]))
                if iy + 1 < m:
                    ent.append((p, p + m, n + nx + yface[iy, ix]))
                for r, c, s in sorted(ent, key=lambda e: e[1]):
                    rows.append(r)
                    cols.append(c)
                    src.append(s)
        rp = np.zeros(n + 1, dtype=np.int32)
        np.cumsum(np.bincount(np.array(rows), minlength=n), out=rp[1:])
        self.row_ptr = torch.as_tensor(rp, device=self.device)
        self.col = torch.as_tensor(np.array(cols, dtype=np.int32), device=self.device)
        self.src = torch.as_tensor(np.array(src, dtype=np.int64), device=self.device)
        nwall = ((idx % m == 0).astype(int) + (idx % m == m - 1) + (idx // m == 0) + (idx // m == m - 1))
        self.walls = torch.as_tensor(nwall.reshape(-1).astype(np.float64), device=self.device)
        self.pattern = Pattern(self.row_ptr, self.col)

    def values(self, kappa: torch.Tensor) -> torch.Tensor:
        """CSR values of A(kappa) (float64, differentiable in kappa)."""
        m = self.m
        inv_h2 = float(m * m)
        K = kappa.view(m, m)
        tx = 2.0 * K[:, :-1] * K[:, 1:] / (K[:, :-1] + K[:, 1:]) * inv_h2  # (m, m-1)
        ty = 2.0 * K[:-1, :] * K[1:, :] / (K[:-1, :] + K[1:, :]) * inv_h2  # (m-1, m)
        zc = K.new_zeros(m, 1)
        zr = K.new_zeros(1, m)
        diag = (torch.cat([zc, tx], 1) + torch.cat([tx, zc], 1) + torch.cat([zr, ty], 0) + torch.cat([ty, zr], 0))
        diag = diag.reshape(-1) + self.walls * (2.0 * inv_h2) * kappa
        srcv = torch.cat([diag, -tx.reshape(-1), -ty.reshape(-1)])
        return srcv[self.src]

    def matrix(self, kappa: torch.Tensor) -> SparseCSR:
        return SparseCSR(self.values(kappa), self.row_ptr, self.col, pattern=self.pattern)


def regulariser(kappa: torch.Tensor, m: int) -> torch.Tensor:
    """||grad_h kappa||^2 / N: squared differences of neighbouring cells."""
    K = kappa.view(m, m)
    dx = K[:, 1:] - K[:, :-1]
    dy = K[1:, :] - K[:-1, :]
    return ((dx * dx).sum() + (dy * dy).sum()) / (m * m)


class InverseProblem:
    """Learns kappa from u_obs = A(kappa_true)^{-1} f (observed by a GPU
    solve); theta starts at softplus^-1(1), i.e. kappa = 1."""

    def __init__(self, kappa_true: np.ndarray, f: np.ndarray, m: int = 64, device="cuda", rtol: float = 1e-12,
                 lr: float = 5e-2):
        self.m = m
        self.op = VarCoefPoisson2D(m, device)
        dev = self.op.device
        self.rtol = rtol
        self.kappa_true = torch.as_tensor(kappa_true, dtype=torch.float64, device=dev)
        self.f = torch.as_tensor(f, dtype=torch.float64, device=dev)
        with torch.no_grad():
            self.u_obs = self.op.matrix(self.kappa_true).solve(self.f, rtol=rtol, method="cg")
        self.theta = torch.nn.Parameter(torch.full((m * m,), math.log(math.e - 1.0), dtype=torch.float64, device=dev))
        self.opt = torch.optim.Adam([self.theta], lr=lr)

    def kappa(self) -> torch.Tensor:
        return torch.nn.functional.softplus(self.theta)

    def loss(self, theta: torch.Tensor | None = None):
        """(L, u) at theta (default: the parameter)."""
        th = self.theta if theta is None else theta
        kappa = torch.nn.functional.softplus(th)
        u = self.op.matrix(kappa).solve(self.f, rtol=self.rtol, method="cg")
        e = u - self.u_obs
        return (e * e).sum() + REG * regulariser(kappa, self.m), u

    def step(self) -> float:
        self.opt.zero_grad(set_to_none=True)
        loss, _ = self.loss()
        loss.backward()
        self.opt.step()
        return float(loss.detach())

    def errors(self):
        """(||kappa - kappa*|| / ||kappa*||, ||u(kappa) - u_obs|| / ||u_obs||, min kappa, max kappa)."""
        with torch.no_grad():
            k = self.kappa()
            u = self.op.matrix(k).solve(self.f, rtol=self.rtol, method="cg")
            ek = float(torch.linalg.norm(k - self.kappa_true) / torch.linalg.norm(self.kappa_true))
            eu = float(torch.linalg.norm(u - self.u_obs) / torch.linalg.norm(self.u_obs))
            return ek, eu, float(k.min()), float(k.max())
