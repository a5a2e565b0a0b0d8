"""Oracle of the inverse coefficient problem (Sec. "End-to-End: Inverse
Coefficient Learning", Eq. for -div(kappa grad u) = f with u = 0 on the
boundary of (0, 1)^2).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: plain numpy loops and the
C oracle's CG and adjoint; nothing here is shared with the GPU path.

Readings (the paper names the discretisation only as cell-centred five-point
finite differences on a 64 x 64 grid):

* cells of size h = 1/m, unknown u_P at the centre of cell P;
* the flux coefficient of the face between cells P and Q is the harmonic
  mean 2 kappa_P kappa_Q / (kappa_P + kappa_Q), divided by h^2;
* a face on the boundary lies h/2 from the cell centre, where u = 0: its
  coefficient is 2 kappa_P / h^2;
* (A u)_P = sum over P's faces of t_face (u_P - u_other), u_other = 0 on the
  boundary; f = 1;
* loss L = ||u - u_obs||^2 + 1e-3 ||grad_h kappa||^2 / N, grad_h the
  differences of kappa between neighbouring cells (not divided by h: divided
  by h, the term is about 5e-3 at kappa* and would outweigh a misfit small
  enough for the paper's 0.23% coefficient error), N = m^2;
* kappa = softplus(theta), theta starts at softplus^-1(1) (kappa = 1).
"""
from __future__ import annotations

import numpy as np

import oracle
from workloads import Csr

REG = 1e-3


def softplus(theta):
    return np.log1p(np.exp(theta))


def faces(m: int):
    """Interior faces (P, Q) with Q = P + 1 (x) or P + m (y), in a fixed order."""
    out = []
    for iy in range(m):
        for ix in range(m):
            p = iy * m + ix
            if ix + 1 < m:
                out.append((p, p + 1))
            if iy + 1 < m:
                out.append((p, p + m))
    return out


def walls(m: int):
    """Number of boundary faces of every cell."""
    w = np.zeros(m * m, dtype=np.int64)
    for iy in range(m):
        for ix in range(m):
            w[iy * m + ix] = (ix == 0) + (ix == m - 1) + (iy == 0) + (iy == m - 1)
    return w


def assemble(kappa, m: int) -> Csr:
    """A(kappa) in canonical CSR (columns ascending in every row)."""
    n = m * m
    h2 = (1.0 / m) ** 2
    rows = {p: {} for p in range(n)}
    diag = np.zeros(n)
    for p, q in faces(m):
        t = 2.0 * kappa[p] * kappa[q] / (kappa[p] + kappa[q]) / h2
        rows[p][q] = -t
        rows[q][p] = -t
        diag[p] += t
        diag[q] += t
    w = walls(m)
    for p in range(n):
        diag[p] += w[p] * 2.0 * kappa[p] / h2
        rows[p][p] = diag[p]
    rp = np.zeros(n + 1, dtype=np.int32)
    col, val = [], []
    for p in range(n):
        for q in sorted(rows[p]):
            col.append(q)
            val.append(rows[p][q])
        rp[p + 1] = len(col)
    return Csr(n, rp, np.array(col, dtype=np.int32), np.array(val))


def regulariser(kappa, m: int):
    """||grad_h kappa||^2 / N and its gradient with respect to kappa."""
    r = 0.0
    g = np.zeros(m * m)
    for p, q in faces(m):
        d = kappa[q] - kappa[p]
        r += d * d
        g[q] += 2.0 * d
        g[p] -= 2.0 * d
    return r / (m * m), g / (m * m)


def observe(m: int, kappa_true, f, rtol=1e-12):
    return oracle.cg(assemble(kappa_true, m), f, precond="jacobi", rtol=rtol).x


def loss_and_grad(theta, m: int, u_obs, f, rtol=1e-12):
    """(L, dL/dtheta, u): forward solve, adjoint (A symmetric: CG on A), the
    on-pattern gradient dL/dA_ij = -lambda_i u_j (Eq. adjoint_linear), and
    the chain rule through the face coefficients, kappa and softplus."""
    kappa = softplus(theta)
    a = assemble(kappa, m)
    u = oracle.cg(a, f, precond="jacobi", rtol=rtol).x
    e = u - u_obs
    reg, greg = regulariser(kappa, m)
    loss = float(e @ e) + REG * reg
    gA, _, _ = oracle.adjoint(a, u, 2.0 * e, method="cg", precond="jacobi", rtol=rtol)
    # dL/dA for each (row, col) of the pattern
    g = {}
    for p in range(a.n):
        for k in range(a.row_ptr[p], a.row_ptr[p + 1]):
            g[(p, int(a.col[k]))] = gA[k]
    h2 = (1.0 / m) ** 2
    gk = REG * greg
    for p, q in faces(m):
        # t enters A_pp, A_qq with +1 and A_pq, A_qp with -1
        dt = g[(p, p)] + g[(q, q)] - g[(p, q)] - g[(q, p)]
        s = kappa[p] + kappa[q]
        gk[p] += dt * 2.0 * kappa[q] ** 2 / (s * s) / h2
        gk[q] += dt * 2.0 * kappa[p] ** 2 / (s * s) / h2
    w = walls(m)
    for p in range(a.n):
        gk[p] += g[(p, p)] * w[p] * 2.0 / h2
    sig = 1.0 / (1.0 + np.exp(-theta))
    return loss, gk * sig, u


def adam(theta, grad, state, lr=5e-2, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in place; state = {"t", "m", "v"}."""
    state["t"] += 1
    state["m"] = b1 * state["m"] + (1 - b1) * grad
    state["v"] = b2 * state["v"] + (1 - b2) * grad * grad
    mh = state["m"] / (1 - b1 ** state["t"])
    vh = state["v"] / (1 - b2 ** state["t"])
    theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta
