"""Oracle of s-step (communication-avoiding) CG.

TEST INFRASTRUCTURE: only tests/ use this module; it shares nothing with the
GPU path.

The paper names pipelined and communication-avoiding CG as the way forward
after its Algorithm "Distributed CG" (Appendix "Distributed Conjugate
Gradient and Halo Exchange"), without giving steps.  This follows the s-step
formulation of Chronopoulos and Gear as written out by Carson and Demmel
(CA-CG): per outer iteration

  1. a basis Y of the Krylov spaces of the current direction p (s + 1
     vectors) and residual r (s vectors), built with matrix products only;
  2. one Gram matrix G = Y^T Y -- the only reduction of the outer iteration;
  3. s CG steps carried out on coordinate vectors (length 2s + 1) in that
     basis: A Y c = Y (B c) for a fixed change-of-basis matrix B, so every
     inner product is c1^T G c2 and no vector is touched;
  4. the vectors recovered from the basis: x += Y x_c, r = Y r_c, p = Y p_c.

In exact arithmetic the k-th iterate is CG's k-th iterate.

Basis: Chebyshev polynomials on [0, 2]: T_0 = v, T_1 = (A - I) v,
T_{j+1} = 2 (A - I) T_j - T_{j-1}; hence A T_0 = T_0 + T_1 and
A T_j = (T_{j-1} + T_{j+1}) / 2 + T_j (j >= 1), which is B.  The interval
holds the spectrum of a Jacobi-scaled, diagonally dominant operator.

Jacobi preconditioning runs CG on A^ = S A S with S = D^{-1/2} and
b^ = S b (Jacobi-PCG on A in exact arithmetic); x = S x^.  The stop test is
taken after every inner step on the unscaled residual: ||S^{-1} r^||^2 =
r_c^T (Y^T S^{-2} Y) r_c.

Generic in the number type: float (numpy float64) or fractions.Fraction
(numpy object arrays) for exact arithmetic on tiny systems; precond "jacobi"
needs square roots and is float only.
"""
from __future__ import annotations

import math

import numpy as np

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 1, 2, 3


class SStepResult:
    def __init__(self, x, status, iters, relres):
        self.x, self.status, self.iters, self.relres = x, status, iters, relres

    def __repr__(self):
        return f"SStepResult(status={self.status}, iters={self.iters})"


def _matvec(rows, col, val, v):
    """y = A v, one product per stored entry (generic number type)."""
    y = np.zeros(len(v), dtype=v.dtype)
    if y.dtype == object:
        y[:] = [0 * v[0]] * len(v)
        for k in range(len(val)):
            y[rows[k]] = y[rows[k]] + val[k] * v[col[k]]
        return y
    np.add.at(y, rows, val * v[col])
    return y


def change_of_basis(s):
    """B with A Y c = Y (B c) for the basis [T_0..T_s of p, T_0..T_{s-1} of
    r]; the image of each block's last vector is not in the basis and is
    never needed (after j < s inner steps the coordinates of p use the first
    j + 1 entries of the p block and those of r the first j entries of the r
    block)."""
    nb = 2 * s + 1
    Bm = np.zeros((nb, nb), dtype=object)
    Bm[:, :] = 0
    for start, length in ((0, s + 1), (s + 1, s)):
        for j in range(length - 1):
            c = start + j
            if j == 0:
                Bm[c, c] = 1
                Bm[c + 1, c] = 1
            else:
                Bm[c - 1, c] = _half()
                Bm[c, c] = 1
                Bm[c + 1, c] = _half()
    return Bm


def _half():
    from fractions import Fraction

    return Fraction(1, 2)


def sstep_cg(a, b, s=4, precond="jacobi", rtol=1e-10, atol=0.0, max_iter=None, exact=False):
    """s-step CG on A x = b from x0 = 0.  `a` is a CSR (n, row_ptr, col,
    val); with exact=True the values and b are taken as exact rationals
    (precond "none" only).  max_iter caps the inner steps (default
    min(10 n, 100000)); the k-th iterate of a run capped at k is returned
    with status NOT_CONVERGED."""
    from fractions import Fraction

    n = a.n
    rows = np.repeat(np.arange(n), np.diff(a.row_ptr))
    col = np.asarray(a.col)
    if max_iter is None:
        max_iter = min(10 * n, 100000)
    if exact:
        if precond != "none":
            raise ValueError("exact arithmetic runs without the Jacobi scaling")
        val = np.array([Fraction(v) for v in a.val], dtype=object)
        bb = np.array([Fraction(v) for v in b], dtype=object)
        Bm = change_of_basis(s)
        zero = Fraction(0)
    else:
        val = np.asarray(a.val, dtype=np.float64)
        bb = np.asarray(b, dtype=np.float64)
        Bm = change_of_basis(s).astype(np.float64)
        zero = 0.0
    # Jacobi scaling: A^ = S A S, b^ = S b
    if precond == "jacobi":
        diag = np.zeros(n)
        for k in range(len(val)):
            if rows[k] == col[k]:
                diag[rows[k]] = val[k]
        if np.any(diag <= 0):
            return SStepResult(np.zeros(n), BREAKDOWN, 0, 1.0)
        S = 1.0 / np.sqrt(diag)
        ahat = val * S[rows] * S[col]
        w = 1.0 / (S * S)  # weights of the unscaled residual norm
        bh = S * bb
    else:
        S, ahat, bh = None, val, bb
        w = None
    bn2 = np.dot(bb, bb)
    bn = math.sqrt(float(bn2))
    tol = max(rtol * bn, atol)
    x = np.array([zero] * n, dtype=bh.dtype) if exact else np.zeros(n)
    r = bh.copy()
    p = r.copy()
    if bn <= tol:
        return SStepResult(x if S is None else S * x, OK, 0, 1.0 if bn > 0 else 0.0)
    if max_iter <= 0:
        return SStepResult(x if S is None else S * x, NOT_CONVERGED, 0, 1.0)
    nb = 2 * s + 1
    it, status, rr = 0, NOT_CONVERGED, bn2
    while True:
        # 1. basis: Chebyshev polynomials in (A^ - I) of p and of r
        Y = []
        for v0, length in ((p, s + 1), (r, s)):
            prev, cur = None, v0
            Y.append(cur)
            for j in range(1, length):
                t = _matvec(rows, col, ahat, cur) - cur
                nxt = t if j == 1 else 2 * t - prev
                prev, cur = cur, nxt
                Y.append(cur)
        Y = np.array(Y, dtype=bh.dtype)
        # 2. the Gram matrices (plain and with the unscaled-norm weights)
        G = Y @ Y.T
        Gw = G if w is None else (Y * w) @ Y.T
        # 3. s steps on coordinates
        pc = np.array([zero] * nb, dtype=Y.dtype)
        rc = pc.copy()
        xc = pc.copy()
        pc[0] = 1
        rc[s + 1] = 1
        rho = rc @ G @ rc
        stop = False
        for _ in range(s):
            bp = Bm @ pc
            sigma = pc @ G @ bp
            if not exact and not np.isfinite(sigma):
                status, stop = NONFINITE, True
                break
            if not sigma > 0:
                status, stop = BREAKDOWN, True
                break
            alpha = rho / sigma
            xc = xc + alpha * pc
            rc = rc - alpha * bp
            it += 1
            rr = rc @ Gw @ rc
            if exact:
                done = rr <= tol * tol
            else:
                if not np.isfinite(rr):
                    status, stop = NONFINITE, True
                    break
                done = math.sqrt(max(rr, 0.0)) <= tol
            if done:
                status, stop = OK, True
                break
            if it >= max_iter:
                status, stop = NOT_CONVERGED, True
                break
            rho_new = rc @ G @ rc
            beta = rho_new / rho
            rho = rho_new
            pc = rc + beta * pc
        # 4. recovery
        x = x + Y.T @ xc
        if stop:
            break
        r = Y.T @ rc
        p = Y.T @ pc
    xo = x if S is None else S * x
    rel = math.sqrt(max(float(rr), 0.0)) / bn if bn > 0 else math.sqrt(max(float(rr), 0.0))
    return SStepResult(xo, status, it, rel)
