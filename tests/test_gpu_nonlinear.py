"""Nonlinear solve with the adjoint gradient on the GPU (F(u) = A u + u^2 -
f, Newton; Sec. "Adjoint Differentiation", paragraph "Nonlinear systems"):
u, the Newton step count and dL/dA, dL/df against the oracle, the paper's
finite-difference protocol (epsilon = 1e-5) through the GPU, and the
one-node autograd graph."""
import warnings

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, rel, t32, t64  # noqa: E402
import paper_2601_13994_amd as hs  # noqa: E402
from paper_2601_13994_amd import nonlinear  # noqa: E402
from oracle import nonlinear as ON  # noqa: E402


def _problem(m, seed):
    p = W.poisson2d(m)
    a = p.with_values(p.val * (m + 1) ** 2)
    r = np.random.default_rng(seed)
    return a, 1.0 + 0.5 * r.standard_normal(a.n), r


@pytest.mark.parametrize("m", [12, 64])
def test_newton_and_gradients_match_oracle(orc, m):
    a, f, r = _problem(m, 5)
    ustar = r.standard_normal(a.n)
    vals = t64(a.val).requires_grad_(True)
    ft = t64(f).requires_grad_(True)
    A = hs.SparseCSR(vals, t32(a.row_ptr), t32(a.col))
    info = {}
    u = nonlinear.newton_solve(A, ft, tol=1e-13, lin_rtol=1e-14, info=info)
    uo, its = ON.newton(a, f, tol=1e-13)
    assert rel(u.detach().cpu().numpy(), uo) <= 1e-10
    assert abs(info["newton_steps"] - its) <= 1 and its <= 8
    loss = 0.5 * ((u - t64(ustar)) ** 2).sum()
    assert type(u.grad_fn).__name__ == "NewtonSolveFnBackward"  # one node for all Newton steps
    loss.backward()
    gA, gf = ON.gradients(a, uo, uo - ustar)
    assert rel(vals.grad.cpu().numpy(), gA) <= 1e-6
    assert rel(ft.grad.cpu().numpy(), gf) <= 1e-6


def test_paper_fd_protocol():
    """Central differences at epsilon = 1e-5 on 16 random entries of A and
    of f, every L evaluated by GPU Newton solves: relative error of the
    2-norm over the picks below 1e-5 (the paper reports 4.7e-7)."""
    m = 16
    a, f, r = _problem(m, 6)
    c = t64(r.standard_normal(a.n))
    rp, col = t32(a.row_ptr), t32(a.col)
    pat = hs.Pattern(rp, col)

    def L(v, ff):
        with torch.no_grad():
            A = hs.SparseCSR(v, rp, col, pattern=pat)
            return float(c @ nonlinear.newton_solve(A, ff, tol=1e-14, lin_rtol=1e-14))

    vals = t64(a.val).requires_grad_(True)
    ft = t64(f).requires_grad_(True)
    u = nonlinear.newton_solve(hs.SparseCSR(vals, rp, col, pattern=pat), ft, tol=1e-14, lin_rtol=1e-14)
    (c @ u).backward()
    eps = 1e-5
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        ka = r.choice(a.nnz, 16, replace=False)
        fa = []
        for k in ka:
            vp, vm = t64(a.val), t64(a.val)
            vp[k] += eps
            vm[k] -= eps
            fa.append((L(vp, t64(f)) - L(vm, t64(f))) / (2 * eps))
        kf = r.choice(a.n, 16, replace=False)
        ff = []
        for k in kf:
            fp, fm = t64(f), t64(f)
            fp[k] += eps
            fm[k] -= eps
            ff.append((L(t64(a.val), fp) - L(t64(a.val), fm)) / (2 * eps))
    ga = vals.grad.cpu().numpy()[ka]
    gf = ft.grad.cpu().numpy()[kf]
    ea = np.linalg.norm(np.array(fa) - ga) / np.linalg.norm(ga)
    ef = np.linalg.norm(np.array(ff) - gf) / np.linalg.norm(gf)
    print("[nonlinear] fd", ea, ef, flush=True)
    assert ea <= 1e-5 and ef <= 1e-5
