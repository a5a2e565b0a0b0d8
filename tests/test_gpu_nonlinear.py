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


# ---------------------------------------------------------------- general residuals

def test_general_residual_cubic_with_parameter(orc):
    """F(u; values, f, k) = A(values) u + k u^3 - f with k inside the
    nonlinearity, solved by newton_solve_residual (Jacobian from colored
    forward-mode products through SparseCSR.mv): u and the gradients w.r.t.
    every stored value, f and k against the dense oracle."""
    a, f, r = _problem(16, 8)
    w = r.standard_normal(a.n)
    vals = t64(a.val).requires_grad_(True)
    ft = t64(f).requires_grad_(True)
    kt = torch.tensor(0.8, dtype=torch.float64, device=dev(), requires_grad=True)
    A = hs.SparseCSR(vals, t32(a.row_ptr), t32(a.col))

    def res(u, v, ff, kk):
        return A.with_values(v).mv(u) + kk * u ** 3 - ff

    info = {}
    u = nonlinear.newton_solve_residual(res, (vals, ft, kt), pattern=A.pattern, tol=1e-13, lin_rtol=1e-14,
                                        info=info)
    (t64(w) * u).sum().backward()
    rows = torch.as_tensor(a.rows())
    cols = torch.as_tensor(a.col.astype(np.int64))

    def res_dense(uu, v, ff, kk):
        Ad = torch.zeros(a.n, a.n, dtype=torch.float64).index_put((rows, cols), v)
        return Ad @ uu + kk * uu ** 3 - ff

    pc = (torch.as_tensor(a.val), torch.as_tensor(f), torch.tensor(0.8, dtype=torch.float64))
    u_ref, its = ON.newton_general(res_dense, a.n, pc)
    assert rel(u.detach().cpu().numpy(), u_ref) <= 1e-10
    assert 5 <= info["colors"] <= 9 and info["newton_steps"] <= its + 1
    (gv, gf, gk), _ = ON.gradients_general(res_dense, u_ref, pc, w)
    assert rel(vals.grad.cpu().numpy(), gv) <= 1e-8
    assert rel(ft.grad.cpu().numpy(), gf) <= 1e-8
    assert abs(float(kt.grad) - float(gk)) <= 1e-8 * abs(float(gk))


def test_general_residual_nonlinear_diffusion(orc):
    """A residual with a nonsymmetric Jacobian on the 5-point pattern
    (kappa depends on u on every face): u and dL/dkappa, dL/df against the
    dense oracle; the Newton steps' linear solves run BiCGStab."""
    from test_oracle_nonlinear import nl_diffusion

    m = 14
    pat_a = W.poisson2d(m)
    r = np.random.default_rng(9)
    kap = np.exp(0.3 * r.standard_normal(m * m))
    f = 1.0 + 0.3 * r.standard_normal(m * m)
    w = r.standard_normal(m * m)
    kt = t64(kap).requires_grad_(True)
    ft = t64(f).requires_grad_(True)
    from gpu_common import pattern
    pat = pattern(pat_a)

    def res(u, kk, ff):
        return nl_diffusion(u, kk, ff, m)

    info = {}
    u = nonlinear.newton_solve_residual(res, (kt, ft), pattern=pat, tol=1e-13, lin_rtol=1e-14, info=info)
    (t64(w) * u).sum().backward()
    pc = (torch.as_tensor(kap), torch.as_tensor(f))
    u_ref, _ = ON.newton_general(lambda uu, a1, a2: nl_diffusion(uu, a1, a2, m), m * m, pc)
    assert rel(u.detach().cpu().numpy(), u_ref) <= 1e-10
    (gk, gf), _ = ON.gradients_general(lambda uu, a1, a2: nl_diffusion(uu, a1, a2, m), u_ref, pc, w)
    assert rel(kt.grad.cpu().numpy(), gk) <= 1e-8
    assert rel(ft.grad.cpu().numpy(), gf) <= 1e-8


def test_general_residual_matches_semilinear_path():
    """On F = A u + u^2 - f the general solve and the semilinear one agree:
    u, dL/dA and dL/df."""
    a, f, r = _problem(24, 10)
    w = t64(r.standard_normal(a.n))
    out = []
    for general in (False, True):
        vals = t64(a.val).requires_grad_(True)
        ft = t64(f).requires_grad_(True)
        A = hs.SparseCSR(vals, t32(a.row_ptr), t32(a.col))
        if general:
            u = nonlinear.newton_solve_residual(lambda uu, v, ff: A.with_values(v).mv(uu) + uu * uu - ff,
                                                (vals, ft), pattern=A.pattern, tol=1e-13, lin_rtol=1e-14)
        else:
            u = nonlinear.newton_solve(A, ft, tol=1e-13, lin_rtol=1e-14)
        (w * u).sum().backward()
        out.append((u.detach().cpu().numpy(), vals.grad.cpu().numpy(), ft.grad.cpu().numpy()))
    assert rel(out[1][0], out[0][0]) <= 1e-10
    assert rel(out[1][1], out[0][1]) <= 1e-8
    assert rel(out[1][2], out[0][2]) <= 1e-8
