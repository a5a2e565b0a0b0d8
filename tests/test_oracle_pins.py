"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each check is independent of the oracle's own code: closed forms (DST
diagonalisation and eigenvalues of the Dirichlet Laplacian), library
routines (numpy dense products and solves, scipy triangular solves), exact
integer arithmetic, finite termination of CG, and adjoint identities.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _int_csr(n, density, seed, explicit_zeros=True, empty_rows=True):
    r = np.random.default_rng(seed)
    row_ptr, col = W.random_pattern(n, density, r, diag=not empty_rows)
    val = r.integers(-(2 ** 20), 2 ** 20, size=len(col)).astype(np.float64)
    if explicit_zeros and len(val):
        val[r.random(len(val)) < 0.1] = 0.0
    return W.Csr(n, row_ptr, col, val)


# ---------------------------------------------------------------- SpMV (exact)

@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (7, 0.3, 1), (64, 0.05, 2), (300, 0.02, 3), (50, 0.0, 4)])
def test_spmv_integer_exact(orc, n, density, seed):
    """Integer values <= 2^20 and x <= 2^20: every product and partial sum is
    an exact integer below 2^53, so y equals the dense numpy product bitwise."""
    a = _int_csr(n, density, seed)
    x = np.random.default_rng(seed + 100).integers(-(2 ** 20), 2 ** 20, size=n).astype(np.float64)
    y = orc.spmv(a, x)
    assert np.array_equal(y, a.to_dense() @ x)


def test_spmv_empty_rows(orc):
    a = W.Csr(3, np.array([0, 0, 2, 2], np.int32), np.array([0, 2], np.int32), np.array([2.0, 3.0]))
    assert np.array_equal(orc.spmv(a, np.array([1.0, 5.0, 7.0])), np.array([0.0, 23.0, 0.0]))


# ---------------------------------------------------------------- transpose

@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (40, 0.1, 5), (200, 0.03, 6)])
def test_transpose_round_trip(orc, n, density, seed):
    a = _int_csr(n, density, seed)
    t, src = orc.transpose(a)
    assert np.array_equal(t.to_dense(), a.to_dense().T)
    assert np.array_equal(np.sort(src), np.arange(a.nnz))  # bijection
    assert np.array_equal(t.val, a.val[src])
    tt, _ = orc.transpose(t)
    assert np.array_equal(tt.row_ptr, a.row_ptr) and np.array_equal(tt.col, a.col)
    assert np.array_equal(tt.val, a.val)
    # canonical: strictly increasing columns per row
    for i in range(n):
        seg = t.col[t.row_ptr[i]:t.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_symmetry_detection(orc):
    a = W.poisson2d(5)
    assert orc.is_symmetric(a)
    b = a.with_values(a.val.copy())
    b.val[3] += 1e-16 * 4
    assert not orc.is_symmetric(b)
    assert not orc.is_symmetric(W.diffusion3d(3, velocity=1.0))


# ---------------------------------------------------------------- gradient index map

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adjoint_grad_index_map(orc, seed):
    """gA[k] = -lambda[row(k)] * x[col(k)] exactly, for integer lambda, x:
    compare against the dense outer product -lambda x^T sampled on the pattern."""
    a = _int_csr(80, 0.07, seed)
    r = np.random.default_rng(seed)
    lam = r.integers(-1000, 1000, size=a.n).astype(np.float64)
    x = r.integers(-1000, 1000, size=a.n).astype(np.float64)
    g = orc.adjoint_grad(a, lam, x)
    assert np.array_equal(g, -np.outer(lam, x)[a.rows(), a.col])


# ---------------------------------------------------------------- CG closed forms

def _dst_solve_2d(m, b):
    """x = A^{-1} b for the m x m Dirichlet 5-point Laplacian via the DST-I
    eigendecomposition A = (S (x) S) diag(Lambda) (S (x) S)."""
    j = np.arange(1, m + 1)
    S = math.sqrt(2.0 / (m + 1)) * np.sin(np.outer(j, j) * math.pi / (m + 1))
    mu = 4.0 * np.sin(j * math.pi / (2 * (m + 1))) ** 2
    Lam = mu[:, None] + mu[None, :]  # [ky, kx]
    B = b.reshape(m, m)  # [y, x]
    X = S @ ((S @ B @ S) / Lam) @ S
    return X.ravel()


def test_dst_closed_form_is_exact_inverse():
    """Sanity of the pin itself: A x_DST == b to rounding."""
    m = 16
    a = W.poisson2d(m)
    b = np.random.default_rng(0).standard_normal(a.n)
    x = _dst_solve_2d(m, b)
    assert np.linalg.norm(a.to_dense() @ x - b) <= 1e-13 * np.linalg.norm(b)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_cg_poisson2d_dst(orc, precond):
    """Workload-1 operator (64 x 64, b ~ N(0,1)): ||x - x_DST|| / ||x_DST|| <= kappa * rtol."""
    a, b = W.poisson2d_workload(64)
    rtol = 1e-12
    res = orc.cg(a, b, precond=precond, rtol=rtol)
    assert res.status == orc.OK
    kappa = 1.0 / math.tan(math.pi / 130) ** 2
    assert _rel(res.x, _dst_solve_2d(64, b)) <= kappa * rtol
    assert res.relres <= 1.5 * rtol


def _lanczos_ritz(alphas, betas):
    k = len(alphas)
    d = np.empty(k)
    e = np.empty(k - 1)
    for i in range(k):
        d[i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i < k - 1:
            e[i] = math.sqrt(betas[i]) / alphas[i]
    return scipy.linalg.eigvalsh_tridiagonal(d, e)


def test_cg_ritz_values_2d(orc):
    """Extreme Ritz values of CG's Lanczos tridiagonal converge to the
    closed-form extremes 8 sin^2(pi/130), 8 cos^2(pi/130) of the 64^2 operator."""
    a, b = W.poisson2d_workload(64)
    res = orc.cg(a, b, rtol=1e-12, history=True)
    ritz = _lanczos_ritz(res.alphas, res.betas)
    lo = 8 * math.sin(math.pi / 130) ** 2
    hi = 8 * math.cos(math.pi / 130) ** 2
    assert abs(ritz[0] - lo) <= 1e-6 * lo
    assert abs(ritz[-1] - hi) <= 1e-9 * hi


def test_cg_ritz_values_1d(orc):
    """1D operator of order 100, eigenvalues 4 sin^2(k pi / 2(n+1)): with a
    generic right-hand side, n CG steps recover the extreme eigenvalues."""
    n = 100
    a = W.poisson1d(n)
    b = np.random.default_rng(3).standard_normal(n)
    res = orc.cg(a, b, rtol=1e-14, max_iter=n, history=True)
    ritz = _lanczos_ritz(res.alphas, res.betas)
    k = np.arange(1, n + 1)
    exact = 4 * np.sin(k * math.pi / (2 * (n + 1))) ** 2
    assert abs(ritz[0] - exact[0]) <= 1e-8
    assert abs(ritz[-1] - exact[-1]) <= 1e-8


def test_cg_finite_termination(orc):
    n = 50
    eye = W.from_dense(np.eye(n))
    b = np.random.default_rng(1).standard_normal(n)
    r = orc.cg(eye, b, rtol=1e-14)
    assert r.iters == 1 and np.array_equal(r.x, b)
    d = np.random.default_rng(2).uniform(1, 100, n)
    diag = W.from_dense(np.diag(d))
    r = orc.cg(diag, b, precond="jacobi", rtol=1e-14)
    assert r.iters == 1 and np.allclose(r.x, b / d, rtol=1e-15, atol=0)
    blk = np.array([[4.0, 1.0], [1.0, 3.0]])
    bd = scipy.linalg.block_diag(*([blk] * 25))
    r = orc.cg(W.from_dense(bd), b, rtol=1e-13)
    assert r.iters == 2
    assert _rel(r.x, np.linalg.solve(bd, b)) < 1e-13


# ---------------------------------------------------------------- dense + brute force

@pytest.mark.parametrize("n", [1, 5, 40])
def test_dense_direct_vs_numpy(orc, n):
    r = np.random.default_rng(n)
    M = r.standard_normal((n, n))
    spd = M @ M.T + n * np.eye(n)
    b = r.standard_normal(n)
    assert _rel(orc.dense_solve(spd, b, spd=True), np.linalg.solve(spd, b)) < 1e-12
    assert _rel(orc.dense_solve(M + 3 * np.eye(n), b), np.linalg.solve(M + 3 * np.eye(n), b)) < 1e-10
    assert _rel(orc.dense_solve(M + 3 * np.eye(n), b, trans=True), np.linalg.solve((M + 3 * np.eye(n)).T, b)) < 1e-10


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_krylov_vs_dense(orc, seed, precond):
    r = np.random.default_rng(seed)
    a = W.random_spd(120, 0.05, r)
    b = r.standard_normal(a.n)
    xd = np.linalg.solve(a.to_dense(), b)
    kappa = np.linalg.cond(a.to_dense())
    res = orc.cg(a, b, precond=precond, rtol=1e-12)
    assert res.status == orc.OK and _rel(res.x, xd) <= kappa * 1e-12
    ns = W.random_nonsym(120, 0.05, r)
    xn = np.linalg.solve(ns.to_dense(), b)
    res = orc.bicgstab(ns, b, precond=precond, rtol=1e-12)
    assert res.status == orc.OK
    assert _rel(res.x, xn) <= np.linalg.cond(ns.to_dense()) * 1e-12
    assert res.relres <= 1e-12


def test_bicgstab_on_spd_matches_cg_solution(orc):
    a, b = W.poisson2d_workload(32)
    x1 = orc.cg(a, b, rtol=1e-13).x
    x2 = orc.bicgstab(a, b, rtol=1e-13).x
    assert _rel(x2, x1) < 1e-9


def test_pure_upwind_is_triangular(orc):
    """Pure upwind convection (no diffusion) is lower triangular in
    lexicographic order: forward substitution gives x exactly."""
    a = W.diffusion3d(6, velocity=10.0, diffusion=False)
    d = a.to_dense()
    assert np.array_equal(d, np.tril(d))
    b = np.random.default_rng(7).standard_normal(a.n)
    x = scipy.linalg.solve_triangular(d, b, lower=True)
    for pc in ["none", "jacobi"]:
        res = orc.bicgstab(a, b, precond=pc, rtol=1e-14)
        assert _rel(res.x, x) <= 1e-10


def test_upwind_diffusion_bicgstab(orc):
    a = W.diffusion3d(8, W.diffusion3d_kappa(8), velocity=10.0)
    b = np.random.default_rng(8).standard_normal(a.n)
    xd = np.linalg.solve(a.to_dense(), b)
    res = orc.bicgstab(a, b, precond="jacobi", rtol=1e-12)
    assert res.status == orc.OK and _rel(res.x, xd) < 1e-10


# ---------------------------------------------------------------- status codes

def test_status_codes(orc):
    a, b = W.poisson2d_workload(16)
    assert orc.cg(a, b, max_iter=1).status == orc.NOT_CONVERGED
    r = orc.cg(a, np.zeros(a.n))
    assert r.status == orc.OK and r.iters == 0 and not r.x.any()
    bad = b.copy()
    bad[3] = np.nan
    assert orc.cg(a, bad).status == orc.NONFINITE
    assert orc.bicgstab(a, bad).status == orc.NONFINITE
    indef = a.with_values(-a.val)
    assert orc.cg(indef, b).status == orc.BREAKDOWN
    nodiag = W.Csr(2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    assert orc.cg(nodiag, np.ones(2), precond="jacobi").status == orc.BAD_INPUT


def test_bicgstab_breakdown_restart(orc):
    """[[0,1],[1,0]] x = (1,0): without preconditioning r_hat.v = 0 at the
    first step (v = A r is orthogonal to r); one restart cannot help, so the
    solver reports breakdown rather than dividing by zero."""
    a = W.from_dense(np.array([[0.0, 1.0], [1.0, 0.0]]), keep=np.ones((2, 2), bool))
    r = orc.bicgstab(a, np.array([1.0, 0.0]))
    assert r.status == orc.BREAKDOWN and np.all(np.isfinite(r.x))


# ---------------------------------------------------------------- adjoint identities

@pytest.mark.parametrize("kind", ["spd", "nonsym"])
def test_adjoint_vs_dense(orc, kind):
    r = np.random.default_rng(11)
    a = W.random_spd(60, 0.08, r) if kind == "spd" else W.random_nonsym(60, 0.08, r)
    b = r.standard_normal(a.n)
    gx = r.standard_normal(a.n)
    x = np.linalg.solve(a.to_dense(), b)
    gA, gb, res = orc.adjoint(a, x, gx, precond="jacobi", rtol=1e-13)
    lam = np.linalg.solve(a.to_dense().T, gx)
    assert _rel(gb, lam) < 1e-10
    assert _rel(gA, (-np.outer(lam, x))[a.rows(), a.col]) < 1e-10
    gA2, lam2 = orc.dense_adjoint(a, x, gx, spd=(kind == "spd"))
    assert _rel(lam2, lam) < 1e-12


def test_adjoint_jacobian_identity(orc):
    """The adjoint with gx = e_k is dx_k/db, i.e. row k of the Jacobian
    J = dx/db = A^{-1}; stacking the rows, A J = I."""
    a = W.random_nonsym(30, 0.15, np.random.default_rng(4))
    x = np.zeros(a.n)
    J = np.stack([orc.adjoint(a, x, np.eye(a.n)[k], rtol=1e-14)[1] for k in range(a.n)])
    assert np.abs(a.to_dense() @ J - np.eye(a.n)).max() < 1e-10


def test_adjoint_identity_matrix(orc):
    """A = I: x = b, lambda = gx, gA_ij = -gx_i b_j on the pattern."""
    n = 20
    a = W.from_dense(np.eye(n))
    r = np.random.default_rng(5)
    b, gx = r.standard_normal(n), r.standard_normal(n)
    x = orc.cg(a, b, rtol=1e-14).x
    gA, gb, _ = orc.adjoint(a, x, gx, rtol=1e-14)
    assert np.array_equal(gb, gx)
    assert np.array_equal(gA, -gx * b)


def _fd_correction(orc, a, xt, b, xstar, k, h, on="A"):
    """Central FD of L = 1/2 ||x - x*||^2 by correction solves: with converged
    x~, (A + dA) (x~ + d) = b is solved for d against the small residual
    b - A x~ - dA x~, so no O(1) quantity is differenced."""
    rows = a.rows()
    out = []
    for sgn in (+1.0, -1.0):
        if on == "A":
            v = a.val.copy()
            v[k] += sgn * h
            ap = a.with_values(v)
            rhs = b - orc.spmv(a, xt)
            rhs[rows[k]] -= sgn * h * xt[a.col[k]]
        else:
            ap = a
            rhs = b - orc.spmv(a, xt)
            rhs[k] += sgn * h
        d = orc.bicgstab(ap, rhs, precond="jacobi", rtol=1e-13).x
        out.append(d)
    dp, dm = out
    dl = (dp - dm) @ (xt - xstar) + 0.5 * (dp @ dp - dm @ dm)
    return dl / (2 * h)


def test_adjoint_vs_fd(orc):
    """Finite differences (h = 1e-6 on raw values) on a small 3D log-normal
    diffusion system: relative error of the 2-norm over picked entries <= 1e-6."""
    m = 6
    a = W.diffusion3d(m, W.diffusion3d_kappa(m, cfg=4, sample=0))
    r = np.random.default_rng(99)
    b = r.standard_normal(a.n)
    xstar = r.standard_normal(a.n)
    xt = orc.cg(a, b, precond="jacobi", rtol=1e-14).x
    gA, gb, _ = orc.adjoint(a, xt, xt - xstar, precond="jacobi", rtol=1e-14)
    picks = r.choice(a.nnz, 24, replace=False)
    fd = np.array([_fd_correction(orc, a, xt, b, xstar, int(k), 1e-6) for k in picks])
    assert np.linalg.norm(fd - gA[picks]) <= 1e-6 * np.linalg.norm(gA[picks])
    pb = r.choice(a.n, 8, replace=False)
    fdb = np.array([_fd_correction(orc, a, xt, b, xstar, int(k), 1e-6, on="b") for k in pb])
    assert np.linalg.norm(fdb - gb[pb]) <= 1e-6 * np.linalg.norm(gb[pb])


# ---------------------------------------------------------------- FSAI + probe loss

def test_fsai_diagonal(orc):
    d = np.random.default_rng(0).uniform(0.5, 9.0, 30)
    a = W.from_dense(np.diag(d))
    _, _, g = orc.fsai(a)
    assert np.allclose(g, 1 / np.sqrt(d), rtol=1e-15, atol=0)


def test_fsai_block_cholesky(orc):
    """2x2 SPD blocks with full lower pattern: G = L^{-1} (A = L L^T), so
    G A G^T = I and FSAI-PCG converges in one iteration."""
    r = np.random.default_rng(1)
    blocks = []
    for _ in range(20):
        M = r.standard_normal((2, 2))
        blocks.append(M @ M.T + np.eye(2))
    D = scipy.linalg.block_diag(*blocks)
    a = W.from_dense(D, keep=D != 0)
    rpL, colL, g = orc.fsai(a)
    G = W.Csr(a.n, rpL, colL, g).to_dense()
    Linv = np.linalg.inv(np.linalg.cholesky(D))
    assert np.abs(G - Linv).max() < 1e-13
    b = r.standard_normal(a.n)
    res = orc.fsai_pcg(a, rpL, colL, g, b, rtol=1e-12)
    assert res.iters == 1 and res.status == orc.OK


def test_fsai_unit_diagonal_and_apply(orc):
    a = W.aniso2d(8, 30.0, 0.4)
    rpL, colL, g = orc.fsai(a)
    G = W.Csr(a.n, rpL, colL, g).to_dense()
    M = G @ a.to_dense() @ G.T
    assert np.allclose(np.diag(M), 1.0, atol=1e-13)
    rvec = np.random.default_rng(2).standard_normal(a.n)
    assert _rel(orc.fsai_apply(rpL, colL, g, rvec), G.T @ (G @ rvec)) < 1e-14
    b = np.random.default_rng(3).standard_normal(a.n)
    res = orc.fsai_pcg(a, rpL, colL, g, b, rtol=1e-10)
    assert res.status == orc.OK
    assert _rel(res.x, np.linalg.solve(a.to_dense(), b)) < 1e-7


def test_probe_loss_expectation(orc):
    """Averaged over all 2^n Rademacher probes, ||B z||^2 equals ||B||_F^2
    exactly (B = G A G^T - I), n = 9."""
    a = W.aniso2d(3, 5.0, 1.0)
    rpL, colL, g = orc.fsai(a)
    g = g * (1 + 0.1 * np.random.default_rng(0).standard_normal(len(g)))
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=a.n)))
    loss = orc.probe_loss(a, rpL, colL, g, Z, grad=False)
    G = W.Csr(a.n, rpL, colL, g).to_dense()
    B = G @ a.to_dense() @ G.T - np.eye(a.n)
    assert abs(loss / len(Z) - np.sum(B * B)) < 1e-12 * np.sum(B * B)


def test_probe_loss_gradient_fd(orc):
    a = W.aniso2d(5, 20.0, 0.7)
    a = a.with_values(a.val)
    rpL, colL, g = orc.fsai(a)
    r = np.random.default_rng(4)
    g = g * (1 + 0.2 * r.standard_normal(len(g)))
    Z = W.rademacher(r, (3, a.n))
    _, grad = orc.probe_loss(a, rpL, colL, g, Z)
    h = 1e-6
    for k in r.choice(len(g), 12, replace=False):
        gp, gm = g.copy(), g.copy()
        gp[k] += h
        gm[k] -= h
        fd = (orc.probe_loss(a, rpL, colL, gp, Z, grad=False) - orc.probe_loss(a, rpL, colL, gm, Z, grad=False)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(grad[k]))
    # dense form of the same gradient (nonsymmetric A exercises A^T)
    ns = W.random_nonsym(20, 0.2, r)
    rpL2, colL2, _ = orc.lower_pattern(ns)
    g2 = r.standard_normal(len(colL2))
    Z2 = W.rademacher(r, (2, ns.n))
    _, grad2 = orc.probe_loss(ns, rpL2, colL2, g2, Z2)
    G = W.Csr(ns.n, rpL2, colL2, g2).to_dense()
    A = ns.to_dense()
    dense = np.zeros_like(G)
    for z in Z2:
        u = A @ G.T @ z
        e = G @ u - z
        y = A.T @ G.T @ e
        dense += 2 * (np.outer(e, u) + np.outer(z, y))
    rowsL = np.repeat(np.arange(ns.n), np.diff(rpL2))
    assert _rel(grad2, dense[rowsL, colL2]) < 1e-13


def test_residual_norm_integer_exact(orc):
    """||b - A x||_2 with integer data: every product, row sum and square is
    exact, so the oracle equals the sum of squares numpy forms from the dense
    product, up to the final square root (correctly rounded both ways)."""
    r = np.random.default_rng(21)
    rp, col = W.random_pattern(300, 0.03, r)
    a = W.Csr(300, rp, col, r.integers(-50, 50, len(col)).astype(np.float64))
    x = r.integers(-100, 100, a.n).astype(np.float64)
    b = r.integers(-10000, 10000, a.n).astype(np.float64)
    e = b - a.to_dense() @ x
    assert orc.residual_norm(a, b, x) == np.sqrt(float(np.sum(e * e)))
    assert orc.residual_norm(a, a.to_dense() @ x, x) == 0.0


# ------------------------------------------------------------------ threaded mode

def test_threaded_mode_changes_only_summation_order(orc):
    """With several threads the oracle splits rows and element-wise loops
    (no result changes: SpMV bitwise equal to one thread, and integer data
    stays exact) and sums inner products as per-thread partials: each
    within n * eps * sum|a_i b_i| of the exactly rounded sum (math.fsum)."""
    a = W.diffusion3d(12, W.diffusion3d_kappa(12))
    r = np.random.default_rng(5)
    x = r.standard_normal(a.n)
    y1 = orc.spmv(a, x)
    with orc.threads(7):
        y7 = orc.spmv(a, x)
        for n in (1, 6, 7, 1000, a.n):
            u, v = r.standard_normal(n), r.standard_normal(n)
            exact = math.fsum(u * v)
            assert abs(orc.dot(u, v) - exact) <= n * 2.3e-16 * float(np.sum(np.abs(u * v)))
        bi = r.integers(-1000, 1000, a.n).astype(np.float64)
        xi = r.integers(-1000, 1000, a.n).astype(np.float64)
        ai = a.with_values(r.integers(-1000, 1000, a.nnz).astype(np.float64))
        res = bi - ai.to_dense() @ xi
        assert orc.residual_norm(ai, bi, xi) == math.sqrt(math.fsum(res * res))
    assert np.array_equal(y1, y7)


@pytest.mark.parametrize("threads", [3, 8])
def test_threaded_cg_and_bicgstab_match_closed_forms(orc, threads):
    """The threaded solvers still meet the pins the sequential ones do: CG on
    the 64^2 Poisson operator against the DST-I closed form within kappa *
    rtol, BiCGStab on the pure-upwind (lower triangular) operator against
    forward substitution, and both against the one-thread solve to rounding
    with iteration counts within max(2, 2%)."""
    m = 64
    a = W.poisson2d(m)
    b = W.rng(1, 1).standard_normal(a.n)
    seq = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    with orc.threads(threads):
        par = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    kappa = 1.0 / math.tan(math.pi / 130) ** 2
    assert par.status == orc.OK
    assert _rel(par.x, _dst_solve_2d(m, b)) <= kappa * 1e-12
    assert _rel(par.x, seq.x) <= 1e-10
    assert abs(par.iters - seq.iters) <= max(2, int(0.02 * seq.iters))
    u = W.diffusion3d(10, velocity=10.0, diffusion=False)
    keep = u.val != 0
    d = np.zeros((u.n, u.n))
    d[u.rows()[keep], u.col[keep]] = u.val[keep]
    bu = W.rng(2, 1, 3).standard_normal(u.n)
    with orc.threads(threads):
        pu = orc.bicgstab(u, bu, precond="jacobi", rtol=1e-13)
    assert pu.status == orc.OK
    assert _rel(pu.x, scipy.linalg.solve_triangular(d, bu, lower=True)) <= 1e-10
