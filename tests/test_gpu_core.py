"""GPU parity of the core path (SpMV, pattern ingest, CG/PCG, BiCGStab,
adjoint) against the CPU oracle, through the C ABI."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, iters_close, pattern, rel, solve, t32, t64  # noqa: E402
from paper_2601_13994_amd import _lib  # noqa: E402


def _rand_csr(n, density, seed, long_rows=(), int_vals=False):
    r = np.random.default_rng(seed)
    m = r.random((n, n)) < density
    for i in long_rows:
        m[i, :] = True
    np.fill_diagonal(m, True)
    a = W.from_dense(np.where(m, 1.0, 0.0), keep=m)
    a.val = (r.integers(-1000, 1000, a.nnz).astype(np.float64) if int_vals else r.standard_normal(a.nnz))
    return a


# ---------------------------------------------------------------- pattern ingest

def test_pattern_rejects_invalid_csr():
    good = W.poisson2d(5)
    cases = []
    rp = good.row_ptr.copy(); rp[3], rp[4] = rp[4], rp[3]; cases.append((rp, good.col))   # decreasing
    c = good.col.copy(); c[7] = good.n; cases.append((good.row_ptr, c))                     # out of range
    c = good.col.copy(); c[0], c[1] = c[1], c[0]; cases.append((good.row_ptr, c))           # unsorted
    c = good.col.copy(); c[1] = c[0]; cases.append((good.row_ptr, c))                       # duplicate
    rp = good.row_ptr.copy(); rp[-1] -= 1; cases.append((rp, good.col))                     # rp[n] != nnz
    c = good.col.copy(); c[5] = -3; cases.append((good.row_ptr, c))                         # negative
    for rp, c in cases:
        with pytest.raises(_lib.HslaError) as e:
            _lib.Pattern(t32(rp), t32(c))
        assert e.value.status == _lib.ERR_INVALID_CSR


def test_pattern_transpose_exact(orc):
    for seed, (n, d) in enumerate([(1, 1.0), (57, 0.08), (700, 0.01)]):
        a = _rand_csr(n, d, seed)
        pat = pattern(a)
        rpT, colT, src = pat.transpose()
        t, srco = orc.transpose(a)
        assert np.array_equal(rpT.cpu().numpy(), t.row_ptr)
        assert np.array_equal(colT.cpu().numpy(), t.col)
        assert np.array_equal(src.cpu().numpy(), srco)
        assert pat.nnz_lower == int(np.sum(a.col <= a.rows()))
    assert pattern(W.poisson2d(6)).pattern_symmetric
    assert not pattern(_rand_csr(40, 0.1, 9)).pattern_symmetric


def test_pattern_lower_exact(orc):
    """The lower triangle (the layout of FSAI factors and the network's
    output) equals the oracle's bit for bit, with each entry's position in A."""
    for seed, (n, d) in enumerate([(1, 1.0), (57, 0.08), (700, 0.01)]):
        a = _rand_csr(n, d, seed)
        rpL, colL, pos = pattern(a).lower()
        ro, co, po = orc.lower_pattern(a)
        assert np.array_equal(rpL.cpu().numpy(), ro)
        assert np.array_equal(colL.cpu().numpy(), co)
        assert np.array_equal(pos.cpu().numpy(), po)


def test_pattern_csr_only_flag(orc):
    """HSLA_PATTERN_CSR: no offset-mask form is derived (a stencil pattern
    reports none), SpMV and solves still match the oracle; unknown flag bits
    are rejected."""
    import ctypes
    a, b = W.poisson2d_workload(20)
    assert pattern(a).stencil == (True, 5)
    pat = _lib.Pattern(t32(a.row_ptr), t32(a.col), csr_only=True)
    assert pat.stencil == (False, 0)
    x = np.random.default_rng(3).standard_normal(a.n)
    assert np.array_equal(_lib.spmv(pat, t64(a.val), t64(x)).cpu().numpy(), orc.spmv(a, x))
    xs, info, st = solve(a, b, pat=pat, rtol=1e-12, persistent=False)
    assert st == 0 and info[0]["spmv_form"] == "tiles"
    assert rel(xs, orc.cg(a, b, precond="jacobi", rtol=1e-12).x) <= 1e-8
    p = ctypes.c_void_p()
    rp, col = t32(a.row_ptr), t32(a.col)
    st = _lib.load().hsla_pattern_create(pat.h, a.n, a.nnz, rp.data_ptr(), col.data_ptr(), 6, None, ctypes.byref(p))
    assert st == _lib.ERR_INVALID_ARG and not p.value


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (63, 0.1, 1), (64, 0.1, 2), (1000, 0.005, 3),
                                            (4097, 0.001, 4)])
def test_spmv_bitwise(orc, n, density, seed):
    """Each row adds its rounded products in ascending column order, exactly
    as the oracle does, so the results agree bit for bit for any values."""
    a = _rand_csr(n, density, seed)
    x = np.random.default_rng(seed + 7).standard_normal(n)
    y = _lib.spmv(pattern(a), t64(a.val), t64(x)).cpu().numpy()
    assert np.array_equal(y, orc.spmv(a, x))


def test_spmv_long_rows_and_empty_rows(orc):
    """Rows longer than one LDS tile (split across lanes) with integer data
    (exact under any order), and empty rows."""
    a = _rand_csr(1500, 0.002, 5, long_rows=(3, 700, 1499), int_vals=True)
    x = np.random.default_rng(1).integers(-1000, 1000, a.n).astype(np.float64)
    y = _lib.spmv(pattern(a), t64(a.val), t64(x)).cpu().numpy()
    assert np.array_equal(y, orc.spmv(a, x))
    e = W.Csr(4, np.array([0, 0, 2, 2, 3], np.int32), np.array([0, 3, 1], np.int32), np.array([2.0, 3.0, 5.0]))
    y = _lib.spmv(pattern(e), t64(e.val), t64(np.array([1.0, 2.0, 3.0, 4.0]))).cpu().numpy()
    assert np.array_equal(y, np.array([0.0, 14.0, 0.0, 10.0]))


def test_spmv_long_rows_random_values(orc):
    """Rows of 513 to 1500 entries (longer than one LDS tile, summed in
    pieces) with random FP64 values: still ascending per-row sums, bitwise
    equal to the oracle; also through the solvers' SpMV+dot on the CSR form."""
    a = _rand_csr(1500, 0.002, 6, long_rows=(3, 700, 1499))
    lens = np.diff(a.row_ptr)
    assert lens.max() > 512
    x = np.random.default_rng(2).standard_normal(a.n)
    pat = pattern(a)
    y = _lib.spmv(pat, t64(a.val), t64(x)).cpu().numpy()
    assert np.array_equal(y, orc.spmv(a, x))
    pat.set_format("csr")
    y = _lib.spmv(pat, t64(a.val), t64(x)).cpu().numpy()
    assert np.array_equal(y, orc.spmv(a, x))


def test_spmv_batched(orc):
    a = W.diffusion3d(7, W.diffusion3d_kappa(7))
    r = np.random.default_rng(3)
    V = np.stack([a.val * r.uniform(0.5, 2.0) for _ in range(3)])
    X = r.standard_normal((3, a.n))
    Y = _lib.spmv(pattern(a), t64(V), t64(X)).cpu().numpy()
    for s in range(3):
        assert np.array_equal(Y[s], orc.spmv(a.with_values(V[s]), X[s]))


# ---------------------------------------------------------------- CG / PCG

@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_cg_poisson2d_parity(orc, precond, persistent):
    """2D 5-point Poisson 64 x 64 (n = 4096), the small adjoint-check problem
    of the paper: ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-8 at rtol 1e-12."""
    a, b = W.poisson2d_workload(64)
    x, info, st = solve(a, b, method="cg", precond=precond, rtol=1e-12, persistent=persistent)
    ref = orc.cg(a, b, precond=precond, rtol=1e-12)
    assert st == 0 and info[0]["status"] == 0
    assert rel(x, ref.x) <= 1e-8
    assert iters_close(info[0]["iters"], ref.iters)
    assert info[0]["true_residual"] <= 2e-12


@pytest.mark.parametrize("make", [lambda: W.poisson2d(20), lambda: W.poisson2d(30), lambda: W.poisson2d(45),
                                  lambda: W.poisson2d(64), lambda: W.diffusion3d(8, W.diffusion3d_kappa(8)),
                                  lambda: W.diffusion3d(10, W.diffusion3d_kappa(10)),
                                  lambda: W.diffusion3d(12, W.diffusion3d_kappa(12))],
                         ids=["p20", "p30", "p45", "p64", "d8", "d10", "d12"])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("method", ["cg", "cg_sr"])
def test_small_systems_matrix_in_registers(orc, make, precond, method):
    """Small systems with rows of at most 5 (n <= 4096) or 8 (n <= 2048)
    entries run with the matrix held in registers, 1, 2, 4 or 8 rows per
    thread, by CG and by the single-reduction recurrence (up to 4 rows per
    thread; p64 runs it in the LDS kernel): the oracle's solution and
    iteration count, the k-th iterate at a cap, breakdown on -A, b = 0, and
    a batch member bitwise equal to its own solve."""
    a = make()
    r = np.random.default_rng(a.n)
    b = r.standard_normal(a.n)
    pat = pattern(a)
    x, info, st = solve(a, b, pat=pat, method=method, precond=precond, rtol=1e-12)
    ref = orc.cg(a, b, precond=precond, rtol=1e-12)
    assert st == 0 and info[0]["spmv_form"] == "persistent" and info[0]["method"] == method
    assert rel(x, ref.x) <= 1e-8
    assert iters_close(info[0]["iters"], ref.iters), (info[0]["iters"], ref.iters)
    assert info[0]["true_residual"] <= 5e-12
    for k in (1, 5):
        xk, ik, sk = solve(a, b, pat=pat, method=method, precond=precond, rtol=1e-14, max_iter=k)
        refk = orc.cg(a, b, precond=precond, rtol=1e-14, max_iter=k)
        assert sk == _lib.NOT_CONVERGED and ik[0]["iters"] == k and rel(xk, refk.x) <= 1e-12
    V = np.stack([a.val * 2.0, a.val, -a.val])
    Bm = np.stack([r.standard_normal(a.n), b, b])
    X, infos, st = _lib.solve(pat, t64(V), t64(Bm), _lib.make_opts(method=method, precond=precond, rtol=1e-12))
    assert st == _lib.BREAKDOWN and infos[2]["status"] == _lib.BREAKDOWN
    assert infos[0]["status"] == 0 and infos[1]["status"] == 0
    assert np.array_equal(X[1].cpu().numpy(), x)
    x0, i0, st = solve(a, np.zeros(a.n), pat=pat, method=method, precond=precond)
    assert st == 0 and i0[0]["iters"] == 0 and not x0.any()


@pytest.mark.parametrize("persistent", [True, False])
def test_pcg_diffusion3d_parity(orc, persistent):
    """3D log-normal diffusion (the large workload's operator) at m = 24."""
    m = 24
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    b = W.rng(2, 1).standard_normal(a.n)
    x, info, st = solve(a, b, precond="jacobi", rtol=1e-12, persistent=persistent)
    ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    assert st == 0 and info[0]["method"] == "cg"
    assert rel(x, ref.x) <= 1e-8
    assert iters_close(info[0]["iters"], ref.iters)


@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("seed", [0, 1])
def test_cg_random_spd_parity(orc, seed, persistent):
    r = np.random.default_rng(seed)
    a = W.random_spd(300, 0.02, r)
    b = r.standard_normal(a.n)
    x, info, st = solve(a, b, precond="jacobi", rtol=1e-12, persistent=persistent)
    ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    assert st == 0 and rel(x, ref.x) <= 1e-8


def test_cg_finite_termination():
    n = 300
    b = np.random.default_rng(1).standard_normal(n)
    x, info, st = solve(W.from_dense(np.eye(n)), b, method="cg", precond="none", rtol=1e-14)
    assert info[0]["iters"] == 1 and np.array_equal(x, b)
    d = np.random.default_rng(2).uniform(1, 100, n)
    x, info, _ = solve(W.from_dense(np.diag(d)), b, precond="jacobi", rtol=1e-14)
    assert info[0]["iters"] == 1 and rel(x, b / d) < 1e-15


# ---------------------------------------------------------------- BiCGStab

@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_bicgstab_upwind_parity(orc, precond):
    m = 12
    a = W.diffusion3d(m, W.diffusion3d_kappa(m), velocity=10.0)
    b = W.rng(2, 1).standard_normal(a.n)
    x, info, st = solve(a, b, precond=precond, rtol=1e-12)
    ref = orc.bicgstab(a, b, precond=precond, rtol=1e-12)
    assert st == 0 and info[0]["method"] == "bicgstab"
    assert rel(x, ref.x) <= 1e-8
    assert iters_close(info[0]["iters"], ref.iters)


def test_bicgstab_pure_upwind_exact():
    """Triangular operator: the solution from forward substitution."""
    import scipy.linalg

    a = W.diffusion3d(10, velocity=10.0, diffusion=False)
    b = np.random.default_rng(7).standard_normal(a.n)
    xe = scipy.linalg.solve_triangular(a.to_dense(), b, lower=True)
    x, info, st = solve(a, b, precond="jacobi", rtol=1e-14)
    assert rel(x, xe) <= 1e-10


def test_bicgstab_random_nonsym(orc):
    r = np.random.default_rng(5)
    a = W.random_nonsym(400, 0.02, r)
    b = r.standard_normal(a.n)
    x, info, st = solve(a, b, precond="jacobi", rtol=1e-12)
    ref = orc.bicgstab(a, b, precond="jacobi", rtol=1e-12)
    assert st == 0 and rel(x, ref.x) <= 1e-8


def test_bicgstab_breakdown_reported():
    a = W.from_dense(np.array([[0.0, 1.0], [1.0, 0.0]]), keep=np.ones((2, 2), bool))
    x, info, st = solve(a, np.array([1.0, 0.0]), method="bicgstab", precond="none")
    assert st == _lib.BREAKDOWN and np.all(np.isfinite(x))


# ---------------------------------------------------------------- status codes

@pytest.mark.parametrize("persistent", [True, False])
def test_status_codes(persistent):
    kw = dict(persistent=persistent)
    a, b = W.poisson2d_workload(16)
    pat = pattern(a)
    x, info, st = solve(a, b, pat=pat, max_iter=1, **kw)
    assert st == _lib.NOT_CONVERGED and info[0]["iters"] == 1
    x, info, st = solve(a, np.zeros(a.n), pat=pat, **kw)
    assert st == 0 and info[0]["iters"] == 0 and not x.any()
    bad = b.copy()
    bad[3] = np.nan
    with pytest.raises(_lib.HslaError) as e:
        solve(a, bad, pat=pat, **kw)
    assert e.value.status == _lib.ERR_NONFINITE
    x, info, st = solve(a, b, pat=pat, values=t64(-a.val), method="cg", **kw)
    assert st == _lib.BREAKDOWN
    # one negative Jacobi diagonal: BREAKDOWN before the first iteration, x = 0
    v = a.val.copy()
    v[(a.rows() == 7) & (a.col == 7)] *= -1.0
    x, info, st = solve(a, b, pat=pat, values=t64(v), method="cg", precond="jacobi", **kw)
    assert st == _lib.BREAKDOWN and info[0]["iters"] == 0 and not x.any()
    nodiag = W.Csr(2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    with pytest.raises(_lib.HslaError) as e:
        solve(nodiag, np.ones(2), precond="jacobi", **kw)
    assert e.value.status == _lib.ERR_ZERO_DIAGONAL


def test_empty_system():
    e = W.Csr(0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0))
    x, info, st = solve(e, np.zeros(0))
    assert st == 0 and x.size == 0


# ---------------------------------------------------------------- determinism, graphs, batches

def test_deterministic_and_graph_equal():
    m = 20
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    b = W.rng(2, 1).standard_normal(a.n)
    pat = pattern(a)
    kw = dict(pat=pat, rtol=1e-10, persistent=False)
    x1, i1, _ = solve(a, b, graph=True, **kw)
    x2, i2, _ = solve(a, b, graph=True, **kw)
    x3, i3, _ = solve(a, b, graph=False, **kw)
    x4, i4, _ = solve(a, b, graph=False, check_every=5, **kw)
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3) and np.array_equal(x1, x4)
    assert i1[0]["iters"] == i3[0]["iters"] == i4[0]["iters"]
    # the persistent launch: run to run identical, same iterations to within rounding
    x5, i5, _ = solve(a, b, pat=pat, rtol=1e-10)
    x6, i6, _ = solve(a, b, pat=pat, rtol=1e-10)
    assert np.array_equal(x5, x6) and i5[0]["iters"] == i6[0]["iters"]
    assert iters_close(i5[0]["iters"], i1[0]["iters"]) and rel(x5, x1) <= 1e-9


@pytest.mark.parametrize("persistent", [True, False])
def test_batched_masks_and_independence(orc, persistent):
    """Systems with very different iteration counts, a zero right-hand side
    and an easy one, iterated in lock step: each equals its own solve bit for
    bit and matches the oracle."""
    m = 14
    base = W.diffusion3d(m)
    r = np.random.default_rng(11)
    vals, bs = [], []
    for s in range(5):
        if s == 3:
            vals.append(W.diffusion3d(m, np.full(m ** 3, 5.0)).val)  # constant coefficient
        else:
            vals.append(W.diffusion3d(m, np.exp((s + 0.5) * r.standard_normal(m ** 3))).val)
        bs.append(np.zeros(base.n) if s == 2 else r.standard_normal(base.n))
    V, Bm = np.stack(vals), np.stack(bs)
    pat = pattern(base)
    opts = _lib.make_opts(precond="jacobi", rtol=1e-11, persistent=persistent)
    X, infos, st = _lib.solve(pat, t64(V), t64(Bm), opts)
    X = X.cpu().numpy()
    assert st == 0
    its = [f["iters"] for f in infos]
    assert its[2] == 0 and not X[2].any()
    assert len(set(its)) >= 3
    for s in range(5):
        xs, inf, _ = _lib.solve(pat, t64(V[s]), t64(Bm[s]), opts)
        assert np.array_equal(xs.cpu().numpy(), X[s])
        assert inf[0]["iters"] == its[s]
        if s != 2:
            ref = orc.cg(base.with_values(V[s]), Bm[s], precond="jacobi", rtol=1e-11)
            assert rel(X[s], ref.x) <= 1e-7


# ---------------------------------------------------------------- adjoint

def test_outer_on_pattern_bitwise(orc):
    a = _rand_csr(500, 0.01, 3)
    r = np.random.default_rng(0)
    lam = r.integers(-1000, 1000, a.n).astype(np.float64)
    x = r.standard_normal(a.n)
    g = _lib.outer_on_pattern(pattern(a), t64(lam), t64(x)).cpu().numpy()
    assert np.array_equal(g, orc.adjoint_grad(a, lam, x))


@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("kind", ["spd", "nonsym"])
def test_adjoint_parity(orc, kind, persistent):
    m = 10
    if kind == "spd":
        a = W.diffusion3d(m, W.diffusion3d_kappa(m, cfg=4))
    else:
        a = W.diffusion3d(m, W.diffusion3d_kappa(m, cfg=4), velocity=10.0)
    r = np.random.default_rng(2)
    b, xs = r.standard_normal(a.n), r.standard_normal(a.n)
    x = orc.solve(a, b, precond="jacobi", rtol=1e-13).x
    gx = x - xs
    pat = pattern(a)
    opts = _lib.make_opts(precond="jacobi", rtol=1e-13, persistent=persistent)
    gA, gb, infos, st = _lib.adjoint(pat, t64(a.val), t64(x), t64(gx), opts)
    gA_o, gb_o, _ = orc.adjoint(a, x, gx, precond="jacobi", rtol=1e-13)
    assert st == 0
    assert rel(gb.cpu().numpy(), gb_o) <= 1e-6
    assert rel(gA.cpu().numpy(), gA_o) <= 1e-6
    # dense brute force
    lam = np.linalg.solve(a.to_dense().T, gx)
    assert rel(gb.cpu().numpy(), lam) <= 1e-8


def test_autograd_one_node_and_gradients(orc):
    import paper_2601_13994_amd as hs

    m = 8
    a = W.diffusion3d(m, W.diffusion3d_kappa(m, cfg=4))
    r = np.random.default_rng(4)
    b_np, xs_np = r.standard_normal(a.n), r.standard_normal(a.n)
    vals = t64(a.val).requires_grad_(True)
    b = t64(b_np).requires_grad_(True)
    A = hs.SparseCSR(vals, t32(a.row_ptr), t32(a.col), shape=(a.n, a.n))
    x = A.solve(b, rtol=1e-13)
    assert type(x.grad_fn).__name__ == "SolveFnBackward"
    assert all(f[0] is None or "AccumulateGrad" in type(f[0]).__name__ for f in x.grad_fn.next_functions)
    loss = 0.5 * ((x - t64(xs_np)) ** 2).sum()
    loss.backward()
    xo = orc.cg(a, b_np, precond="jacobi", rtol=1e-13).x
    gA_o, gb_o, _ = orc.adjoint(a, xo, xo - xs_np, precond="jacobi", rtol=1e-13)
    assert rel(vals.grad.cpu().numpy(), gA_o) <= 1e-6
    assert rel(b.grad.cpu().numpy(), gb_o) <= 1e-6


def test_workspace_growth_between_solves(orc):
    """Solves of increasing size on one handle grow its workspace each time;
    every solve must match the oracle (regression: the zero-fill of a grown
    workspace once ran unordered with the solve that followed)."""
    for m in (6, 10, 14, 18, 22, 26):
        a = W.diffusion3d(m, W.diffusion3d_kappa(m))
        b = W.rng(2, 1, m).standard_normal(a.n)
        x, info, st = solve(a, b, precond="jacobi", rtol=1e-12)
        ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
        assert st == 0 and rel(x, ref.x) <= 1e-8 and iters_close(info[0]["iters"], ref.iters)


def test_torch_allocator_and_workspace_size(orc):
    """Workspaces come from torch's caching allocator once it is set, and a
    reservation of hsla_workspace_size bytes covers the solve that follows
    (no further allocation)."""
    m = 20
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    b = W.rng(2, 1).standard_normal(a.n)
    pat = pattern(a)
    cnt = {}
    _lib.use_torch_allocator(dev(), counter=cnt)
    try:
        for persistent in (False, True):
            opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-12, persistent=persistent)
            need = _lib.workspace_size(pat, 3, opts)
            _lib.reserve(need, dev())
            allocs = cnt.get("alloc", 0)
            assert allocs >= 1
            x, infos, st = _lib.solve(pat, t64(np.stack([a.val] * 3)), t64(np.stack([b] * 3)), opts)
            assert st == 0 and cnt["alloc"] == allocs
            ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
            assert rel(x[0].cpu().numpy(), ref.x) <= 1e-8
    finally:
        _lib.use_torch_allocator(dev(), enable=False)
    assert cnt.get("free", 0) >= 1


def test_backward_memory_flat_in_iterations():
    """The autograd node keeps only (values, x): device memory of forward +
    backward does not grow with the number of CG iterations.  2D Poisson
    N = 640,000 (800^2), plain CG forced to k iterations, all workspaces
    drawn from torch's allocator so that they are counted."""
    import paper_2601_13994_amd as hs

    a = W.poisson2d(800)
    b = np.random.default_rng(3).standard_normal(a.n)
    rp, col = t32(a.row_ptr), t32(a.col)
    pat = hs.SparseCSR(t64(a.val), rp, col).pattern
    _lib.use_torch_allocator(dev())
    try:
        peaks = []
        for k in (10, 10, 100, 1000):  # the first run sizes the workspaces
            vals = t64(a.val).requires_grad_()
            bt = t64(b).requires_grad_()
            A = hs.SparseCSR(vals, rp, col, pattern=pat)
            torch.cuda.synchronize()
            torch.cuda.reset_peak_memory_stats()
            base = torch.cuda.memory_allocated()
            with pytest.warns(RuntimeWarning):
                x = A.solve(bt, rtol=0.0, max_iter=k, method="cg", precond="none", allow_unconverged=True)
                (x * x).sum().backward()
            torch.cuda.synchronize()
            peaks.append(torch.cuda.max_memory_allocated() - base)
            assert vals.grad is not None and bt.grad is not None
        peaks = peaks[1:]
        assert max(peaks) <= min(peaks) * 1.01 + (1 << 20), peaks
    finally:
        _lib.use_torch_allocator(dev(), enable=False)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_persistent_single_reduction(orc, precond):
    """CG_SR in the general persistent kernel (shared-pattern mode, one
    workgroup per system, one reduction per iteration): sampled systems
    match the oracle's CG, the k-th iterate at a cap, breakdown, b = 0."""
    m = 20
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    B = 300
    r = np.random.default_rng(9)
    V = np.stack([a.val] * B)
    V[5] = -a.val  # not SPD: breakdown (Jacobi: negative diagonal)
    bs = r.standard_normal((B, a.n))
    bs[7] = 0.0
    pat = pattern(a)
    kw = dict(method="cg_sr", precond=precond, rtol=1e-12)
    x, inf, st = _lib.solve(pat, t64(V), t64(bs), _lib.make_opts(**kw))
    assert st == _lib.BREAKDOWN
    assert all(f["spmv_form"] == "persistent" and f["method"] == "cg_sr" for f in inf)
    assert inf[5]["status"] == _lib.BREAKDOWN
    assert inf[7]["status"] == 0 and inf[7]["iters"] == 0 and not x[7].any()
    for s in (0, 150, 299):
        ref = orc.cg(a, bs[s], precond=precond, rtol=1e-12)
        assert inf[s]["status"] == 0
        assert rel(x[s].cpu().numpy(), ref.x) <= 1e-8
        assert iters_close(inf[s]["iters"], ref.iters), (inf[s]["iters"], ref.iters)
    for k in (1, 2, 7):
        xk, ik, sk = _lib.solve(pat, t64(V), t64(bs), _lib.make_opts(max_iter=k, **kw))
        refk = orc.cg(a, bs[0], precond=precond, rtol=1e-12, max_iter=k)
        assert ik[0]["status"] == _lib.NOT_CONVERGED and ik[0]["iters"] == k
        assert rel(xk[0].cpu().numpy(), refk.x) <= 1e-10, (k, rel(xk[0].cpu().numpy(), refk.x))


def test_persistent_shared_mode_batch(orc):
    """A batch with one system per compute unit and more runs the general
    persistent kernel in shared-pattern mode (n > 4096): sampled systems
    match the oracle and the per-iteration kernels."""
    m = 24
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    B = 320
    r = np.random.default_rng(8)
    V = np.stack([a.val] * B)
    bs = r.standard_normal((B, a.n))
    pat = pattern(a)
    x1, i1, s1 = _lib.solve(pat, t64(V), t64(bs), _lib.make_opts(method="cg", precond="jacobi", rtol=1e-12))
    x2, i2, s2 = _lib.solve(pat, t64(V), t64(bs),
                            _lib.make_opts(method="cg", precond="jacobi", rtol=1e-12, persistent=False))
    assert s1 == s2 == 0
    assert all(f["spmv_launches"] == 0 for f in i1)
    for s in (0, 157, 319):
        ref = orc.cg(a, bs[s], precond="jacobi", rtol=1e-12)
        assert rel(x1[s].cpu().numpy(), ref.x) <= 1e-8
        assert rel(x2[s].cpu().numpy(), ref.x) <= 1e-8
        assert iters_close(i1[s]["iters"], ref.iters)


@pytest.mark.parametrize("name,make", [
    ("poisson64", lambda: W.poisson2d(64)),                 # matrix in registers, 8 rows per thread
    ("poisson30", lambda: W.poisson2d(30)),                 # in registers, 2 rows per thread
    ("poisson40", lambda: W.poisson2d(40)),                 # in registers, 4 rows per thread
    ("aniso9", lambda: W.aniso2d(60, 50.0, 0.6)),           # 9 entries per row: matrix streamed, K = 16
    ("diff15", lambda: W.diffusion3d(15, W.diffusion3d_kappa(15))),  # n = 3375, 7 entries: streamed, K = 8
])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_cg_single_reduction_parity(orc, name, make, precond):
    """CG_SR (the Chronopoulos-Gear recurrence in the small-system kernels)
    against the oracle's Algorithm-1 CG: same solution, iteration counts
    within max(2, 2%), reported as CG_SR; capped and singular cases."""
    a = make()
    b = np.random.default_rng(13).standard_normal(a.n)
    x, info, st = solve(a, b, method="cg_sr", precond=precond, rtol=1e-12)
    ref = orc.cg(a, b, precond=precond, rtol=1e-12)
    assert st == 0 and info[0]["method"] == "cg_sr"
    assert rel(x, ref.x) <= 1e-8
    assert iters_close(info[0]["iters"], ref.iters), (info[0]["iters"], ref.iters)
    assert info[0]["true_residual"] <= 5e-12
    pat = pattern(a)
    x, info, st = solve(a, b, pat=pat, method="cg_sr", precond=precond, rtol=1e-12, max_iter=3)
    ref3 = orc.cg(a, b, precond=precond, rtol=1e-12, max_iter=3)
    assert st == _lib.NOT_CONVERGED and info[0]["iters"] == 3 and rel(x, ref3.x) <= 1e-12
    x, info, st = solve(a, b, pat=pat, values=t64(-a.val), method="cg_sr", precond=precond)
    assert st == _lib.BREAKDOWN
    x, info, st = solve(a, np.zeros(a.n), pat=pat, method="cg_sr", precond=precond)
    assert st == 0 and info[0]["iters"] == 0 and not x.any()


@pytest.mark.parametrize("fmt", ["auto", "csr"])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_cg_single_reduction_per_iteration(orc, fmt, precond):
    """CG_SR on the per-iteration kernels (w = A r with r.r and w.r in one
    launch, one finalize, one vector sweep) in the diagonal-major and tile
    forms: the oracle's CG solution, iteration counts within max(2, 2%),
    graph replay bitwise equal to plain launches, a batch member bitwise
    equal to its own solve, the k-th iterate at a cap, breakdown and b = 0."""
    m = 20
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    r = np.random.default_rng(14)
    b = r.standard_normal(a.n)
    pat = pattern(a)
    pat.set_format(fmt)
    kw = dict(method="cg_sr", precond=precond, rtol=1e-12, persistent=False)
    # leave NaN in the work vectors first: a CG solve whose SpMV meets a NaN
    # value stops as non-finite after writing q = A p
    bad = a.val.copy()
    bad[1] = np.nan
    with pytest.raises(_lib.HslaError):
        solve(a, b, pat=pat, values=t64(bad), method="cg", precond="none", persistent=False)
    x, info, st = solve(a, b, pat=pat, **kw)
    ref = orc.cg(a, b, precond=precond, rtol=1e-12)
    assert st == 0 and info[0]["method"] == "cg_sr", info
    assert info[0]["spmv_form"] != "persistent"
    assert rel(x, ref.x) <= 1e-8
    assert iters_close(info[0]["iters"], ref.iters), (info[0]["iters"], ref.iters)
    assert info[0]["true_residual"] <= 5e-12
    xg, _, _ = solve(a, b, pat=pat, graph=False, **kw)
    assert np.array_equal(x, xg)
    # a batch: each member is its own solve
    V = np.stack([a.val, W.diffusion3d_values(m, W.diffusion3d_kappa(m, sample=1)), a.val])
    bs = np.stack([r.standard_normal(a.n), b, b])
    xb, ib, sb = _lib.solve(pat, t64(V), t64(bs), _lib.make_opts(**kw))
    assert sb == 0 and np.array_equal(xb[2].cpu().numpy(), x)
    ref1 = orc.cg(a.with_values(V[1]), b, precond=precond, rtol=1e-12)
    assert rel(xb[1].cpu().numpy(), ref1.x) <= 1e-8 and iters_close(ib[1]["iters"], ref1.iters)
    # the k-th iterate of a capped run is CG's k-th iterate
    for k in (1, 2, 7):
        xk, ik, sk = solve(a, b, pat=pat, **dict(kw, max_iter=k))
        refk = orc.cg(a, b, precond=precond, rtol=1e-12, max_iter=k)
        assert sk == _lib.NOT_CONVERGED and ik[0]["iters"] == k and rel(xk, refk.x) <= 1e-10, (k, rel(xk, refk.x))
    _, _, st = solve(a, b, pat=pat, values=t64(-a.val), **dict(kw, precond="none"))
    assert st == _lib.BREAKDOWN
    x0, i0, st = solve(a, np.zeros(a.n), pat=pat, **kw)
    assert st == 0 and i0[0]["iters"] == 0 and not x0.any()


@pytest.mark.parametrize("s", [2, 3, 4])
@pytest.mark.parametrize("fmt", ["auto", "csr"])
def test_sstep_cg(orc, s, fmt):
    """s-step CG (Chebyshev basis on [0, 2], one Gram reduction per s inner
    steps) on the per-iteration kernels, diagonal-major and tile forms:
    against the s-step oracle the solution at rtol 1e-10 and the iteration
    count (within max(2, 2%)), against the oracle's Jacobi-PCG the solution,
    the k-th iterate at k = s (an outer boundary) and s + 1 (inside an outer
    step), graph replay bitwise equal to plain launches, a batch member
    bitwise equal to its own solve, b = 0, and the rejected options."""
    from oracle import sstep
    m = 20
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    r = np.random.default_rng(21)
    b = r.standard_normal(a.n)
    pat = pattern(a)
    pat.set_format(fmt)
    kw = dict(method="cg_sstep", precond="jacobi", s_step=s, persistent=False)
    try:
        x, info, st = solve(a, b, pat=pat, rtol=1e-10, **kw)
        ref = sstep.sstep_cg(a, b, s=s, precond="jacobi", rtol=1e-10)
        assert st == 0 and info[0]["method"] == "cg_sstep", info[0]
        assert rel(x, ref.x) <= 1e-9
        assert iters_close(info[0]["iters"], ref.iters), (info[0]["iters"], ref.iters)
        assert info[0]["true_residual"] <= 2e-10
        pcg = orc.cg(a, b, precond="jacobi", rtol=1e-10)
        assert rel(x, pcg.x) <= 1e-8
        xg, _, _ = solve(a, b, pat=pat, rtol=1e-10, graph=False, **kw)
        assert np.array_equal(x, xg)
        for k in (s, s + 1):
            xk, ik, sk = solve(a, b, pat=pat, rtol=1e-14, max_iter=k, **kw)
            refk = sstep.sstep_cg(a, b, s=s, precond="jacobi", rtol=1e-14, max_iter=k)
            assert sk == _lib.NOT_CONVERGED and ik[0]["iters"] == k
            assert rel(xk, refk.x) <= 1e-11, (k, rel(xk, refk.x))
        V = np.stack([a.val, W.diffusion3d_values(m, W.diffusion3d_kappa(m, sample=1)), a.val])
        bs = np.stack([r.standard_normal(a.n), b, b])
        xb, ib, sb = _lib.solve(pat, t64(V), t64(bs), _lib.make_opts(rtol=1e-10, **kw))
        assert sb == 0 and np.array_equal(xb[2].cpu().numpy(), x)
        ref1 = sstep.sstep_cg(a.with_values(V[1]), b, s=s, precond="jacobi", rtol=1e-10)
        assert rel(xb[1].cpu().numpy(), ref1.x) <= 1e-9
        x0, i0, st0 = solve(a, np.zeros(a.n), pat=pat, **kw)
        assert st0 == 0 and i0[0]["iters"] == 0 and not x0.any()
    finally:
        pat.set_format("auto")
    with pytest.raises(_lib.HslaError):
        solve(a, b, pat=pat, **dict(kw, precond="none"))
    with pytest.raises(_lib.HslaError):
        solve(a, b, pat=pat, **dict(kw, s_step=5))


def test_cg_single_reduction_fsai_runs_cg(orc):
    """FSAI preconditioning keeps the two-reduction recurrence and says so."""
    from oracle import mpnn
    pa, slots = W.aniso_pattern(21)
    a = pa.with_values(W.aniso_stencil(100.0, 0.4)[slots])
    rpL, colL, gh = orc.fsai(mpnn.scaled(a))
    pat = pattern(a)
    G, GT = _lib.fsai_factors(pat, t64(a.val), torch.as_tensor(gh.astype(np.float32)).to(dev()))
    b = np.random.default_rng(15).standard_normal(a.n)
    x, info, st = _lib.solve(pat, t64(a.val), t64(b),
                             _lib.make_opts(method="cg_sr", precond="fsai", rtol=1e-12, G=G, GT=GT))
    assert st == 0 and info[0]["method"] == "cg"
    ref = orc.fsai_pcg(a, rpL, colL, G.cpu().numpy().astype(np.float64), b, rtol=1e-12)
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8


def _random_csr(n, density, seed):
    rp, col = W.random_pattern(n, density, np.random.default_rng(seed))
    return W.Csr(n, rp, col, np.ones(len(col)))


@pytest.mark.parametrize("make", [lambda: W.poisson2d(17), lambda: W.diffusion3d(9), lambda: _random_csr(500, 0.02, 3)])
def test_pattern_colors_separate_columns_sharing_a_row(make):
    """hsla_pattern_colors: no two columns stored in the same row share a
    color, and the greedy coloring uses at least the longest row's length
    and few colors on stencils."""
    a = make()
    pat = pattern(a)
    color, nc = pat.colors()
    color = color.cpu().numpy()
    assert color.shape == (a.n,) and color.min() >= 0 and color.max() == nc - 1
    for i in range(a.n):
        cs = color[a.col[a.row_ptr[i]:a.row_ptr[i + 1]]]
        assert len(set(cs.tolist())) == len(cs)
    longest = int(np.diff(a.row_ptr).max())
    assert nc >= longest
    if a.n in (17 * 17, 9 ** 3):
        assert nc <= 2 * longest
