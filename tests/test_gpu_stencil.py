"""The offset-mask forms of structured-grid patterns: detection, fallback to
CSR, bitwise equal SpMV in every form (mask tiles, diagonal-major copy,
CSR), and solves in the diagonal-major form (CG, BiCGStab, the
nonsymmetric adjoint on A^T, FSAI-PCG) against the CSR form and the
oracle.  Solves compare to rounding: their dot products are reduced in an
order that depends on each form's grid."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, iters_close, pattern, rel, t64  # noqa: E402
from paper_2601_13994_amd import _lib  # noqa: E402
from oracle import mpnn  # noqa: E402


def _both(pat, fn):
    """fn() with the offset-mask forms in use, then with CSR."""
    pat.set_format("auto")
    a = fn()
    pat.set_format("csr")
    try:
        b = fn()
    finally:
        pat.set_format("auto")
    return a, b


@pytest.mark.parametrize("name,make,nofs", [
    ("poisson2d", lambda: W.poisson2d(37), 5),
    ("diffusion3d", lambda: W.diffusion3d(13, W.diffusion3d_kappa(13)), 7),
    ("aniso9", lambda: W.aniso2d(29, 30.0, 0.7), 9),
    ("upwind", lambda: W.diffusion3d(11, W.diffusion3d_kappa(11), velocity=10.0), 7),
    # even n: the diagonal-major copy runs two adjacent rows per thread
    ("poisson2d_even", lambda: W.poisson2d(38), 5),
    ("diffusion3d_even", lambda: W.diffusion3d(14, W.diffusion3d_kappa(14)), 7),
    ("upwind_even", lambda: W.diffusion3d(12, W.diffusion3d_kappa(12), velocity=10.0), 7),
    # odd offsets m - 1, m + 1 with even n
    ("aniso9_even", lambda: W.aniso2d(30, 30.0, 0.7), 9),
])
def test_stencil_spmv_bitwise(orc, name, make, nofs):
    a = make()
    pat = pattern(a)
    assert pat.stencil == (True, nofs)
    r = np.random.default_rng(1)
    B = 3
    V = np.stack([a.val * (1 + 0.1 * r.standard_normal(a.nnz)) for _ in range(B)])
    X = r.standard_normal((B, a.n))
    ys = {}
    for fmt in ("auto", "diagonal", "csr"):
        pat.set_format(fmt)
        ys[fmt] = _lib.spmv(pat, t64(V), t64(X)).cpu().numpy()
    pat.set_format("auto")
    assert np.array_equal(ys["auto"], ys["csr"]) and np.array_equal(ys["diagonal"], ys["csr"])
    for s in range(B):
        assert np.array_equal(ys["csr"][s], orc.spmv(a.with_values(V[s]), X[s]))


def test_stencil_detection_falls_back(orc):
    # a random pattern has far more than 16 diagonals
    a = W.random_spd(500, 0.02, np.random.default_rng(3))
    assert pattern(a).stencil == (False, 0)
    # a 2D stencil plus one entry on a diagonal that no sampled row has: the
    # device check over all rows rejects the candidate set
    m = 100
    p = W.poisson2d(m)
    r2 = np.concatenate([p.rows(), [2500]])
    c2 = np.concatenate([p.col, [2537]])
    o = np.lexsort((c2, r2))
    r2, c2 = r2[o], c2[o]
    rp = np.zeros(m * m + 1, np.int64)
    np.cumsum(np.bincount(r2, minlength=m * m), out=rp[1:])
    q = W.Csr(m * m, rp.astype(np.int32), c2.astype(np.int32),
              np.random.default_rng(1).standard_normal(len(c2)))
    pat = pattern(q)
    assert pat.stencil == (False, 0)
    x = np.random.default_rng(0).standard_normal(q.n)
    assert np.array_equal(_lib.spmv(pat, t64(q.val), t64(x)).cpu().numpy(), orc.spmv(q, x))
    # the same matrix without the extra entry is a 5-diagonal stencil
    assert pattern(p).stencil == (True, 5)


def _close(r1, r2, cg=True):
    """Two solves of the same systems that differ only in the order their dot
    products are reduced.  CG iteration counts agree to max(2, 2%); those of
    BiCGStab, whose residual is erratic near the FP64 floor, are not compared
    (its iterates are not pinned), only the solutions."""
    (x1, i1, s1), (x2, i2, s2) = r1, r2
    assert s1 == s2 == 0
    assert rel(x1.cpu().numpy(), x2.cpu().numpy()) <= 1e-10
    if cg:
        assert all(iters_close(f["iters"], g["iters"]) for f, g in zip(i1, i2)), \
            [(f["iters"], g["iters"]) for f, g in zip(i1, i2)]


@pytest.mark.parametrize("method,precond", [("cg", "jacobi"), ("cg", "none"), ("bicgstab", "jacobi")])
def test_stencil_solves(orc, method, precond):
    """Per-iteration kernels (persistent launch off) on the diagonal-major
    copy vs on CSR tiles, a batch of 3, and the oracle."""
    m = 14
    conv = 10.0 if method == "bicgstab" else 0.0
    a = W.diffusion3d(m, W.diffusion3d_kappa(m), velocity=conv)
    r = np.random.default_rng(2)
    V = np.stack([a.val * (1 + 0.05 * r.random(a.nnz)) if s else a.val for s in range(3)])
    if method == "cg":
        V = np.stack([W.diffusion3d(m, np.exp(r.standard_normal(m ** 3))).val if s else a.val for s in range(3)])
    b = r.standard_normal((3, a.n))
    pat = pattern(a)
    opts = _lib.make_opts(method=method, precond=precond, rtol=1e-12, persistent=False)
    res = _both(pat, lambda: _lib.solve(pat, t64(V), t64(b), opts))
    _close(*res, cg=method == "cg")
    ref = orc.solve(a, b[0], method=method, precond=precond, rtol=1e-12)
    assert rel(res[0][0][0].cpu().numpy(), ref.x) <= 1e-8


def test_stencil_adjoint_transpose():
    """The nonsymmetric adjoint iterates on A^T's diagonal-major copy."""
    a = W.diffusion3d(12, W.diffusion3d_kappa(12), velocity=10.0)
    r = np.random.default_rng(4)
    x, gx = r.standard_normal(a.n), r.standard_normal(a.n)
    pat = pattern(a)
    opts = _lib.make_opts(method="bicgstab", precond="jacobi", rtol=1e-12)
    (g1, l1, i1, s1), (g2, l2, i2, s2) = _both(pat, lambda: _lib.adjoint(pat, t64(a.val), t64(x), t64(gx), opts))
    assert s1 == s2 == 0
    assert rel(l1.cpu().numpy(), l2.cpu().numpy()) <= 1e-10
    assert rel(g1.cpu().numpy(), g2.cpu().numpy()) <= 1e-10
    dense = np.linalg.solve(a.to_dense().T, gx)
    assert rel(l1.cpu().numpy(), dense) <= 1e-8


@pytest.mark.parametrize("m", [21, 22])
def test_stencil_fsai(orc, m):
    """FSAI-PCG with factors on the 9-point stencil's lower and upper
    triangles (main diagonal at one end), odd and even n, against the
    oracle with the same factor."""
    pa, slots = W.aniso_pattern(m)
    a = pa.with_values(W.aniso_stencil(100.0, 0.4)[slots])
    ah = mpnn.scaled(a)
    rpL, colL, gh = orc.fsai(ah)
    pat = pattern(a)
    G, GT = _lib.fsai_factors(pat, t64(a.val), torch.as_tensor(gh.astype(np.float32)).to(dev()))
    b = np.random.default_rng(5).standard_normal(a.n)
    opts = _lib.make_opts(method="cg", precond="fsai", rtol=1e-12, G=G, GT=GT)
    res = _both(pat, lambda: _lib.solve(pat, t64(a.val), t64(b), opts))
    _close(*res)
    ref = orc.fsai_pcg(a, rpL, colL, G.cpu().numpy().astype(np.float64), b, rtol=1e-12)
    assert rel(res[0][0].cpu().numpy(), ref.x) <= 1e-8


def test_autotune_choice_applies(orc):
    """The autotuner picks a measured configuration, and solves on the tuned
    pattern still match the oracle."""
    m = 24
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    pat = pattern(a)
    t = pat.autotune(B=2, effort=3)
    assert t["form"] in ("diagonal", "diagonal-half", "tiles") and t["blocks_per_cu"] in (1, 2, 3, 4, 8, 16, 32)
    assert 0 < t["best_us"] <= t["default_us"]
    b = np.random.default_rng(6).standard_normal(a.n)
    x, infos, st = _lib.solve(pat, t64(a.val), t64(b),
                              _lib.make_opts(method="cg", precond="jacobi", rtol=1e-12, persistent=False))
    ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    assert st == 0 and rel(x.cpu().numpy(), ref.x) <= 1e-8
    # a pattern without a stencil form is tuned among the row tiles only
    q = W.random_spd(400, 0.03, np.random.default_rng(7))
    assert pattern(q).autotune(B=1, effort=2)["form"] == "tiles"


def test_tuning_cache_across_patterns(tmp_path):
    """Signatures: equal patterns agree, a one-index change differs.  The
    autotuner's choice is stored in a JSON cache keyed by signature, batch
    size and device, and a second pattern object with the same indices (as
    in a later process) takes it from the file without timing; a record
    from another pattern is refused."""
    m = 16
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    p1, p2 = pattern(a), pattern(a)
    assert p1.signature == p2.signature != 0
    # the same n and nnz, one column index moved by one within its row
    c = a.col.copy()
    k = int(a.row_ptr[100])
    assert c[k] + 1 < c[k + 1]
    c[k] += 1
    assert pattern(W.Csr(a.n, a.row_ptr, c, a.val)).signature != p1.signature
    other = W.poisson2d(64)
    assert pattern(other).signature != p1.signature
    cache = str(tmp_path / "tune.json")
    t1 = p1.autotune(B=2, effort=2, cache=cache)
    assert t1["cached"] is False
    t2 = p2.autotune(B=2, effort=2, cache=cache)
    assert t2["cached"] is True
    assert p2.get_tuning() == p1.get_tuning() and p2.get_tuning()["tuned"] == 1
    assert p2.autotune(B=3, effort=2, cache=cache)["cached"] is False  # another batch size: timed
    q = pattern(other)
    with pytest.raises(_lib.HslaError):
        q.set_tuning(p1.get_tuning())
    bad = dict(p1.get_tuning(), dia_cu=0)
    with pytest.raises(_lib.HslaError):
        p1.set_tuning(bad)


def _grid7(nx, ny, nz, seed, keep=None):
    """7-point SPD operator on an nx x ny x nz grid with random face
    coefficients (bitwise symmetric values), optionally cut to its first
    `keep` unknowns (a partial last plane and a partial last row chunk)."""
    r = np.random.default_rng(seed)
    n = nx * ny * nz
    idx = np.arange(n)
    coord = (idx % nx, (idx // nx) % ny, idx // (nx * ny))
    rows, cols, vals = [], [], []
    diag = np.full(n, 0.1)
    for d, st, lim in ((0, 1, nx), (1, nx, ny), (2, nx * ny, nz)):
        i = idx[coord[d] < lim - 1]
        c = r.uniform(0.5, 2.0, i.size)
        rows += [i, i + st]
        cols += [i + st, i]
        vals += [-c, -c]
        np.add.at(diag, i, c)
        np.add.at(diag, i + st, c)
    rows = np.concatenate(rows + [idx])
    cols = np.concatenate(cols + [idx])
    vals = np.concatenate(vals + [diag])
    m = n if keep is None else keep
    k = (rows < m) & (cols < m)
    rows, cols, vals = rows[k], cols[k], vals[k]
    o = np.lexsort((cols, rows))
    rp = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    return W.Csr(m, rp.astype(np.int32), cols[o].astype(np.int32), vals[o])


@pytest.mark.parametrize("shape,keep", [((32, 32, 37), None), ((32, 32, 37), 37788), ((512, 20, 1), None),
                                        ((16, 32, 29), 14500), ((64, 64, 21), 85000), ((37, 41, 1), None),
                                        ((100, 30, 7), 20000), ((256, 16, 5), None), ((256, 16, 5), 18000),
                                        ((256, 12, 4), None)])
def test_half_form_spmv_bitwise(orc, shape, keep):
    """The symmetric half form (main + upper diagonals stored; pencil walk
    when the largest offset is a whole number of 512-row chunks, chunk walk
    otherwise) equals the CSR SpMV bit for bit; nonsymmetric values on the
    same pattern take the full copy, also bitwise."""
    a = _grid7(*shape, seed=11, keep=keep)
    pat = pattern(a)
    assert pat.stencil[0]
    r = np.random.default_rng(2)
    B = 3
    V = np.stack([a.val * (1.0 + s) for s in range(B)])  # still symmetric
    X = r.standard_normal((B, a.n))
    ys = {}
    for fmt in ("diagonal", "csr"):
        pat.set_format(fmt)
        ys[fmt] = _lib.spmv(pat, t64(V), t64(X)).cpu().numpy()
    assert np.array_equal(ys["diagonal"], ys["csr"])
    assert np.array_equal(ys["csr"][1], orc.spmv(a.with_values(V[1]), X[1]))
    Vn = V * (1 + 0.01 * r.standard_normal(V.shape))
    pat.set_format("diagonal")
    yd = _lib.spmv(pat, t64(Vn), t64(X)).cpu().numpy()
    pat.set_format("csr")
    yc = _lib.spmv(pat, t64(Vn), t64(X)).cpu().numpy()
    pat.set_format("auto")
    assert np.array_equal(yd, yc)


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_half_form_solves(orc, method):
    """Jacobi-PCG on symmetric values runs on the half form (reported in the
    info); right-Jacobi BiCGStab iterates on A D^{-1}, which is not
    symmetric, and takes the full copy.  Both agree with the CSR-form solve
    and the oracle; the adjoint on the same system too."""
    a = _grid7(32, 32, 37, seed=5, keep=37788)
    r = np.random.default_rng(8)
    V = np.stack([a.val, a.val * 1.5])
    b = r.standard_normal((2, a.n))
    pat = pattern(a)
    opts = _lib.make_opts(method=method, precond="jacobi", rtol=1e-12, persistent=False)
    res = _both(pat, lambda: _lib.solve(pat, t64(V), t64(b), opts))
    form = "diagonal-half-unit" if method == "cg" else "diagonal-unit"
    assert all(f["spmv_form"] == form for f in res[0][1])
    assert all(f["spmv_form"] == "tiles" for f in res[1][1])
    _close(*res, cg=method == "cg")
    ref = orc.solve(a, b[0], method=method, precond="jacobi", rtol=1e-12)
    assert rel(res[0][0][0].cpu().numpy(), ref.x) <= 1e-8
    if method == "cg":
        x = res[0][0]
        gx = t64(r.standard_normal((2, a.n)))
        gA, gb, bi, st = _lib.adjoint(pat, t64(V), x, gx, opts)
        assert st == _lib.OK and all(f["spmv_form"] == "diagonal-half-unit" for f in bi)
        gA_o, gb_o, _ = orc.adjoint(a, x[0].cpu().numpy(), gx[0].cpu().numpy(), method="cg", precond="jacobi",
                                    rtol=1e-12)
        assert rel(gb[0].cpu().numpy(), gb_o) <= 1e-8
        assert rel(gA[0].cpu().numpy(), gA_o) <= 1e-8


@pytest.mark.parametrize("fmt", ["auto", "csr"])
@pytest.mark.parametrize("precond", ["jacobi", "none", "fsai"])
def test_truncated_iterates_match_oracle(orc, fmt, precond):
    """Runs cut at k = 1, 2, 7 iterations (status NOT_CONVERGED) return the
    k-th iterate, x included (the direction kernel applies the stopping
    iteration's x += alpha p), in the half, full and tile forms."""
    m = 14
    a = W.diffusion3d(m, W.diffusion3d_kappa(m))
    b = np.random.default_rng(12).standard_normal(a.n)
    pat = pattern(a)
    pat.set_format(fmt)
    kw = {}
    if precond == "fsai":
        rpL, colL, gh = orc.fsai(mpnn.scaled(a))
        G, GT = _lib.fsai_factors(pat, t64(a.val), torch.as_tensor(gh.astype(np.float32)).to(dev()))
        kw = dict(G=G, GT=GT)
    try:
        for k in (1, 2, 7):
            opts = _lib.make_opts(method="cg", precond=precond, rtol=1e-14, max_iter=k, persistent=False, **kw)
            x, infos, st = _lib.solve(pat, t64(a.val), t64(b), opts)
            assert st == _lib.NOT_CONVERGED and infos[0]["iters"] == k
            if precond == "fsai":
                ref = orc.fsai_pcg(a, rpL, colL, G.cpu().numpy().astype(np.float64), b, rtol=1e-14, max_iter=k)
            else:
                ref = orc.cg(a, b, precond=precond, rtol=1e-14, max_iter=k)
            assert rel(x.cpu().numpy(), ref.x) <= 1e-12, (k, rel(x.cpu().numpy(), ref.x))
    finally:
        pat.set_format("auto")


@pytest.mark.parametrize("m,paired", [(14, True), (13, False)])
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_paired_layout(orc, m, paired, method):
    """A 7-point grid with even n runs the diagonal forms two adjacent rows
    per thread without row masks (hsla_info.spmv_paired), odd n two rows
    256 apart with masks; both match the oracle, and CG's truncated iterate
    too."""
    a = W.diffusion3d(m, W.diffusion3d_kappa(m), velocity=10.0 if method == "bicgstab" else 0.0)
    b = np.random.default_rng(m).standard_normal(a.n)
    pat = pattern(a)
    opts = _lib.make_opts(method=method, precond="jacobi", rtol=1e-12, persistent=False)
    x, infos, st = _lib.solve(pat, t64(a.val), t64(b), opts)
    assert st == _lib.OK and infos[0]["spmv_paired"] is paired
    assert infos[0]["spmv_form"] == ("diagonal-half-unit" if method == "cg" else "diagonal-unit")
    ref = orc.solve(a, b, method=method, precond="jacobi", rtol=1e-12)
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    if method == "cg":
        assert iters_close(infos[0]["iters"], ref.iters)
        k = 7
        opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-14, max_iter=k, persistent=False)
        xk, fk, st = _lib.solve(pat, t64(a.val), t64(b), opts)
        refk = orc.cg(a, b, precond="jacobi", rtol=1e-14, max_iter=k)
        assert st == _lib.NOT_CONVERGED and fk[0]["iters"] == k
        assert rel(xk.cpu().numpy(), refk.x) <= 1e-12


@pytest.mark.parametrize("m", [30, 29])
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_odd_offset_stencil(orc, m, method):
    """The 9-point anisotropic stencil (offsets -m-1 .. m+1, odd ones beyond
    -1/+1) keeps the two-rows-256-apart layout with row masks for even and
    odd n (half copy of S A S for CG, full copy of A D^{-1} for BiCGStab);
    the half-form SpMV is bitwise the CSR one; solves and CG's truncated
    iterate match the oracle."""
    paired = False
    a = W.aniso2d(m, 50.0, 0.6)
    pat = pattern(a)
    assert pat.stencil == (True, 9)
    r = np.random.default_rng(m)
    X = r.standard_normal((2, a.n))
    V = np.stack([a.val, 2.0 * a.val])  # symmetric: the half form
    ys = {}
    for fmt in ("diagonal", "csr"):
        pat.set_format(fmt)
        ys[fmt] = _lib.spmv(pat, t64(V), t64(X)).cpu().numpy()
    pat.set_format("auto")
    assert np.array_equal(ys["diagonal"], ys["csr"])
    b = r.standard_normal(a.n)
    if method == "bicgstab":
        a = a.with_values(a.val * (1 + 0.05 * r.standard_normal(a.nnz)))
    opts = _lib.make_opts(method=method, precond="jacobi", rtol=1e-12, persistent=False)
    x, infos, st = _lib.solve(pat, t64(a.val), t64(b), opts)
    assert st == _lib.OK and infos[0]["spmv_paired"] is paired
    assert infos[0]["spmv_form"] == ("diagonal-half-unit" if method == "cg" else "diagonal-unit")
    ref = orc.solve(a, b, method=method, precond="jacobi", rtol=1e-12)
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    if method == "cg":
        assert iters_close(infos[0]["iters"], ref.iters)
        for k in (1, 7):
            opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-14, max_iter=k, persistent=False)
            xk, fk, st = _lib.solve(pat, t64(a.val), t64(b), opts)
            refk = orc.cg(a, b, precond="jacobi", rtol=1e-14, max_iter=k)
            assert st == _lib.NOT_CONVERGED and fk[0]["iters"] == k
            assert rel(xk.cpu().numpy(), refk.x) <= 1e-12
