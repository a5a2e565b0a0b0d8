"""The FP64 true residual ||b - A x||_2 (and ||b||_2) on the GPU against the
oracle on the same seeded inputs, single and batched, on the stencil and CSR
forms; and the true residual every solver path reports against it."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import pattern, t32, t64  # noqa: E402
import paper_2601_13994_amd as hs  # noqa: E402
from paper_2601_13994_amd import _lib  # noqa: E402


def _close(u, v, tol=1e-12):
    return abs(u - v) <= tol * max(abs(v), 1e-300)


def _cases():
    return [("poisson2d_40", W.poisson2d(40)),
            ("diffusion3d_12", W.diffusion3d(12, W.diffusion3d_kappa(12))),
            ("random_spd", W.random_spd(2000, 0.004, np.random.default_rng(31)))]


@pytest.mark.parametrize("fmt", ["auto", "csr"])
def test_residual_norms_vs_oracle(orc, fmt):
    """Random x (no cancellation) and the oracle's converged x (the residual
    is a cancellation of nearly equal terms): each row's b_i - (Ax)_i has the
    same bits on both sides (ascending-order row sums), so the norms differ
    only by the order of the sum of squares."""
    for name, a in _cases():
        r = np.random.default_rng(5)
        b = r.standard_normal(a.n)
        xr = r.standard_normal(a.n)
        xs = orc.solve(a, b, precond="jacobi", rtol=1e-12).x
        pat = pattern(a)
        pat.set_format(fmt)
        for x in (xr, xs):
            rn, bn = _lib.residual_norms(pat, t64(a.val), t64(b), t64(x))
            assert _close(rn[0], orc.residual_norm(a, b, x)), (name, rn[0], orc.residual_norm(a, b, x))
            assert _close(bn[0], np.sqrt(orc.dot(b, b)))
        # batched: three value sets, right-hand sides and iterates
        V = np.stack([a.val * s for s in (1.0, 0.5, 3.0)])
        Bm = r.standard_normal((3, a.n))
        X = r.standard_normal((3, a.n))
        rn, bn = _lib.residual_norms(pat, t64(V), t64(Bm), t64(X))
        for s in range(3):
            want = orc.residual_norm(a.with_values(V[s]), Bm[s], X[s])
            assert _close(rn[s], want), (name, s)
            assert _close(bn[s], np.sqrt(orc.dot(Bm[s], Bm[s])))


@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_reported_true_residual(persistent, method):
    """hsla_info.true_residual (computed by each solver path: persistent
    small-system kernel, per-iteration kernels, batched) equals
    ||b - A x|| / ||b|| from hsla_residual_norms on the returned x."""
    for name, a in _cases():
        r = np.random.default_rng(7)
        pat = pattern(a)
        b = r.standard_normal(a.n)
        x, infos, st = _lib.solve(pat, t64(a.val), t64(b),
                                  _lib.make_opts(method=method, rtol=1e-12, persistent=persistent))
        assert st == _lib.OK
        rn, bn = _lib.residual_norms(pat, t64(a.val), t64(b), x)
        assert _close(infos[0]["true_residual"], rn[0] / bn[0], 1e-10), (name, infos[0]["true_residual"], rn[0] / bn[0])
        V = np.stack([a.val * s for s in (1.0, 2.0)] * 40)
        Bm = r.standard_normal((80, a.n))
        X, infos, st = _lib.solve(pat, t64(V), t64(Bm), _lib.make_opts(method=method, rtol=1e-12, persistent=persistent))
        assert st == _lib.OK
        rn, bn = _lib.residual_norms(pat, t64(V), t64(Bm), X)
        for s in (0, 41, 79):
            assert _close(infos[s]["true_residual"], rn[s] / bn[s], 1e-10), (name, s)


@pytest.mark.parametrize("persistent", [True, False])
def test_ragged_true_residual(persistent):
    """The ragged paths' reported true residual against hsla_residual_norms
    of each system on its own pattern."""
    systems = [W.knn_system(s, n_lo=300, n_hi=3000) for s in range(5)]
    L = hs.SparseCSRList([(t64(a.val), t32(a.row_ptr), t32(a.col)) for a, _ in systems])
    xs, infos, st = L.solve([t64(b) for _, b in systems], rtol=1e-12, persistent=persistent)
    assert st == _lib.OK
    for (a, b), x, f in zip(systems, xs, infos):
        rn, bn = _lib.residual_norms(pattern(a), t64(a.val), t64(b), x)
        assert _close(f["true_residual"], rn[0] / bn[0], 1e-10), (f["true_residual"], rn[0] / bn[0])
