"""GPU parity of the ragged persistent batch against the CPU oracle."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, iters_close, rel, t32, t64  # noqa: E402
import paper_2601_13994_amd as hs  # noqa: E402
from paper_2601_13994_amd import _lib  # noqa: E402


def _knn(sample, lo, hi):
    return W.knn_system(sample, n_lo=lo, n_hi=hi)


def test_ragged_knn_parity(orc):
    """k-NN Laplacians of different sizes, a zero right-hand side and an
    empty system: each result matches the oracle's CG and does not depend on
    the batch (bitwise equal when solved alone)."""
    systems = [_knn(s, 100, 3000) for s in range(9)]
    systems[4] = (systems[4][0], np.zeros(systems[4][0].n))
    empty = W.Csr(0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0))
    systems.insert(6, (empty, np.zeros(0)))
    mats = [(t64(a.val), t32(a.row_ptr), t32(a.col)) for a, _ in systems]
    L = hs.SparseCSRList(mats)
    xs, infos, st = L.solve([t64(b) for _, b in systems], rtol=1e-12)
    assert st == 0
    for (a, b), x, f in zip(systems, xs, infos):
        if a.n == 0:
            assert f["status"] == 0 and x.numel() == 0
            continue
        ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
        if not b.any():
            assert f["iters"] == 0 and not x.cpu().numpy().any()
            continue
        assert rel(x.cpu().numpy(), ref.x) <= 1e-8
        assert iters_close(f["iters"], ref.iters)
        assert f["true_residual"] <= 2e-12
    # alone vs in the batch: bitwise equal
    a, b = systems[2]
    alone = hs.SparseCSRList([(t64(a.val), t32(a.row_ptr), t32(a.col))])
    x1, _, _ = alone.solve([t64(b)], rtol=1e-12)
    assert torch.equal(x1[0], xs[2])
    # run to run: bitwise equal
    xs2, _, _ = L.solve([t64(b) for _, b in systems], rtol=1e-12)
    assert all(torch.equal(u, v) for u, v in zip(xs, xs2))


def test_ragged_rejects_invalid_system():
    a, b = _knn(0, 100, 200)
    c = a.col.copy()
    c[3], c[4] = c[4], c[3]
    good = (t64(a.val), t32(a.row_ptr), t32(a.col))
    badm = (t64(a.val), t32(a.row_ptr), t32(c))
    L = hs.SparseCSRList([good, badm])
    with pytest.raises(_lib.HslaError) as e:
        L.solve([t64(b), t64(b)])
    assert e.value.status == _lib.ERR_INVALID_CSR and "system 1" in str(e.value)


def test_ragged_status_codes():
    a, b = _knn(1, 200, 300)
    L = hs.SparseCSRList([(t64(a.val), t32(a.row_ptr), t32(a.col))])
    _, infos, st = L.solve([t64(b)], max_iter=2)
    assert st == _lib.NOT_CONVERGED and infos[0]["iters"] == 2
    L2 = hs.SparseCSRList([(t64(-a.val), t32(a.row_ptr), t32(a.col))])
    _, infos, st = L2.solve([t64(b)])
    assert st == _lib.BREAKDOWN
