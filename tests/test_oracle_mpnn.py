"""Pins of the FP64 preconditioner-network reference (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import mpnn


def _sys(m=5, ratio=30.0, angle=0.7):
    return W.aniso2d(m, ratio, angle)


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(20000) * np.logspace(-30, 30, 20000)
    x[:3] = [0.0, -0.0, 1.0]
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mpnn.bf16(x), ref)


def test_closed_form_head_only():
    """All matrices zero: every off-diagonal value is c2, every diagonal softplus(c2)."""
    a = _sys()
    p = {k: np.zeros_like(v) for k, v in mpnn.init_params(0).items()}
    p["c2"] = np.array([0.3])
    g, _ = mpnn.forward(p, a)
    rows, col, _, _, lower = mpnn.graph(a)
    diag = col[lower] == rows[lower]
    assert np.allclose(g[diag], np.log1p(np.exp(0.3)), rtol=1e-15)
    assert np.all(g[~diag] == 0.3)


def test_graph_scaling_unit_diagonal():
    a = _sys()
    rows, col, ah, f, lower = mpnn.graph(a)
    assert np.allclose(ah[rows == col], 1.0)
    d = a.to_dense()
    dd = np.sqrt(np.diag(d))
    assert np.allclose(mpnn.scaled(a).to_dense(), d / np.outer(dd, dd), rtol=1e-14)
    assert len(lower) == int(np.sum(a.col <= rows))


@pytest.mark.parametrize("name", mpnn.MATS + ["b0", "b1", "b3", "c1", "c2"])
def test_backward_vs_finite_differences(name):
    a = _sys(m=4)
    p = mpnn.init_params(3)
    for k in p:
        if k.startswith(("b", "c")):
            p[k] = np.random.default_rng(7).standard_normal(p[k].shape) * 0.1
    g, cache = mpnn.forward(p, a)
    dg = np.random.default_rng(1).standard_normal(g.shape)
    grads = mpnn.backward(cache, dg)
    r = np.random.default_rng(2)
    flat = p[name].reshape(-1)
    for idx in r.choice(flat.size, min(6, flat.size), replace=False):
        h = 1e-6
        old = flat[idx]
        flat[idx] = old + h
        gp, _ = mpnn.forward(p, a)
        flat[idx] = old - h
        gm, _ = mpnn.forward(p, a)
        flat[idx] = old
        fd = (dg @ gp - dg @ gm) / (2 * h)
        an = grads[name].reshape(-1)[idx]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)


def test_bf16_forward_close_to_fp64():
    a = _sys(m=6)
    p = mpnn.init_params(1)
    g64, _ = mpnn.forward(p, a, bf=False)
    g16, _ = mpnn.forward(p, a, bf=True)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)
